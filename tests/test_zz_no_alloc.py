"""The allocation-free FP32 prediction entry point (ds_predict_f32_noalloc) against
ds_predict in DS_PREC_F32 on the same points: two calls in a row, the second with a
smaller input, through the C ABI."""
import numpy as np
import pytest
import torch

import paper_1709_05418_amd as ds
from paper_1709_05418_amd import synth
from _util import Workload, rel_l2

pytestmark = pytest.mark.gpu


def test_noalloc_prediction_matches_ds_predict():
    # K = 10, W = 200: chunks of 2880 points, so 7000 points span three chunks and a tail
    w = Workload(48, 48.0, L=7, K=10, P=7000, seed_cloud=9, seed_pts=90)
    ctx = ds.Context(0)
    cloud = ds.Cloud(ctx, w.density.cuda(), w.sigma_max, w.aabb_min, w.h0, w.L, w.K, w.mips)
    net = ds.Net(ctx, w.K, 200, 3)
    net.set_params(synth.init_params(w.K, 200, 3, 17, branch_scale=0.3, out_scale=0.2,
                                     out_bias=0.5))
    try:
        pos, view, light = w.cuda_inputs()
        view[5] = 0.0  # an invalid point
        # before the cloud's float32 cells exist the call refuses (building them allocates)
        with pytest.raises(ds.DSError):
            ds.ds_predict_f32_noalloc(ctx.h, cloud.h, net.h, pos[:64], view[:64], light[:64])
        ds.ds_predict_reserve(ctx.h, cloud.h, net.h, ds.DS_PREC_F32, w.P)
        for n in (w.P, 1000):  # two calls in a row, the second smaller
            g_ref, pre_ref, fl_ref = ds.ds_predict(ctx.h, cloud.h, net.h, ds.DS_PREC_F32,
                                                   pos[:n], view[:n], light[:n])
            out = torch.full((n,), -7.0, device="cuda")
            pre = torch.full((n,), -7.0, device="cuda")
            fl = torch.full((n,), 255, dtype=torch.uint8, device="cuda")
            ds.ds_predict_f32_noalloc(ctx.h, cloud.h, net.h, pos[:n], view[:n], light[:n],
                                      out=out, pre=pre, flags=fl)
            torch.cuda.synchronize()
            e = rel_l2(pre.cpu().numpy(), pre_ref.cpu().numpy())
            print(f"n={n}: relative L2 against ds_predict {e:.2e}")
            assert e <= 1e-5
            assert rel_l2(out.cpu().numpy(), g_ref.cpu().numpy()) <= 1e-5
            assert torch.equal(fl, fl_ref)
            assert out[5].item() == 0.0 and fl[5].item() & ds.DS_FLAG_INVALID
        # no flags and no pre-activation requested
        out2, _, _ = ds.ds_predict_f32_noalloc(ctx.h, cloud.h, net.h, pos[:300], view[:300],
                                               light[:300], want_pre=False, want_flags=False)
        torch.cuda.synchronize()
        assert rel_l2(out2.cpu().numpy(), g_ref[:300].cpu().numpy()) <= 1e-5
    finally:
        net.close()
        cloud.close()
        ctx.close()
