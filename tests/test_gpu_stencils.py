"""Coarser stencils trained on the 5 x 5 x 9 layout (Fig. 10, right) on the GPU: with the
dropped descriptor entries zero and their weights zero at the start, training steps (BF16
and FP32 operands) leave those weights exactly zero, and the trained network gives the same
outputs on the full descriptor as on the masked one, i.e. it is the coarser stencil's RPNN."""
import numpy as np
import pytest
import torch

import paper_1709_05418_amd as ds
from paper_1709_05418_amd import learn
from _util import Workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = ds.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("prec", [ds.DS_PREC_BF16, ds.DS_PREC_F32])
@pytest.mark.parametrize("shape", [(3, 3, 5), (2, 2, 3)])
def test_dropped_weights_stay_zero(ctx, prec, shape):
    w = Workload(64, 64.0, L=6, K=4, P=600, seed_cloud=2, seed_pts=41)
    z, _ = w.oracle_z()
    z = z.astype(np.float32)
    K, W = w.K, 48
    keep = learn.stencil_points(shape)
    drop = np.setdiff1d(np.arange(225), keep)
    zm = z.copy()
    for k in range(K):
        zm[:, k * 225 + drop] = 0.0
    t = np.log1p(np.random.default_rng(3).random(w.P) * 1.5).astype(np.float32)
    net = ds.Net(ctx, K, W, 3)
    try:
        net.set_params(learn.stencil_params(K, W, 9, keep, 0.5))
        ds.ds_net_set_train_precision(net.h, prec)
        opt = ds.ds_adam_create(net.h, 1e-3)
        zt, tt = torch.from_numpy(zm).cuda(), torch.from_numpy(t).cuda()
        l0, _ = ds.ds_loss_grad(net.h, zt, tt, net.n_params, want_grad=False)
        for i in range(30):
            ds.ds_train_step(net.h, opt, zt[(i % 2) * 256:(i % 2) * 256 + 256],
                             tt[(i % 2) * 256:(i % 2) * 256 + 256])
        ds.ds_adam_destroy(opt)
        theta = net.get_params()
        l1, _ = ds.ds_loss_grad(net.h, zt, tt, net.n_params, want_grad=False)
        assert l1.item() < l0.item()
        for V in learn.stencil_blocks(theta, K, W):
            assert np.all(V[:, drop] == 0.0)
            assert np.any(V[:, keep] != 0.0)
        a, pa = ds.ds_forward(ctx.h, net.h, torch.from_numpy(z).cuda())
        b, pb = ds.ds_forward(ctx.h, net.h, zt)
        assert torch.equal(pa, pb) and torch.equal(a, b)
    finally:
        net.close()
