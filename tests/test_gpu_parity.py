"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element by
element on the same seeded inputs.  Tolerances (relative L2 over all points):
1e-5 for FP32, 2e-2 for BF16 (the gates stated for this method's GPU path)."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1709_05418_amd as ds
from paper_1709_05418_amd import synth
from _util import Workload, rel_l2

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5
TOL_BF16 = 2e-2


@pytest.fixture(scope="module")
def ctx():
    c = ds.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def tiny():
    # 64^3 fBm cloud, sigma_max 64/unit, 6 levels, K = 6; a ragged point count
    return Workload(64, 64.0, L=6, K=6, P=4096 + 37, seed_cloud=1, seed_pts=3)


@pytest.fixture(scope="module")
def tiny_cloud(ctx, tiny):
    c = ds.Cloud(ctx, tiny.density.cuda(), tiny.sigma_max, tiny.aabb_min, tiny.h0, tiny.L, tiny.K,
                 tiny.mips)
    yield c
    c.close()


def _net(ctx, K, W, H=3, seed=2, out_bias=0.05):
    theta = synth.init_params(K, W, H, seed)
    theta[-1] = out_bias
    net = ds.Net(ctx, K, W, H)
    net.set_params(theta)
    return net, theta.astype(np.float64)


def test_cloud_mean_and_pyramid(ctx, tiny, tiny_cloud):
    info = tiny_cloud.info
    print("mean gpu", info["mean_mu_t"], "oracle", tiny.mean)
    assert info["mean_mu_t"] == pytest.approx(tiny.mean, rel=1e-6)
    assert info["mip_of_level"] == list(tiny.mips)
    pyr, dims, offs = tiny.pyr
    for i in range(tiny.L):
        got = tiny_cloud.level(i).cpu().numpy()
        ref = O.level(pyr, dims, offs, i)
        e = rel_l2(got, ref)
        print(f"level {i} dims {got.shape} rel_l2 {e:.2e}")
        assert got.shape == ref.shape
        assert e <= TOL_F32
        assert np.max(np.abs(got - ref)) <= 1e-5 * np.abs(ref).max()


def test_gather_f32_matches_oracle(ctx, tiny, tiny_cloud):
    pos, view, light = tiny.cuda_inputs()
    z, fl = ds.ds_gather(ctx.h, tiny_cloud.h, pos, view, light, tiny.K)
    zr, flr = tiny.oracle_z()
    z = z.cpu().numpy()
    e = rel_l2(z, zr)
    print("gather f32 rel_l2", e, "per level",
          [f"{rel_l2(z[:, k * 225:(k + 1) * 225], zr[:, k * 225:(k + 1) * 225]):.1e}"
           for k in range(tiny.K)])
    assert e <= TOL_F32
    # gamma: acos of an FP32 dot product; its rounding grows like 1/sin(gamma)
    assert rel_l2(z[:, -1], zr[:, -1]) <= 1e-6
    assert np.max(np.abs(z[:, -1] - zr[:, -1])) <= 2e-5
    mism = np.flatnonzero(fl.cpu().numpy() != flr)
    assert mism.size <= 2, mism  # only points whose stencil corner touches a face may differ


def test_gather_bf16_output(ctx, tiny, tiny_cloud):
    pos, view, light = tiny.cuda_inputs()
    z, _ = ds.ds_gather(ctx.h, tiny_cloud.h, pos, view, light, tiny.K, out_dtype=torch.bfloat16)
    zr, _ = tiny.oracle_z()
    e = rel_l2(z.float().cpu().numpy(), zr)
    print("gather bf16 rel_l2", e)
    assert e <= 4e-3


def test_packed_gather_matches_oracle(ctx, tiny, tiny_cloud):
    # the fused kernel's gather schedule (BF16 corner cells, BF16 weights) in canonical order
    pos, view, light = tiny.cuda_inputs()
    z = ds.ds_gather_packed(ctx.h, tiny_cloud.h, pos, view, light, tiny.K).cpu().numpy()
    zr, _ = tiny.oracle_z()
    per = [rel_l2(z[:, k * 225:(k + 1) * 225], zr[:, k * 225:(k + 1) * 225]) for k in range(tiny.K)]
    bad = np.argmax(np.abs(z - zr).max(0))
    print("packed gather rel_l2", rel_l2(z, zr), "per level", [f"{e:.1e}" for e in per],
          "worst column", bad)
    assert rel_l2(z, zr) <= 4e-3


def test_forward_f32_on_oracle_descriptors(ctx, tiny):
    net, theta = _net(ctx, tiny.K, 64)
    zr, _ = tiny.oracle_z()
    g, pre = ds.ds_forward(ctx.h, net.h, torch.from_numpy(zr.astype(np.float32)).cuda())
    gr, prer = O.forward(theta, tiny.K, 64, 3, zr.astype(np.float32).astype(np.float64))
    e = rel_l2(pre.cpu().numpy(), prer)
    print("forward f32 pre rel_l2", e, "alive", (gr > 0).mean())
    assert e <= TOL_F32
    assert rel_l2(g.cpu().numpy(), gr) <= TOL_F32
    net.close()


@pytest.mark.parametrize("prec,tol", [(ds.DS_PREC_F32, TOL_F32), (ds.DS_PREC_BF16, TOL_BF16)])
def test_predict_tiny(ctx, tiny, tiny_cloud, prec, tol):
    net, theta = _net(ctx, tiny.K, 64)
    pos, view, light = tiny.cuda_inputs()
    g, pre, fl = ds.ds_predict(ctx.h, tiny_cloud.h, net.h, prec, pos, view, light)
    zr, flr = tiny.oracle_z()
    gr, prer = O.forward(theta, tiny.K, 64, 3, zr)
    e_pre, e_g = rel_l2(pre.cpu().numpy(), prer), rel_l2(g.cpu().numpy(), gr)
    print(f"predict prec={prec} pre rel_l2 {e_pre:.2e} g rel_l2 {e_g:.2e} alive {(gr > 0).mean():.2f}")
    assert e_pre <= tol and e_g <= tol
    assert np.count_nonzero(fl.cpu().numpy() != flr) <= 2
    net.close()


@pytest.fixture(scope="module")
def paper_width():
    # 128^3 fBm + Worley cloud, 8 levels, K = 10, W = 200; 1000 points (ragged tiles)
    return Workload(128, 128.0, L=8, K=10, P=1000, seed_cloud=7, seed_pts=30, worley=0.3)


@pytest.mark.parametrize("prec,tol", [(ds.DS_PREC_F32, TOL_F32), (ds.DS_PREC_BF16, TOL_BF16)])
def test_predict_paper_width(ctx, paper_width, prec, tol):
    w = paper_width
    cloud = ds.Cloud(ctx, w.density.cuda(), w.sigma_max, w.aabb_min, w.h0, w.L, w.K, w.mips)
    net, theta = _net(ctx, w.K, 200, seed=12)
    pos, view, light = w.cuda_inputs()
    g, pre, fl = ds.ds_predict(ctx.h, cloud.h, net.h, prec, pos, view, light)
    zr, flr = w.oracle_z()
    gr, prer = O.forward(theta, w.K, 200, 3, zr)
    e_pre, e_g = rel_l2(pre.cpu().numpy(), prer), rel_l2(g.cpu().numpy(), gr)
    print(f"paper width prec={prec} pre {e_pre:.2e} g {e_g:.2e} alive {(gr > 0).mean():.2f}")
    assert e_pre <= tol and e_g <= tol
    net.close()
    cloud.close()


def _biased_params(K, W, H, seed):
    # the reduced-precision recipe (R21) with every bias drawn from N(0, 0.2^2): the fused
    # kernel carries the biases inside its weight chunks (a BF16 high and low part, the
    # dense layers' only when the tile count is odd), which zero biases would not test
    theta = synth.init_params(K, W, H, seed, branch_scale=1 / np.sqrt(K), out_scale=0.2,
                              out_bias=0.5)
    rng = np.random.default_rng(seed + 100)
    o = 0
    for name, r, c in synth.layer_shapes(K, W, H):
        n = r * (c if c else 1)
        if c == 0 and name != f"bh{H - 1}":
            theta[o:o + n] = rng.normal(0.0, 0.2, n)
        o += n
    return theta


@pytest.mark.parametrize("W", [16, 64, 200])
def test_predict_with_nonzero_biases(ctx, tiny, tiny_cloud, W):
    # W = 16 and 200: odd tile counts (every bias in the chunks); W = 64: even (b1 only).
    # The FP8 form is checked where it is specified (K = 6 at W = 64 here; K = 10 at W = 200
    # in the FP8 tests): on this 6-block network it misses its gate at W = 16 and W = 200
    # with or without biases (7 % and 16-18 %, the same with biases as vector loads)
    w = tiny
    theta = _biased_params(w.K, W, 3, 40 + W)
    net = ds.Net(ctx, w.K, W, 3)
    try:
        net.set_params(theta)
        pos, view, light = w.cuda_inputs()
        zr, _ = w.oracle_z()
        gr, prer = O.forward(theta.astype(np.float64), w.K, W, 3, zr)
        ds.ds_net_quantize(ctx.h, net.h, tiny_cloud.h, ds.DS_PREC_FP8, pos[::3].contiguous(),
                           view[::3].contiguous(), light[::3].contiguous())
        precs = [(ds.DS_PREC_BF16, TOL_BF16)] + ([(ds.DS_PREC_FP8, 5e-2)] if W == 64 else [])
        for prec, tol in precs:
            g, pre, _ = ds.ds_predict(ctx.h, tiny_cloud.h, net.h, prec, pos, view, light)
            e = rel_l2(pre.cpu().numpy(), prer)
            print(f"W={W} precision {prec}: relative L2 of the pre-activation {e:.2e}", flush=True)
            assert e <= tol
    finally:
        net.close()


def test_degenerate_and_invalid_inputs(ctx, tiny, tiny_cloud):
    net, theta = _net(ctx, tiny.K, 64)
    pos = tiny.pos[:8].copy()
    view = tiny.view[:8].copy()
    light = tiny.light[:8].copy()
    pos[0] = np.nan
    view[1] = 0.0
    light[2] = [np.inf, 0, 0]
    pos[3] = [3.0, 0.0, 0.0]          # outside the grid box: all samples of level 1 are zero
    view[4] = light[4] * 2.5           # view parallel to the light: degenerate frame
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    for prec in (ds.DS_PREC_F32, ds.DS_PREC_BF16):
        g, pre, fl = ds.ds_predict(ctx.h, tiny_cloud.h, net.h, prec, t(pos), t(view), t(light))
        g, pre, fl = g.cpu().numpy(), pre.cpu().numpy(), fl.cpu().numpy()
        assert fl[0] == fl[1] == fl[2] == ds.DS_FLAG_INVALID
        assert np.all(g[:3] == 0) and np.all(pre[:3] == 0)
        assert fl[3] & ds.DS_FLAG_OUTSIDE and fl[3] & ds.DS_FLAG_FALLBACK
        assert np.all(np.isfinite(g)) and np.all(np.isfinite(pre))
    # the degenerate frame still matches the oracle's choice of basis
    z, _ = ds.ds_gather(ctx.h, tiny_cloud.h, t(pos), t(view), t(light), tiny.K)
    pyr, dims, offs = tiny.pyr
    zr, _ = O.gather(tiny.grid, pyr, dims, offs, tiny.mean, tiny.K, tiny.mips, pos, view, light)
    assert rel_l2(z.cpu().numpy()[3:], zr[3:]) <= TOL_F32
    net.close()


def test_empty_and_single_point(ctx, tiny, tiny_cloud):
    net, theta = _net(ctx, tiny.K, 64)
    e = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    g, pre, fl = ds.ds_predict(ctx.h, tiny_cloud.h, net.h, ds.DS_PREC_BF16, e, e, e)
    assert g.numel() == 0
    pos, view, light = (a[:1] for a in tiny.cuda_inputs())
    zr, _ = tiny.oracle_z(slice(0, 1))
    gr, prer = O.forward(theta, tiny.K, 64, 3, zr)
    for prec, tol in ((ds.DS_PREC_F32, TOL_F32), (ds.DS_PREC_BF16, TOL_BF16)):
        g, pre, fl = ds.ds_predict(ctx.h, tiny_cloud.h, net.h, prec, pos, view, light)
        assert abs(pre.item() - prer[0]) <= tol * max(abs(prer[0]), 1e-3)
    net.close()


def test_mismatched_levels_rejected(ctx, tiny, tiny_cloud):
    net = ds.Net(ctx, tiny.K + 1, 64)
    pos, view, light = tiny.cuda_inputs()
    with pytest.raises(ds.DSError):
        ds.ds_predict(ctx.h, tiny_cloud.h, net.h, ds.DS_PREC_BF16, pos, view, light)
    net.close()
