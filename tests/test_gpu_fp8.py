"""FP8 form of the fused kernel: W1, W2 and the dense trailing layers on the E4M3
matrix cores with power-of-two scales, the descriptor layers in BF16.  Checked against
the FP64 oracle at the FP8 gate (relative L2 5e-2, on g and on the final
pre-activation), its scales against the calibration activations and the weights, its
state rules, and the batched, autotuned and graph-replayed launches bitwise against
per-cloud prediction.

The parameters are He-uniform with every block's second matrix scaled by 1/sqrt(K) and a
live output unit: with unscaled residual branches the residual stream grows through
the blocks and the final pre-activation cancels, which amplifies rounding in any
reduced precision (BF16 included)."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import paper_1709_05418_amd as ds
from paper_1709_05418_amd import synth
from _util import Workload, rel_l2

pytestmark = pytest.mark.gpu

H = 3
FP8_GATE = 5e-2


def theta_for(K, W, seed, biases=False):
    th = synth.init_params(K, W, H, seed, branch_scale=1.0 / math.sqrt(K), out_scale=0.2,
                           out_bias=0.5)
    if biases:  # every bias but the output's drawn from N(0, 0.2^2)
        rng = np.random.default_rng(seed + 100)
        o = 0
        for name, r, c in synth.layer_shapes(K, W, H):
            n = r * (c if c else 1)
            if c == 0 and name != f"bh{H - 1}":
                th[o:o + n] = rng.normal(0.0, 0.2, n)
            o += n
    return th


def numpy_activation_maxima(theta, K, W, z):
    """Largest |activation| per layer of the FP64 forward (first layer of every block,
    residual stream, dense trailing layers), for checking the calibration."""
    th = theta.astype(np.float64)
    off = 0

    def take(*shape):
        nonlocal off
        n = int(np.prod(shape))
        r = th[off:off + n].reshape(shape)
        off += n
        return r
    o = np.zeros((z.shape[0], W))
    aF, aO = [], 0.0
    for k in range(K):
        V = take(W, 226)
        W1 = take(W, W) if k else None
        b1 = take(W)
        W2 = take(W, W)
        b2 = take(W)
        zk = np.concatenate([z[:, 225 * k:225 * (k + 1)], z[:, -1:]], 1)
        h = zk @ V.T + b1 + (o @ W1.T if k else 0.0)
        F = np.maximum(h, 0.0)
        aF.append(F.max())
        o = np.maximum(F @ W2.T + b2 + o, 0.0)
        aO = max(aO, o.max())
    aH = []
    for m in range(H - 1):
        M, b = take(W, W), take(W)
        o = np.maximum(o @ M.T + b, 0.0)
        aH.append(o.max())
    return aF, aO, aH, th


def layer_mats(th, K, W):
    """The FP8 matrices in the order of the exported matrix exponents."""
    off = 0
    blocks = []
    for k in range(K):
        V = off
        off += W * 226
        W1 = off if k else None
        off += W * W if k else 0
        off += W
        W2 = off
        off += W * W + W
        blocks.append((W1, W2))
    heads = []
    for m in range(H - 1):
        heads.append(off)
        off += W * W + W
    mats = [th[b[0]:b[0] + W * W] for b in blocks[1:]]
    mats += [th[b[1]:b[1] + W * W] for b in blocks]
    mats += [th[h:h + W * W] for h in heads]
    return mats


@pytest.fixture(scope="module")
def ctx():
    c = ds.Context(0)
    yield c
    c.close()


CASES = {
    # 64^3 fBm, sigma 64, 6 levels, 6 x 64 network, 4096 points
    "tiny": dict(n=64, sigma=64.0, L=6, K=6, W=64, P=4096, seed_cloud=1, seed_pts=3, worley=0.0),
    # paper width on a 128^3 fBm + Worley cloud
    "paper_width": dict(n=128, sigma=128.0, L=8, K=10, W=200, P=3000, seed_cloud=10,
                        seed_pts=11, worley=0.3),
}


@pytest.mark.parametrize("biases", [False, True])
@pytest.mark.parametrize("name", list(CASES))
def test_fp8_prediction_matches_oracle(ctx, name, biases):
    c = CASES[name]
    K, W = c["K"], c["W"]
    w = Workload(c["n"], c["sigma"], L=c["L"], K=K, P=c["P"], seed_cloud=c["seed_cloud"],
                 seed_pts=c["seed_pts"], worley=c["worley"])
    theta = theta_for(K, W, 12, biases)
    cloud = ds.Cloud(ctx, w.density.cuda(), w.sigma_max, w.aabb_min, w.h0, w.L, K, w.mips)
    net = ds.Net(ctx, K, W, H)
    try:
        net.set_params(theta)
        pos, view, light = w.cuda_inputs()
        ncal = 1024  # calibration points; the rest are held out
        ds.ds_net_quantize(ctx.h, net.h, cloud.h, ds.DS_PREC_FP8, pos[:ncal], view[:ncal],
                           light[:ncal])
        g8, p8, fl8 = ds.ds_predict(ctx.h, cloud.h, net.h, ds.DS_PREC_FP8, pos, view, light)
        g16, p16, _ = ds.ds_predict(ctx.h, cloud.h, net.h, ds.DS_PREC_BF16, pos, view, light)
        torch.cuda.synchronize()
        z, flr = w.oracle_z()
        gr, pr = O.forward(theta.astype(np.float64), K, W, H, z)
        sl = slice(ncal, None)
        e8 = (rel_l2(g8.cpu().numpy()[sl], gr[sl]), rel_l2(p8.cpu().numpy()[sl], pr[sl]))
        e16 = (rel_l2(g16.cpu().numpy()[sl], gr[sl]), rel_l2(p16.cpu().numpy()[sl], pr[sl]))
        assert max(e16) < 2e-2
        print(f"{name}, biases {biases}: fp8 g {e8[0]:.3e} pre {e8[1]:.3e}; bf16 g {e16[0]:.3e} "
              f"pre {e16[1]:.3e}; "
              f"alive {(gr > 0).mean():.2f}", flush=True)
        assert max(e8) < FP8_GATE
        assert np.array_equal(fl8.cpu().numpy(), flr)
        assert bool(torch.isfinite(g8).all())
    finally:
        net.close()
        cloud.close()


def test_fp8_scales_follow_calibration_and_weights(ctx):
    c = CASES["tiny"]
    K, W = c["K"], c["W"]
    w = Workload(c["n"], c["sigma"], L=c["L"], K=K, P=1024, seed_cloud=c["seed_cloud"],
                 seed_pts=c["seed_pts"])
    theta = theta_for(K, W, 12)
    cloud = ds.Cloud(ctx, w.density.cuda(), w.sigma_max, w.aabb_min, w.h0, w.L, K, w.mips)
    net = ds.Net(ctx, K, W, H)
    try:
        net.set_params(theta)
        pos, view, light = w.cuda_inputs()
        ds.ds_net_quantize(ctx.h, net.h, cloud.h, ds.DS_PREC_FP8, pos, view, light)
        ex = ds.ds_net_fp8_scales(net.h, K, H)
        assert ex.size == 3 * K + 2 * H - 2
        f, o, h = ex[:K], int(ex[K]), ex[K + 1:K + H]
        mexp = ex[K + H:]
        z, _ = w.oracle_z()
        aF, aO, aH, th = numpy_activation_maxima(theta, K, W, z)
        # matrix exponent = output unit - input unit
        want = [f[k] - o for k in range(1, K)] + [o - f[k] for k in range(K)]
        want += [h[m] - (o if m == 0 else h[m - 1]) for m in range(H - 1)]
        assert list(mexp) == want
        # nothing overflows: weights and calibration activations fit under 448
        for M, e in zip(layer_mats(th, K, W), mexp):
            assert np.abs(M).max() * 2.0 ** e <= 448.0
        rng = lambda a: math.floor(math.log2(448.0 / a))
        for k in range(K):
            assert aF[k] * 2.0 ** f[k] <= 448.0 * (1 + 1e-5)
        assert aO * 2.0 ** o <= 448.0 * (1 + 1e-5)
        # with these weights no matrix bound is active: every unit fills its range
        assert [int(v) for v in f] == [rng(a) for a in aF] and o == rng(aO)
        assert [int(v) for v in h] == [rng(a) for a in aH]
    finally:
        net.close()
        cloud.close()


def test_fp8_state_rules(ctx):
    K, W = 5, 64
    w = Workload(32, 32.0, L=5, K=K, P=256, seed_cloud=4, seed_pts=5)
    cloud = ds.Cloud(ctx, w.density.cuda(), w.sigma_max, w.aabb_min, w.h0, w.L, K, w.mips)
    net = ds.Net(ctx, K, W, H)
    try:
        pos, view, light = w.cuda_inputs()
        with pytest.raises(ds.DSError) as e:  # no parameters yet
            ds.ds_net_quantize(ctx.h, net.h, cloud.h, ds.DS_PREC_FP8, pos, view, light)
        assert e.value.status == -5
        net.set_params(theta_for(K, W, 3))
        with pytest.raises(ds.DSError) as e:  # not quantised yet
            ds.ds_predict(ctx.h, cloud.h, net.h, ds.DS_PREC_FP8, pos, view, light)
        assert e.value.status == -5
        with pytest.raises(ds.DSError):
            ds.ds_net_quantize(ctx.h, net.h, cloud.h, ds.DS_PREC_BF16, pos, view, light)
        with pytest.raises(ds.DSError):
            ds.ds_net_fp8_scales(net.h, K, H)
        ds.ds_net_quantize(ctx.h, net.h, cloud.h, ds.DS_PREC_FP8, pos, view, light)
        a, _, _ = ds.ds_predict(ctx.h, cloud.h, net.h, ds.DS_PREC_FP8, pos, view, light)
        # new parameters drop the FP8 form until the next quantisation
        net.set_params(theta_for(K, W, 4))
        with pytest.raises(ds.DSError) as e:
            ds.ds_predict(ctx.h, cloud.h, net.h, ds.DS_PREC_FP8, pos, view, light)
        assert e.value.status == -5
        ds.ds_net_quantize(ctx.h, net.h, cloud.h, ds.DS_PREC_FP8, pos, view, light)
        b, _, _ = ds.ds_predict(ctx.h, cloud.h, net.h, ds.DS_PREC_FP8, pos, view, light)
        torch.cuda.synchronize()
        assert not torch.equal(a, b)
    finally:
        net.close()
        cloud.close()


def test_fp8_batched_variants_and_graph(ctx):
    K, W = 5, 64
    sizes, counts = [24, 40, 32], [1000 + 3, 0, 2048 + 77]
    ws, clouds = [], []
    for i, (n, P) in enumerate(zip(sizes, counts)):
        w = Workload(n, float(n), L=5, K=K, P=max(P, 1), seed_cloud=80 + i, seed_pts=90 + i)
        ws.append(w)
        clouds.append(ds.Cloud(ctx, w.density.cuda(), w.sigma_max, w.aabb_min, w.h0, w.L, K,
                               w.mips))
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    pos = t(np.concatenate([w.pos[:P] for w, P in zip(ws, counts)]))
    view = t(np.concatenate([w.view[:P] for w, P in zip(ws, counts)]))
    light = t(np.concatenate([w.light[:P] for w, P in zip(ws, counts)]))
    N = int(offsets[-1])
    theta = theta_for(K, W, 9)
    net = ds.Net(ctx, K, W, H)
    b = None
    try:
        net.set_params(theta)
        ds.ds_net_quantize(ctx.h, net.h, clouds[0].h, ds.DS_PREC_FP8, pos[:512], view[:512],
                           light[:512])
        per = []
        for c, (a0, a1) in zip(clouds, zip(offsets[:-1], offsets[1:])):
            if a1 > a0:
                o, _, _ = ds.ds_predict(ctx.h, c.h, net.h, ds.DS_PREC_FP8, pos[a0:a1],
                                        view[a0:a1], light[a0:a1], want_pre=False,
                                        want_flags=False)
                per.append(o)
        per = torch.cat(per)
        b = ds.ds_batch_create(ctx.h, net.h, [c.h for c in clouds], offsets)
        for kind, waves in ((ds.DS_KERNEL_REGISTER, 4), (ds.DS_KERNEL_REGISTER, 8),
                            (ds.DS_KERNEL_TEAMS, 8)):
            for grid in (0, 1, 3, 64):
                print("fp8 variant", kind, waves, grid, flush=True)
                ds.ds_batch_set_config(b, kind, waves, grid)
                out = torch.full((N,), -1.0, device="cuda")
                ds.ds_batch_predict(b, ds.DS_PREC_FP8, pos, view, light, out)
                assert torch.equal(out, per), (kind, waves, grid)
        ds.ds_batch_set_config(b, ds.DS_KERNEL_PIPELINED, 4, 0)
        with pytest.raises(ds.DSError) as e:  # the FP8 form: register and two-team kernels
            ds.ds_batch_predict(b, ds.DS_PREC_FP8, pos, view, light, out)
        assert e.value.status == -4
        cfg = ds.ds_batch_autotune(b, ds.DS_PREC_FP8, pos, view, light, out, 2)
        assert cfg["kernel"] in (ds.DS_KERNEL_REGISTER, ds.DS_KERNEL_TEAMS) and cfg["ms"] > 0
        out.fill_(-1.0)
        ds.ds_batch_capture(b, ds.DS_PREC_FP8, pos, view, light, out)
        for r in range(3):
            out.fill_(-1.0)
            ds.ds_batch_replay(b)
            torch.cuda.synchronize()
            assert torch.equal(out, per), r
            _ = (pos * 2).sum()  # eager work between replays
        # against the oracle, cloud by cloud
        got, want = [], []
        for w, P, a0 in zip(ws, counts, offsets):
            if P == 0:
                continue
            idx = np.arange(0, P, 5)
            z, _ = w.oracle_z(idx)
            g, _ = O.forward(theta.astype(np.float64), K, W, H, z)
            want.append(g)
            got.append(per.cpu().numpy()[a0 + idx])
        err = rel_l2(np.concatenate(got), np.concatenate(want))
        print(f"batched fp8 rel L2 {err:.3e}", flush=True)
        assert err < FP8_GATE
    finally:
        if b is not None:
            ds.ds_batch_destroy(b)
        net.close()
        for c in clouds:
            c.close()
