"""Batched uneven prediction: several clouds of different sizes and uneven point
counts in one launch of the fused kernel, every kernel variant, the autotuner and
graph capture/replay, against per-cloud prediction and the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1709_05418_amd as ds
from paper_1709_05418_amd import synth
from _util import Workload, rel_l2

pytestmark = pytest.mark.gpu

K, W, H = 5, 64, 3


@pytest.fixture(scope="module")
def ctx():
    c = ds.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def setup(ctx):
    # four clouds (24^3 .. 48^3, one BF16 grid), uneven ragged point counts, one empty
    sizes = [24, 40, 32, 48]
    counts = [1000 + 3, 0, 4096 + 77, 257]
    ws, clouds = [], []
    for i, (n, P) in enumerate(zip(sizes, counts)):
        dens = synth.cloud_density(n, 60 + i)
        if i == 2:
            dens = dens.to(torch.bfloat16)
        w = Workload(n, float(n), L=5, K=K, P=max(P, 1), seed_cloud=60 + i, seed_pts=70 + i,
                     density=dens)
        ws.append(w)
        clouds.append(ds.Cloud(ctx, dens.cuda(), w.sigma_max, w.aabb_min, w.h0, w.L, K, w.mips))
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    pos = np.concatenate([w.pos[:P] for w, P in zip(ws, counts)])
    view = np.concatenate([w.view[:P] for w, P in zip(ws, counts)])
    light = np.concatenate([w.light[:P] for w, P in zip(ws, counts)])
    net = ds.Net(ctx, K, W, H)
    theta = synth.init_params(K, W, H, 9, branch_scale=0.5, out_scale=0.2, out_bias=0.5)
    net.set_params(theta)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    yield dict(ws=ws, clouds=clouds, counts=counts, offsets=offsets, pos=t(pos), view=t(view),
               light=t(light), net=net, theta=theta)
    net.close()
    for c in clouds:
        c.close()


def _batch(ctx, s):
    return ds.ds_batch_create(ctx.h, s["net"].h, [c.h for c in s["clouds"]], s["offsets"])


def _per_cloud(ctx, s, prec):
    outs = []
    for c, (a, b) in zip(s["clouds"], zip(s["offsets"][:-1], s["offsets"][1:])):
        if b == a:
            continue
        o, _, _ = ds.ds_predict(ctx.h, c.h, s["net"].h, prec, s["pos"][a:b], s["view"][a:b],
                                s["light"][a:b], want_pre=False, want_flags=False)
        outs.append(o)
    return torch.cat(outs)


def test_batched_equals_per_cloud_and_oracle(ctx, setup):
    s = setup
    N = int(s["offsets"][-1])
    b = _batch(ctx, s)
    try:
        out = torch.empty(N, dtype=torch.float32, device="cuda")
        pre = torch.empty(N, dtype=torch.float32, device="cuda")
        fl = torch.empty(N, dtype=torch.uint8, device="cuda")
        ds.ds_batch_predict(b, ds.DS_PREC_BF16, s["pos"], s["view"], s["light"], out, pre, fl)
        ref = _per_cloud(ctx, s, ds.DS_PREC_BF16)
        # each point's arithmetic does not depend on which tile carries it
        assert torch.equal(out, ref)
        out32 = torch.empty_like(out)
        ds.ds_batch_predict(b, ds.DS_PREC_F32, s["pos"], s["view"], s["light"], out32)
        assert torch.equal(out32, _per_cloud(ctx, s, ds.DS_PREC_F32))
        # against the oracle, cloud by cloud
        got, got32, want = [], [], []
        for w, P, a in zip(s["ws"], s["counts"], s["offsets"]):
            if P == 0:
                continue
            idx = np.arange(0, P, 7)
            z, _ = w.oracle_z(idx)
            g, _ = O.forward(s["theta"].astype(np.float64), K, W, H, z)
            want.append(g)
            got.append(out.cpu().numpy()[a + idx])
            got32.append(out32.cpu().numpy()[a + idx])
        want = np.concatenate(want)
        assert rel_l2(np.concatenate(got32), want) < 1e-5
        assert rel_l2(np.concatenate(got), want) < 2e-2
    finally:
        ds.ds_batch_destroy(b)


def test_every_variant_and_grid_agrees(ctx, setup):
    s = setup
    N = int(s["offsets"][-1])
    b = _batch(ctx, s)
    try:
        base = torch.empty(N, dtype=torch.float32, device="cuda")
        ds.ds_batch_predict(b, ds.DS_PREC_BF16, s["pos"], s["view"], s["light"], base)
        for kind in (ds.DS_KERNEL_REGISTER, ds.DS_KERNEL_PIPELINED, ds.DS_KERNEL_WIDE,
                     ds.DS_KERNEL_TEAMS):
            for waves in {ds.DS_KERNEL_WIDE: (4,), ds.DS_KERNEL_TEAMS: (8,)}.get(kind, (4, 8)):
                for grid in (0, 1, 3, 64):
                    print("variant", kind, waves, grid, flush=True)
                    ds.ds_batch_set_config(b, kind, waves, grid)
                    out = torch.full((N,), -1.0, device="cuda")
                    ds.ds_batch_predict(b, ds.DS_PREC_BF16, s["pos"], s["view"], s["light"], out)
                    assert torch.equal(out, base), (kind, waves, grid)
        with pytest.raises(ds.DSError):
            ds.ds_batch_set_config(b, 4, 4, 0)
        with pytest.raises(ds.DSError):
            ds.ds_batch_set_config(b, ds.DS_KERNEL_WIDE, 8, 0)
        with pytest.raises(ds.DSError):
            ds.ds_batch_set_config(b, ds.DS_KERNEL_TEAMS, 4, 0)
        with pytest.raises(ds.DSError):
            ds.ds_batch_set_config(b, 0, 6, 0)
    finally:
        ds.ds_batch_destroy(b)


def test_autotune_then_graph_replay(ctx, setup):
    s = setup
    N = int(s["offsets"][-1])
    b = _batch(ctx, s)
    try:
        eager = torch.empty(N, dtype=torch.float32, device="cuda")
        ds.ds_batch_predict(b, ds.DS_PREC_BF16, s["pos"], s["view"], s["light"], eager)
        cfg = ds.ds_batch_autotune(b, ds.DS_PREC_BF16, s["pos"], s["view"], s["light"], eager, 2)
        # any available variant may win on timing, the two-team kernel (3) included
        assert cfg["ms"] > 0 and cfg["waves"] in (4, 8) and cfg["kernel"] in (0, 1, 2, 3)
        out = torch.full((N,), -1.0, device="cuda")
        pos = s["pos"].clone()
        ds.ds_batch_capture(b, ds.DS_PREC_BF16, pos, s["view"], s["light"], out)
        for r in range(3):
            out.fill_(-1.0)
            ds.ds_batch_replay(b)
            torch.cuda.synchronize()
            assert torch.equal(out, eager), r
            _ = (pos * 2).sum()  # unrelated eager work between replays
        # the graph reads the arrays it was captured with: new contents, new results
        pos[: s["counts"][0]] += 0.01
        ds.ds_batch_replay(b)
        torch.cuda.synchronize()
        moved = torch.empty_like(out)
        ds.ds_batch_predict(b, ds.DS_PREC_BF16, pos, s["view"], s["light"], moved)
        assert torch.equal(out, moved) and not torch.equal(out, eager)
        with pytest.raises(ds.DSError):
            ds.ds_batch_capture(b, ds.DS_PREC_F32, pos, s["view"], s["light"], out)
    finally:
        ds.ds_batch_destroy(b)


def test_spatial_order_is_bitwise_the_input_order(ctx, setup):
    # the spatial order only changes which tile carries a point: outputs, pre-activations
    # and flags stay bitwise those of the input order, for every kernel kind, eagerly and
    # through a captured graph; points outside the box and a non-finite position included
    s = setup
    N = int(s["offsets"][-1])
    pos = s["pos"].clone()
    pos[5] = torch.tensor([9.0, -9.0, 0.0])          # outside its cloud's box
    pos[s["counts"][0] + 7, 1] = float("nan")        # unusable position
    b = _batch(ctx, s)
    try:
        def run(order, kind=ds.DS_KERNEL_REGISTER, waves=4, grid=0):
            ds.ds_batch_set_order(b, order)
            ds.ds_batch_set_config(b, kind, waves, grid)
            out = torch.full((N,), -1.0, device="cuda")
            pre = torch.full((N,), -1.0, device="cuda")
            fl = torch.full((N,), 255, dtype=torch.uint8, device="cuda")
            ds.ds_batch_predict(b, ds.DS_PREC_BF16, pos, s["view"], s["light"], out, pre, fl)
            return out, pre, fl
        ref = run(ds.DS_ORDER_INPUT)
        assert int(ref[2][5]) & ds.DS_FLAG_OUTSIDE and int(ref[2][s["counts"][0] + 7]) & \
            ds.DS_FLAG_INVALID
        for kind, waves, grid in [(ds.DS_KERNEL_REGISTER, 4, 0), (ds.DS_KERNEL_REGISTER, 8, 3),
                                  (ds.DS_KERNEL_PIPELINED, 4, 64), (ds.DS_KERNEL_WIDE, 4, 0),
                                  (ds.DS_KERNEL_TEAMS, 8, 0), (ds.DS_KERNEL_TEAMS, 8, 3)]:
            got = run(ds.DS_ORDER_SPATIAL, kind, waves, grid)
            for g, r in zip(got, ref):
                assert torch.equal(g, r), (kind, waves, grid)
        # captured with the order inside the graph
        ds.ds_batch_set_config(b, ds.DS_KERNEL_REGISTER, 4, 0)
        out = torch.full((N,), -1.0, device="cuda")
        ds.ds_batch_capture(b, ds.DS_PREC_BF16, pos, s["view"], s["light"], out)
        for r in range(3):
            out.fill_(-1.0)
            ds.ds_batch_replay(b)
            torch.cuda.synchronize()
            assert torch.equal(out, ref[0]), r
            _ = (pos * 2).nan_to_num().sum()  # unrelated eager work between replays
        # back to the input order: the graph is dropped, results unchanged
        ds.ds_batch_set_order(b, ds.DS_ORDER_INPUT)
        with pytest.raises(ds.DSError):
            ds.ds_batch_replay(b)
        assert torch.equal(run(ds.DS_ORDER_INPUT)[0], ref[0])
        with pytest.raises(ds.DSError):
            ds.ds_batch_set_order(b, 2)
    finally:
        ds.ds_batch_destroy(b)


def test_batch_argument_checks(ctx, setup):
    s = setup
    with pytest.raises(ds.DSError):
        ds.ds_batch_create(ctx.h, s["net"].h, [s["clouds"][0].h] * 17, list(range(18)))
    with pytest.raises(ds.DSError):
        ds.ds_batch_create(ctx.h, s["net"].h, [c.h for c in s["clouds"][:2]], [0, 5, 3])
    with pytest.raises(ds.DSError):
        ds.ds_batch_create(ctx.h, s["net"].h, [c.h for c in s["clouds"][:2]], [1, 5, 6])
    other = ds.Net(ctx, K + 1, W, H)
    try:
        with pytest.raises(ds.DSError):
            ds.ds_batch_create(ctx.h, other.h, [c.h for c in s["clouds"][:2]], [0, 5, 6])
    finally:
        other.close()
    b = _batch(ctx, s)
    try:
        with pytest.raises(ds.DSError):
            ds.ds_batch_replay(b)
    finally:
        ds.ds_batch_destroy(b)
    # the two-team kernel needs an even number of weight chunks per tile: K = 5, W = 16
    # has 47
    odd = ds.Net(ctx, K, 16, H)
    try:
        b = ds.ds_batch_create(ctx.h, odd.h, [c.h for c in s["clouds"][:2]], [0, 5, 6])
        try:
            with pytest.raises(ds.DSError):
                ds.ds_batch_set_config(b, ds.DS_KERNEL_TEAMS, 8, 0)
        finally:
            ds.ds_batch_destroy(b)
    finally:
        odd.close()


def _fast(info, h0):
    """Whether every level of a cloud gets a zero border wide enough for the unclamped pass:
    the library's rule (a border of ceil(E + 1/2) + 1 cells, E = sqrt(11) 2^k / mean / h for
    each stencil level k on that level, kept only while at most 256 cells and not growing
    the level beyond 1.5 times or 2^21 cells), restated to check that a test builds both
    kinds of cloud."""
    mean, mips = info["mean_mu_t"], info["mip_of_level"]
    for i, (nx, ny, nz) in enumerate(info["dims"]):
        ext = max([3.3166248 * 2.0 ** k / mean / (h0 * 2.0 ** i)
                   for k, m in enumerate(mips) if m == i], default=0.0)
        if ext > 0.0:
            want = np.ceil(ext + 0.5) + 1.0
            base = (nx + 2) * (ny + 2) * (nz + 2)
            grown = (nx + 2 * want) * (ny + 2 * want) * (nz + 2 * want)
            if not (want <= 256 and (grown <= 1.5 * base or grown <= 1 << 21)):
                return False
    return True


def test_variants_orders_with_a_clamped_cloud_and_invalid_points(ctx):
    # The two-pass launches leave clouds whose borders are too narrow, and tiles holding a
    # point outside the grid box, to the clamped pass; the two-team kernel then walks such
    # a cloud's chunks idle, and its clamped pass recomputes 64-point halves of its 128-point
    # tiles.  A batch with a thin cloud between two dense ones and invalid points in ragged
    # tiles: every variant in both point orders, bitwise the per-cloud default launches
    # (outputs, pre-activations and flags), BF16 and FP8.  With 55 tiles of 64 points and a
    # grid of one workgroup, the clamped pass screens its tiles in two batches of 32.
    specs = [(32, 32.0, 1300, 81), (24, 0.5, 900, 82), (40, 40.0, 1260, 83)]
    ws, clouds = [], []
    try:
        for n, sig, P, seed in specs:
            w = Workload(n, sig, L=5, K=K, P=P, seed_cloud=seed, seed_pts=seed + 10)
            ws.append(w)
            clouds.append(ds.Cloud(ctx, w.density.cuda(), sig, w.aabb_min, w.h0, w.L, K))
        assert [_fast(c.info, w.h0) for c, w in zip(clouds, ws)] == [True, False, True]
        counts = [w.P for w in ws]
        offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        pos = np.concatenate([w.pos for w in ws]).astype(np.float32)
        view = np.concatenate([w.view for w in ws]).astype(np.float32)
        light = np.concatenate([w.light for w in ws]).astype(np.float32)
        pos[3] = np.nan                                       # invalid, first tile
        pos[70] = ws[0].aabb_min - 0.25                       # outside the box, second half
        view[131] = 0.0                                       # invalid, third half
        light[1300 + 65] = [np.inf, 0.0, 0.0]                 # invalid, in the thin cloud
        pos[2200 + 1200] = ws[2].aabb_min + np.float32(2.0)   # outside, second batch of tiles
        view[2200 + 7] = light[2200 + 7] * 3.0                # view parallel to the light
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        pos, view, light = t(pos), t(view), t(light)
        N = int(offsets[-1])
        net = ds.Net(ctx, K, W, H)
        net.set_params(synth.init_params(K, W, H, 19, branch_scale=0.5, out_scale=0.2,
                                         out_bias=0.5))
        try:
            # calibrated on valid points of the first cloud
            ds.ds_net_quantize(ctx.h, net.h, clouds[0].h, ds.DS_PREC_FP8, pos[140:300],
                               view[140:300], light[140:300])
            variants = {ds.DS_PREC_BF16: [(0, 4, 0), (0, 4, 1), (0, 4, 3), (0, 8, 0), (1, 4, 0),
                                          (2, 4, 0), (3, 8, 0), (3, 8, 1), (3, 8, 5)],
                        ds.DS_PREC_FP8: [(0, 4, 0), (0, 4, 1), (0, 8, 2), (3, 8, 0), (3, 8, 5)]}
            for prec, vs in variants.items():
                ref = [[], [], []]
                for c, a, b in zip(clouds, offsets[:-1], offsets[1:]):
                    for r, x in zip(ref, ds.ds_predict(ctx.h, c.h, net.h, prec, pos[a:b],
                                                       view[a:b], light[a:b])):
                        r.append(x)
                ref = [torch.cat(r) for r in ref]
                fl = ref[2].cpu().numpy()
                assert fl[3] == fl[131] == fl[1365] == ds.DS_FLAG_INVALID
                assert fl[70] & ds.DS_FLAG_OUTSIDE and fl[3400] & ds.DS_FLAG_OUTSIDE
                for order in (ds.DS_ORDER_INPUT, ds.DS_ORDER_SPATIAL):
                    bt = ds.ds_batch_create(ctx.h, net.h, [c.h for c in clouds], offsets)
                    try:
                        ds.ds_batch_set_order(bt, order)
                        for v in vs:
                            print("precision", prec, "order", order, "variant", v, flush=True)
                            ds.ds_batch_set_config(bt, *v)
                            got = [torch.full((N,), -1.0, device="cuda"),
                                   torch.full((N,), -1.0, device="cuda"),
                                   torch.full((N,), 255, dtype=torch.uint8, device="cuda")]
                            ds.ds_batch_predict(bt, prec, pos, view, light, *got)
                            for g, r in zip(got, ref):
                                assert torch.equal(g, r), (prec, order, v)
                    finally:
                        ds.ds_batch_destroy(bt)
        finally:
            net.close()
    finally:
        for c in clouds:
            c.close()


@pytest.fixture(scope="module")
def paper_width_batch(ctx):
    # the batched configuration's shape at sizes the oracle handles: five BF16 clouds of
    # 48^3 .. 128^3 (sigma_max = n / unit, fBm + Worley), log-uniform point counts, K = 10
    # stencil levels with the mip levels clamped on the small clouds, W = 200
    sizes = [48, 64, 80, 96, 128]
    rng = np.random.default_rng(210)
    counts = np.exp(rng.uniform(np.log(300), np.log(5000), len(sizes))).astype(np.int64).tolist()
    Kp, Wp = 10, 200
    ws, clouds = [], []
    for i, (n, P) in enumerate(zip(sizes, counts)):
        dens = synth.cloud_density(n, 110 + i, worley=0.3).to(torch.bfloat16)
        L = int(np.ceil(np.log2(n))) + 1
        w = Workload(n, float(n), L=L, K=Kp, P=P, seed_cloud=110 + i, seed_pts=310 + i,
                     density=dens)
        ws.append(w)
        clouds.append(ds.Cloud(ctx, dens.cuda(), w.sigma_max, w.aabb_min, w.h0, w.L, Kp, w.mips))
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    cat = lambda k: torch.from_numpy(np.concatenate([getattr(w, k) for w in ws])).cuda()
    net = ds.Net(ctx, Kp, Wp, 3)
    theta = synth.init_params(Kp, Wp, 3, 12, branch_scale=1 / np.sqrt(Kp), out_scale=0.2,
                              out_bias=0.5)
    net.set_params(theta)
    yield dict(ws=ws, clouds=clouds, counts=counts, offsets=offsets, pos=cat("pos"),
               view=cat("view"), light=cat("light"), net=net, theta=theta, K=Kp, W=Wp)
    net.close()
    for c in clouds:
        c.close()


@pytest.mark.parametrize("prec", [ds.DS_PREC_BF16, ds.DS_PREC_FP8])
def test_paper_width_teams_kernel_matches_register_kernel(ctx, paper_width_batch, prec):
    # the two-team kernel at paper width (ring of ten 13 KB chunks, team lag 6): bitwise the
    # four-wave register kernel's outputs, on one workgroup per tile and on a persistent grid
    s = paper_width_batch
    N = int(s["offsets"][-1])
    if prec == ds.DS_PREC_FP8:
        a, b = int(s["offsets"][-2]), int(s["offsets"][-1])
        ds.ds_net_quantize(ctx.h, s["net"].h, s["clouds"][-1].h, ds.DS_PREC_FP8,
                           s["pos"][a:b].contiguous(), s["view"][a:b].contiguous(),
                           s["light"][a:b].contiguous())
    bt = ds.ds_batch_create(ctx.h, s["net"].h, [c.h for c in s["clouds"]], s["offsets"])
    try:
        ref = torch.full((N,), -1.0, device="cuda")
        ds.ds_batch_predict(bt, prec, s["pos"], s["view"], s["light"], ref)
        for grid in (0, 7, 256):
            print("two-team kernel, precision", prec, "grid", grid, flush=True)
            ds.ds_batch_set_config(bt, ds.DS_KERNEL_TEAMS, 8, grid)
            out = torch.full((N,), -1.0, device="cuda")
            ds.ds_batch_predict(bt, prec, s["pos"], s["view"], s["light"], out)
            assert torch.equal(out, ref), grid
    finally:
        ds.ds_batch_destroy(bt)


@pytest.mark.parametrize("order", [ds.DS_ORDER_INPUT, ds.DS_ORDER_SPATIAL])
@pytest.mark.parametrize("prec,tol", [(ds.DS_PREC_BF16, 2e-2), (ds.DS_PREC_FP8, 5e-2)])
def test_paper_width_batch_autotuned_graph_matches_oracle(ctx, paper_width_batch, prec, tol,
                                                          order):
    s = paper_width_batch
    N = int(s["offsets"][-1])
    if prec == ds.DS_PREC_FP8:  # calibrated on the largest cloud's points, as the bench does
        a, b = int(s["offsets"][-2]), int(s["offsets"][-1])
        ds.ds_net_quantize(ctx.h, s["net"].h, s["clouds"][-1].h, ds.DS_PREC_FP8,
                           s["pos"][a:b].contiguous(), s["view"][a:b].contiguous(),
                           s["light"][a:b].contiguous())
    bt = ds.ds_batch_create(ctx.h, s["net"].h, [c.h for c in s["clouds"]], s["offsets"])
    try:
        ds.ds_batch_set_order(bt, order)
        out = torch.full((N,), -1.0, device="cuda")
        pre = torch.full((N,), -1.0, device="cuda")
        cfg = ds.ds_batch_autotune(bt, prec, s["pos"], s["view"], s["light"], out, 2)
        ds.ds_batch_capture(bt, prec, s["pos"], s["view"], s["light"], out, pre)
        out.fill_(-1.0)
        pre.fill_(-1.0)
        ds.ds_batch_replay(bt)
        torch.cuda.synchronize()
        got, gotp, want, wantp = [], [], [], []
        for w, P, a in zip(s["ws"], s["counts"], s["offsets"]):
            idx = np.arange(0, P, 3)
            z, _ = w.oracle_z(idx)
            g, p = O.forward(s["theta"].astype(np.float64), s["K"], s["W"], 3, z)
            want.append(g)
            wantp.append(p)
            got.append(out.cpu().numpy()[a + idx])
            gotp.append(pre.cpu().numpy()[a + idx])
        e = rel_l2(np.concatenate(gotp), np.concatenate(wantp))
        eg = rel_l2(np.concatenate(got), np.concatenate(want))
        print(f"paper-width batch, precision {prec}, order {order}, {cfg}: relative L2 "
              f"pre-activation {e:.2e}, "
              f"g {eg:.2e}", flush=True)
        assert e <= tol and eg <= tol
    finally:
        ds.ds_batch_destroy(bt)
