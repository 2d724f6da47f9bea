"""Training-record estimators on the GPU beyond fixed-count L_i (Sec. 5.1, Sec. 7): the
all-in-scattered target L_s and the progressive estimate that stops at +-rel with
normal-quantile confidence, against the FP64 oracle on the same random streams."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1709_05418_amd as ds
from _util import Workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = ds.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def small():
    return Workload(32, 32.0, L=5, K=5, P=96 + 5, seed_cloud=4, seed_pts=21)


@pytest.fixture(scope="module")
def small_cloud(ctx, small):
    c = ds.Cloud(ctx, small.density.cuda(), small.sigma_max, small.aabb_min, small.h0, small.L,
                 small.K, small.mips)
    yield c
    c.close()


def _agree(m, v, mo, vo, z=5.0):
    tol = z * np.sqrt(v + vo) + 1e-7 * max(1.0, np.abs(mo).max())
    return np.flatnonzero(np.abs(m - mo) > tol)


@pytest.mark.parametrize("mode", [0, 1])
def test_ls_records_match_oracle(ctx, small_cloud, small, mode):
    spp, seed = 48, 77
    prm = ds.TracerParams(0.95, 0.85, 1.5, mode, 0, include_direct=1)
    pos, view, light = small.cuda_inputs()
    m, v = ds.ds_trace_li(ctx.h, small_cloud.h, prm, pos, view, light, spp, seed)
    m, v = m.cpu().numpy(), v.cpu().numpy()
    mo, vo = O.trace_li(small.grid, small.pos, small.view, small.light, albedo=0.95, g=0.85,
                        irradiance=1.5, light_mode=mode, spp=spp, seed=seed, include_direct=True)
    assert _agree(m, v, mo, vo).size == 0
    assert np.median(np.abs(m - mo) / np.maximum(np.abs(mo), 1e-6)) < 1e-3
    # L_s exceeds L_i on average by the direct term
    mi, _ = ds.ds_trace_li(ctx.h, small_cloud.h, ds.TracerParams(0.95, 0.85, 1.5, mode, 0), pos,
                           view, light, spp, seed)
    assert m.sum() > mi.cpu().numpy().sum()


@pytest.mark.parametrize("include_direct,batch", [(0, 32), (1, 32), (0, 64), (1, 128)])
def test_adaptive_matches_oracle(ctx, small_cloud, small, include_direct, batch):
    # batches of 32 paths: one batch per round; 64 and 128 (whole blocks): rounds of several
    # batches for the records still running, the rule applied after each batch in order
    top, rel, zq, seed = 1024, 0.3, 1.96, 5
    prm = ds.TracerParams(0.95, 0.85, 1.0, 0, 0, include_direct)
    ad = ds.Adaptive(batch, top, rel, zq)
    pos, view, light = small.cuda_inputs()
    m, v, n = (t.cpu().numpy() for t in ds.ds_trace_li_adaptive(ctx.h, small_cloud.h, prm, ad,
                                                                  pos, view, light, seed))
    mo, vo, no = O.trace_li_adaptive(small.grid, small.pos, small.view, small.light, batch=batch,
                                     max_spp=top, rel=rel, zq=zq, albedo=0.95, g=0.85,
                                     seed=seed, include_direct=bool(include_direct))
    assert np.all(n % batch == 0) and np.all((n >= batch) & (n <= top))
    assert len(set(n.tolist())) > 2
    # the same stopping point on (nearly) every record: decided on FP32 paths here and
    # FP64 paths in the oracle, so a record at the boundary may stop a batch apart
    same = n == no
    assert same.mean() > 0.95, same.mean()
    assert _agree(m[same], v[same], mo[same], vo[same]).size == 0
    assert np.median(np.abs(m[same] - mo[same]) / np.maximum(np.abs(mo[same]), 1e-6)) < 1e-3
    # every record that stopped early meets the rule with its own estimate
    early = n < top
    assert np.all(zq * np.sqrt(v[early]) <= rel * np.abs(m[early]) * (1 + 1e-12))
    # and its estimate is the fixed-count one at that many paths, up to summation order
    k = int(np.median(n[early]))
    sel = n == k
    mf, _ = ds.ds_trace_li(ctx.h, small_cloud.h, prm, pos, view, light, k, seed)
    np.testing.assert_allclose(m[sel], mf.cpu().numpy()[sel], rtol=1e-12, atol=1e-15)


def test_make_records_adaptive(ctx, small_cloud, small):
    N, seed, stride, off = 300, 41, 2, 1
    prm = ds.TracerParams(0.95, 0.85, 1.0, 0, 0)
    ad = ds.Adaptive(32, 512, 0.3, 1.96)
    D = 225 * small.K + 1
    z = torch.full((off + (N - 1) * stride + 1, D), -7.0, dtype=torch.float32, device="cuda")
    t = torch.full((z.shape[0],), -7.0, dtype=torch.float32, device="cuda")
    (pos, view, light), (m, v, n) = ds.ds_make_records(ctx.h, small_cloud.h, prm, N, ad, seed, z,
                                                       t, offset=off, stride=stride,
                                                       want_records=True, want_li=True)
    # the same records and descriptors as the fixed-count call
    z2 = torch.zeros_like(z)
    t2 = torch.zeros_like(t)
    (pos2, _, _), _ = ds.ds_make_records(ctx.h, small_cloud.h, prm, N, 64, seed, z2, t2,
                                         offset=off, stride=stride, want_records=True)
    rows = off + stride * np.arange(N)
    assert torch.equal(pos, pos2) and torch.equal(z[rows], z2[rows])
    tc, m, v, n = t.cpu().numpy(), m.cpu().numpy(), v.cpu().numpy(), n.cpu().numpy()
    assert np.allclose(tc[rows], np.log1p(m.astype(np.float32)), rtol=1e-6, atol=1e-7)
    assert np.all(np.delete(tc, rows) == -7.0)
    # the progressive estimate on the records' own streams (the derived key of the seed)
    _, _, n_again = ds.ds_trace_li_adaptive(ctx.h, small_cloud.h, prm, ad, pos, view, light,
                                            derived_key(seed))
    np.testing.assert_array_equal(n, n_again.cpu().numpy())
    assert len(set(n.tolist())) > 2


def derived_key(seed, which=0):
    M64 = (1 << 64) - 1
    z = (seed + 0x9E3779B97F4A7C15 * (which + 1)) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def test_render_calls_reject_ls_params(ctx, small_cloud):
    prm = ds.TracerParams(0.9, 0.85, 1.0, 0, 0, include_direct=1)
    o = torch.zeros((4, 3), dtype=torch.float32, device="cuda")
    d = torch.ones((4, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(ds.DSError):
        ds.ds_render_mc(ctx.h, small_cloud.h, prm, (1, 0, 0), o, d, 4, 1)
    with pytest.raises(ds.DSError):
        ds.ds_first_hits(ctx.h, small_cloud.h, prm, (1, 0, 0), o, d, 1)
    with pytest.raises(ds.DSError):
        ds.ds_trace_li_adaptive(ctx.h, small_cloud.h, ds.TracerParams(), ds.Adaptive(32, 100),
                                o, d, d, 1)


def test_adaptive_rounds_do_not_change_results(ctx, small_cloud):
    # batches of 64 paths are whole blocks, so a round may trace several batches ahead: 16
    # at once for 101 records, fewer while 8192 records still run.  Record i keeps its
    # streams (i * 2^20 + s) either way, so the first 101 records of the large set must give
    # bitwise the estimates and path counts of the 101 alone.
    prm = ds.TracerParams(0.95, 0.85, 1.0, 0, 0)
    ad = ds.Adaptive(64, 1024, 0.2, 1.96)
    pos, view, light, _ = ds.ds_sample_records(ctx.h, small_cloud.h, 8192, 31)
    big = ds.ds_trace_li_adaptive(ctx.h, small_cloud.h, prm, ad, pos, view, light, 9)
    few = ds.ds_trace_li_adaptive(ctx.h, small_cloud.h, prm, ad, pos[:101].contiguous(),
                                  view[:101].contiguous(), light[:101].contiguous(), 9)
    for a, b in zip(big, few):
        assert torch.equal(a[:101], b)
    n = big[2].cpu().numpy()
    assert len(set(n.tolist())) > 3 and (n < 1024).any()
