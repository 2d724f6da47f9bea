"""Pins of the oracle's training-record estimators beyond L_i (Sec. 5.1, Sec. 7): the
progressive estimate that stops once the mean lies within +-2 % at 95 % confidence,
against the fixed-count estimator on the same streams and its own stopping rule; and
the all-in-scattered target L_s = L_d + L_i against the closed-form direct term of a
homogeneous box and the white furnace.  CPU only."""
import math

import numpy as np

import oracle as O
from paper_1709_05418_amd import synth

from test_oracle_tracer import ramp_int


def small_records(P=40, seed=3):
    n = 16
    d = synth.cloud_density(n, seed=7).numpy()
    grid = O.Grid(d, 16.0, [-0.5] * 3, 1.0 / n)
    pos, view, light, _ = O.sample_records(grid, P, seed)
    return grid, pos, view, light


def test_adaptive_is_the_fixed_estimator_stopped_by_its_rule():
    grid, pos, view, light = small_records()
    batch, top, rel, zq = 32, 2048, 0.3, 1.96   # a loose interval, so that records stop early
    m, v, n = O.trace_li_adaptive(grid, pos, view, light, batch=batch, max_spp=top, rel=rel,
                                  zq=zq, albedo=0.95, g=0.85, seed=9)
    assert np.all(n % batch == 0) and np.all((n >= batch) & (n <= top))
    assert len(set(n.tolist())) > 2          # the records stop at different counts
    for k in sorted(set(n.tolist())):
        sel = n == k
        # the result at n paths is the fixed-count estimate on the same streams (the
        # streams depend on the record index, so the whole set is traced)
        mf, vf = O.trace_li(grid, pos, view, light, albedo=0.95, g=0.85, spp=k, seed=9)
        np.testing.assert_array_equal(m[sel], mf[sel])
        np.testing.assert_array_equal(v[sel], vf[sel])
        met = zq * np.sqrt(vf[sel]) <= rel * np.abs(mf[sel])
        assert np.all(met) if k < top else True
        if k > batch:   # one batch earlier the rule did not hold yet
            mp, vp = O.trace_li(grid, pos, view, light, albedo=0.95, g=0.85, spp=k - batch,
                                seed=9)
            assert not np.any(zq * np.sqrt(vp[sel]) <= rel * np.abs(mp[sel]))


def test_adaptive_stops_at_once_without_scattering_and_flags_bad_records():
    grid, pos, view, light = small_records(P=10)
    view = view.copy()
    view[3] = 0.0
    m, v, n = O.trace_li_adaptive(grid, pos, view, light, batch=16, max_spp=256, albedo=0.0,
                                  seed=2)
    # no path survives its first collision: every estimate is exactly zero after one batch
    assert np.all(m == 0) and np.all(v == 0)
    assert n[3] == 0 and np.all(np.delete(n, 3) == 16)


def test_ls_adds_the_closed_form_direct_term():
    # homogeneous box, light along +z: L_s - L_i at x is p(-w . w_l) exp(-sigma depth) E
    n = 12
    h = 1.0 / n
    grid = O.Grid(np.ones((n, n, n), np.float32), 1.7, [-0.5] * 3, h)
    sigma, gg, E = 1.7, 0.6, 2.0
    zs = np.linspace(-0.3, 0.3, 4)
    pos = np.stack([np.full(4, 0.05), np.full(4, 0.05), zs], 1).astype(np.float32)
    view = np.tile(np.array([[0.6, 0.0, 0.8]], np.float32), (4, 1))
    light = np.tile(np.array([[0.0, 0.0, 1.0]], np.float32), (4, 1))
    spp = 20000
    ms, vs = O.trace_li(grid, pos, view, light, albedo=0.9, g=gg, irradiance=E, spp=spp, seed=4,
                        include_direct=True)
    mi, vi = O.trace_li(grid, pos, view, light, albedo=0.9, g=gg, irradiance=E, spp=spp, seed=5)
    depth = np.array([ramp_int(z + 0.5, 1.0, n, h) for z in zs])
    want = O.hg(gg, -0.8) * np.exp(-sigma * depth) * E
    assert np.all(np.abs((ms - mi) - want) < 5 * np.sqrt(vs + vi)), (ms - mi, want)


def test_ls_white_furnace():
    # albedo 1 in a uniform environment: every path ends by escaping with the
    # environment radiance, so L_s is E exactly with zero variance
    grid, pos, view, light = small_records(P=12)
    m, v = O.trace_li(grid, pos, view, light, albedo=1.0, g=0.85, irradiance=0.75, light_mode=1,
                      spp=64, seed=6, include_direct=True)
    assert np.all(m == 0.75) and np.all(v == 0.0)
    mi, _ = O.trace_li(grid, pos, view, light, albedo=1.0, g=0.85, irradiance=0.75, light_mode=1,
                       spp=64, seed=6)
    assert np.all(mi <= 0.75) and np.any(mi < 0.75)   # L_i misses the uncollided part
    assert math.isfinite(float(mi.sum()))
