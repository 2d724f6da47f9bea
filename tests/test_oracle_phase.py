"""Pins of the oracle's tabulated phase functions (Sec. 5.1: a chopped Lorenz-Mie
table for data generation and rendering, the unchopped one for the direct term at the
first collision, in the optically thinner medium of Sec. 3.1): the table's normalisation
and chopped mass, its sampling against the table's own moments, a Henyey-Greenstein table
against the analytic function inside the tracer, and the chopped set-up against the full
function's single-scattering integral in a thin homogeneous box.  CPU only."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O
from paper_1709_05418_amd import synth

from test_oracle_tracer import ramp_int


def hg_table(g, n=3601):
    theta = np.linspace(0, math.pi, n)
    return np.array([O.hg(g, c) for c in np.cos(theta)])


@pytest.fixture
def clean_phase():
    yield
    O.set_phase(None)


def test_table_normalisation_and_chop():
    theta, p, _ = synth.cloud_droplet_phase(n_theta=1801, n_r=60)
    t = O.phase_table(p)
    assert t["removed"] == 0.0 and t["cdf"][0] == 0.0 and t["cdf"][-1] == 1.0
    assert np.all(np.diff(t["cdf"]) >= 0)
    t0 = O.phase_table(p, chop_deg=0.0)
    np.testing.assert_array_equal(t0["p"], t["p"])
    c = O.phase_table(p, chop_deg=5.0)
    ic = int(round(math.radians(5.0) / (math.pi / 1800)))
    # above the chop angle the chopped function is the original over (1 - f)
    np.testing.assert_allclose(c["p"][ic:] * (1 - c["removed"]), t["p"][ic:], rtol=1e-12)
    assert np.all(c["p"][:ic] == c["p"][ic])
    assert 0.2 < c["removed"] < 0.6            # the diffraction peak holds a large share
    assert c["g"] < t["g"]


@pytest.mark.parametrize("g", [0.0, 0.5, 0.857])
def test_hg_table_moments_and_sampling(g):
    t = O.phase_table(hg_table(g))
    assert t["g"] == pytest.approx(g, abs=2e-3)
    us = (np.arange(20000) + 0.5) / 20000
    mus = np.array([O.tab_sample(t, u) for u in us])
    assert np.all(np.diff(mus) <= 1e-15)        # monotone in u
    assert mus.mean() == pytest.approx(t["g"], abs=1e-3)
    # the drawn cosines follow the analytic inverse CDF of HG (the table walks theta
    # upward, the analytic form mu upward: u and 1 - u)
    ref = np.array([O.hg_sample_cos(g, 1 - u) for u in us[::97]])
    np.testing.assert_allclose(mus[::97], ref, atol=5e-3)


def test_table_lookup_is_linear_in_theta_between_nodes():
    # a table sampled from a function linear in theta is read back exactly between its
    # nodes, and any table is read back at its nodes (coarse, so that a lookup that does
    # not interpolate is far off)
    n = 7
    theta = np.linspace(0, math.pi, n)
    rng = np.random.default_rng(5)
    for th in np.concatenate([rng.uniform(0, math.pi, 60), theta]):
        assert O.tab_eval(0.3 + 0.5 * theta, math.cos(th)) == pytest.approx(0.3 + 0.5 * th,
                                                                         rel=1e-7)
    p = rng.uniform(0.1, 2.0, n)
    for i, th in enumerate(theta):
        assert O.tab_eval(p, math.cos(th)) == pytest.approx(p[i], rel=1e-7)


def test_table_sampling_inverts_the_piecewise_linear_cdf():
    # coarse table: the drawn angle follows the density p sin(theta) taken linear in theta
    # between the nodes (the density that the trapezoid cdf integrates exactly); checked
    # by quadrature of that density up to the drawn angle
    n = 6
    p = np.random.default_rng(8).uniform(0.2, 3.0, n)
    t = O.phase_table(p)
    theta = np.linspace(0, math.pi, n)
    f = t["p"] * np.sin(theta)

    def dens(x):
        return np.interp(x, theta, f)

    total = integrate.quad(dens, 0, math.pi, points=theta[1:-1], limit=200)[0]
    for u in (0.03, 0.2, 0.41, 0.5, 0.66, 0.9, 0.99):
        th = math.acos(O.tab_sample(t, u))
        inner = [x for x in theta[1:-1] if x < th]
        F = integrate.quad(dens, 0, th, points=inner or None, limit=200)[0]
        assert F / total == pytest.approx(u, abs=1e-8)


def test_hg_table_in_the_tracer_matches_analytic_hg(clean_phase):
    n = 16
    d = synth.cloud_density(n, seed=7).numpy()
    grid = O.Grid(d, 16.0, [-0.5] * 3, 1.0 / n)
    pos, view, light, _ = O.sample_records(grid, 24, 3)
    m0, v0 = O.trace_li(grid, pos, view, light, albedo=0.95, g=0.7, spp=3000, seed=2)
    O.set_phase(O.phase_table(hg_table(0.7)))
    m1, v1 = O.trace_li(grid, pos, view, light, albedo=0.95, g=0.7, spp=3000, seed=2)
    assert np.all(np.abs(m0 - m1) < 5 * np.sqrt(v0 + v1) + 1e-12)
    assert np.any(m0 != m1)


def _thin_box_full_model(sigma, albedo, p_first, E, n, h, z0):
    """Expected first-collision direct term of one camera ray along +x through a homogeneous
    box (trilinear density rx(x) ry(y) rz(z), ry = rz = 1 at the ray) lit from +z, for the
    unchopped phase function and the unreduced medium: the integral over the collision point
    of sigma r(x) exp(-sigma R(x)) (collision density), times albedo p E exp(-sigma r(x) Rz)
    (transmittance to the light), by adaptive quadrature."""
    Rz = ramp_int(z0 + 0.5, 1.0, n, h)

    def r(s):
        return min(1.0, 0.5 + s / h, 0.5 + (1.0 - s) / h)

    def f(s):
        return sigma * r(s) * math.exp(-sigma * ramp_int(0.0, s, n, h)) * math.exp(-sigma * r(s) * Rz)

    val, _ = integrate.quad(f, 0.0, 1.0, points=[h / 2, 1.0 - h / 2], epsabs=1e-14, limit=200)
    return albedo * p_first * E * val, Rz


@pytest.mark.parametrize("chop", [0.5, 5.0, 20.0])
def test_chopped_set_up_matches_full_function_in_a_thin_medium(clean_phase, chop):
    # Sec. 3.1: the chopped function in the thinner medium with the full function at the
    # first bounce stands in for the full function in the original medium.  Single
    # scattering dominates an optically thin medium, so there the set-up's first-collision
    # direct term must equal the full model's single-scattering integral, up to the
    # attenuation the thinner medium saves: 1 <= ratio <= exp(sigma (1 + Rz)).  A dropped
    # first-collision weight (x (1 - f)), an unreduced albedo (x (1 - a f) / (1 - f)) or
    # extinction scaled by 1 - f would leave that band by tens of per cent (f = 0.44 at 5 deg).
    n, h, sigma, albedo, E = 8, 1.0 / 8, 0.03, 0.5, 2.0
    grid = O.Grid(np.ones((n, n, n), np.float32), sigma, [-0.5] * 3, h)
    _, p, _ = synth.cloud_droplet_phase(n_theta=1801, n_r=60)
    full, chopped = O.phase_table(p), O.phase_table(p, chop_deg=chop)
    assert chopped["removed"] > 0.0
    p90 = full["p"][900]                         # theta = 90 degrees is node 900
    want, Rz = _thin_box_full_model(sigma, albedo, p90, E, n, h, 0.1)
    N = 1 << 20
    o = np.tile(np.array([[-0.9, 0.05, 0.1]], np.float32), (N, 1))
    d = np.tile(np.array([[1.0, 0.0, 0.0]], np.float32), (N, 1))

    def mean_se(table, first):
        O.set_phase(table, first=first)
        _, _, direct, _ = O.first_hits(grid, o, d, [0, 0, 1], albedo=albedo, irradiance=E, seed=9)
        return direct.mean(), direct.std() / math.sqrt(N)

    m_full, se_full = mean_se(full, None)        # the full model itself, unthinned
    assert abs(m_full - want) < 5 * se_full
    m, se = mean_se(chopped, full)
    assert want - 5 * se <= m <= want * math.exp(sigma * (1.0 + Rz)) + 5 * se, (m, want)
    # without the full function at the first bounce the chopped set-up is (1 - f) darker
    m_c, se_c = mean_se(chopped, None)
    assert m_c == pytest.approx(m * (1 - chopped["removed"]) * chopped["p"][900] / p90, rel=1e-9)


def test_unchopped_table_leaves_the_medium_alone(clean_phase):
    # f = 0: no thinning, no weight; the full table as "chopped" table and first table gives
    # exactly the full set-up's estimates on the same streams
    n, h = 8, 1.0 / 8
    grid = O.Grid(np.ones((n, n, n), np.float32), 3.0, [-0.5] * 3, h)
    _, p, _ = synth.cloud_droplet_phase(n_theta=1801, n_r=60)
    full, zero = O.phase_table(p), O.phase_table(p, chop_deg=0.0)
    assert zero["removed"] == 0.0
    o = np.tile(np.array([[-0.9, 0.05, 0.1]], np.float32), (4096, 1))
    d = np.tile(np.array([[1.0, 0.0, 0.0]], np.float32), (4096, 1))
    O.set_phase(full)
    a = O.first_hits(grid, o, d, [0, 0, 1], albedo=0.7, irradiance=1.0, seed=3)
    O.set_phase(zero, first=full)
    b = O.first_hits(grid, o, d, [0, 0, 1], albedo=0.7, irradiance=1.0, seed=3)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_first_collision_closed_form_of_the_reading(clean_phase):
    # The reading's closed form in a thicker homogeneous box, rays along +x, light along +z
    # (restates the reading, so it is a consistency check; the thin-medium test above is
    # the independent pin): with a chopped table the medium is thinned to extinction
    # sigma (1 - a f) and the direct term of a collision has mean
    # a (1 - f) / (1 - a f) / (1 - f) p_first(90 deg) exp(-sigma (1 - a f) depth) E.
    n = 12
    h = 1.0 / n
    grid = O.Grid(np.ones((n, n, n), np.float32), 1.7, [-0.5] * 3, h)
    theta, p, _ = synth.cloud_droplet_phase(n_theta=1801, n_r=60)
    full, chop = O.phase_table(p), O.phase_table(p, chop_deg=5.0)
    O.set_phase(chop, first=full)
    a, f = 0.9, chop["removed"]
    R, S = 4, 2500
    zs = np.linspace(-0.3, 0.3, R)
    o = np.stack([np.full(R, -0.9), np.full(R, 0.05), zs], 1).astype(np.float32)
    dirs = np.tile(np.array([[1.0, 0, 0]], np.float32), (R, 1))
    hits, dsum = np.zeros(R), np.zeros(R)
    for s in range(S):
        _, _, direct, hit = O.first_hits(grid, o, dirs, [0, 0, 1], albedo=a, irradiance=2.0,
                                         seed=4, sample=s)
        hits += hit == 1
        dsum += direct
    p90 = full["p"][900]
    assert p90 != chop["p"][900]
    T = np.exp(-1.7 * (1 - a * f) * np.array([ramp_int(z + 0.5, 1.0, n, h) for z in zs]))
    w = a * (1 - f) / (1 - a * f) / (1 - f)
    want = w * p90 * T * 2.0
    sd = w * p90 * 2.0 * np.sqrt(T * (1 - T) / hits)
    assert np.all(np.abs(dsum / hits - want) < 5 * sd + 1e-12)


@pytest.mark.skipif(not __import__("os").path.exists(__import__("paper_1709_05418_amd").LIB_PATH),
                    reason="libdeepscatter.so not built")
@pytest.mark.parametrize("chop", [0.0, 5.0, 20.0])
def test_library_phase_table_matches_oracle(chop):
    import paper_1709_05418_amd as ds
    theta, p, _ = synth.cloud_droplet_phase(n_theta=1801, n_r=60)
    q, c, rem, g = ds.ds_phase_build(p, chop)
    t = O.phase_table(p, chop_deg=chop)
    np.testing.assert_allclose(q, t["p"], rtol=1e-12)
    np.testing.assert_allclose(c, t["cdf"], rtol=1e-12, atol=1e-15)
    assert rem == pytest.approx(t["removed"], rel=1e-10, abs=1e-15)
    assert g == pytest.approx(t["g"], rel=1e-12)
    for bad in ([1.0], [1.0, 2.0], [1.0, -1.0, 1.0], [np.nan, 1.0, 1.0]):
        with pytest.raises(ds.DSError):
            ds.ds_phase_build(bad)
