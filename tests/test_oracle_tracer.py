"""Pins of the oracle's Monte Carlo transport (Sec. 3.2 Eq. 1, Sec. 4, Sec. 4.4,
Sec. 5.1) against closed forms, quadrature and exact invariants."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O
from paper_1709_05418_amd import synth


def fib_sphere(n):
    i = np.arange(n) + 0.5
    z = 1 - 2 * i / n
    r = np.sqrt(1 - z * z)
    phi = np.pi * (3 - np.sqrt(5)) * i
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], 1)


def ramp(s, n, h):
    """1-D voxel-centred linear interpolation of an all-ones row of n voxels with zero
    padding, at position s measured from the grid face."""
    u = s / h - 0.5
    return np.clip(np.minimum(u + 1.0, n - u), 0.0, 1.0)


def ramp_int(a, b, n, h):
    """Integral of ramp() over [a, b] (closed form, piecewise linear)."""
    def F(s):  # antiderivative on [0, n h]
        s = np.clip(s, 0.0, n * h)
        lo = np.minimum(s, h / 2)
        val = (lo / h + 0.5) * lo - lo * lo / (2 * h)  # int_0^lo (x/h + 1/2) dx
        val = val + np.clip(np.minimum(s, n * h - h / 2) - h / 2, 0, None)
        t = np.clip(s - (n * h - h / 2), 0, h / 2)
        val = val + t - t * t / h  # ramp falls from 1 to 1/2 over the last half voxel
        return val
    return F(b) - F(a)


# ---------------------------------------------------------------- phase function
@pytest.mark.parametrize("g", [0.0, 0.3, 0.85, 0.857, -0.5])
def test_hg_normalised_mean_cosine_and_inverse_cdf(g):
    norm = 2 * np.pi * integrate.quad(lambda m: O.hg(g, m), -1, 1, epsabs=1e-13, limit=200)[0]
    assert norm == pytest.approx(1.0, abs=1e-9)
    mean = 2 * np.pi * integrate.quad(lambda m: m * O.hg(g, m), -1, 1, epsabs=1e-13, limit=200)[0]
    assert mean == pytest.approx(g, abs=1e-9)
    for u in (0.01, 0.2, 0.5, 0.77, 0.99):
        c = O.hg_sample_cos(g, u)
        cdf = 2 * np.pi * integrate.quad(lambda m: O.hg(g, m), -1, c, epsabs=1e-13, limit=200)[0]
        assert cdf == pytest.approx(u, abs=1e-7)
    # stratified sampling reproduces the mean cosine g
    us = (np.arange(200000) + 0.5) / 200000
    cs = np.array([O.hg_sample_cos(g, u) for u in us[::50]])
    assert cs.mean() == pytest.approx(g, abs=2e-3)


# ---------------------------------------------------------------- transmittance
def test_slab_transmittance_closed_form():
    n = 16
    h = 1.0 / n
    prof = np.random.default_rng(1).uniform(0.1, 1.0, n)  # density varies along x only
    d = np.broadcast_to(prof[None, None, :], (n, n, n)).astype(np.float32).copy()
    sigma = 3.0
    g = O.Grid(d, sigma, [-0.5] * 3, h)
    v = prof.astype(np.float32).astype(np.float64)
    tau = sigma * h * (3.0 / 8.0 * (v[0] + v[-1]) + 0.5 * np.sum(v[:-1] + v[1:]))
    R = 8
    rng = np.random.default_rng(2)
    yz = rng.uniform(-0.5 + h, 0.5 - h, (R, 2))
    orig = np.stack([np.full(R, -0.9), yz[:, 0], yz[:, 1]], 1)
    dirs = np.tile([1.0, 0, 0], (R, 1))
    spp = 20000
    ratio, esc = O.transmittance(g, orig, dirs, spp=spp, seed=3)
    T = math.exp(-tau)
    sd = math.sqrt(T * (1 - T) / spp)
    assert np.all(np.abs(esc - T) < 5 * sd)
    assert np.all(np.abs(ratio - T) < 5 * sd)
    assert abs(esc.mean() - T) < 5 * sd / math.sqrt(R)


def test_homogeneous_box_transmittance_along_each_axis():
    n = 12
    h = 1.0 / n
    d = np.ones((n, n, n), np.float32)
    sigma = 1.7
    g = O.Grid(d, sigma, [-0.5] * 3, h)
    T = math.exp(-sigma * (1.0 - h / 4))  # interior sigma, linear fall-off in the outer half voxels
    orig = np.array([[-0.8, 0.1, -0.05], [0.05, 0.9, 0.2], [0.1, -0.1, -3.0]])
    dirs = np.array([[1.0, 0, 0], [0, -2.0, 0], [0, 0, 0.5]])
    spp = 20000
    ratio, esc = O.transmittance(g, orig, dirs, spp=spp, seed=9)
    sd = math.sqrt(T * (1 - T) / spp)
    assert np.all(np.abs(esc - T) < 5 * sd) and np.all(np.abs(ratio - T) < 5 * sd)


@pytest.mark.parametrize("vary,along", [(2, 0), (0, 1), (1, 2)])
def test_transmittance_across_a_profile_reads_the_interpolated_density(vary, along):
    # density varies along axis `vary` only and rays run along axis `along`, at heights
    # that fall at known fractions between two voxel centres: the extinction the ray sees
    # is the linear interpolation of the two voxel values (closed form), constant along the
    # ray except for the half-voxel fall-off at the two faces it crosses
    n = 10
    h = 1.0 / n
    rng = np.random.default_rng(21)
    prof = np.where(np.arange(n) % 2 == 0, 0.2, 0.9) * rng.uniform(0.9, 1.1, n)
    shape = [1, 1, 1]
    shape[2 - vary] = n  # arrays are [z][y][x]
    d = np.broadcast_to(prof.reshape(shape), (n, n, n)).astype(np.float32).copy()
    v = prof.astype(np.float32).astype(np.float64)
    sigma = 1.3
    g = O.Grid(d, sigma, [-0.5] * 3, h)
    other = 3 - vary - along
    cells = [(2, 0.2), (3, 0.8), (5, 0.35), (6, 0.9), (1, 0.6), (7, 0.1)]
    R = len(cells)
    orig = np.zeros((R, 3))
    orig[:, along] = -0.9
    orig[:, other] = rng.uniform(-0.5 + h, 0.5 - h, R)
    orig[:, vary] = [-0.5 + (i + 0.5 + f) * h for i, f in cells]
    dirs = np.zeros((R, 3))
    dirs[:, along] = 1.0
    c = np.array([(1 - f) * v[i] + f * v[i + 1] for i, f in cells])
    T = np.exp(-sigma * c * (1.0 - h / 4))
    spp = 20000
    ratio, esc = O.transmittance(g, orig, dirs, spp=spp, seed=22)
    sd = np.sqrt(T * (1 - T) / spp)
    assert np.all(np.abs(esc - T) < 5 * sd) and np.all(np.abs(ratio - T) < 5 * sd)


# ---------------------------------------------------------------- furnace and zero cases
def test_furnace_every_camera_path_returns_one():
    n = 16
    d = synth.cloud_density(n, 5).numpy()
    g = O.Grid(d, 40.0, [-0.5] * 3, 1.0 / n)
    o = np.tile([0.0, 0.0, 2.0], (32, 1)).astype(np.float32)
    dirs = np.concatenate([fib_sphere(64)[:32] * [0.3, 0.3, 0] + [0, 0, -1.0]]).astype(np.float32)
    mean, var = O.render_pixels(g, o, dirs, [0, 0, 1.0], albedo=1.0, g=0.85, light_mode=1, spp=16,
                                seed=4)
    np.testing.assert_array_equal(mean, 1.0)
    np.testing.assert_array_equal(var, 0.0)


def test_zero_albedo_or_empty_medium_gives_zero():
    n = 8
    d = np.ones((n, n, n), np.float32)
    g = O.Grid(d, 10.0, [-0.5] * 3, 1.0 / n)
    pos = np.zeros((2, 3), np.float32)
    view = np.array([[0, 0, 1], [1, 0, 0]], np.float32)
    light = np.array([[0, 1, 0], [0, 0, -1]], np.float32)
    m, v = O.trace_li(g, pos, view, light, albedo=0.0, spp=64)
    np.testing.assert_array_equal(m, 0.0)
    g0 = O.Grid(np.zeros((n, n, n), np.float32), 10.0, [-0.5] * 3, 1.0 / n)
    m, v = O.trace_li(g0, pos, view, light, albedo=1.0, spp=64)
    np.testing.assert_array_equal(m, 0.0)


# ---------------------------------------------------------------- L_i against quadrature
def _cube_tau(x, dirs, n, h, sigma, steps=3000):
    """Optical depth from x to the box exit along each direction (midpoint rule)."""
    amin = -0.5
    with np.errstate(divide="ignore"):
        tx = np.where(dirs > 0, (0.5 - x) / dirs, np.where(dirs < 0, (-0.5 - x) / dirs, np.inf))
    tmax = tx.min(1)
    out = np.zeros(len(dirs))
    for i in range(len(dirs)):
        t = (np.arange(steps) + 0.5) / steps * tmax[i]
        p = x[None, :] + t[:, None] * dirs[i][None, :] - amin
        mu = sigma * ramp(p[:, 0], n, h) * ramp(p[:, 1], n, h) * ramp(p[:, 2], n, h)
        out[i] = mu.sum() * tmax[i] / steps
    return out


@pytest.mark.parametrize("gph", [0.0, 0.6])
def test_environment_li_at_box_centre_matches_quadrature(gph):
    # With albedo 1 under a uniform environment, L_i = 1 - int p(w.w') T(x, -w') dw'.
    n, sigma = 10, 1.4
    h = 1.0 / n
    g = O.Grid(np.ones((n, n, n), np.float32), sigma, [-0.5] * 3, h)
    x = np.zeros(3)
    w = np.array([0.0, 0.6, 0.8])
    dirs = fib_sphere(6000)
    tau = _cube_tau(x, -dirs, n, h, sigma, steps=600)
    pw = np.array([O.hg(gph, c) for c in dirs @ w])
    expect = 1.0 - np.sum(pw * np.exp(-tau)) * 4 * np.pi / len(dirs)
    spp = 40000
    m, v = O.trace_li(g, x[None].astype(np.float32), w[None].astype(np.float32),
                      np.array([[0, 0, 1.0]], np.float32), albedo=1.0, g=gph, light_mode=1,
                      spp=spp, seed=11)
    assert abs(m[0] - expect) < 5 * math.sqrt(v[0]) + 2e-3, (m[0], expect, math.sqrt(v[0]))


@pytest.mark.parametrize("gph", [0.0, 0.6])
def test_single_scatter_li_matches_quadrature(gph):
    # One interaction, light along +z, an off-centre point in a homogeneous box:
    # L_i = albedo int dw' p(w.w') int du mu(x_u) exp(-tau(x, x_u)) p(w'.(-w_l)) T_light(x_u).
    n, sigma, albedo = 10, 2.0, 0.8
    h = 1.0 / n
    g = O.Grid(np.ones((n, n, n), np.float32), sigma, [-0.5] * 3, h)
    x = np.array([0.2, -0.1, 0.15])
    w = np.array([1.0, 0.0, 0.0])
    dirs = fib_sphere(6000)
    total = 0.0
    steps = 400
    for dw in dirs:
        pw = O.hg(gph, dw @ w) * O.hg(gph, -dw[2])
        back = -dw
        with np.errstate(divide="ignore"):
            tx = np.where(back > 0, (0.5 - x) / back, np.where(back < 0, (-0.5 - x) / back, np.inf))
        tmax = tx.min()
        u = (np.arange(steps) + 0.5) / steps * tmax
        p = x[None, :] + u[:, None] * back[None, :] + 0.5
        rx, ry, rz = ramp(p[:, 0], n, h), ramp(p[:, 1], n, h), ramp(p[:, 2], n, h)
        mu = sigma * rx * ry * rz
        tau = np.concatenate([[0.0], np.cumsum(mu)[:-1]]) * tmax / steps + mu * tmax / steps / 2
        tl = sigma * rx * ry * ramp_int(p[:, 2], 1.0, n, h)  # column optical depth toward +z
        total += pw * np.sum(mu * np.exp(-tau) * np.exp(-tl)) * tmax / steps
    expect = albedo * total * 4 * np.pi / len(dirs)
    spp = 100000
    m, v = O.trace_li(g, x[None].astype(np.float32), w[None].astype(np.float32),
                      np.array([[0, 0, 1.0]], np.float32), albedo=albedo, g=gph, light_mode=0,
                      max_interactions=1, spp=spp, seed=12)
    assert abs(m[0] - expect) < 5 * math.sqrt(v[0]) + 1e-3 * expect, (m[0], expect, math.sqrt(v[0]))


# ---------------------------------------------------------------- record sampler
def test_record_sampler_places_points_in_the_medium():
    n = 24
    d = synth.cloud_density(n, 8).numpy()
    g = O.Grid(d, 60.0, [-0.5] * 3, 1.0 / n)
    N = 3000
    pos, view, light, att = O.sample_records(g, N, seed=5)
    assert np.all(np.isfinite(pos)) and np.all(att >= 1)
    assert np.all(np.abs(pos) <= 0.5 + 1e-6)
    # collisions happen only where the interpolated density is positive
    u = (pos.astype(np.float64) + 0.5) * n - 0.5
    i0 = np.floor(u).astype(int)
    f = u - i0
    val = np.zeros(N)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                c = i0 + [dx, dy, dz]
                ok = np.all((c >= 0) & (c < n), 1)
                w = np.where(dx, f[:, 0], 1 - f[:, 0]) * np.where(dy, f[:, 1], 1 - f[:, 1]) * \
                    np.where(dz, f[:, 2], 1 - f[:, 2])
                cc = np.clip(c, 0, n - 1)
                val += np.where(ok, w * d[cc[:, 2], cc[:, 1], cc[:, 0]], 0)
    assert np.all(val > 0)
    np.testing.assert_allclose(np.linalg.norm(view, axis=1), 1, atol=1e-6)
    np.testing.assert_allclose(np.linalg.norm(light, axis=1), 1, atol=1e-6)
    # light directions are uniform: mean ~ 0, second moments ~ 1/3
    assert np.all(np.abs(light.mean(0)) < 5 / math.sqrt(3 * N))
    np.testing.assert_allclose((light.astype(np.float64) ** 2).mean(0), 1 / 3, atol=0.03)
    # the same seed reproduces the same records
    pos2, _, _, _ = O.sample_records(g, 50, seed=5)
    np.testing.assert_array_equal(pos2, pos[:50])


# ---------------------------------------------------------------- camera samples
def test_first_hits_homogeneous_box_closed_forms():
    # rays along +x through a homogeneous box, light along +z: a ray collides with
    # probability 1 - exp(-tau) and, given a collision, the direct term has mean
    # albedo * p(0) * exp(-sigma * depth toward the light) * E, the same for every
    # collision of that ray because the depth depends on z only
    n = 12
    h = 1.0 / n
    d = np.ones((n, n, n), np.float32)
    sigma, albedo, gg, E = 1.7, 0.9, 0.6, 2.5
    grid = O.Grid(d, sigma, [-0.5] * 3, h)
    R, S = 6, 3000
    zs = np.linspace(-0.35, 0.35, R)
    o = np.stack([np.full(R, -0.9), np.full(R, 0.05), zs], 1).astype(np.float32)
    dirs = np.tile(np.array([[1.0, 0, 0]], np.float32), (R, 1))
    hits = np.zeros(R)
    dsum = np.zeros(R)
    for s in range(S):
        pos, view, direct, hit = O.first_hits(grid, o, dirs, [0, 0, 1], albedo=albedo, g=gg,
                                              irradiance=E, seed=4, sample=s)
        h1 = hit == 1
        assert np.all(np.abs(pos[h1, 1:] - o[h1, 1:]) < 1e-6)   # on the ray
        assert np.all(view[h1] == [-1, 0, 0]) and np.all(direct[~h1] == 0)
        hits += h1
        dsum += direct
    T_ray = math.exp(-sigma * (1.0 - h / 4))
    p_hit = 1 - T_ray
    sd = math.sqrt(p_hit * (1 - p_hit) / S)
    assert np.all(np.abs(hits / S - p_hit) < 5 * sd)
    depth = np.array([ramp_int(z + 0.5, 1.0, n, h) for z in zs])  # optical depth / sigma to the top
    T_up = np.exp(-sigma * depth)
    want = albedo * O.hg(gg, 0.0) * T_up * E
    mean = dsum / hits
    sd_d = albedo * O.hg(gg, 0.0) * E * np.sqrt(T_up * (1 - T_up) / hits) + 1e-12
    assert np.all(np.abs(mean - want) < 5 * sd_d), (mean, want)
