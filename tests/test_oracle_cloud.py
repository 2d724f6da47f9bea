"""Pins of the oracle's scale normalisation (Sec. 4.2 / Sec. 5) and Gaussian
mipmap (Sec. 6) against closed forms, brute force and invariants."""
import math

import numpy as np
import pytest

import oracle as O


def grid(d, sigma_max=8.0):
    n = d.shape
    h0 = 1.0 / max(n)
    amin = [-0.5 * n[2] * h0, -0.5 * n[1] * h0, -0.5 * n[0] * h0]
    return O.Grid(d.astype(np.float32), sigma_max, amin, h0)


# ---------------------------------------------------------------- normalisation
def test_normalize_half_filled_closed_form():
    d = np.zeros((6, 5, 4), np.float32)
    d[:3] = 0.375
    m, c = O.normalize(grid(d, sigma_max=16.0))
    assert c == 3 * 5 * 4
    assert m == pytest.approx(16.0 * 0.375, rel=1e-15)


def test_normalize_mixed_values_ignores_zeros():
    d = np.zeros((4, 4, 4), np.float32)
    d[0, 0, 0], d[1, 2, 3], d[3, 3, 3] = 0.25, 0.5, 1.0
    m, c = O.normalize(grid(d, sigma_max=10.0))
    assert c == 3
    assert m == pytest.approx(10.0 * (0.25 + 0.5 + 1.0) / 3, rel=1e-15)


def test_normalize_bf16_input():
    d = np.zeros((4, 4, 4), np.float32)
    d[1] = 0.75  # exactly representable in bf16
    bits = (d.view(np.uint32) >> 16).astype(np.uint16)
    g = O.Grid(bits, 4.0, [-0.5] * 3, 0.25)
    m, c = O.normalize(g)
    assert c == 16 and m == pytest.approx(3.0, rel=1e-15)


def test_normalize_empty_grid_is_an_error():
    with pytest.raises(ValueError):
        O.normalize(grid(np.zeros((3, 3, 3), np.float32)))


# ---------------------------------------------------------------- pyramid
def test_level_dims_and_layout():
    dims, offs, total = O.pyramid_layout(100, 37, 64, 8)
    assert dims[0].tolist() == [100, 37, 64]
    assert dims[1].tolist() == [50, 19, 32]
    assert dims[3].tolist() == [13, 5, 8]
    assert dims[7].tolist() == [1, 1, 1]
    assert offs[0] == 0 and total == sum(int(np.prod(d)) for d in dims)


@pytest.mark.parametrize("level", [0, 1, 2, 5, 9])
def test_gauss_norm_matches_integral(level):
    # The normaliser sums the kernel over the lattice within 3 sigma; by the midpoint
    # rule it equals sigma*sqrt(2 pi)*erf(3/sqrt 2) up to O(1/sigma^2).
    s = 2.0 ** level
    approx = s * math.sqrt(2 * math.pi) * math.erf(3 / math.sqrt(2))
    z = O.gauss_norm(level)
    if level == 0:
        exact = sum(math.exp(-t * t / 2) for t in range(-3, 4))
        assert z == pytest.approx(exact, rel=1e-15)
    else:
        assert abs(z / approx - 1) < 0.2 / s ** 2 + 1e-12


def _brute_level(rho, level):
    """Non-separable 3-D sum of the normalised, truncated Gaussian, per output voxel."""
    nz, ny, nx = rho.shape
    s = 2.0 ** level
    lattice = np.arange(-int(3 * s) - 1, int(3 * s) + 2, dtype=np.float64)
    lattice = lattice if level == 0 else lattice + 0.5
    lattice = lattice[np.abs(lattice) <= 3 * s]
    Z = np.exp(-lattice ** 2 / (2 * s * s)).sum()
    dims = [max(1, -(-n // int(s))) for n in (nx, ny, nz)]
    out = np.zeros((dims[2], dims[1], dims[0]))
    jz, jy, jx = (np.arange(n) + 0.5 for n in (nz, ny, nx))
    for mz in range(dims[2]):
        for my in range(dims[1]):
            for mx in range(dims[0]):
                tz = jz - (mz + 0.5) * s
                ty = jy - (my + 0.5) * s
                tx = jx - (mx + 0.5) * s
                w = np.exp(-(tz[:, None, None] ** 2 + ty[None, :, None] ** 2 + tx[None, None, :] ** 2)
                           / (2 * s * s))
                w *= (np.abs(tz)[:, None, None] <= 3 * s) & (np.abs(ty)[None, :, None] <= 3 * s) \
                    & (np.abs(tx)[None, None, :] <= 3 * s)
                out[mz, my, mx] = (w * rho).sum() / Z ** 3
    return out


@pytest.mark.parametrize("shape", [(8, 9, 10), (12, 12, 12), (16, 11, 7)])
def test_pyramid_equals_bruteforce_3d_sum(shape):
    rng = np.random.default_rng(7)
    d = rng.random(shape).astype(np.float32)
    d[d < 0.3] = 0
    g = grid(d, sigma_max=5.0)
    m, _ = O.normalize(g)
    L = 4
    pyr, dims, offs = O.pyramid(g, m, L)
    rho = 5.0 * d.astype(np.float64) / m
    for lv in range(L):
        ref = _brute_level(rho, lv)
        got = O.level(pyr, dims, offs, lv)
        assert got.shape == ref.shape
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13)


def test_pyramid_constant_field_is_constant_in_interior():
    n = 64
    d = np.full((n, n, n), 0.5, np.float32)
    g = grid(d, sigma_max=4.0)
    m, _ = O.normalize(g)
    assert m == pytest.approx(2.0)
    pyr, dims, offs = O.pyramid(g, m, 4)
    for lv in range(4):
        s = 2 ** lv
        P = O.level(pyr, dims, offs, lv)
        c = (np.arange(P.shape[0]) + 0.5) * s - 0.5  # centre in base-index units
        inside = (c - 3 * s >= -0.5) & (c + 3 * s <= n - 0.5)
        sub = P[np.ix_(inside, inside, inside)]
        assert sub.size > 0
        np.testing.assert_allclose(sub, 1.0, rtol=0, atol=1e-13)
        # at the faces the zero padding darkens the value (no renormalisation)
        assert P[0, P.shape[1] // 2, P.shape[2] // 2] < 1.0 - 1e-3


def test_pyramid_preserves_affine_field_in_interior():
    n = 48
    z, y, x = np.meshgrid(*(np.arange(n) + 0.5,) * 3, indexing="ij")
    d = (0.2 + 0.004 * x + 0.006 * y + 0.003 * z).astype(np.float32)
    g = grid(d, sigma_max=3.0)
    m, _ = O.normalize(g)
    rho = 3.0 * d.astype(np.float64) / m
    a = np.array([0.004, 0.006, 0.003]) * 3.0 / m  # d rho / d index along x, y, z
    pyr, dims, offs = O.pyramid(g, m, 3)
    for lv in range(3):
        s = 2 ** lv
        P = O.level(pyr, dims, offs, lv)
        c = (np.arange(P.shape[0]) + 0.5) * s  # centre in base *position* units (index + 0.5)
        inside = (c - 3 * s >= 0) & (c + 3 * s <= n)
        cz, cy, cx = np.meshgrid(c, c, c, indexing="ij")
        # affine field evaluated at the level-i voxel centre
        f = 3.0 * 0.2 / m + a[0] * cx + a[1] * cy + a[2] * cz
        # rho was built from float32 d, so compare against the float32 field's own affine fit
        sel = np.ix_(inside, inside, inside)
        np.testing.assert_allclose(P[sel], f[sel], rtol=2e-6)
    assert rho.max() > 0


def test_pyramid_impulse_response_is_sampled_gaussian():
    n = 40
    d = np.zeros((n, n, n), np.float32)
    j = (17, 22, 19)  # (z, y, x)
    d[j] = 1.0
    g = grid(d, sigma_max=2.0)
    m, _ = O.normalize(g)
    assert m == 2.0
    pyr, dims, offs = O.pyramid(g, m, 4)
    for lv in range(4):
        s = 2.0 ** lv
        Z = O.gauss_norm(lv)
        P = O.level(pyr, dims, offs, lv)
        mz, my, mx = np.meshgrid(*(np.arange(k) for k in P.shape), indexing="ij")
        t = [(j[0] + 0.5) - (mz + 0.5) * s, (j[1] + 0.5) - (my + 0.5) * s, (j[2] + 0.5) - (mx + 0.5) * s]
        w = np.ones_like(P)
        for ta in t:
            w = w * np.where(np.abs(ta) <= 3 * s, np.exp(-ta * ta / (2 * s * s)), 0.0) / Z
        np.testing.assert_allclose(P, w, rtol=1e-12, atol=1e-300)


def test_default_mip_rule():
    # level-1 stencil spacing 0.5/mean; 0.5/(mean*h0) = 1 voxel -> delta 0, one level per k
    assert O.default_mips(32.0, 1 / 64, 6, 6).tolist() == [0, 1, 2, 3, 4, 5]
    # spacing of 2 voxels -> delta 1, clamped at the top
    assert O.default_mips(16.0, 1 / 64, 6, 6).tolist() == [1, 2, 3, 4, 5, 5]
    # very dense cloud: spacing a quarter voxel -> negative delta clamps to level 0
    assert O.default_mips(128.0, 1 / 64, 4, 6).tolist() == [0, 0, 0, 1]
