"""Coarser stencils of the same extent as sub-lattices of the 5 x 5 x 9 one (Sec. 4.2 and
Fig. 10, right): point counts, spacings and extents from the offsets' definition, and the
parameter layout that keeps the dropped points' weights at zero."""
import numpy as np
import pytest

from paper_1709_05418_amd import learn, synth


def _offsets(idx):
    ix, iy, iz = idx % 5, (idx // 5) % 5, idx // 25
    return np.stack([-1 + ix / 2, -1 + iy / 2, -1 + iz / 2], 1)


@pytest.mark.parametrize("shape,spacing", [((5, 5, 9), 0.5), ((3, 3, 5), 1.0), ((2, 2, 3), 2.0)])
def test_sub_lattices(shape, spacing):
    idx = learn.stencil_points(shape)
    assert idx.size == np.prod(shape) == np.unique(idx).size
    o = _offsets(idx)
    # same extent in mean free paths, regular spacing on every axis
    np.testing.assert_array_equal(o.min(0), [-1, -1, -1])
    np.testing.assert_array_equal(o.max(0), [1, 1, 3])
    for a, n in zip(range(3), shape):
        np.testing.assert_allclose(np.unique(o[:, a]), -1 + spacing * np.arange(n))


def test_not_a_sub_lattice():
    with pytest.raises(ValueError):
        learn.stencil_points((4, 4, 9))


def test_stencil_params_zero_the_dropped_columns():
    K, W = 3, 8
    keep = learn.stencil_points((3, 3, 5))
    full = learn.stencil_params(K, W, 5, learn.stencil_points((5, 5, 9)), 0.1)
    theta = learn.stencil_params(K, W, 5, keep, 0.1)
    assert theta.size == synth.n_params(K, W, 3)
    drop = np.setdiff1d(np.arange(225), keep)
    for V, Vf in zip(learn.stencil_blocks(theta, K, W), learn.stencil_blocks(full, K, W)):
        assert V.shape == (W, 226)
        assert np.all(V[:, drop] == 0)
        # the kept columns are the full initialisation rescaled for the smaller fan-in
        np.testing.assert_allclose(V[:, keep], Vf[:, keep] * np.sqrt(226 / 46), rtol=1e-6)
        np.testing.assert_array_equal(V[:, 225], Vf[:, 225])
    # everything outside the input matrices is unchanged
    mask = np.ones(theta.size, bool)
    off = 0
    for name, r, c in synth.layer_shapes(K, W, 3):
        n = r * (c if c else 1)
        if name.startswith("V"):
            mask[off:off + n] = False
        off += n
    np.testing.assert_array_equal(theta[mask], full[mask])
