"""Environment maps as light sets (Sec. 4.4): the texel solid angles against closed-form
integrals over the sphere, directions, dropping of dark texels, and the synthetic map's lobe."""
import numpy as np
import pytest

from paper_1709_05418_amd import synth


def test_constant_map_integrates_to_four_pi():
    dirs, E = synth.envmap_lights(np.full((16, 32), 0.7))
    assert dirs.shape == (512, 3) and E.shape == (512,)
    assert E.sum() == pytest.approx(4.0 * np.pi * 0.7, rel=1e-12)
    np.testing.assert_allclose(np.linalg.norm(dirs, axis=1), 1.0, atol=1e-6)
    # rows are bands of the polar angle from +y: the first row is near the top
    assert np.all(dirs[:32, 1] > 0.98) and np.all(dirs[-32:, 1] < -0.98)


def test_cosine_map_integrates_to_pi():
    # L = max(0, y) at the texel centres: the integral over the sphere is pi
    H, W = 128, 256
    th = np.pi * (np.arange(H) + 0.5) / H
    L = np.broadcast_to(np.maximum(np.cos(th), 0.0)[:, None], (H, W))
    _, E = synth.envmap_lights(L)
    assert E.sum() == pytest.approx(np.pi, rel=1e-4)
    # irradiance on an up-facing plane: integral of y max(0, y) = 2 pi / 3
    dirs, E = synth.envmap_lights(L, min_radiance=0.0)
    assert np.sum(E * dirs[:, 1]) == pytest.approx(2.0 * np.pi / 3.0, rel=1e-3)
    assert np.all(dirs[:, 1] > 0)   # the lower half is dropped


def test_single_texel():
    L = np.zeros((8, 16))
    L[2, 5] = 3.0
    dirs, E = synth.envmap_lights(L)
    assert E.shape == (1,)
    th, ph = np.pi * 2.5 / 8, 2 * np.pi * 5.5 / 16
    np.testing.assert_allclose(dirs[0], [np.sin(th) * np.cos(ph), np.cos(th),
                                         np.sin(th) * np.sin(ph)], atol=1e-6)
    dw = (np.cos(np.pi * 2 / 8) - np.cos(np.pi * 3 / 8)) * 2 * np.pi / 16
    assert E[0] == pytest.approx(3.0 * dw, rel=1e-12)


def test_synthetic_map_lobe_carries_its_power():
    sun = synth.table1_lights()["side"]
    lobe_only = synth.synthetic_envmap(sun, H=256, W=512, sky_radiance=0.0)
    _, E = synth.envmap_lights(lobe_only)
    # the lobe integrates to 2 pi S w^2 (1 - exp(-2 / w^2)) = lobe_power (1 - exp(-200));
    # the rest is the midpoint rule on 0.7-degree texels
    assert E.sum() == pytest.approx(1.0, rel=2e-2)
    full = synth.synthetic_envmap(sun)
    assert full.shape == (32, 64) and np.all(full > 0)
