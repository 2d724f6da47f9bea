"""Pins of the Lorenz-Mie input generator (synth.mie_amplitudes, cloud_droplet_phase)
against limits and identities of Mie theory: the Rayleigh limit, the optical theorem,
energy conservation for a non-absorbing sphere, the extinction paradox, and the angular
integral of the amplitudes against the series for Q_sca.  CPU only."""
import math

import numpy as np
import pytest

from paper_1709_05418_amd import synth

M = 1.333 + 0j


def test_rayleigh_limit():
    x = 0.01
    mu = np.linspace(-1, 1, 9)
    S1, S2, qe, qs = synth.mie_amplitudes(x, M, mu)
    K = (M * M - 1) / (M * M + 2)
    assert qs == pytest.approx(8.0 / 3.0 * x ** 4 * abs(K) ** 2, rel=1e-4)
    p = (np.abs(S1) ** 2 + np.abs(S2) ** 2) / (2 * math.pi * x * x * qs)
    np.testing.assert_allclose(p, 3.0 / (16 * math.pi) * (1 + mu * mu), rtol=1e-4)


@pytest.mark.parametrize("x", [0.5, 3.0, 17.0, 120.0])
def test_optical_theorem_and_no_absorption(x):
    S1, S2, qe, qs = synth.mie_amplitudes(x, M, np.array([1.0]))
    assert S1[0] == pytest.approx(S2[0], rel=1e-12)
    assert qe == pytest.approx(4.0 / x ** 2 * S1[0].real, rel=1e-10)
    assert qe == pytest.approx(qs, rel=1e-9)


@pytest.mark.parametrize("x", [2.0, 25.0])
def test_angular_integral_matches_the_series(x):
    theta = np.linspace(0, math.pi, 40001)
    S1, S2, _, qs = synth.mie_amplitudes(x, M, np.cos(theta))
    tot = np.trapezoid((np.abs(S1) ** 2 + np.abs(S2) ** 2) * np.sin(theta), theta) * 2 * math.pi
    assert tot == pytest.approx(2 * math.pi * x * x * qs, rel=1e-5)


def test_extinction_paradox():
    _, _, qe, _ = synth.mie_amplitudes(400.0, M, np.array([1.0]))
    assert qe == pytest.approx(2.0, abs=0.05)


def test_droplet_population_phase():
    theta, p, g = synth.cloud_droplet_phase(n_theta=1801, n_r=80)
    norm = np.trapezoid(2 * math.pi * p * np.sin(theta), theta)
    assert norm == pytest.approx(1.0, abs=2e-3)
    assert np.all(p > 0) and p[0] > 1000 * p[len(p) // 2]     # the forward diffraction peak
    # cumulus droplets at 0.55 um: a mean cosine near the 0.857 the paper matches with HG
    assert 0.84 < g < 0.88
