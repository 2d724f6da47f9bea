"""The sphere-and-box judge scene (Sec. 7, non-cloud shaped objects): the occupied volume
against the closed-form volume of the union, and the values on and off the two shapes."""
import math

import numpy as np
import torch

from paper_1709_05418_amd import synth


def test_sphere_box_volume_and_values():
    n = 96
    d = synth.sphere_box_density(n)
    assert d.shape == (n, n, n) and d.dtype == torch.float32
    assert set(torch.unique(d).tolist()) == {0.0, 1.0}
    # union volume: sphere + box - their overlap, the overlap by Monte Carlo in FP64
    (cx, cy, cz), r = (-0.14, 0.0, 0.0), 0.2
    lo, hi = np.array([0.02, -0.15, -0.15]), np.array([0.32, 0.15, 0.15])
    p = np.random.default_rng(0).uniform(lo, hi, (400000, 3))
    in_sphere = ((p - [cx, cy, cz]) ** 2).sum(1) <= r * r
    v_box = float(np.prod(hi - lo))
    v_union = 4.0 / 3.0 * math.pi * r ** 3 + v_box - v_box * in_sphere.mean()
    frac = float(d.double().mean())
    assert abs(frac - v_union) < 0.03 * v_union, (frac, v_union)
    # voxel centres: inside the sphere, inside the box, and the empty corner
    c = lambda x: int((x + 0.5) * n)
    assert d[c(0.0), c(0.0), c(-0.14)] == 1.0
    assert d[c(0.1), c(0.1), c(0.25)] == 1.0
    assert d[c(0.4), c(0.4), c(0.4)] == 0.0
    assert d[c(0.0), c(0.3), c(-0.14)] == 0.0


def test_sphere_box_bf16_and_slabs_agree():
    a = synth.sphere_box_density(40, slab=7)
    b = synth.sphere_box_density(40, dtype=torch.bfloat16)
    assert torch.equal(a, b.float())
