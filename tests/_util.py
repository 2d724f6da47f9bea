"""Shared helpers for the tests: seeded workloads built from the synthetic input
generators, oracle references, and error metrics."""
from __future__ import annotations

import numpy as np
import torch

import oracle as O
from paper_1709_05418_amd import synth


def rel_l2(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / (den if den > 0 else 1.0))


def max_rel(got, ref, floor_frac=1e-3):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    floor = floor_frac * max(np.abs(ref).max(), 1e-30)
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), floor)))


class Workload:
    """A seeded cloud, its oracle normalisation and pyramid, and shading points."""

    def __init__(self, n, sigma_max, L, K, P, seed_cloud=1, seed_pts=3, worley=0.0,
                 device="cpu", density=None):
        if density is None:
            density = synth.cloud_density(n, seed_cloud, worley=worley, device=device)
        self.density = density
        self.d = density.float().cpu().numpy()
        self.n = self.d.shape[::-1]
        self.aabb_min, self.h0 = synth.unit_box(self.n)
        self.sigma_max = float(sigma_max)
        self.L, self.K, self.P = L, K, P
        if density.dtype == torch.bfloat16:
            bits = density.cpu().view(torch.int16).numpy().view(np.uint16)
            self.grid = O.Grid(bits, sigma_max, self.aabb_min, self.h0)
        else:
            self.grid = O.Grid(self.d, sigma_max, self.aabb_min, self.h0)
        self.mean, self.count = O.normalize(self.grid)
        self.mips = O.default_mips(self.mean, self.h0, K, L)
        self._pyr = None
        self.pos = synth.points_in_density(self.d, P, seed_pts, self.aabb_min, self.h0)
        self.view = synth.uniform_dirs(P, seed_pts + 1)
        self.light = synth.uniform_dirs(P, seed_pts + 2)

    @property
    def pyr(self):
        if self._pyr is None:
            self._pyr = O.pyramid(self.grid, self.mean, self.L)
        return self._pyr

    def oracle_z(self, idx=None):
        pyr, dims, offs = self.pyr
        sel = slice(None) if idx is None else idx
        return O.gather(self.grid, pyr, dims, offs, self.mean, self.K, self.mips, self.pos[sel],
                        self.view[sel], self.light[sel])

    def cuda_inputs(self):
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        return t(self.pos), t(self.view), t(self.light)
