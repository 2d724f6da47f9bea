"""FP64 CPU oracle for the Deep Scattering radiance-prediction path.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The GPU library never imports, links or runs it,
and it shares no code with the library (`oracle.c` is compiled on its own with
gcc).  Inputs are host numpy arrays; results are float64.

What each part follows in the paper and what pins it (tests/test_oracle_*.py):
  normalize       Sec. 4.2 / Sec. 5 scale normalisation     closed form on constructed grids
  pyramid         Sec. 6 Gaussian mipmap, sigma_i = 2^i     brute-force 3-D sum, constant/affine
                                                            fields, impulse response, unit mass
  frame           Sec. 4.2 local frame, gamma               closed form (0, sin g, cos g), det +1
  gather          Sec. 4.2 / Fig. 5 hierarchical stencil    affine-field exactness, constant grid,
                                                            cube-rotation invariance, axial symmetry,
                                                            fall-back flag at known face distances
  forward         Sec. 4.3 / Fig. 6 progressive residual    numpy matmul, bias-only closed form,
                  blocks + trailing layers                  hand-computed K=1, W=2 case
  loss_grad       Sec. 5.2 loss and its gradient            central finite differences
  adam            Sec. 5.2 (Kingma and Ba, Alg. 1)          first-step closed form, 1-D recursion
  philox          Salmon et al. 2011                        published known-answer vectors
  trace_li etc.   Sec. 3.2 Eq. 1, Sec. 4, Sec. 4.4, 5.1     slab transmittance, furnace, sphere
                                                            closed form, single-scatter quadrature,
                                                            HG moments and CDF, transmittance
                                                            across a density profile (interpolated
                                                            value between voxel centres)
  first_hits      Sec. 4.4 camera sample: first collision   homogeneous box: hit fraction
                  and direct single scattering              1 - exp(-sigma L), direct term against
                                                            albedo p exp(-sigma s) E
  trace_li_       Sec. 5.1 progressive estimate (+-2 % at   equals the fixed-count estimate at its
  adaptive        95 %), Sec. 7 target L_s = L_d + L_i      path count, rule fails one batch
                                                            earlier; L_s - L_i against the direct
                                                            closed form, L_s furnace = E exactly
  light_table,    Sec. 4.4 distant emitter as directional   p_j w_j = E_j exactly, thresholds within
                                                            1/2 of the exact running fraction, all
                                                            2^24 draws
  *_lights        lights, one drawn per estimate            counted, homogeneous-box closed form,
                                                            one-light set = directional renderer,
                                                            linearity in the lights
  mlp_forward,    Sec. 7 / Fig. 10 all-at-once MLPs         equal to forward / loss_grad of a K = 1
  mlp_loss_grad   (numpy, FP64)                             RPNN (same parameter vector), central
                                                            finite differences
  phase_table,    Sec. 3.1 / 5.1 tabulated (chopped)        normalisation, chopped mass, HG table
  set_phase       Lorenz-Mie phase function: the chop's     against analytic HG (moments, CDF and
                  thinner medium and albedo, the unchopped  the tracer's estimates); in a thin
                  function at the first collision when      homogeneous box the chopped set-up's
                  rendering                                 first-collision pixel equals the full
                                                            function's single-scattering integral
                                                            (quadrature), f -> 0 gives the full one;
                                                            coarse tables: linear-in-theta lookup
                                                            read back exactly, drawn angles invert
                                                            the piecewise-linear cdf (quadrature)
  e4m3_encode     OCP 8-bit floating point, E4M3 format     torch.float8_e4m3fn cast, hand values,
                  (round to nearest even, saturating)       decode/encode round trip of every code

That the pins can see a mistake is itself tested: tests/test_oracle_mutants.py plants one
plausible mistake at a time in a copy of this package (46 of them, across every part
above) and requires a pin to fail for each.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

FLAG_INVALID, FLAG_OUTSIDE, FLAG_FALLBACK = 1, 2, 4
STENCIL_N = 225


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (FP64, OpenMP, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE",
               "-ffp-contract=off", "-Wall", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        P, I, D, I64, U64 = C.c_void_p, C.c_int, C.c_double, C.c_int64, C.c_uint64
        sig = {
            "dso_num_threads": (I, []),
            "dso_set_threads": (None, [I]),
            "dso_normalize": (I, [P, I, I, I, I, D, P, P]),
            "dso_pyramid_layout": (I64, [I, I, I, I, P, P]),
            "dso_gauss_norm": (D, [I]),
            "dso_pyramid": (I, [P, I, I, I, I, D, D, I, P]),
            "dso_default_mips": (None, [D, D, I, I, P]),
            "dso_frame": (I, [P, P, P, P, P, P]),
            "dso_stencil_offset": (None, [I, P]),
            "dso_gather": (I, [P, P, P, I, P, D, I, I, I, D, I, P, P, P, P, I64, P, P]),
            "dso_param_count": (I64, [I, I, I]),
            "dso_forward": (I, [P, I, I, I, P, I64, P, P]),
            "dso_loss_grad": (I, [P, I, I, I, P, P, I64, P, P]),
            "dso_adam": (None, [P, P, P, P, I64, I64, D, D, D, D]),
            "dso_philox4x32_10": (None, [P, P, P]),
            "dso_hg": (D, [D, D]),
            "dso_hg_sample_cos": (D, [D, D]),
            "dso_trace_li": (I, [P, I, I, I, I, D, P, D, D, D, D, I, I, I, I, U64, P, P, P, I64, P,
                                 P]),
            "dso_trace_li_adaptive": (I, [P, I, I, I, I, D, P, D, D, D, D, I, I, I, I, I, D, D, U64,
                                          P, P, P, I64, P, P, P]),
            "dso_transmittance": (I, [P, I, I, I, I, D, P, D, P, P, I64, I, U64, P, P]),
            "dso_sample_records": (I, [P, I, I, I, I, D, P, D, I64, U64, P, P, P, P]),
            "dso_render_pixels": (I, [P, I, I, I, I, D, P, D, D, D, D, I, I, P, P, P, I64, I, U64,
                                      P, P]),
            "dso_first_hits": (I, [P, I, I, I, I, D, P, D, D, D, D, P, P, P, I64, U64, U64, P, P,
                                   P, P]),
            "dso_set_phase": (None, [I, P, P, D, I, P, P, D]),
            "dso_tab_sample": (D, [I, P, P, D]),
            "dso_tab_eval": (D, [I, P, D]),
            "dso_render_pixels_lights": (I, [P, I, I, I, I, D, P, D, D, D, D, I, I, P, P, P, P, P,
                                             I64, I, U64, P, P]),
            "dso_first_hits_lights": (I, [P, I, I, I, I, D, P, D, D, D, D, I, P, P, P, I, P, P,
                                          I64, U64, U64, P, P, P, P, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with status {rc}")


def threads() -> int:
    return lib().dso_num_threads()


def set_threads(n: int) -> None:
    lib().dso_set_threads(int(n))


# --------------------------------------------------------------------------------------
class Grid:
    """A density grid on the host: float32 or bf16 bit patterns (uint16), [z][y][x]."""

    def __init__(self, d, sigma_max: float, aabb_min, h0: float):
        d = np.ascontiguousarray(d)
        if d.dtype == np.float32:
            self.dtype = 0
        elif d.dtype == np.uint16:
            self.dtype = 1
        else:
            raise TypeError("density must be float32 or bf16 bit patterns as uint16")
        self.d = d
        self.nz, self.ny, self.nx = d.shape
        self.sigma_max = float(sigma_max)
        self.aabb_min = np.ascontiguousarray(np.asarray(aabb_min, np.float64))
        self.h0 = float(h0)

    def args(self):
        return (_p(self.d), self.dtype, self.nx, self.ny, self.nz, self.sigma_max)


def normalize(grid: Grid):
    """(mean extinction over non-zero voxels, number of such voxels)."""
    m = np.zeros(1, np.float64)
    c = np.zeros(1, np.int64)
    _check(lib().dso_normalize(*grid.args(), _p(m), _p(c)), "normalize")
    return float(m[0]), int(c[0])


def pyramid_layout(nx, ny, nz, L):
    dims = np.zeros((L, 3), np.int32)
    offs = np.zeros(L, np.int64)
    total = lib().dso_pyramid_layout(nx, ny, nz, L, _p(dims), _p(offs))
    return dims, offs, int(total)


def gauss_norm(level: int) -> float:
    return lib().dso_gauss_norm(int(level))


def pyramid(grid: Grid, mean_mu_t: float, L: int):
    """Concatenated float64 levels plus (dims[L][3] as (nx, ny, nz), offsets[L])."""
    dims, offs, total = pyramid_layout(grid.nx, grid.ny, grid.nz, L)
    out = np.zeros(total, np.float64)
    _check(lib().dso_pyramid(*grid.args(), float(mean_mu_t), int(L), _p(out)), "pyramid")
    return out, dims, offs


def level(pyr, dims, offs, i):
    nx, ny, nz = (int(v) for v in dims[i])
    return pyr[offs[i]:offs[i] + nx * ny * nz].reshape(nz, ny, nx)


def default_mips(mean_mu_t: float, h0: float, K: int, L: int) -> np.ndarray:
    out = np.zeros(K, np.int32)
    lib().dso_default_mips(float(mean_mu_t), float(h0), int(K), int(L), _p(out))
    return out


def frame(view, light):
    v = np.ascontiguousarray(np.asarray(view, np.float64))
    l_ = np.ascontiguousarray(np.asarray(light, np.float64))
    X, Y, Z = (np.zeros(3, np.float64) for _ in range(3))
    g = np.zeros(1, np.float64)
    ok = lib().dso_frame(_p(v), _p(l_), _p(X), _p(Y), _p(Z), _p(g))
    if not ok:
        return None
    return X, Y, Z, float(g[0])


def stencil_offset(n: int) -> np.ndarray:
    o = np.zeros(3, np.float64)
    lib().dso_stencil_offset(int(n), _p(o))
    return o


def gather(grid: Grid, pyr, dims, offs, mean_mu_t, K, mips, pos, view, light):
    """Descriptor rows [Sigma^1 .. Sigma^K, gamma] (P, 225K+1) and per-point flags."""
    pos = np.ascontiguousarray(pos, np.float32)
    view = np.ascontiguousarray(view, np.float32)
    light = np.ascontiguousarray(light, np.float32)
    mips = np.ascontiguousarray(mips, np.int32)
    P = pos.shape[0]
    z = np.zeros((P, STENCIL_N * K + 1), np.float64)
    flags = np.zeros(P, np.uint8)
    dims = np.ascontiguousarray(dims, np.int32)
    offs = np.ascontiguousarray(offs, np.int64)
    _check(lib().dso_gather(_p(pyr), _p(dims), _p(offs), int(dims.shape[0]), _p(grid.aabb_min),
                            grid.h0, grid.nx, grid.ny, grid.nz, float(mean_mu_t), int(K), _p(mips),
                            _p(pos), _p(view), _p(light), P, _p(z), _p(flags)), "gather")
    return z, flags


def param_count(K, W, H=3) -> int:
    return int(lib().dso_param_count(K, W, H))


def forward(theta, K, W, H, z):
    """Network output g and the final layer's pre-activation, both (P,)."""
    th = np.ascontiguousarray(theta, np.float64)
    if th.size != param_count(K, W, H):
        raise ValueError("parameter vector has the wrong length")
    z = np.ascontiguousarray(z, np.float64)
    P = z.shape[0]
    g = np.zeros(P, np.float64)
    pre = np.zeros(P, np.float64)
    _check(lib().dso_forward(_p(th), K, W, H, _p(z), P, _p(g), _p(pre)), "forward")
    return g, pre


def loss_grad(theta, K, W, H, z, target_log1p, want_grad=True):
    th = np.ascontiguousarray(theta, np.float64)
    z = np.ascontiguousarray(z, np.float64)
    t = np.ascontiguousarray(target_log1p, np.float64)
    B = z.shape[0]
    loss = np.zeros(1, np.float64)
    grad = np.zeros(th.size, np.float64) if want_grad else None
    _check(lib().dso_loss_grad(_p(th), K, W, H, _p(z), _p(t), B, _p(loss), _p(grad)), "loss_grad")
    return float(loss[0]), grad


# ------------------------------------------------------------ all-at-once MLP baselines
def mlp_param_count(widths) -> int:
    """widths: input width first, output width (1) last.  Per layer W [out][in], b [out]."""
    return int(sum(o * i + o for i, o in zip(widths[:-1], widths[1:])))


def _mlp_layers(theta, widths):
    th = np.asarray(theta, np.float64)
    if th.size != mlp_param_count(widths):
        raise ValueError("parameter vector has the wrong length")
    out, at = [], 0
    for i, o in zip(widths[:-1], widths[1:]):
        W = th[at:at + o * i].reshape(o, i)
        at += o * i
        b = th[at:at + o]
        at += o
        out.append((W, b))
    return out


def mlp_forward(theta, widths, z):
    """The comparison networks of Sec. 7 (Fig. 10): the whole descriptor enters the first
    layer, every layer is ReLU(W h + b), the last one included (as the RPNN's).  Returns
    (g, final pre-activation), both (P,)."""
    h = np.asarray(z, np.float64)
    pre = None
    for W, b in _mlp_layers(theta, widths):
        pre = h @ W.T + b
        h = np.maximum(pre, 0.0)
    return h[:, 0], pre[:, 0]


def mlp_loss_grad(theta, widths, z, target_log1p):
    """Loss of Sec. 5.2, mean over the batch of (log(1 + g) - t)^2, and its gradient by
    backpropagation in FP64 (ReLU' = 1 where the pre-activation is > 0)."""
    layers = _mlp_layers(theta, widths)
    z = np.asarray(z, np.float64)
    t = np.asarray(target_log1p, np.float64)
    B = z.shape[0]
    hs, pres = [z], []
    for W, b in layers:
        pres.append(hs[-1] @ W.T + b)
        hs.append(np.maximum(pres[-1], 0.0))
    g = hs[-1][:, 0]
    r = np.log1p(g) - t
    loss = float(np.mean(r * r))
    d = (2.0 * r / (B * (1.0 + g)))[:, None]          # d loss / d g
    grads = []
    for l in range(len(layers) - 1, -1, -1):
        d = d * (pres[l] > 0)                          # through the ReLU
        grads.append((d.T @ hs[l], d.sum(0)))          # dW, db
        d = d @ layers[l][0]                           # d loss / d input of layer l
    out = []
    for dW, db in reversed(grads):
        out += [dW.reshape(-1), db]
    return loss, np.concatenate(out)


def adam(theta, m, v, grad, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays; t is the 1-based step number."""
    for a in (theta, m, v, grad):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().dso_adam(_p(theta), _p(m), _p(v), _p(grad), theta.size, int(t), lr, b1, b2, eps)


def philox(ctr, key):
    c = np.ascontiguousarray(np.asarray(ctr, np.uint32))
    k = np.ascontiguousarray(np.asarray(key, np.uint32))
    out = np.zeros(4, np.uint32)
    lib().dso_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def hg(g, mu):
    return lib().dso_hg(float(g), float(mu))


def hg_sample_cos(g, u):
    return lib().dso_hg_sample_cos(float(g), float(u))


def trace_li(grid: Grid, pos, view, light, albedo=0.999, g=0.85, irradiance=1.0, light_mode=0,
             max_interactions=0, spp=64, seed=1, include_direct=False):
    """Per record: mean of spp path estimates of L_i (of L_s = L_d + L_i with
    include_direct) and the variance of that mean."""
    pos = np.ascontiguousarray(pos, np.float32)
    view = np.ascontiguousarray(view, np.float32)
    light = np.ascontiguousarray(light, np.float32)
    P = pos.shape[0]
    mean = np.zeros(P, np.float64)
    var = np.zeros(P, np.float64)
    _check(lib().dso_trace_li(*grid.args(), _p(grid.aabb_min), grid.h0, albedo, g, irradiance,
                              light_mode, max_interactions, int(include_direct), spp, seed,
                              _p(pos), _p(view), _p(light), P, _p(mean), _p(var)), "trace_li")
    return mean, var


def trace_li_adaptive(grid: Grid, pos, view, light, batch=64, max_spp=4096, rel=0.02, zq=1.96,
                      albedo=0.999, g=0.85, irradiance=1.0, light_mode=0, max_interactions=0,
                      seed=1, include_direct=False):
    """Progressive estimates: batches of paths until zq * sqrt(var of mean) <= rel * |mean|
    (the mean within +-rel at the confidence of zq) or max_spp paths.  Returns (mean,
    variance of the mean, paths used)."""
    pos = np.ascontiguousarray(pos, np.float32)
    view = np.ascontiguousarray(view, np.float32)
    light = np.ascontiguousarray(light, np.float32)
    P = pos.shape[0]
    mean = np.zeros(P, np.float64)
    var = np.zeros(P, np.float64)
    n = np.zeros(P, np.int32)
    _check(lib().dso_trace_li_adaptive(*grid.args(), _p(grid.aabb_min), grid.h0, albedo, g,
                                       irradiance, light_mode, max_interactions,
                                       int(include_direct), batch, max_spp, rel, zq, seed,
                                       _p(pos), _p(view), _p(light), P, _p(mean), _p(var), _p(n)),
           "trace_li_adaptive")
    return mean, var, n


def transmittance(grid: Grid, orig, dirs, spp=256, seed=1):
    o = np.ascontiguousarray(orig, np.float64)
    d = np.ascontiguousarray(dirs, np.float64)
    R = o.shape[0]
    rm = np.zeros(R, np.float64)
    ef = np.zeros(R, np.float64)
    _check(lib().dso_transmittance(*grid.args(), _p(grid.aabb_min), grid.h0, _p(o), _p(d), R, spp,
                                   seed, _p(rm), _p(ef)), "transmittance")
    return rm, ef


def sample_records(grid: Grid, N, seed):
    pos = np.zeros((N, 3), np.float32)
    view = np.zeros((N, 3), np.float32)
    light = np.zeros((N, 3), np.float32)
    att = np.zeros(N, np.int32)
    _check(lib().dso_sample_records(*grid.args(), _p(grid.aabb_min), grid.h0, N, seed, _p(pos),
                                    _p(view), _p(light), _p(att)), "sample_records")
    return pos, view, light, att


def first_hits(grid: Grid, ray_o, ray_d, light_dir, albedo=0.999, g=0.85, irradiance=1.0, seed=1,
               sample=0):
    """First collision, view direction and NEE direct term per ray (one sample)."""
    o = np.ascontiguousarray(ray_o, np.float32)
    d = np.ascontiguousarray(ray_d, np.float32)
    ld = np.ascontiguousarray(np.asarray(light_dir, np.float64))
    N = o.shape[0]
    pos = np.zeros((N, 3))
    view = np.zeros((N, 3))
    direct = np.zeros(N)
    hit = np.zeros(N, np.uint8)
    _check(lib().dso_first_hits(*grid.args(), _p(grid.aabb_min), grid.h0, albedo, g, irradiance,
                                _p(ld), _p(o), _p(d), N, seed, sample, _p(pos), _p(view),
                                _p(direct), _p(hit)), "first_hits")
    return pos, view, direct, hit


def render_pixels(grid: Grid, ray_o, ray_d, light_dir, albedo=0.999, g=0.85, irradiance=1.0,
                  light_mode=0, max_interactions=0, spp=16, seed=1):
    o = np.ascontiguousarray(ray_o, np.float32)
    d = np.ascontiguousarray(ray_d, np.float32)
    ld = np.ascontiguousarray(np.asarray(light_dir, np.float64))
    N = o.shape[0]
    mean = np.zeros(N, np.float64)
    var = np.zeros(N, np.float64)
    _check(lib().dso_render_pixels(*grid.args(), _p(grid.aabb_min), grid.h0, albedo, g, irradiance,
                                   light_mode, max_interactions, _p(ld), _p(o), _p(d), N, spp,
                                   seed, _p(mean), _p(var)), "render_pixels")
    return mean, var


# ------------------------------------------------------------------- tabulated phases
def phase_table(p, chop_deg=0.0):
    """Tracer table of a phase function given at theta_i = i pi / (n - 1) (per steradian):
    normalised so that the trapezoid rule on 2 pi p sin(theta) gives 1; with chop_deg > 0
    the forward peak is chopped (Sec. 5.1's chopped Lorenz-Mie function): below the node
    nearest chop_deg the value is held at that node's, the lost fraction f of the
    scattering is reported and the rest renormalised (the medium then scatters (1 - f) of
    its original scattering, the chopped part travelling on as if unscattered).  Returns a
    dict: p, cdf (normalised running trapezoid sums), removed (f), g (mean cosine)."""
    p = np.asarray(p, np.float64)
    n = p.size
    if n < 3 or not np.all(np.isfinite(p)) or np.any(p < 0):
        raise ValueError("a phase table needs at least three finite non-negative values")
    theta = np.arange(n) * (np.pi / (n - 1))

    def integral(q):
        f = 2 * np.pi * q * np.sin(theta)
        return float(np.sum(0.5 * (f[1:] + f[:-1])) * (np.pi / (n - 1)))

    q = p / integral(p)
    removed = 0.0
    if chop_deg > 0:
        ic = int(round(np.radians(chop_deg) / (np.pi / (n - 1))))
        q = q.copy()
        q[:ic] = q[ic]
        removed = 1.0 - integral(q)
        q = q / (1.0 - removed)
    f = 2 * np.pi * q * np.sin(theta)
    c = np.concatenate([[0.0], np.cumsum(0.5 * (f[1:] + f[:-1]) * (np.pi / (n - 1)))])
    cdf = c / c[-1]
    g = float(np.sum(0.5 * ((f * np.cos(theta))[1:] + (f * np.cos(theta))[:-1])) * (np.pi / (n - 1)))
    return {"p": q, "cdf": cdf, "removed": removed, "g": g}


def set_phase(table=None, first=None):
    """Use `table` (from phase_table) for every scattering and `first` for the direct
    term at the first collision of camera rays in all later tracer calls; None restores
    Henyey-Greenstein (first falls back to table).  While a chopped table is set, every
    tracer call takes its albedo argument as the medium's own single-scattering albedo a
    and traces the optically thinner medium of Sec. 3.1: extinction times 1 - a f, albedo
    a (1 - f) / (1 - a f), f = table["removed"]; `first` is weighted by
    (1 - first["removed"]) / (1 - f) (the C oracle's chop_reduce and first_scale)."""
    L = lib()
    keep = []

    def args(t):
        if t is None:
            return [0, None, None, 0.0]
        a, b = np.ascontiguousarray(t["p"]), np.ascontiguousarray(t["cdf"])
        keep.extend([a, b])
        return [a.size, _p(a), _p(b), float(t.get("removed", 0.0))]

    L.dso_set_phase(*args(table), *args(first))


def tab_eval(p, mu):
    """p(mu) the tracer reads from the values p at theta_i = i pi / (n - 1)."""
    a = np.ascontiguousarray(p, np.float64)
    if a.size < 2:
        raise ValueError("a table needs at least two values")
    return lib().dso_tab_eval(a.size, _p(a), float(mu))


def tab_sample(table, u):
    """cos(theta) the tracer draws from `table` for the uniform u."""
    a, b = np.ascontiguousarray(table["p"]), np.ascontiguousarray(table["cdf"])
    return lib().dso_tab_sample(a.size, _p(a), _p(b), float(u))


# ---------------------------------------------------------------------------- light sets
def light_table(irradiance):
    """Selection table of a set of directional lights (Sec. 4.4: a distant emitter
    approximated by directional samples), for drawing light j with probability close
    to E_j / sum(E) from the top 24 bits k of one uniform: j is the first index with
    k < thr[j].  thr[j] is the running sum of E up to j (in order, FP64) over the
    total, times 2^24, rounded half up, then kept at least one above thr[j-1] and low
    enough to leave one step for each later light, so every light has a nonzero
    probability p_j = (thr[j] - thr[j-1]) / 2^24 and thr[-1] = 2^24.  The weight
    w[j] = E_j / p_j makes one draw an unbiased estimate of the sum over the set."""
    E = np.asarray(irradiance, np.float64).reshape(-1)
    m = E.size
    if m < 1 or m > 65536 or not np.all(np.isfinite(E)) or not np.all(E > 0):
        raise ValueError("a light set needs 1..65536 finite positive irradiances")
    thr = np.zeros(m, np.uint32)
    w = np.zeros(m, np.float64)
    total = 0.0
    for j in range(m):
        total += E[j]
    run, prev = 0.0, 0
    for j in range(m):
        run += E[j]
        t = int(np.floor(run / total * 16777216.0 + 0.5))
        t = min(max(t, prev + 1), (1 << 24) - (m - 1 - j))
        thr[j] = t
        w[j] = E[j] / ((t - prev) / 16777216.0)
        prev = t
    return thr, w


def light_pick(thr, k):
    """The light drawn by the 24-bit integer k: the first j with k < thr[j]."""
    for j, t in enumerate(thr):
        if k < int(t):
            return j
    raise ValueError("k must be below 2^24")


def _light_args(dirs, irradiance):
    d = np.asarray(dirs, np.float64).reshape(-1, 3)
    n = np.linalg.norm(d, axis=1, keepdims=True)
    if not np.all(np.isfinite(d)) or not np.all(n > 0):
        raise ValueError("unusable light direction")
    d = np.ascontiguousarray(d / n)
    thr, w = light_table(irradiance)
    if thr.size != d.shape[0]:
        raise ValueError("one irradiance per light direction")
    return d, thr, w


def render_pixels_lights(grid: Grid, ray_o, ray_d, dirs, irradiances, albedo=0.999, g=0.85,
                         irradiance=1.0, max_interactions=0, spp=16, seed=1):
    """Path-traced pixels under a set of directional lights (one light drawn per
    next-event estimate)."""
    o = np.ascontiguousarray(ray_o, np.float32)
    d = np.ascontiguousarray(ray_d, np.float32)
    ld, thr, w = _light_args(dirs, irradiances)
    N = o.shape[0]
    mean = np.zeros(N, np.float64)
    var = np.zeros(N, np.float64)
    _check(lib().dso_render_pixels_lights(*grid.args(), _p(grid.aabb_min), grid.h0, albedo, g,
                                          irradiance, max_interactions, ld.shape[0], _p(ld),
                                          _p(thr), _p(w), _p(o), _p(d), N, spp, seed, _p(mean),
                                          _p(var)), "render_pixels_lights")
    return mean, var


def first_hits_lights(grid: Grid, ray_o, ray_d, dirs, irradiances, draws, albedo=0.999, g=0.85,
                      irradiance=1.0, seed=1, sample=0):
    """First collision, view direction, `draws` lights drawn from the set (rows
    i * draws + q: direction and weight) and the averaged NEE direct term per ray."""
    o = np.ascontiguousarray(ray_o, np.float32)
    d = np.ascontiguousarray(ray_d, np.float32)
    ld, thr, w = _light_args(dirs, irradiances)
    N = o.shape[0]
    pos = np.zeros((N, 3))
    view = np.zeros((N, 3))
    light = np.zeros((N * draws, 3))
    weight = np.zeros(N * draws)
    direct = np.zeros(N)
    hit = np.zeros(N, np.uint8)
    _check(lib().dso_first_hits_lights(*grid.args(), _p(grid.aabb_min), grid.h0, albedo, g,
                                       irradiance, ld.shape[0], _p(ld), _p(thr), _p(w), draws,
                                       _p(o), _p(d), N, seed, sample, _p(pos), _p(view),
                                       _p(light), _p(weight), _p(direct), _p(hit)),
           "first_hits_lights")
    return pos, view, light, weight, direct, hit


# ----------------------------------------------------------------------------- FP8 E4M3
def e4m3_value(code: int) -> float:
    """Value of a finite OCP E4M3 code 0..126 (sign bit clear): exponent bias 7, three
    mantissa bits, subnormals m * 2^-9; 0x7F is NaN and there are no infinities."""
    e, m = code >> 3, code & 7
    return m * 2.0 ** -9 if e == 0 else (1.0 + m / 8.0) * 2.0 ** (e - 7)


def e4m3_encode(x) -> np.ndarray:
    """OCP E4M3 codes of x: the nearest of the 127 finite magnitudes, ties to the even
    code (even mantissa), magnitudes above 448 saturated to 448, NaN to 0x7F, the sign in
    bit 7.  Written as a search over the value table so that it can be read against the
    format's definition."""
    x = np.asarray(x, dtype=np.float64)
    vals = np.array([e4m3_value(c) for c in range(127)])
    a = np.minimum(np.abs(x), vals[-1])
    hi = np.clip(np.searchsorted(vals, a, side="left"), 0, 126)
    lo = np.clip(hi - 1, 0, 126)
    dlo, dhi = a - vals[lo], vals[hi] - a
    code = np.where(dhi < dlo, hi, np.where(dlo < dhi, lo, np.where(hi % 2 == 0, hi, lo)))
    code = code.astype(np.uint8) | (np.signbit(x).astype(np.uint8) << 7)
    return np.where(np.isnan(x), np.uint8(0x7F), code).astype(np.uint8)

