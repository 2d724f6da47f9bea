"""Seeded synthetic inputs: procedural cloud densities, shading points, directions
and network parameters.

This module is the only code shared by the GPU path's tests/benchmarks and the
FP64 oracle.  It produces *inputs* only and holds none of the method's
arithmetic (no normalisation, filtering, stencil, network or transport).

The paper trains and tests on 80 procedural, simulated and artist-made clouds
(Sec. 5) that are not available here; the fBm + Worley clouds below stand in
for them: cumulus-like blobs with the paper's resolution range, fitted to the
unit box (Sec. 5).

Conventions shared with the library and the oracle:
  * density grids are indexed [z][y][x] with x fastest, values in [0, 1];
  * the grid is fitted to the unit box: voxel size h0 = 1 / max(nx, ny, nz),
    centred on the origin, so aabb_min = -0.5 * (nx, ny, nz) * h0;
  * points and directions are float32 arrays of shape (P, 3) (x, y, z per row).
"""
from __future__ import annotations

import math

import numpy as np
import torch

_MASK32 = 0xFFFFFFFF


# --------------------------------------------------------------------------------------
# integer hashing (exact in int64 on any device)
# --------------------------------------------------------------------------------------
def _hash3(ix: torch.Tensor, iy: torch.Tensor, iz: torch.Tensor, salt: int) -> torch.Tensor:
    """32-bit integer hash of lattice coordinates; all intermediate products
    stay below 2**63, so the result is identical on CPU and GPU."""
    h = (ix * 73856093) ^ (iy * 19349663) ^ (iz * 83492791) ^ (salt & _MASK32)
    h = h & _MASK32
    h = ((h >> 16) ^ h) * 0x45D9F3B & _MASK32
    h = ((h >> 16) ^ h) * 0x45D9F3B & _MASK32
    h = (h >> 16) ^ h
    return h


def _salt(seed: int, octave: int, which: int) -> int:
    x = (seed * 0x9E3779B1 + octave * 0x85EBCA77 + which * 0xC2B2AE3D + 0x27D4EB2F) & _MASK32
    x ^= x >> 15
    x = (x * 0x2C1B3C6D) & _MASK32
    x ^= x >> 12
    return x


def _value_noise(px, py, pz, salt):
    """Value noise in [0, 1): hashed lattice values, quintic-faded trilinear blend."""
    fx, fy, fz = torch.floor(px), torch.floor(py), torch.floor(pz)
    tx, ty, tz = px - fx, py - fy, pz - fz
    ix = fx.to(torch.int64) + 4096
    iy = fy.to(torch.int64) + 4096
    iz = fz.to(torch.int64) + 4096

    def fade(t):
        return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)

    ux, uy, uz = fade(tx), fade(ty), fade(tz)
    out = None
    for dz in (0, 1):
        wz = uz if dz else (1.0 - uz)
        for dy in (0, 1):
            wy = uy if dy else (1.0 - uy)
            for dx in (0, 1):
                wx = ux if dx else (1.0 - ux)
                v = _hash3(ix + dx, iy + dy, iz + dz, salt).to(px.dtype) * (1.0 / 4294967296.0)
                term = wx * wy * wz * v
                out = term if out is None else out + term
    return out


def _worley_f1(px, py, pz, salt):
    """Distance to the nearest feature point, one jittered point per unit cell."""
    fx, fy, fz = torch.floor(px), torch.floor(py), torch.floor(pz)
    ix = fx.to(torch.int64) + 4096
    iy = fy.to(torch.int64) + 4096
    iz = fz.to(torch.int64) + 4096
    best = torch.full_like(px, 1e9)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                cx, cy, cz = ix + dx, iy + dy, iz + dz
                hx = _hash3(cx, cy, cz, salt).to(px.dtype) * (1.0 / 4294967296.0)
                hy = _hash3(cx, cy, cz, salt ^ 0x5BD1E995).to(px.dtype) * (1.0 / 4294967296.0)
                hz = _hash3(cx, cy, cz, salt ^ 0x1B873593).to(px.dtype) * (1.0 / 4294967296.0)
                qx = (cx - 4096).to(px.dtype) + hx - px
                qy = (cy - 4096).to(px.dtype) + hy - py
                qz = (cz - 4096).to(px.dtype) + hz - pz
                best = torch.minimum(best, qx * qx + qy * qy + qz * qz)
    return torch.sqrt(best)


def cloud_density(n, seed: int, worley: float = 0.0, device="cpu",
                  dtype=torch.float32, slab: int = 16) -> torch.Tensor:
    """Seeded cumulus-like density in [0, 1], shape (nz, ny, nx).

    d = clamp((shape + fBm detail - tau) / (1 - tau), 0, 1), where `shape` is an
    ellipsoidal falloff and the fBm has 2**(log2 n - 2) ... octaves (capped at 7),
    lacunarity 2 and gain 0.5; with `worley` > 0 an F1 cellular term erodes the
    body.  Computed in float64 slab by slab, returned in `dtype` (bf16 by RNE).
    """
    if isinstance(n, int):
        nx = ny = nz = n
    else:
        nx, ny, nz = n
    nmax = max(nx, ny, nz)
    octaves = int(min(7, max(2, round(math.log2(nmax)) - 2)))
    base_freq = 4.0
    out = torch.empty((nz, ny, nx), dtype=dtype, device=device)
    f64 = torch.float64
    xs = (torch.arange(nx, device=device, dtype=f64) + 0.5) / nmax
    ys = (torch.arange(ny, device=device, dtype=f64) + 0.5) / nmax
    cx, cy, cz = 0.5 * nx / nmax, 0.45 * ny / nmax, 0.5 * nz / nmax
    for z0 in range(0, nz, slab):
        z1 = min(nz, z0 + slab)
        zs = (torch.arange(z0, z1, device=device, dtype=f64) + 0.5) / nmax
        pz, py, px = torch.meshgrid(zs, ys, xs, indexing="ij")
        fbm = torch.zeros_like(px)
        amp, norm, freq = 1.0, 0.0, base_freq
        for o in range(octaves):
            fbm = fbm + amp * _value_noise(px * freq, py * freq, pz * freq, _salt(seed, o, 0))
            norm += amp
            amp *= 0.5
            freq *= 2.0
        fbm = fbm / norm
        ex = (px - cx) / 0.40
        ey = (py - cy) / 0.27
        ez = (pz - cz) / 0.40
        # flatter bottom, puffier top: the vertical radius shrinks below the centre
        ey = torch.where(ey < 0, ey * 1.6, ey)
        r = torch.sqrt(ex * ex + ey * ey + ez * ez)
        shape = 1.0 - r
        d = shape + 0.9 * (fbm - 0.5)
        if worley > 0.0:
            f1 = _worley_f1(px * 6.0, py * 6.0, pz * 6.0, _salt(seed, 99, 1))
            d = d - worley * f1
        tau = 0.08
        d = torch.clamp((d - tau) / (0.45 - tau), 0.0, 1.0)
        out[z0:z1] = d.to(dtype)
    return out


def unit_box(n):
    """(aabb_min[3], h0) of a grid with dims n = (nx, ny, nz) fitted to the unit box."""
    if isinstance(n, int):
        n = (n, n, n)
    h0 = 1.0 / max(n)
    aabb_min = [-0.5 * n[0] * h0, -0.5 * n[1] * h0, -0.5 * n[2] * h0]
    return np.asarray(aabb_min, dtype=np.float32), float(h0)


# --------------------------------------------------------------------------------------
# directions, points, parameters
# --------------------------------------------------------------------------------------
def uniform_dirs(P: int, seed: int) -> np.ndarray:
    """Directions uniform on the unit sphere: z = 1 - 2u, phi = 2 pi v."""
    rng = np.random.default_rng(seed)
    u = rng.random(P)
    v = rng.random(P)
    z = 1.0 - 2.0 * u
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = 2.0 * np.pi * v
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1).astype(np.float32)


def points_in_density(d, P: int, seed: int, aabb_min, h0: float) -> np.ndarray:
    """Shading points: a uniformly chosen voxel with d > 0, jittered uniformly inside it."""
    dn = d.detach().to("cpu").float().numpy() if isinstance(d, torch.Tensor) else np.asarray(d)
    nz, ny, nx = dn.shape
    idx = np.flatnonzero(dn.reshape(-1) > 0)
    if idx.size == 0:
        raise ValueError("density grid has no non-zero voxel")
    rng = np.random.default_rng(seed)
    pick = idx[rng.integers(0, idx.size, size=P)]
    iz, rem = np.divmod(pick, ny * nx)
    iy, ix = np.divmod(rem, nx)
    jit = rng.random((P, 3))
    pos = np.empty((P, 3), dtype=np.float64)
    pos[:, 0] = aabb_min[0] + (ix + jit[:, 0]) * h0
    pos[:, 1] = aabb_min[1] + (iy + jit[:, 1]) * h0
    pos[:, 2] = aabb_min[2] + (iz + jit[:, 2]) * h0
    return pos.astype(np.float32)


def points_in_density_device(d: torch.Tensor, P: int, seed: int, aabb_min, h0: float):
    """Same distribution as points_in_density for grids too large to scan on the
    host: voxels drawn uniformly on the device, kept where d > 0 (rejection),
    jittered inside the voxel.  Returns a (P, 3) float32 device tensor."""
    nz, ny, nx = d.shape
    g = torch.Generator(device=d.device).manual_seed(seed)
    flat = d.reshape(-1)
    got = []
    have = 0
    while have < P:
        m = max(4 * (P - have), 4096)
        cand = torch.randint(0, flat.numel(), (m,), generator=g, device=d.device)
        cand = cand[flat[cand] > 0][: P - have]
        got.append(cand)
        have += cand.numel()
        if have == 0 and m > 64 * P + 4096:
            raise ValueError("density grid looks empty")
    pick = torch.cat(got)
    iz = pick // (ny * nx)
    rem = pick % (ny * nx)
    iy, ix = rem // nx, rem % nx
    jit = torch.rand((P, 3), generator=g, device=d.device, dtype=torch.float64)
    lo = torch.as_tensor(np.asarray(aabb_min, np.float64), device=d.device)
    idx = torch.stack([ix, iy, iz], 1).to(torch.float64)
    return (lo + (idx + jit) * h0).to(torch.float32)


def layer_shapes(K: int, W: int, H: int = 3, n_in: int = 226):
    """(name, rows, cols) of every weight matrix / bias vector in canonical order:
    per block k: V[W][226], W1[W][W] (k > 1 only), b1[W], W2[W][W], b2[W];
    head: H-1 layers W x W plus bias, then a 1 x W layer plus a 1-vector bias."""
    shapes = []
    for k in range(K):
        shapes.append((f"V{k}", W, n_in))
        if k > 0:
            shapes.append((f"W1_{k}", W, W))
        shapes.append((f"b1_{k}", W, 0))
        shapes.append((f"W2_{k}", W, W))
        shapes.append((f"b2_{k}", W, 0))
    for m in range(H):
        rows = 1 if m == H - 1 else W
        shapes.append((f"Wh{m}", rows, W))
        shapes.append((f"bh{m}", rows, 0))
    return shapes


def n_params(K: int, W: int, H: int = 3) -> int:
    return sum(r * (c if c else 1) for _, r, c in layer_shapes(K, W, H))


def init_params(K: int, W: int, H: int, seed: int, bias: float = 0.0, branch_scale: float = 1.0,
                out_scale: float = 1.0, out_bias: float | None = None) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), constant biases; float32 vector.
    For training runs: branch_scale multiplies the second matrix of every residual
    block (keeps the residual stream from growing with depth), out_scale the final
    layer's weights, and out_bias sets the final bias (a starting prediction that
    keeps the output unit alive)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, r, c in layer_shapes(K, W, H):
        if c == 0:
            v = out_bias if (name == f"bh{H - 1}" and out_bias is not None) else bias
            parts.append(np.full(r, v, dtype=np.float64))
        else:
            b = math.sqrt(6.0 / c)
            w = rng.uniform(-b, b, size=r * c)
            if name.startswith("W2_"):
                w = w * branch_scale
            if name == f"Wh{H - 1}":
                w = w * out_scale
            parts.append(w)
    return np.concatenate(parts).astype(np.float32)


# --------------------------------------------------------------------------------------
# camera primary hits (shading points of a rendered view)
# --------------------------------------------------------------------------------------
def _morton_key8(px: np.ndarray, py: np.ndarray) -> np.ndarray:
    """Sort key: 8x8 pixel tiles in row-major order, Morton order inside a tile."""
    tx, ty = px >> 3, py >> 3
    lx, ly = px & 7, py & 7
    m = np.zeros_like(px)
    for b in range(3):
        m |= ((lx >> b) & 1) << (2 * b)
        m |= ((ly >> b) & 1) << (2 * b + 1)
    return (ty * 1_000_003 + tx) * 64 + m


def camera_rays(res: int, cam_pos, look_at, fov_deg: float, px, py, jx, jy):
    """Pinhole camera: world-space unit ray directions for pixel (px, py) + jitter."""
    cam_pos = np.asarray(cam_pos, np.float64)
    fwd = np.asarray(look_at, np.float64) - cam_pos
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, [0.0, 1.0, 0.0])
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    t = math.tan(math.radians(fov_deg) * 0.5)
    sx = (2.0 * (px + jx) / res - 1.0) * t
    sy = (1.0 - 2.0 * (py + jy) / res) * t
    d = fwd[None, :] + sx[:, None] * right[None, :] + sy[:, None] * up[None, :]
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def camera_hits(d, sigma_max: float, res: int, P: int, seed: int, aabb_min, h0: float,
                cam_pos=(0.0, 0.12, 2.3), look_at=(0.0, 0.0, 0.0), fov_deg: float = 42.0,
                device="cpu", shuffle: bool = False):
    """Shading points of a res x res view: for jittered pinhole rays, march the
    nearest-voxel density with half-voxel steps until the optical depth reaches
    an exponential deviate; rays that leave the grid first are re-drawn at
    random pixels until P hits exist.  Points come back in 8x8 Morton-tiled pixel
    order (or shuffled).  Returns (pos, view_dir) float32 (P, 3); view_dir is the
    direction the radiance travels toward the camera (minus the ray direction)."""
    rng = np.random.default_rng(seed)
    dt = d if isinstance(d, torch.Tensor) else torch.as_tensor(d)
    dt = dt.to(device)
    nz, ny, nx = dt.shape
    dims = np.array([nx, ny, nz], np.float64)
    amin = np.asarray(aabb_min, np.float64)
    amax = amin + dims * h0
    cam = np.asarray(cam_pos, np.float64)
    got_pos, got_dir, got_key = [], [], []
    have = 0
    first = True
    flat = dt.reshape(-1)
    while have < P:
        if first:
            n = res * res
            pix = np.arange(n, dtype=np.int64)
            first = False
        else:
            n = min(4 * (P - have) + 1024, res * res)
            pix = rng.integers(0, res * res, size=n)
        px, py = pix % res, pix // res
        jx, jy = rng.random(n), rng.random(n)
        dirs = camera_rays(res, cam, look_at, fov_deg, px, py, jx, jy)
        target = -np.log1p(-rng.random(n))
        # slab intersection with the grid box
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / dirs
            t0 = (amin[None, :] - cam[None, :]) * inv
            t1 = (amax[None, :] - cam[None, :]) * inv
        tn = np.nanmax(np.minimum(t0, t1), axis=1)
        tf = np.nanmin(np.maximum(t0, t1), axis=1)
        ok = tf > np.maximum(tn, 0.0)
        tn = np.maximum(tn, 0.0)
        step = 0.5 * h0
        T = lambda a: torch.as_tensor(a, device=device, dtype=torch.float64)
        o = T(cam)
        dd, tcur, tend, tau_t = T(dirs), T(tn), T(tf), T(target)
        alive = T(ok.astype(np.float64)) > 0
        tau = torch.zeros_like(tcur)
        hit_t = torch.full_like(tcur, -1.0)
        n_steps = int(math.ceil((np.max(tf[ok] - tn[ok]) if ok.any() else 0.0) / step)) + 2
        lo = T(amin)
        for _ in range(n_steps):
            if not bool(alive.any()):
                break
            tm = tcur + 0.5 * step
            p = o[None, :] + tm[:, None] * dd
            g = torch.floor((p - lo[None, :]) / h0).to(torch.int64)
            gx = g[:, 0].clamp(0, nx - 1)
            gy = g[:, 1].clamp(0, ny - 1)
            gz = g[:, 2].clamp(0, nz - 1)
            mu = flat[(gz * ny + gy) * nx + gx].to(torch.float64) * sigma_max
            mu = torch.where(alive, mu, torch.zeros_like(mu))
            seg = torch.minimum(torch.full_like(tcur, step), tend - tcur).clamp_min(0.0)
            newtau = tau + mu * seg
            crossed = alive & (newtau >= tau_t) & (mu > 0)
            th = tcur + (tau_t - tau) / torch.where(mu > 0, mu, torch.ones_like(mu))
            hit_t = torch.where(crossed, th, hit_t)
            alive = alive & ~crossed
            tau = newtau
            tcur = tcur + step
            alive = alive & (tcur < tend)
        ht = hit_t.cpu().numpy()
        m = ht >= 0
        pos = cam[None, :] + ht[m, None] * dirs[m]
        got_pos.append(pos)
        got_dir.append(-dirs[m])
        got_key.append(_morton_key8(px[m], py[m]) * 8 + (0 if have == 0 else 1))
        have += int(m.sum())
    pos = np.concatenate(got_pos)[:P]
    vdir = np.concatenate(got_dir)[:P]
    key = np.concatenate(got_key)[:P]
    order = rng.permutation(P) if shuffle else np.argsort(key, kind="stable")
    return pos[order].astype(np.float32), vdir[order].astype(np.float32)


def table1_lights(cam_pos=(0.0, 0.12, 2.3), look_at=(0.0, 0.0, 0.0)):
    """Directions toward a distant light placed to the side of, in front of
    (behind the camera) and behind the cloud, relative to the camera (the three
    directional-light set-ups of the paper's Table 1)."""
    cam = np.asarray(cam_pos, np.float64)
    fwd = np.asarray(look_at, np.float64) - cam
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, [0.0, 1.0, 0.0])
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)

    def nrm(v):
        return (v / np.linalg.norm(v)).astype(np.float32)

    return {
        "side": nrm(right + 0.35 * up),
        "front": nrm(-fwd + 0.35 * up + 0.2 * right),
        "back": nrm(fwd + 0.35 * up + 0.2 * right),
    }


def sun_sky_lights(sun_dir, sun_irradiance: float = 1.0, sky_radiance: float = 0.08,
                   n_bands: int = 8, n_az: int = 16, ground: float = 0.25):
    """A synthetic sun and sky as a set of directional lights (the paper's sun-sky
    illumination, Fig. 7, approximated by directions): the sun as one light of
    irradiance sun_irradiance, plus the sphere cut into n_bands equal-height bands of
    the up coordinate y times n_az equal azimuth sectors (equal solid angle 4 pi /
    (n_bands n_az) each), one light at each cell centre with irradiance radiance times
    that solid angle.  Sky radiance (y > 0): sky_radiance * (0.6 + 0.4 (1 - y)) * (1 + 2
    exp(-3 angle to the sun)), brighter toward the horizon and around the sun; below the
    horizon a constant ground * sky_radiance.  Input data only: returns (dirs (m, 3)
    float32, irradiance (m,) float64)."""
    s = np.asarray(sun_dir, np.float64)
    s = s / np.linalg.norm(s)
    dirs, E = [s], [float(sun_irradiance)]
    dw = 4.0 * np.pi / (n_bands * n_az)
    for b in range(n_bands):
        y = -1.0 + (2.0 * b + 1.0) / n_bands
        r = np.sqrt(max(0.0, 1.0 - y * y))
        for a in range(n_az):
            phi = 2.0 * np.pi * (a + 0.5) / n_az
            v = np.array([r * np.cos(phi), y, r * np.sin(phi)])
            if y > 0:
                ang = np.arccos(np.clip(v @ s, -1.0, 1.0))
                L = sky_radiance * (0.6 + 0.4 * (1.0 - y)) * (1.0 + 2.0 * np.exp(-3.0 * ang))
            else:
                L = ground * sky_radiance
            dirs.append(v)
            E.append(L * dw)
    return np.asarray(dirs, np.float32), np.asarray(E, np.float64)


def envmap_lights(radiance, min_radiance: float = 0.0):
    """An environment map as a set of directional lights (Sec. 4.4: a distant emitter of
    any shape is a set of directions).  radiance is an equirectangular map (H, W): row i
    covers polar angles [i, i + 1] pi / H from the up axis +y, column j azimuths
    [j, j + 1] 2 pi / W.  One light per texel at its centre (mid polar angle, mid
    azimuth), with irradiance radiance times the texel's exact solid angle
    (cos theta_i - cos theta_{i+1}) 2 pi / W; texels at or below min_radiance are
    dropped.  Input data only: returns (dirs (m, 3) float32, irradiance (m,) float64)."""
    L = np.asarray(radiance, np.float64)
    H, W = L.shape
    t0 = np.pi * np.arange(H) / H
    t1 = np.pi * np.arange(1, H + 1) / H
    dw = (np.cos(t0) - np.cos(t1)) * 2.0 * np.pi / W
    th = 0.5 * (t0 + t1)
    ph = 2.0 * np.pi * (np.arange(W) + 0.5) / W
    st, ct = np.sin(th)[:, None], np.cos(th)[:, None]
    dirs = np.stack(np.broadcast_arrays(st * np.cos(ph)[None, :], ct, st * np.sin(ph)[None, :]),
                    -1).reshape(-1, 3)
    E = (L * dw[:, None]).reshape(-1)
    keep = L.reshape(-1) > min_radiance
    return dirs[keep].astype(np.float32), E[keep]


def synthetic_envmap(sun_dir, H: int = 32, W: int = 64, lobe_power: float = 1.0,
                     lobe_width: float = 0.1, sky_radiance: float = 0.08,
                     ground: float = 0.25) -> np.ndarray:
    """A synthetic HDR environment map (H, W) in the layout of envmap_lights: a bright
    lobe around sun_dir, radiance S exp((cos a - 1) / w^2) at angle a with S = lobe_power
    / (2 pi w^2) (the lobe integrates to lobe_power (1 - exp(-2 / w^2)) over the sphere),
    over a sky of sky_radiance (0.6 + 0.4 (1 - y)) above the horizon and ground *
    sky_radiance below it, each evaluated at the texel centre.  Input data only."""
    s = np.asarray(sun_dir, np.float64)
    s = s / np.linalg.norm(s)
    th = np.pi * (np.arange(H) + 0.5) / H
    ph = 2.0 * np.pi * (np.arange(W) + 0.5) / W
    x = np.sin(th)[:, None] * np.cos(ph)[None, :]
    y = np.broadcast_to(np.cos(th)[:, None], (H, W))
    z = np.sin(th)[:, None] * np.sin(ph)[None, :]
    cos_a = x * s[0] + y * s[1] + z * s[2]
    lobe = lobe_power / (2.0 * np.pi * lobe_width ** 2) * np.exp((cos_a - 1.0) / lobe_width ** 2)
    sky = np.where(y > 0, sky_radiance * (0.6 + 0.4 * (1.0 - y)), ground * sky_radiance)
    return lobe + sky


def init_mlp(widths, seed: int, out_scale: float = 1.0, out_bias: float = 0.0) -> np.ndarray:
    """He-uniform weights and zero biases for an all-at-once MLP (widths: input first,
    output last; per layer W [out][in] then b [out]); out_scale multiplies the last
    layer's weights and out_bias sets its bias.  float32 vector."""
    rng = np.random.default_rng(seed)
    parts = []
    L = len(widths) - 1
    for l, (i, o) in enumerate(zip(widths[:-1], widths[1:])):
        b = math.sqrt(6.0 / i)
        w = rng.uniform(-b, b, size=o * i)
        bias = np.zeros(o)
        if l == L - 1:
            w = w * out_scale
            bias[:] = out_bias
        parts += [w, bias]
    return np.concatenate(parts).astype(np.float32)


# --------------------------------------------------------------------------------------
# Lorenz-Mie phase function of a cloud droplet population (input data for the tracer)
# --------------------------------------------------------------------------------------
def mie_amplitudes(x: float, m: complex, mu: np.ndarray):
    """Lorenz-Mie scattering of a homogeneous sphere of size parameter x = 2 pi r / lambda
    and relative refractive index m, by the series of Bohren and Huffman (1983, Ch. 4 and
    App. A): a_n, b_n from the logarithmic derivative D_n(m x) (downward recurrence) and
    the Riccati-Bessel functions (upward recurrence), the angle functions pi_n, tau_n by
    their recurrences in mu = cos(theta).  Returns (S1(mu), S2(mu), Q_ext, Q_sca)."""
    mu = np.asarray(mu, np.float64)
    y = m * x
    nstop = int(x + 4.0 * x ** (1.0 / 3.0) + 2.0)
    nmx = int(max(nstop, abs(y))) + 16
    D = np.zeros(nmx + 1, complex)
    for n in range(nmx, 0, -1):
        D[n - 1] = n / y - 1.0 / (D[n] + n / y)
    psi0, psi1 = np.cos(x), np.sin(x)          # psi_{-1}, psi_0
    chi0, chi1 = -np.sin(x), np.cos(x)         # chi_{-1}, chi_0
    xi1 = complex(psi1, -chi1)
    pi0, pi1 = np.zeros_like(mu), np.ones_like(mu)
    S1 = np.zeros(mu.shape, complex)
    S2 = np.zeros(mu.shape, complex)
    qext = qsca = 0.0
    for n in range(1, nstop + 1):
        psi = (2 * n - 1) / x * psi1 - psi0
        chi = (2 * n - 1) / x * chi1 - chi0
        xi = complex(psi, -chi)
        da = D[n] / m + n / x
        db = D[n] * m + n / x
        an = (da * psi - psi1) / (da * xi - xi1)
        bn = (db * psi - psi1) / (db * xi - xi1)
        tau = n * mu * pi1 - (n + 1) * pi0
        f = (2 * n + 1) / (n * (n + 1))
        S1 += f * (an * pi1 + bn * tau)
        S2 += f * (an * tau + bn * pi1)
        qext += (2 * n + 1) * (an + bn).real
        qsca += (2 * n + 1) * (abs(an) ** 2 + abs(bn) ** 2)
        pi0, pi1 = pi1, ((2 * n + 1) * mu * pi1 - (n + 1) * pi0) / n
        psi0, psi1, chi0, chi1, xi1 = psi1, psi, chi1, chi, xi
    return S1, S2, 2.0 * qext / x ** 2, 2.0 * qsca / x ** 2


def cloud_droplet_phase(n_theta: int = 3601, wavelength_um: float = 0.55,
                        r_eff_um: float = 8.0, v_eff: float = 0.1, m: complex = 1.333 + 0j,
                        n_r: int = 160):
    """Phase function (per steradian, unpolarised light) of water droplets following the
    gamma size distribution of Hansen and Travis (1974), n(r) ~ r^((1 - 3 v) / v)
    exp(-r / (r_eff v)), on n_theta angles theta_i = i pi / (n_theta - 1).  The paper's
    own droplet parameters are not given; these are typical of cumulus.  Radii: n_r
    Gauss-Legendre nodes over [r_eff / 20, r_eff (1 + 12 sqrt(v))].  Returns (theta,
    p(theta), mean cosine)."""
    theta = np.linspace(0.0, np.pi, n_theta)
    mu = np.cos(theta)
    lo, hi = r_eff_um / 20.0, r_eff_um * (1.0 + 12.0 * math.sqrt(v_eff))
    t, w = np.polynomial.legendre.leggauss(n_r)
    r = 0.5 * (hi - lo) * t + 0.5 * (hi + lo)
    w = 0.5 * (hi - lo) * w
    nr = r ** ((1.0 - 3.0 * v_eff) / v_eff) * np.exp(-r / (r_eff_um * v_eff))
    num = np.zeros(n_theta)
    den = 0.0
    for ri, wi, ni in zip(r, w, nr):
        x = 2.0 * math.pi * ri / wavelength_um
        S1, S2, _, qs = mie_amplitudes(x, m, mu)
        num += wi * ni * (np.abs(S1) ** 2 + np.abs(S2) ** 2)
        den += wi * ni * 2.0 * math.pi * x * x * qs
    p = num / den
    g = float(np.trapezoid(2.0 * math.pi * p * mu * np.sin(theta), theta))
    return theta, p, g
