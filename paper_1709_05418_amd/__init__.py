"""Python binding of libdeepscatter (MI355X / gfx950 radiance prediction).

Thin ctypes layer over the C ABI in include/deepscatter.h: every ds_* function
here marshals torch device tensors (data pointers) and the current HIP stream and
calls the C entry point of the same name.  All computation happens in the HIP
kernels of libdeepscatter.so; there is no CPU fallback.  Importing works without
the library, but every call raises if libdeepscatter.so has not been built
(python -m paper_1709_05418_amd.build).

The small classes at the end (Context, Cloud, Net) only own handles and call the
same functions.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdeepscatter.so")

DS_OK = 0
DS_ERR_INVALID_ARG, DS_ERR_OOM, DS_ERR_DEVICE, DS_ERR_UNSUPPORTED, DS_ERR_STATE = -1, -2, -3, -4, -5
DS_F32, DS_BF16 = 0, 1
DS_PREC_F32, DS_PREC_BF16, DS_PREC_FP8 = 0, 1, 2
DS_FLAG_INVALID, DS_FLAG_OUTSIDE, DS_FLAG_FALLBACK = 1, 2, 4
DS_LIGHT_DIRECTIONAL, DS_LIGHT_ENVIRONMENT = 0, 1
DS_KERNEL_REGISTER, DS_KERNEL_PIPELINED, DS_KERNEL_WIDE, DS_KERNEL_TEAMS = 0, 1, 2, 3
DS_ORDER_INPUT, DS_ORDER_SPATIAL = 0, 1
STENCIL_N = 225

_lib = None


class DSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def lib():
    """Load libdeepscatter.so (raises if it is missing: no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_1709_05418_amd.build")
    L = C.CDLL(LIB_PATH)
    P, I, F, D, I64, S = C.c_void_p, C.c_int, C.c_float, C.c_double, C.c_int64, C.c_int32
    sig = {
        "ds_last_error": (C.c_char_p, []),
        "ds_version": (C.c_char_p, []),
        "ds_create": (S, [I, P, P]),
        "ds_set_stream": (S, [P, P]),
        "ds_synchronize": (S, [P]),
        "ds_destroy": (S, [P]),
        "ds_cloud_create": (S, [P, P, I, I, I, I, F, P, F, I, P, I, P]),
        "ds_cloud_info": (S, [P, P, P, P, P, P]),
        "ds_cloud_level": (S, [P, P, I, P]),
        "ds_cloud_destroy": (S, [P]),
        "ds_net_param_count": (I64, [P]),
        "ds_net_create": (S, [P, P, P]),
        "ds_net_set_params": (S, [P, P, I64]),
        "ds_net_get_params": (S, [P, P, I64]),
        "ds_net_destroy": (S, [P]),
        "ds_gather": (S, [P, P, P, P, P, I64, I, P, P]),
        "ds_gather_packed": (S, [P, P, P, P, P, I64, P]),
        "ds_forward": (S, [P, P, P, I64, P, P]),
        "ds_predict": (S, [P, P, P, I, P, P, P, I64, P, P, P]),
        "ds_predict_reserve": (S, [P, P, P, I, I64]),
        "ds_predict_f32_noalloc": (S, [P, P, P, P, P, P, I64, P, P, P]),
        "ds_adam_create": (S, [P, F, F, F, F, P]),
        "ds_adam_destroy": (S, [P]),
        "ds_adam_set_lr": (S, [P, F]),
        "ds_adam_steps": (S, [P, P]),
        "ds_loss_grad": (S, [P, P, P, I, P, P]),
        "ds_train_step": (S, [P, P, P, P, I, P]),
        "ds_train_capture": (S, [P, P, P, P, I, P]),
        "ds_train_replay": (S, [P]),
        "ds_net_set_train_precision": (S, [P, I]),
        "ds_net_quantize": (S, [P, P, P, I, P, P, P, I64]),
        "ds_net_fp8_scales": (S, [P, P, S]),
        "ds_fp8_e4m3_encode": (S, [P, I64, S, P]),
        "ds_cloud_majorant": (S, [P, P]),
        "ds_tracer_truncated": (S, [P, P, I]),
        "ds_trace_li": (S, [P, P, P, P, P, P, I64, I, C.c_uint64, P, P]),
        "ds_sample_records": (S, [P, P, I64, C.c_uint64, P, P, P, P]),
        "ds_render_mc": (S, [P, P, P, P, P, P, I64, I, C.c_uint64, P, P]),
        "ds_first_hits": (S, [P, P, P, P, P, P, I64, C.c_uint64, C.c_uint64, P, P, P, P]),
        "ds_philox4x32_10": (S, [P, P, I64, P]),
        "ds_batch_create": (S, [P, P, I, P, P, P]),
        "ds_batch_destroy": (S, [P]),
        "ds_batch_set_config": (S, [P, S, S, S]),
        "ds_batch_get_config": (S, [P, P, P, P, P]),
        "ds_batch_predict": (S, [P, I, P, P, P, P, P, P]),
        "ds_batch_autotune": (S, [P, I, P, P, P, P, I]),
        "ds_batch_capture": (S, [P, I, P, P, P, P, P, P]),
        "ds_batch_replay": (S, [P]),
        "ds_batch_set_order": (S, [P, S]),
        "ds_make_records": (S, [P, P, P, I64, I, C.c_uint64, I64, P, P, P, P, P, P, P]),
        "ds_render_rpnn": (S, [P, P, P, I, P, P, P, P, I64, I, C.c_uint64, I, P, P, P, P]),
        "ds_trace_li_adaptive": (S, [P, P, P, P, P, P, P, I64, C.c_uint64, P, P, P]),
        "ds_make_records_adaptive": (S, [P, P, P, P, I64, C.c_uint64, I64, P, P, P, P, P, P, P,
                                         P]),
        "ds_net_param_count_mlp": (I64, [S, S, P]),
        "ds_net_create_mlp": (S, [P, S, S, P, P]),
        "ds_phase_build": (S, [S, P, D, P, P, P, P]),
        "ds_phase_create": (S, [P, S, P, D, P]),
        "ds_phase_info": (S, [P, P, P]),
        "ds_phase_destroy": (S, [P]),
        "ds_lights_create": (S, [P, S, P, P, P]),
        "ds_light_table": (S, [S, P, P, P]),
        "ds_lights_destroy": (S, [P]),
        "ds_render_mc_lights": (S, [P, P, P, P, P, P, I64, I, C.c_uint64, P, P]),
        "ds_first_hits_lights": (S, [P, P, P, P, S, P, P, I64, C.c_uint64, C.c_uint64, P, P, P,
                                     P, P, P]),
        "ds_render_rpnn_lights": (S, [P, P, P, I, P, P, S, P, P, I64, I, C.c_uint64, I, P, P, P,
                                      P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


class _NetDesc(C.Structure):
    _fields_ = [("K", C.c_int), ("W", C.c_int), ("H", C.c_int)]


class TracerParams(C.Structure):
    """ds_tracer_params: albedo, HG g, light irradiance (or environment radiance),
    light_mode (DS_LIGHT_DIRECTIONAL / DS_LIGHT_ENVIRONMENT), max_interactions (0: none),
    include_direct (record estimates of L_s = L_d + L_i instead of L_i)."""
    _fields_ = [("albedo", C.c_float), ("g", C.c_float), ("irradiance", C.c_float),
                ("light_mode", C.c_int32), ("max_interactions", C.c_int32),
                ("include_direct", C.c_int32), ("phase", C.c_void_p),
                ("phase_first", C.c_void_p)]

    def __init__(self, albedo=0.999, g=0.85, irradiance=1.0, light_mode=0, max_interactions=0,
                 include_direct=0, phase=None, phase_first=None):
        """phase / phase_first: Phase objects (tabulated phase functions) or None."""
        h = lambda ph: None if ph is None else (ph.h.value if hasattr(ph, "h") else ph)
        super().__init__(float(albedo), float(g), float(irradiance), int(light_mode),
                         int(max_interactions), int(include_direct), h(phase),
                         h(phase_first))


class Adaptive(C.Structure):
    """ds_adaptive: paths in batches of batch_spp until z * sqrt(var of mean) <= rel * |mean|
    or max_spp paths (Sec. 5.1 uses rel 0.02 at 95 %, z = 1.96)."""
    _fields_ = [("batch_spp", C.c_int32), ("max_spp", C.c_int32), ("rel", C.c_double),
                ("z", C.c_double)]

    def __init__(self, batch_spp=256, max_spp=65536, rel=0.02, z=1.96):
        super().__init__(int(batch_spp), int(max_spp), float(rel), float(z))


def _check(st):
    if st != DS_OK:
        raise DSError(st, lib().ds_last_error().decode())


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device (cuda) tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _pts(t, P=None):
    import torch
    if t.dtype != torch.float32 or t.dim() != 2 or t.shape[1] != 3:
        raise ValueError("points and directions must be float32 tensors of shape (P, 3)")
    if P is not None and t.shape[0] != P:
        raise ValueError("points and directions must have the same length")
    return _ptr(t)


# ----------------------------------------------------------------------------- C ABI
def ds_version() -> str:
    return lib().ds_version().decode()


def ds_last_error() -> str:
    return lib().ds_last_error().decode()


def ds_create(device: int = 0, stream=None):
    h = C.c_void_p()
    _check(lib().ds_create(device, _stream_handle(stream), C.byref(h)))
    return h


def ds_set_stream(ctx, stream=None):
    _check(lib().ds_set_stream(ctx, _stream_handle(stream)))


def ds_synchronize(ctx):
    _check(lib().ds_synchronize(ctx))


def ds_destroy(ctx):
    _check(lib().ds_destroy(ctx))


def ds_cloud_create(ctx, density, sigma_max, aabb_min, voxel_size, n_levels, K, mip_of_level=None):
    import torch
    if density.dim() != 3:
        raise ValueError("density must be a (nz, ny, nx) tensor")
    dt = {torch.float32: DS_F32, torch.bfloat16: DS_BF16}.get(density.dtype)
    if dt is None:
        raise ValueError("density must be float32 or bfloat16")
    nz, ny, nx = density.shape
    amin = (C.c_float * 3)(*[float(v) for v in aabb_min])
    mips = None
    if mip_of_level is not None:
        mips = (C.c_int * len(mip_of_level))(*[int(v) for v in mip_of_level])
    h = C.c_void_p()
    _check(lib().ds_cloud_create(ctx, _ptr(density), dt, nx, ny, nz, float(sigma_max), amin,
                                 float(voxel_size), int(n_levels), mips, int(K), C.byref(h)))
    return h


def ds_cloud_info(cloud):
    mean = C.c_double()
    L = C.c_int()
    K = C.c_int()
    dims = (C.c_int * 48)()
    mips = (C.c_int * 16)()
    _check(lib().ds_cloud_info(cloud, C.byref(mean), C.byref(L), dims, mips, C.byref(K)))
    return {"mean_mu_t": mean.value, "n_levels": L.value, "K": K.value,
            "dims": [tuple(dims[3 * i:3 * i + 3]) for i in range(L.value)],
            "mip_of_level": list(mips[:K.value])}


def ds_cloud_level(ctx, cloud, level: int):
    import torch
    info = ds_cloud_info(cloud)
    nx, ny, nz = info["dims"][level]
    out = torch.empty((nz, ny, nx), dtype=torch.float32, device="cuda")
    _check(lib().ds_cloud_level(ctx, cloud, int(level), _ptr(out)))
    return out


def ds_cloud_destroy(cloud):
    _check(lib().ds_cloud_destroy(cloud))


def ds_net_param_count(K: int, W: int, H: int = 3) -> int:
    d = _NetDesc(K, W, H)
    return int(lib().ds_net_param_count(C.byref(d)))


def ds_net_create(ctx, K: int, W: int, H: int = 3):
    d = _NetDesc(K, W, H)
    h = C.c_void_p()
    _check(lib().ds_net_create(ctx, C.byref(d), C.byref(h)))
    return h


def ds_net_set_params(net, theta):
    th = np.ascontiguousarray(theta, dtype=np.float32)
    _check(lib().ds_net_set_params(net, C.c_void_p(th.ctypes.data), th.size))


def ds_net_get_params(net, n: int):
    th = np.zeros(n, np.float32)
    _check(lib().ds_net_get_params(net, C.c_void_p(th.ctypes.data), n))
    return th


def ds_net_destroy(net):
    _check(lib().ds_net_destroy(net))


def ds_gather(ctx, cloud, pos, view_dir, light_dir, K: int, out_dtype=None, flags=True):
    import torch
    P = pos.shape[0]
    odt = torch.float32 if out_dtype is None else out_dtype
    code = {torch.float32: DS_F32, torch.bfloat16: DS_BF16}[odt]
    z = torch.empty((P, STENCIL_N * K + 1), dtype=odt, device=pos.device)
    fl = torch.empty(P, dtype=torch.uint8, device=pos.device) if flags else None
    _check(lib().ds_gather(ctx, cloud, _pts(pos), _pts(view_dir, P), _pts(light_dir, P), P, code,
                           _ptr(z), _ptr(fl)))
    return z, fl


def ds_gather_packed(ctx, cloud, pos, view_dir, light_dir, K: int):
    import torch
    P = pos.shape[0]
    z = torch.empty((P, STENCIL_N * K + 1), dtype=torch.float32, device=pos.device)
    _check(lib().ds_gather_packed(ctx, cloud, _pts(pos), _pts(view_dir, P), _pts(light_dir, P), P,
                                  _ptr(z)))
    return z


def ds_forward(ctx, net, z, want_pre=True):
    import torch
    if z.dtype != torch.float32 or z.dim() != 2:
        raise ValueError("z must be a float32 (P, 225K+1) tensor")
    P = z.shape[0]
    out = torch.empty(P, dtype=torch.float32, device=z.device)
    pre = torch.empty(P, dtype=torch.float32, device=z.device) if want_pre else None
    _check(lib().ds_forward(ctx, net, _ptr(z), P, _ptr(out), _ptr(pre)))
    return out, pre


def ds_predict(ctx, cloud, net, precision, pos, view_dir, light_dir, out=None, pre=None,
               flags=None, want_pre=True, want_flags=True):
    import torch
    P = pos.shape[0]
    if out is None:
        out = torch.empty(P, dtype=torch.float32, device=pos.device)
    if pre is None and want_pre:
        pre = torch.empty(P, dtype=torch.float32, device=pos.device)
    if flags is None and want_flags:
        flags = torch.empty(P, dtype=torch.uint8, device=pos.device)
    _check(lib().ds_predict(ctx, cloud, net, int(precision), _pts(pos), _pts(view_dir, P),
                            _pts(light_dir, P), P, _ptr(out), _ptr(pre), _ptr(flags)))
    return out, pre, flags


def ds_predict_reserve(ctx, cloud, net, precision, P):
    """Build ahead what ds_predict with at most P points would create on first use."""
    _check(lib().ds_predict_reserve(ctx, cloud, net, int(precision), int(P)))


def ds_predict_f32_noalloc(ctx, cloud, net, pos, view_dir, light_dir, out=None, pre=None,
                           flags=None, want_pre=True, want_flags=True):
    """ds_predict in FP32 through the library's per-device scratch (no allocation)."""
    import torch
    P = pos.shape[0]
    if out is None:
        out = torch.empty(P, dtype=torch.float32, device=pos.device)
    if pre is None and want_pre:
        pre = torch.empty(P, dtype=torch.float32, device=pos.device)
    if flags is None and want_flags:
        flags = torch.empty(P, dtype=torch.uint8, device=pos.device)
    _check(lib().ds_predict_f32_noalloc(ctx, cloud, net, _pts(pos), _pts(view_dir, P),
                                        _pts(light_dir, P), P, _ptr(out), _ptr(pre),
                                        _ptr(flags)))
    return out, pre, flags


def ds_net_set_train_precision(net, precision):
    _check(lib().ds_net_set_train_precision(net, int(precision)))


def ds_net_quantize(ctx, net, cloud, precision, pos, view_dir, light_dir):
    """Build the FP8 form, calibrated on these points of `cloud` (device tensors)."""
    P = pos.shape[0]
    _check(lib().ds_net_quantize(ctx, net, cloud, int(precision), _pts(pos), _pts(view_dir, P),
                                 _pts(light_dir, P), P))


def ds_net_fp8_scales(net, K: int, H: int):
    """log2 units of the FP8 form's activations, then its matrix exponents (numpy int32)."""
    import numpy as np
    n = 3 * K + 2 * H - 2
    out = np.zeros(n, dtype=np.int32)
    _check(lib().ds_net_fp8_scales(net, out.ctypes.data_as(C.c_void_p), n))
    return out


def ds_fp8_e4m3_encode(x, log2_scale: int = 0):
    """The library's host E4M3 encoder on a float32 numpy array (codes as uint8)."""
    import numpy as np
    x = np.ascontiguousarray(x, dtype=np.float32)
    codes = np.zeros(x.shape, dtype=np.uint8)
    _check(lib().ds_fp8_e4m3_encode(x.ctypes.data_as(C.c_void_p), x.size, int(log2_scale),
                                    codes.ctypes.data_as(C.c_void_p)))
    return codes


def ds_adam_create(net, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    h = C.c_void_p()
    _check(lib().ds_adam_create(net, float(lr), float(beta1), float(beta2), float(eps),
                                C.byref(h)))
    return h


def ds_adam_destroy(opt):
    _check(lib().ds_adam_destroy(opt))


def ds_adam_set_lr(opt, lr):
    _check(lib().ds_adam_set_lr(opt, float(lr)))


def ds_adam_steps(opt) -> int:
    t = C.c_int64()
    _check(lib().ds_adam_steps(opt, C.byref(t)))
    return t.value


def _batch(z, target):
    import torch
    if z.dtype != torch.float32 or z.dim() != 2 or target.dtype != torch.float32:
        raise ValueError("z must be float32 (B, 225K+1) and target float32 (B,)")
    if target.shape[0] != z.shape[0]:
        raise ValueError("z and target have different batch sizes")
    return z.shape[0]


def ds_loss_grad(net, z, target_log1p, n_params, want_grad=True):
    import torch
    B = _batch(z, target_log1p)
    loss = torch.empty(1, dtype=torch.float32, device=z.device)
    grad = torch.empty(n_params, dtype=torch.float32, device=z.device) if want_grad else None
    _check(lib().ds_loss_grad(net, _ptr(z), _ptr(target_log1p), B, _ptr(loss), _ptr(grad)))
    return loss, grad


def ds_train_step(net, opt, z, target_log1p, loss=None):
    import torch
    B = _batch(z, target_log1p)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=z.device)
    _check(lib().ds_train_step(net, opt, _ptr(z), _ptr(target_log1p), B, _ptr(loss)))
    return loss


def ds_train_capture(net, opt, z, target_log1p, loss):
    """Capture one ds_train_step on these buffers (loss: device tensor of one float)."""
    B = _batch(z, target_log1p)
    _check(lib().ds_train_capture(net, opt, _ptr(z), _ptr(target_log1p), B, _ptr(loss)))


def ds_train_replay(opt):
    _check(lib().ds_train_replay(opt))


def ds_tracer_truncated(ctx, reset=False) -> int:
    """Paths stopped at the tracer's bound on tentative collisions (see the header)."""
    n = C.c_int64()
    _check(lib().ds_tracer_truncated(ctx, C.byref(n), int(bool(reset))))
    return n.value


def ds_cloud_majorant(cloud) -> float:
    m = C.c_float()
    _check(lib().ds_cloud_majorant(cloud, C.byref(m)))
    return m.value


def _f64(n, device):
    import torch
    return torch.empty(n, dtype=torch.float64, device=device)


def ds_trace_li(ctx, cloud, params: TracerParams, pos, view_dir, light_dir, spp, seed,
                want_var=True):
    """Per record: (mean of spp path estimates of L_i, variance of that mean), FP64."""
    P = pos.shape[0]
    mean = _f64(P, pos.device)
    var = _f64(P, pos.device) if want_var else None
    _check(lib().ds_trace_li(ctx, cloud, C.byref(params), _pts(pos), _pts(view_dir, P),
                             _pts(light_dir, P), P, int(spp), int(seed), _ptr(mean), _ptr(var)))
    return mean, var


def ds_trace_li_adaptive(ctx, cloud, params: TracerParams, adaptive: Adaptive, pos, view_dir,
                         light_dir, seed, want_var=True):
    """Per record: (mean, variance of the mean, paths used) of the progressive estimate."""
    import torch
    P = pos.shape[0]
    mean = _f64(P, pos.device)
    var = _f64(P, pos.device) if want_var else None
    n = torch.empty(P, dtype=torch.int32, device=pos.device)
    _check(lib().ds_trace_li_adaptive(ctx, cloud, C.byref(params), C.byref(adaptive), _pts(pos),
                                      _pts(view_dir, P), _pts(light_dir, P), P, int(seed),
                                      _ptr(mean), _ptr(var), _ptr(n)))
    return mean, var, n


def ds_sample_records(ctx, cloud, N, seed, device="cuda", want_attempts=True):
    import torch
    pos = torch.empty((N, 3), dtype=torch.float32, device=device)
    view = torch.empty((N, 3), dtype=torch.float32, device=device)
    light = torch.empty((N, 3), dtype=torch.float32, device=device)
    att = torch.empty(N, dtype=torch.int32, device=device) if want_attempts else None
    _check(lib().ds_sample_records(ctx, cloud, int(N), int(seed), _ptr(pos), _ptr(view),
                                   _ptr(light), _ptr(att)))
    return pos, view, light, att


def ds_render_mc(ctx, cloud, params: TracerParams, light_dir, ray_o, ray_d, spp, seed,
                 want_var=True):
    N = ray_o.shape[0]
    ld = (C.c_float * 3)(*[float(v) for v in light_dir])
    mean = _f64(N, ray_o.device)
    var = _f64(N, ray_o.device) if want_var else None
    _check(lib().ds_render_mc(ctx, cloud, C.byref(params), ld, _pts(ray_o), _pts(ray_d, N), N,
                              int(spp), int(seed), _ptr(mean), _ptr(var)))
    return mean, var


def ds_first_hits(ctx, cloud, params: TracerParams, light_dir, ray_o, ray_d, seed, sample=0):
    import torch
    N = ray_o.shape[0]
    ld = (C.c_float * 3)(*[float(v) for v in light_dir])
    dev = ray_o.device
    pos = torch.empty((N, 3), dtype=torch.float32, device=dev)
    view = torch.empty((N, 3), dtype=torch.float32, device=dev)
    direct = torch.empty(N, dtype=torch.float32, device=dev)
    hit = torch.empty(N, dtype=torch.uint8, device=dev)
    _check(lib().ds_first_hits(ctx, cloud, C.byref(params), ld, _pts(ray_o), _pts(ray_d, N), N,
                               int(seed), int(sample), _ptr(pos), _ptr(view), _ptr(direct),
                               _ptr(hit)))
    return pos, view, direct, hit


def ds_batch_create(ctx, net, clouds, offsets):
    """clouds: list of cloud handles; offsets: n + 1 row offsets into the concatenated
    point arrays."""
    n = len(clouds)
    arr = (C.c_void_p * n)(*[c.value if isinstance(c, C.c_void_p) else c for c in clouds])
    off = (C.c_int64 * (n + 1))(*[int(v) for v in offsets])
    h = C.c_void_p()
    _check(lib().ds_batch_create(ctx, net, n, arr, off, C.byref(h)))
    return h


def ds_batch_destroy(batch):
    _check(lib().ds_batch_destroy(batch))


def ds_batch_set_config(batch, kernel, waves, grid):
    _check(lib().ds_batch_set_config(batch, int(kernel), int(waves), int(grid)))


def ds_batch_get_config(batch):
    k, w, g, ms = C.c_int32(), C.c_int32(), C.c_int32(), C.c_float()
    _check(lib().ds_batch_get_config(batch, C.byref(k), C.byref(w), C.byref(g), C.byref(ms)))
    return {"kernel": k.value, "waves": w.value, "grid": g.value, "ms": ms.value}


def ds_batch_predict(batch, precision, pos, view_dir, light_dir, out, pre=None, flags=None):
    P = pos.shape[0]
    _check(lib().ds_batch_predict(batch, int(precision), _pts(pos), _pts(view_dir, P),
                                  _pts(light_dir, P), _ptr(out), _ptr(pre), _ptr(flags)))


def ds_batch_autotune(batch, precision, pos, view_dir, light_dir, out, reps=3):
    P = pos.shape[0]
    _check(lib().ds_batch_autotune(batch, int(precision), _pts(pos), _pts(view_dir, P),
                                   _pts(light_dir, P), _ptr(out), int(reps)))
    return ds_batch_get_config(batch)


def ds_batch_capture(batch, precision, pos, view_dir, light_dir, out, pre=None, flags=None):
    P = pos.shape[0]
    _check(lib().ds_batch_capture(batch, int(precision), _pts(pos), _pts(view_dir, P),
                                  _pts(light_dir, P), _ptr(out), _ptr(pre), _ptr(flags)))


def ds_batch_replay(batch):
    _check(lib().ds_batch_replay(batch))


def ds_batch_set_order(batch, order):
    """DS_ORDER_INPUT or DS_ORDER_SPATIAL (points of each cloud sorted by a 32^3 grid cell
    before every fused launch; outputs stay in input order)."""
    _check(lib().ds_batch_set_order(batch, int(order)))


def ds_make_records(ctx, cloud, params: TracerParams, N, spp, seed, z, target, offset=0,
                    stride=1, want_records=False, want_li=False):
    """Training pairs into rows offset + i * stride of z ((M, 225K+1) float32) and
    target ((M,) float32, log(1 + L_i)).  Optionally returns (pos, view, light) and
    (li_mean, li_var) of the N records.  spp may be an Adaptive (progressive path
    counts); then the second tuple also holds the paths each record used."""
    import torch
    D = z.shape[1]
    if z.dtype != torch.float32 or target.dtype != torch.float32 or z.dim() != 2:
        raise ValueError("z must be float32 (M, 225K+1), target float32 (M,)")
    if N > 0 and (offset + (N - 1) * stride >= z.shape[0] or
                  offset + (N - 1) * stride >= target.shape[0]):
        raise ValueError("z / target too small for N records at this offset and stride")
    dev = z.device
    rec = [torch.empty((N, 3), dtype=torch.float32, device=dev) for _ in range(3)] \
        if want_records else [None, None, None]
    li = [torch.empty(N, dtype=torch.float64, device=dev) for _ in range(2)] \
        if want_li else [None, None]
    zp = C.c_void_p(z.data_ptr() + 4 * D * offset) if N > 0 else None
    tp = C.c_void_p(target.data_ptr() + 4 * offset) if N > 0 else None
    if isinstance(spp, Adaptive):   # progressive path counts (ds_make_records_adaptive)
        n = torch.empty(N, dtype=torch.int32, device=dev) if want_li else None
        _check(lib().ds_make_records_adaptive(ctx, cloud, C.byref(params), C.byref(spp), int(N),
                                              int(seed), int(stride), zp, tp,
                                              *[_ptr(t) for t in rec], *[_ptr(t) for t in li],
                                              _ptr(n)))
        li = li + [n] if want_li else li
    else:
        _check(lib().ds_make_records(ctx, cloud, C.byref(params), int(N), int(spp), int(seed),
                                     int(stride), zp, tp, *[_ptr(t) for t in rec],
                                     *[_ptr(t) for t in li]))
    return (tuple(rec) if want_records else None), (tuple(li) if want_li else None)


def ds_render_rpnn(ctx, cloud, net, precision, params: TracerParams, light_dir, ray_o, ray_d,
                   spp, seed, fallback_spp=0, want_var=True, want_direct=True,
                   count_fallback=False):
    """Per pixel: (mean, variance of the mean, mean of the direct term, fallback count)."""
    N = ray_o.shape[0]
    ld = (C.c_float * 3)(*[float(v) for v in light_dir])
    mean = _f64(N, ray_o.device)
    var = _f64(N, ray_o.device) if want_var else None
    direct = _f64(N, ray_o.device) if want_direct else None
    nfb = C.c_int64(0)
    _check(lib().ds_render_rpnn(ctx, cloud, net, int(precision), C.byref(params), ld,
                                _pts(ray_o), _pts(ray_d, N), N, int(spp), int(seed),
                                int(fallback_spp), _ptr(mean), _ptr(var), _ptr(direct),
                                C.byref(nfb) if count_fallback else None))
    return mean, var, direct, (nfb.value if count_fallback else None)


def ds_lights_create(ctx, dirs, irradiance):
    """dirs: (m, 3) host array; irradiance: m positive values.  Returns the handle."""
    d = np.ascontiguousarray(np.asarray(dirs, np.float32).reshape(-1, 3))
    e = np.ascontiguousarray(np.asarray(irradiance, np.float64).reshape(-1))
    if e.size != d.shape[0]:
        raise ValueError("one irradiance per light direction")
    h = C.c_void_p()
    _check(lib().ds_lights_create(ctx, int(d.shape[0]), d.ctypes.data, e.ctypes.data,
                                  C.byref(h)))
    return h


def ds_light_table(irradiance):
    """The library's selection table of a light set (host only): thresholds, weights."""
    e = np.ascontiguousarray(np.asarray(irradiance, np.float64).reshape(-1))
    thr = np.zeros(e.size, np.uint32)
    w = np.zeros(e.size, np.float64)
    _check(lib().ds_light_table(int(e.size), e.ctypes.data, thr.ctypes.data, w.ctypes.data))
    return thr, w


def ds_lights_destroy(lights):
    _check(lib().ds_lights_destroy(lights))


def ds_render_mc_lights(ctx, cloud, params: TracerParams, lights, ray_o, ray_d, spp, seed,
                        want_var=True):
    N = ray_o.shape[0]
    mean = _f64(N, ray_o.device)
    var = _f64(N, ray_o.device) if want_var else None
    _check(lib().ds_render_mc_lights(ctx, cloud, C.byref(params), lights, _pts(ray_o),
                                     _pts(ray_d, N), N, int(spp), int(seed), _ptr(mean),
                                     _ptr(var)))
    return mean, var


def ds_first_hits_lights(ctx, cloud, params: TracerParams, lights, draws, ray_o, ray_d, seed,
                         sample=0):
    """Per ray and draw (rows i * draws + q): pos, view, light, weight; per ray: direct, hit."""
    import torch
    N = ray_o.shape[0]
    R = N * int(draws)
    dev = ray_o.device
    pos = torch.empty((R, 3), dtype=torch.float32, device=dev)
    view = torch.empty((R, 3), dtype=torch.float32, device=dev)
    light = torch.empty((R, 3), dtype=torch.float32, device=dev)
    weight = torch.empty(R, dtype=torch.float32, device=dev)
    direct = torch.empty(N, dtype=torch.float32, device=dev)
    hit = torch.empty(N, dtype=torch.uint8, device=dev)
    _check(lib().ds_first_hits_lights(ctx, cloud, C.byref(params), lights, int(draws),
                                      _pts(ray_o), _pts(ray_d, N), N, int(seed), int(sample),
                                      _ptr(pos), _ptr(view), _ptr(light), _ptr(weight),
                                      _ptr(direct), _ptr(hit)))
    return pos, view, light, weight, direct, hit


def ds_render_rpnn_lights(ctx, cloud, net, precision, params: TracerParams, lights, draws, ray_o,
                          ray_d, spp, seed, fallback_spp=0, want_var=True, want_direct=True,
                          count_fallback=False):
    """Per pixel: (mean, variance of the mean, mean of the direct term, fallback count)."""
    N = ray_o.shape[0]
    mean = _f64(N, ray_o.device)
    var = _f64(N, ray_o.device) if want_var else None
    direct = _f64(N, ray_o.device) if want_direct else None
    nfb = C.c_int64(0)
    _check(lib().ds_render_rpnn_lights(ctx, cloud, net, int(precision), C.byref(params), lights,
                                       int(draws), _pts(ray_o), _pts(ray_d, N), N, int(spp),
                                       int(seed), int(fallback_spp), _ptr(mean), _ptr(var),
                                       _ptr(direct), C.byref(nfb) if count_fallback else None))
    return mean, var, direct, (nfb.value if count_fallback else None)


def ds_philox4x32_10(ctx, ctr_key):
    """ctr_key: int32/uint32 device tensor (n, 6) = c0 c1 c2 c3 k0 k1; returns (n, 4) words
    (as int32 bit patterns)."""
    import torch
    if ctr_key.dim() != 2 or ctr_key.shape[1] != 6 or ctr_key.element_size() != 4:
        raise ValueError("ctr_key must be a 32-bit (n, 6) tensor")
    n = ctr_key.shape[0]
    out = torch.empty((n, 4), dtype=torch.int32, device=ctr_key.device)
    _check(lib().ds_philox4x32_10(ctx, _ptr(ctr_key), n, _ptr(out)))
    return out


# ----------------------------------------------------------------------------- owners
class Context:
    def __init__(self, device: int = 0, stream=None):
        self.h = ds_create(device, stream)

    def close(self):
        if self.h is not None:
            ds_destroy(self.h)
            self.h = None

    def synchronize(self):
        ds_synchronize(self.h)


class Cloud:
    def __init__(self, ctx: Context, density, sigma_max, aabb_min, voxel_size, n_levels, K,
                 mip_of_level=None):
        self.ctx = ctx
        self.h = ds_cloud_create(ctx.h, density, sigma_max, aabb_min, voxel_size, n_levels, K,
                                 mip_of_level)
        self.info = ds_cloud_info(self.h)
        self.K = K

    def level(self, i):
        return ds_cloud_level(self.ctx.h, self.h, i)

    def close(self):
        if self.h is not None:
            ds_cloud_destroy(self.h)
            self.h = None


class Net:
    def __init__(self, ctx: Context, K: int, W: int, H: int = 3):
        self.ctx, self.K, self.W, self.H = ctx, K, W, H
        self.h = ds_net_create(ctx.h, K, W, H)
        self.n_params = ds_net_param_count(K, W, H)

    def set_params(self, theta):
        ds_net_set_params(self.h, theta)

    def get_params(self):
        return ds_net_get_params(self.h, self.n_params)

    def close(self):
        if self.h is not None:
            ds_net_destroy(self.h)
            self.h = None


def ds_net_param_count_mlp(K, widths):
    w = np.ascontiguousarray(np.asarray(widths, np.int32))
    return int(lib().ds_net_param_count_mlp(int(K), int(w.size), w.ctypes.data))


class NetMLP(Net):
    """An all-at-once MLP on the K-level descriptor (Sec. 7's comparison networks);
    widths are the layer output widths, the last 1."""

    def __init__(self, ctx: Context, K: int, widths):
        w = np.ascontiguousarray(np.asarray(widths, np.int32))
        self.ctx, self.K, self.W, self.H = ctx, K, int(w.max()), int(w.size)
        self.widths = [225 * K + 1] + [int(v) for v in w]
        h = C.c_void_p()
        _check(lib().ds_net_create_mlp(ctx.h, int(K), int(w.size), w.ctypes.data, C.byref(h)))
        self.h = h
        self.n_params = ds_net_param_count_mlp(K, w)


def ds_phase_build(p, chop_deg=0.0):
    """The library's phase table on the host: (p, cdf, removed fraction, mean cosine)."""
    a = np.ascontiguousarray(np.asarray(p, np.float64).reshape(-1))
    q = np.zeros(a.size)
    c = np.zeros(a.size)
    rem, g = C.c_double(), C.c_double()
    _check(lib().ds_phase_build(int(a.size), a.ctypes.data, float(chop_deg), q.ctypes.data,
                                c.ctypes.data, C.byref(rem), C.byref(g)))
    return q, c, rem.value, g.value


class Phase:
    """A tabulated phase function on the device (ds_phase_create)."""

    def __init__(self, ctx: Context, p, chop_deg=0.0):
        a = np.ascontiguousarray(np.asarray(p, np.float64).reshape(-1))
        h = C.c_void_p()
        _check(lib().ds_phase_create(ctx.h, int(a.size), a.ctypes.data, float(chop_deg),
                                     C.byref(h)))
        self.h = h
        rem, g = C.c_double(), C.c_double()
        _check(lib().ds_phase_info(h, C.byref(rem), C.byref(g)))
        self.removed, self.mean_cos = rem.value, g.value

    def close(self):
        if self.h is not None:
            _check(lib().ds_phase_destroy(self.h))
            self.h = None


class Lights:
    """A light set: m directional lights with irradiances (a discretised distant emitter)."""

    def __init__(self, ctx: Context, dirs, irradiance):
        self.ctx = ctx
        self.m = int(np.asarray(irradiance).size)
        self.h = ds_lights_create(ctx.h, dirs, irradiance)

    def close(self):
        if self.h is not None:
            ds_lights_destroy(self.h)
            self.h = None
