"""The learned part end to end, composed from the library's calls (Sec. 5).

  make_dataset   training pairs from several clouds (ds_make_records), interleaved
                 so that every contiguous minibatch mixes all clouds
  train          Adam on contiguous minibatches (ds_train_step), held-out loss
                 (ds_loss_grad), no host synchronisation inside an epoch
  judge          one view rendered with the network (ds_render_rpnn) and by
                 path tracing (ds_render_mc); relative L1 and RMSE of the network
                 image and of the direct-only image against the path-traced one

All arithmetic runs in libdeepscatter's kernels; this module allocates buffers,
slices them and reads scalars back.
"""
from __future__ import annotations

import math
import time

import paper_1709_05418_amd as ds


def make_dataset(ctx, clouds, n_per_cloud, spp, seed, params=None, device="cuda"):
    """Interleaved training pairs: record i of cloud c lands in row i * C + c.
    Returns (z, target) device tensors of C * n_per_cloud rows."""
    import torch
    params = params or ds.TracerParams()
    C = len(clouds)
    K = clouds[0].K
    D = ds.STENCIL_N * K + 1
    M = C * n_per_cloud
    z = torch.empty((M, D), dtype=torch.float32, device=device)
    t = torch.empty(M, dtype=torch.float32, device=device)
    for c, cl in enumerate(clouds):
        if cl.K != K:
            raise ValueError("all clouds need the same number of stencil levels")
        ds.ds_make_records(ctx.h, cl.h, params, n_per_cloud, spp, seed + 7919 * c, z, t,
                           offset=c, stride=C)
    return z, t


def train(net, opt, z, t, steps, batch=1024, val_frac=0.25, eval_every=500, seed=0, log=None):
    """Adam steps on contiguous minibatches of the first (1 - val_frac) rows; each
    pass over the data starts at a different offset.  Returns a dict with the
    per-step training losses and the held-out losses at each evaluation."""
    import torch
    M = z.shape[0]
    n_val = int(M * val_frac)
    n_tr = M - n_val
    if n_tr < batch:
        raise ValueError("not enough training rows for one minibatch")
    zt, tt = z[:n_tr], t[:n_tr]
    zv, tv = z[n_tr:], t[n_tr:]
    losses = torch.zeros(steps, dtype=torch.float32, device=z.device)
    val = []
    per_epoch = n_tr // batch
    g = torch.Generator().manual_seed(seed)
    start = 0

    def held_out():
        if n_val == 0:
            return None
        tot = 0.0
        for a in range(0, n_val, 65536):
            b = min(n_val, a + 65536)
            lo, _ = ds.ds_loss_grad(net.h, zv[a:b], tv[a:b], net.n_params, want_grad=False)
            tot += float(lo.item()) * (b - a)
        return tot / n_val

    t0 = time.time()
    v0 = held_out()
    val.append((0, v0))
    for i in range(steps):
        j = i % per_epoch
        if j == 0:
            start = int(torch.randint(0, batch, (1,), generator=g).item()) \
                if n_tr - per_epoch * batch >= batch else 0
        a = start + j * batch
        ds.ds_train_step(net.h, opt, zt[a:a + batch], tt[a:a + batch], loss=losses[i:i + 1])
        if eval_every and (i + 1) % eval_every == 0:
            v = held_out()
            val.append((i + 1, v))
            if log:
                log(f"step {i + 1}: train {float(losses[max(0, i - 99):i + 1].mean()):.4f} "
                    f"held-out {v:.4f} ({time.time() - t0:.1f}s)")
    torch.cuda.synchronize()
    return {"train": losses.cpu().numpy(), "held_out": val, "seconds": time.time() - t0}


def image_errors(img, ref):
    """Relative L1 (sum |I - R| / sum R) and RMSE of img against ref."""
    import torch
    img = img.double()
    ref = ref.double()
    l1 = float((img - ref).abs().sum() / ref.abs().sum().clamp_min(1e-300))
    rmse = float(torch.sqrt(((img - ref) ** 2).mean()))
    return l1, rmse


def judge(ctx, cloud, net, precision, params, light_dir, ray_o, ray_d, spp, ref_spp, seed,
          fallback_spp=0):
    """Network image vs path-traced reference, and the direct-only image vs the same."""
    t0 = time.time()
    img, var, direct, nfb = ds.ds_render_rpnn(ctx.h, cloud.h, net.h, precision, params, light_dir,
                                              ray_o, ray_d, spp, seed, fallback_spp,
                                              count_fallback=True)
    import torch
    torch.cuda.synchronize()
    t_net = time.time() - t0
    t0 = time.time()
    ref, ref_var = ds.ds_render_mc(ctx.h, cloud.h, params, light_dir, ray_o, ray_d, ref_spp,
                                   seed + 1)
    torch.cuda.synchronize()
    t_ref = time.time() - t0
    l1, rmse = image_errors(img, ref)
    l1d, rmsed = image_errors(direct, ref)
    return {"rel_l1": l1, "rmse": rmse, "rel_l1_direct_only": l1d, "rmse_direct_only": rmsed,
            "ref_noise_rel": float(math.sqrt(float(ref_var.sum())) / max(float(ref.sum()), 1e-300)),
            "fallback_samples": nfb, "seconds_network": t_net, "seconds_reference": t_ref,
            "image": img, "reference": ref, "direct": direct}
