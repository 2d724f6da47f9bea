"""The learned part end to end, composed from the library's calls (Sec. 5).

  make_dataset   training pairs from several clouds (ds_make_records), interleaved
                 so that every contiguous minibatch mixes all clouds
  train          Adam on contiguous minibatches (ds_train_step), held-out loss
                 (ds_loss_grad), no host synchronisation inside an epoch
  judge          one view rendered with the network (ds_render_rpnn) and by
                 path tracing (ds_render_mc); relative L1 and RMSE of the network
                 image and of the direct-only image against the path-traced one,
                 and the time-to-unit-variance speedup; under a light set (a sun and
                 sky as directional lights) through ds_render_rpnn_lights and
                 ds_render_mc_lights

All arithmetic runs in libdeepscatter's kernels; this module allocates buffers,
slices them and reads scalars back.
"""
from __future__ import annotations

import math
import time

import numpy as np

import paper_1709_05418_amd as ds
from paper_1709_05418_amd import synth


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


def train(net, opt, z, t, steps, batch=1024, val_frac=0.25, eval_every=500, seed=0, log=None,
          lr=None, decay_at=(), decay=0.1):
    """Adam steps on contiguous minibatches of the first (1 - val_frac) rows; each
    pass over the data starts at a different offset.  With lr given, the learning
    rate is multiplied by `decay` at each fraction of the run listed in decay_at.
    Returns a dict with the per-step training losses and the held-out losses at each
    evaluation."""
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
    cuts = sorted(int(f * steps) for f in decay_at)
    for i in range(steps):
        if lr is not None and cuts and i == cuts[0]:
            cuts.pop(0)
            lr *= decay
            ds.ds_adam_set_lr(opt, lr)
        j = i % per_epoch
        if j == 0:  # each pass starts at a random offset within the leftover rows
            start = int(torch.randint(0, n_tr - per_epoch * batch + 1, (1,), generator=g).item())
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


def reference(ctx, cloud, params, light_dir, ray_o, ray_d, spp, seed, batch=256, log=None):
    """Path-traced image of spp samples per pixel, rendered in batches of independent
    streams (seed + 1 + b) whose means and variances are combined in FP64.  light_dir is
    one direction, or a ds.Lights set.  Returns (mean, variance of the mean)."""
    import torch
    mean = torch.zeros(ray_o.shape[0], dtype=torch.float64, device=ray_o.device)
    var = torch.zeros_like(mean)
    done = 0
    b = 0
    t0 = time.time()
    while done < spp:
        n = min(batch, spp - done)
        if isinstance(light_dir, ds.Lights):
            m, v = ds.ds_render_mc_lights(ctx.h, cloud.h, params, light_dir.h, ray_o, ray_d, n,
                                          seed + 1 + b)
        else:
            m, v = ds.ds_render_mc(ctx.h, cloud.h, params, light_dir, ray_o, ray_d, n,
                                   seed + 1 + b)
        w = n / (done + n)
        mean = mean * (1 - w) + m * w
        var = var * (1 - w) ** 2 + v * w * w
        done += n
        b += 1
        if log:
            torch.cuda.synchronize()
            log(f"reference: {done}/{spp} samples per pixel ({time.time() - t0:.1f}s)")
    return mean, var


def judge(ctx, cloud, net, precisions, params, light_dir, ray_o, ray_d, spp, ref_spp, seed,
          fallback_spp=0, log=None, draws=8, ls_target=False):
    """Network images (one per (name, precision)) and the direct-only image, each against
    one path-traced reference rendered once.  light_dir is one direction, or a ds.Lights
    set (then `draws` members are drawn per camera sample, Sec. 4.4).  Also the time to
    unit variance (render time times mean pixel variance, Sec. 6) of both renderers and
    its ratio, the speedup over path tracing.  With ls_target the network predicts all
    in-scattered radiance (Sec. 7's ablation): its image is albedo * E * g without the
    renderer's direct term, i.e. the rendered mean minus the mean direct term (the
    variance and TTUV then still describe the image with the direct term)."""
    import torch
    renders = {}
    for name, prec in precisions:
        torch.cuda.synchronize()
        t0 = time.time()
        if isinstance(light_dir, ds.Lights):
            img, var, direct, nfb = ds.ds_render_rpnn_lights(
                ctx.h, cloud.h, net.h, prec, params, light_dir.h, draws, ray_o, ray_d, spp, seed,
                fallback_spp, count_fallback=True)
        else:
            img, var, direct, nfb = ds.ds_render_rpnn(ctx.h, cloud.h, net.h, prec, params,
                                                      light_dir, ray_o, ray_d, spp, seed,
                                                      fallback_spp, count_fallback=True)
        torch.cuda.synchronize()
        renders[name] = (img, var, direct, nfb, time.time() - t0)
    t0 = time.time()
    ref, ref_var = reference(ctx, cloud, params, light_dir, ray_o, ray_d, ref_spp, seed, log=log)
    torch.cuda.synchronize()
    t_ref = time.time() - t0
    noise = float(math.sqrt(float(ref_var.sum())) / max(float(ref.sum()), 1e-300))
    ttuv_ref = t_ref * float(ref_var.mean())
    out = {}
    for name, (img, var, direct, nfb, t_net) in renders.items():
        if ls_target:
            img = img - direct
        l1, rmse = image_errors(img, ref)
        l1d, rmsed = image_errors(direct, ref)
        ttuv = t_net * float(var.mean())
        # brightness bias of the network image: its sum over the reference's sum
        ratio = float(img.double().sum() / ref.sum().clamp_min(1e-300))
        out[name] = {"rel_l1": l1, "rmse": rmse, "mean_ratio": ratio,
                     "rel_l1_direct_only": l1d,
                     "rmse_direct_only": rmsed, "ref_noise_rel": noise, "fallback_samples": nfb,
                     "seconds_network": t_net, "seconds_reference": t_ref,
                     "ttuv_network": ttuv, "ttuv_reference": ttuv_ref,
                     "ttuv_speedup": ttuv_ref / max(ttuv, 1e-300)}
    return out


def quantize_on(ctx, net, cloud, n=65536, seed=77):
    """FP8 form of net, calibrated on records sampled in cloud (the training
    distribution of shading configurations)."""
    pos, view, light, _ = ds.ds_sample_records(ctx.h, cloud.h, n, seed, want_attempts=False)
    ds.ds_net_quantize(ctx.h, net.h, cloud.h, ds.DS_PREC_FP8, pos, view, light)


JUDGE_KEYS = ("rel_l1", "rmse", "mean_ratio", "rel_l1_direct_only", "rmse_direct_only", "ref_noise_rel",
              "seconds_network", "seconds_reference", "fallback_samples", "ttuv_network",
              "ttuv_reference", "ttuv_speedup")


def judge_sun_sky(args, ctx, cloud, net, prm, precs, log, kind="sunsky"):
    """The crop judged under a distant emitter given as a set of directional lights (Fig. 7):
    a synthetic sun and sky (kind "sunsky") or a synthetic HDR environment map with an
    extended bright lobe (kind "envmap", one light per texel).  The network renderer draws
    args.draws members per camera sample, the path tracer one member per next-event
    estimate.  Returns summary entries prefixed with kind."""
    import torch
    sun = synth.table1_lights()["side"]
    if kind == "envmap":
        dirs, E = synth.envmap_lights(synth.synthetic_envmap(sun))
    else:
        dirs, E = synth.sun_sky_lights(sun)
    lights = ds.Lights(ctx, dirs, E)
    label = "sun-sky" if kind == "sunsky" else "env-map"
    out = {f"{kind}_lights": int(E.size), f"{kind}_draws": args.draws,
           f"{kind}_crop": args.sky_crop, f"{kind}_ref_spp": args.sky_ref_spp}
    try:
        o, dd = camera(args.width, args.height, seed=1)
        for name, prec in precs:
            torch.cuda.synchronize()
            tf = time.time()
            ds.ds_render_rpnn_lights(ctx.h, cloud.h, net.h, prec, prm, lights.h, args.draws, o,
                                     dd, args.frame_spp, 5, args.fallback_spp, want_var=False,
                                     want_direct=False)
            torch.cuda.synchronize()
            out[f"{kind}_frame_ms_{name}"] = (time.time() - tf) * 1e3
            log(f"{label} {args.width}x{args.height} frame {name}, {args.frame_spp} spp x "
                f"{args.draws} lights: {out[f'{kind}_frame_ms_{name}']:.1f} ms")
        del o, dd
        c = args.sky_crop
        co, cd = camera(args.width, args.height,
                        crop=((args.width - c) // 2, (args.height - c) // 2, c, c), seed=3)
        js = judge(ctx, cloud, net, precs, prm, lights, co, cd, args.crop_spp, args.sky_ref_spp,
                   13, args.fallback_spp, log=log, draws=args.draws)
    finally:
        lights.close()
    for name, j in js.items():
        for k in JUDGE_KEYS:
            out[f"{kind}_{k}_{name}"] = j[k]
        log(f"{label} crop {c}^2 {name} ({E.size} lights, {args.draws} draws per sample): "
            f"rel L1 {j['rel_l1']:.4f} (direct only {j['rel_l1_direct_only']:.4f}), RMSE "
            f"{j['rmse']:.5f}; reference noise {j['ref_noise_rel']:.4f}; network "
            f"{j['seconds_network']:.2f}s vs reference {j['seconds_reference']:.2f}s; TTUV "
            f"speedup {j['ttuv_speedup']:.1f}x")
    return out


def judge_density(args, dev="cuda"):
    """The held-out judge scene: a seeded cloud."""
    import torch
    return synth.cloud_density(args.judge_n, args.seed + 5000, worley=0.3, device=dev,
                               dtype=torch.bfloat16)


def _close(args, ctx):
    """Free the phase tables of a run, then its context."""
    for ph in getattr(args, "phases", ()):
        if ph is not None:
            ph.close()
    ctx.close()


def camera(width, height, cam_pos=(0.0, 0.12, 2.3), look_at=(0.0, 0.0, 0.0), fov_deg=42.0,
           crop=None, seed=0, device="cuda"):
    """Jittered pinhole rays of a width x height view (fov over the larger side), as
    device tensors (origins, directions); crop = (x0, y0, w, h) keeps a window."""
    import numpy as np
    import torch
    rng = np.random.default_rng(seed)
    x0, y0, w, h = crop if crop else (0, 0, width, height)
    px, py = np.meshgrid(np.arange(x0, x0 + w), np.arange(y0, y0 + h))
    px, py = px.reshape(-1).astype(np.float64), py.reshape(-1).astype(np.float64)
    cam = np.asarray(cam_pos, np.float64)
    fwd = np.asarray(look_at, np.float64) - cam
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, [0.0, 1.0, 0.0])
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    t = math.tan(math.radians(fov_deg) / 2)
    s = max(width, height)
    u = ((px + rng.random(px.size)) / s * 2 - width / s) * t
    v = (height / s - (py + rng.random(py.size)) / s * 2) * t
    d = fwd[None] + u[:, None] * right[None] + v[:, None] * up[None]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.broadcast_to(cam, d.shape)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
    return T(o), T(d)


def main(argv=None):
    """Training pairs from procedural clouds, paper-width training, then a frame of
    a larger held-out cloud rendered with the network and judged against path
    tracing on a crop.  Prints progress and one JSON summary line."""
    import argparse
    import json
    import numpy as np
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--clouds", type=int, default=32)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--records", type=int, default=1 << 19, help="total training pairs")
    ap.add_argument("--spp", type=int, default=256, help="paths per training pair")
    ap.add_argument("--K", type=int, default=10)
    ap.add_argument("--W", type=int, default=200)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--decay-at", type=float, nargs="*", default=[0.6, 0.85],
                    help="fractions of the run at which the learning rate drops tenfold")
    ap.add_argument("--train-precision", default="bf16", choices=["bf16", "fp32"],
                    help="GEMM arithmetic of the training step (FP32 masters either way)")
    ap.add_argument("--judge-n", type=int, default=1024)
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    ap.add_argument("--crop", type=int, default=128)
    ap.add_argument("--frame-spp", type=int, default=4)
    ap.add_argument("--crop-spp", type=int, default=64)
    ap.add_argument("--ref-spp", type=int, default=512)
    ap.add_argument("--fallback-spp", type=int, default=64)
    ap.add_argument("--seed", type=int, default=1000)
    ap.add_argument("--sun-sky", action="store_true",
                    help="also judge a crop under a synthetic sun and sky light set")
    ap.add_argument("--envmap", action="store_true",
                    help="also judge a crop under a synthetic HDR environment map (32 x 64 "
                         "texels, one directional light each)")
    ap.add_argument("--draws", type=int, default=8, help="light-set members per camera sample")
    ap.add_argument("--sky-crop", type=int, default=128)
    ap.add_argument("--sky-ref-spp", type=int, default=1024)
    ap.add_argument("--light", default="side", choices=["side", "front", "back"],
                    help="the judge's directional light (Table 1's set-ups)")
    ap.add_argument("--target", default="li", choices=["li", "ls"],
                    help="train on L_i (indirect, Sec. 4) or on all in-scattered radiance L_s "
                         "(the ablation of Sec. 7); an L_s network replaces the direct term")
    ap.add_argument("--adaptive-rel", type=float, default=0.0,
                    help="> 0: estimate each target progressively until its mean lies within "
                         "+- this fraction at 95 %% confidence (Sec. 5.1), instead of --spp paths")
    ap.add_argument("--adaptive-batch", type=int, default=256)
    ap.add_argument("--adaptive-max", type=int, default=65536)
    ap.add_argument("--phase", default="hg", choices=["hg", "lm"],
                    help="Henyey-Greenstein g = 0.85, or a tabulated Lorenz-Mie function of "
                         "cloud droplets, chopped (the tracer thins the medium, Sec. 3.1) for "
                         "data and rendering and unchopped for the first collision's direct "
                         "term (Sec. 3.1, Sec. 5.1)")
    ap.add_argument("--chop-deg", type=float, default=5.0)
    ap.add_argument("--no-judge", action="store_true", help="stop after training")
    ap.add_argument("--compare-stencils", action="store_true",
                    help="train and judge the RPNN on the 5x5x9, 3x3x5 and 2x2x3 stencils "
                         "(Fig. 10, right) instead of the single network")
    ap.add_argument("--compare", action="store_true",
                    help="train the RPNN and the two all-at-once MLPs of Sec. 7 (23 x 200 and "
                         "[400, 400, 200, 200, 200]) on the same pairs and judge each in FP32")
    ap.add_argument("--phase-study", action="store_true",
                    help="no network: path-trace the judge crop, front- and back-lit, under "
                         "isotropic, HG, full, chopped and chopped-after-first-bounce Lorenz-Mie "
                         "phase functions; equal-time variance and image change (Fig. 3)")
    ap.add_argument("--save-theta", default=None)
    ap.add_argument("--load-theta", default=None,
                    help="judge a network saved by --save-theta instead of training one")
    args = ap.parse_args(argv)
    log = lambda *a: print("[learn]", *a, flush=True)
    dev = "cuda"
    ctx = ds.Context(0)
    albedo, phases = 0.999, (None, None)
    if args.phase == "lm":
        _, p_lm, g_lm = synth.cloud_droplet_phase()
        phases = (ds.Phase(ctx, p_lm, args.chop_deg), ds.Phase(ctx, p_lm))
        f = phases[0].removed
        log(f"Lorenz-Mie phase: mean cosine {g_lm:.4f}; chopped at {args.chop_deg} deg, "
            f"{100 * f:.1f} % of the scattering removed (the tracer thins the medium: extinction "
            f"x{1.0 - albedo * f:.4f}, albedo {albedo * (1.0 - f) / (1.0 - albedo * f):.5f}), "
            f"chopped mean cosine {phases[0].mean_cos:.4f}")
    args.sigma = lambda n: float(n)
    prm = ds.TracerParams(albedo, 0.85, 1.0, ds.DS_LIGHT_DIRECTIONAL, 0, phase=phases[0],
                          phase_first=phases[1])
    args.phases = phases
    K, W = args.K, args.W
    L = int(math.ceil(math.log2(args.n))) + 1
    per = args.records // args.clouds
    if args.phase_study:
        return phase_study(args, ctx, log)
    if args.load_theta:
        net = ds.Net(ctx, K, W, 3)
        net.set_params(np.load(args.load_theta))
        log(f"network loaded from {args.load_theta}")
        return judge_only(args, ctx, net, prm, log)
    D = ds.STENCIL_N * K + 1
    z = torch.empty((per * args.clouds, D), dtype=torch.float32, device=dev)
    t = torch.empty(per * args.clouds, dtype=torch.float32, device=dev)
    rec_prm = ds.TracerParams(albedo, 0.85, 1.0, ds.DS_LIGHT_DIRECTIONAL, 0,
                              include_direct=int(args.target == "ls"), phase=phases[0])
    ad = (ds.Adaptive(args.adaptive_batch, args.adaptive_max, args.adaptive_rel, 1.96)
          if args.adaptive_rel > 0 else None)
    used = []
    t0 = time.time()
    for c in range(args.clouds):
        d = synth.cloud_density(args.n, args.seed + c, worley=0.3, device=dev)
        amin, h0 = synth.unit_box(args.n)
        cl = ds.Cloud(ctx, d, args.sigma(args.n), amin, h0, L, K)
        _, li_out = ds.ds_make_records(ctx.h, cl.h, rec_prm, per, ad or args.spp,
                                       args.seed + 7919 * c, z, t, offset=c, stride=args.clouds,
                                       want_li=ad is not None)
        torch.cuda.synchronize()
        if ad is not None:
            used.append(li_out[2].cpu())
        cl.close()
        del d
        log(f"cloud {c + 1}/{args.clouds}: {per} pairs x "
            f"{'progressive' if ad else args.spp} paths ({time.time() - t0:.1f}s)")
    t_data = time.time() - t0
    stats = {}
    if ad is not None:
        n_used = torch.cat(used).double()
        paths = float(n_used.sum())
        stats = {"adaptive_rel": args.adaptive_rel, "adaptive_batch": args.adaptive_batch,
                 "adaptive_max": args.adaptive_max, "paths_mean": float(n_used.mean()),
                 "paths_median": float(n_used.median()),
                 "at_cap_fraction": float((n_used >= args.adaptive_max).double().mean())}
        log(f"progressive targets: +-{100 * args.adaptive_rel:g} % at 95 %: mean "
            f"{stats['paths_mean']:.0f} paths per pair (median {stats['paths_median']:.0f}), "
            f"{100 * stats['at_cap_fraction']:.1f} % at the cap of {args.adaptive_max}")
    else:
        paths = per * args.clouds * args.spp
    li = torch.expm1(t)
    log(f"data: {z.shape[0]} pairs, {paths:.3e} paths in {t_data:.1f}s "
        f"({paths / t_data:.3e} paths/s); mean {'L_s' if args.target == 'ls' else 'L_i'} "
        f"{float(li.mean()):.4f}")
    if args.steps == 0:   # training data only
        print(json.dumps({"target": args.target, "clouds": args.clouds, "n": args.n,
                          "pairs": per * args.clouds, "spp": args.spp, "data_seconds": t_data,
                          "paths_per_second": paths / t_data, **stats}), flush=True)
        _close(args, ctx)
        return
    if args.compare_stencils:
        return compare_stencils(args, ctx, prm, z, t, float(li.mean()), log,
                                {"data_seconds": t_data, "paths_per_second": paths / t_data,
                                 "pairs": per * args.clouds, "spp": args.spp, **stats})
    if args.compare:
        return compare_architectures(args, ctx, prm, z, t, float(li.mean()), log,
                                     {"data_seconds": t_data, "paths_per_second": paths / t_data,
                                      "pairs": per * args.clouds, "spp": args.spp, **stats})
    net = ds.Net(ctx, K, W, 3)
    net.set_params(synth.init_params(K, W, 3, args.seed + 1, branch_scale=1 / math.sqrt(K),
                                     out_scale=0.01, out_bias=float(li.mean())))
    ds.ds_net_set_train_precision(net.h, ds.DS_PREC_BF16 if args.train_precision == "bf16"
                                  else ds.DS_PREC_F32)
    opt = ds.ds_adam_create(net.h, args.lr)
    res = train(net, opt, z, t, args.steps, args.batch, 0.25, eval_every=max(1, args.steps // 10),
                log=log, lr=args.lr, decay_at=tuple(args.decay_at))
    log(f"training {res['seconds']:.1f}s ({args.steps / res['seconds']:.1f} steps/s)")
    if args.save_theta:
        np.save(args.save_theta, net.get_params())
    del z, t
    torch.cuda.empty_cache()
    base = {"target": args.target, "train_precision": args.train_precision,
            "clouds": args.clouds, "n": args.n, "pairs": per * args.clouds, "spp": args.spp,
            "K": K, "W": W, "steps": args.steps, "batch": args.batch, "data_seconds": t_data,
            "paths_per_second": paths / t_data, "train_seconds": res["seconds"],
            "held_out": res["held_out"], **stats}
    if args.no_judge:
        print(json.dumps(base), flush=True)
        ds.ds_adam_destroy(opt)
        net.close()
        _close(args, ctx)
        return
    # held-out cloud, larger grid, same optical size in mean free paths per unit
    d = judge_density(args, dev)
    amin, h0 = synth.unit_box(args.judge_n)
    Lj = min(16, int(math.ceil(math.log2(args.judge_n))) + 1)
    jc = ds.Cloud(ctx, d, args.sigma(args.n), amin, h0, Lj, K)
    del d
    log(f"judge cloud {args.judge_n}^3 built ({time.time() - t0:.1f}s)")
    light = synth.table1_lights()[args.light]
    o, dd = camera(args.width, args.height, seed=1)
    summary = {}
    quantize_on(ctx, net, jc)
    precs = (("bf16", ds.DS_PREC_BF16), ("fp8", ds.DS_PREC_FP8), ("fp32", ds.DS_PREC_F32))
    for name, prec in precs:
        torch.cuda.synchronize()
        tf = time.time()
        img, _, direct, nfb = ds.ds_render_rpnn(ctx.h, jc.h, net.h, prec, prm, light, o, dd,
                                                args.frame_spp, 5, args.fallback_spp,
                                                count_fallback=True)
        torch.cuda.synchronize()
        summary[f"frame_ms_{name}"] = (time.time() - tf) * 1e3
        summary[f"frame_fallback_samples_{name}"] = nfb
        log(f"{args.width}x{args.height} frame {name}, {args.frame_spp} spp: "
            f"{summary[f'frame_ms_{name}']:.1f} ms, fallback samples {nfb}")
    cx0 = (args.width - args.crop) // 2
    cy0 = (args.height - args.crop) // 2
    co, cd = camera(args.width, args.height, crop=(cx0, cy0, args.crop, args.crop), seed=2)
    js = judge(ctx, jc, net, precs, prm, light, co, cd, args.crop_spp, args.ref_spp, 11,
               args.fallback_spp, log=log, ls_target=args.target == "ls")
    for name, j in js.items():
        for k in JUDGE_KEYS:
            summary[f"crop_{k}_{name}"] = j[k]
        log(f"crop {args.crop}^2 {name}: rel L1 {j['rel_l1']:.4f}, mean ratio "
            f"{j['mean_ratio']:.3f} (direct only "
            f"{j['rel_l1_direct_only']:.4f}), RMSE {j['rmse']:.5f}; reference noise "
            f"{j['ref_noise_rel']:.4f}; network {j['seconds_network']:.2f}s vs reference "
            f"{j['seconds_reference']:.2f}s; TTUV speedup {j['ttuv_speedup']:.0f}x")
    if args.sun_sky and args.target == "li":
        summary.update(judge_sun_sky(args, ctx, jc, net, prm, precs, log))
    if args.envmap and args.target == "li":
        summary.update(judge_sun_sky(args, ctx, jc, net, prm, precs, log, kind="envmap"))
    summary.update(base)
    summary.update({"judge_n": args.judge_n, "frame": [args.width, args.height],
                    "crop": args.crop, "crop_spp": args.crop_spp, "ref_spp": args.ref_spp,
                    "light": args.light, "phase": args.phase})
    print(json.dumps(summary), flush=True)
    ds.ds_adam_destroy(opt)
    net.close()
    jc.close()
    _close(args, ctx)


ARCHS = {"rpnn": None, "mlp_deep_23x200": [200] * 22 + [1],
         "mlp_wide_400_400_200_200_200": [400, 400, 200, 200, 200, 1]}


STENCILS = {"5x5x9": (5, 5, 9), "3x3x5": (3, 3, 5), "2x2x3": (2, 2, 3)}


def stencil_points(shape):
    """Indices n = ix + 5 iy + 25 iz into the 5 x 5 x 9 lattice (Sec. 4.2) of a coarser
    stencil of the same extent, [-1, 1]^2 x [-1, 3] mean free paths: nx x ny x nz points
    with spacings 4 / (nx - 1), 4 / (ny - 1) and 8 / (nz - 1) lattice steps."""
    nx, ny, nz = shape
    if (4 % (nx - 1)) or (4 % (ny - 1)) or (8 % (nz - 1)):
        raise ValueError(f"{shape} is not a sub-lattice of 5 x 5 x 9")
    sx, sy, sz = 4 // (nx - 1), 4 // (ny - 1), 8 // (nz - 1)
    return np.array([ix + 5 * iy + 25 * iz for iz in range(0, 9, sz)
                     for iy in range(0, 5, sy) for ix in range(0, 5, sx)])


def stencil_params(K, W, seed, keep, mean_li):
    """RPNN parameters for a coarser stencil on the 5 x 5 x 9 layout: the V columns of the
    dropped points are zero, the kept ones He-uniform for the kept fan-in.  Trained on
    descriptors whose dropped entries are zero, those weights get zero gradients and Adam
    leaves them at zero, so the network is the RPNN of the coarser stencil."""
    theta = synth.init_params(K, W, 3, seed, branch_scale=1 / math.sqrt(K), out_scale=0.01,
                              out_bias=mean_li)
    if len(keep) == ds.STENCIL_N:
        return theta
    drop = np.setdiff1d(np.arange(ds.STENCIL_N), keep)
    for V in stencil_blocks(theta, K, W):
        V[:, :ds.STENCIL_N] *= math.sqrt(V.shape[1] / (len(keep) + 1))
        V[:, drop] = 0.0
    return theta


def stencil_blocks(theta, K, W):
    """Views of the K input matrices V^k [W][226] inside a parameter vector."""
    off, out = 0, []
    for name, r, c in synth.layer_shapes(K, W, 3):
        n = r * (c if c else 1)
        if name.startswith("V"):
            out.append(theta[off:off + n].reshape(r, c))
        off += n
    return out


def compare_stencils(args, ctx, prm, z, t, mean_li, log, data):
    """Sec. 7, Fig. 10 (right): the RPNN on stencils of different resolution over the same
    extent, trained on the same pairs with the same minibatches and schedule, then judged
    on the same crop.  The coarser stencils are sub-lattices of 5 x 5 x 9: their descriptors
    are the full one with the other entries set to zero."""
    import torch
    K, W = args.K, args.W
    out = dict(data)
    held, nets = {}, {}
    for name, shape in STENCILS.items():
        keep = stencil_points(shape)
        zs = z
        if len(keep) < ds.STENCIL_N:
            drop = torch.from_numpy(np.setdiff1d(np.arange(ds.STENCIL_N), keep)).to(z.device)
            cols = (drop[None, :] + ds.STENCIL_N * torch.arange(K, device=z.device)[:, None])
            zs = z.clone()
            zs[:, cols.reshape(-1)] = 0.0
        net = ds.Net(ctx, K, W, 3)
        net.set_params(stencil_params(K, W, args.seed + 1, keep, mean_li))
        ds.ds_net_set_train_precision(net.h, ds.DS_PREC_BF16 if args.train_precision == "bf16"
                                      else ds.DS_PREC_F32)
        opt = ds.ds_adam_create(net.h, args.lr)
        log(f"stencil {name}: {len(keep)} points per level")
        res = train(net, opt, zs, t, args.steps, args.batch, 0.25,
                    eval_every=max(1, args.steps // 20), log=log, lr=args.lr,
                    decay_at=tuple(args.decay_at))
        ds.ds_adam_destroy(opt)
        del zs
        # the weights of the dropped points must still be exactly zero
        dead = np.setdiff1d(np.arange(ds.STENCIL_N), keep)
        out[f"{name}_dropped_weights_max_abs"] = float(max(
            [float(np.abs(V[:, dead]).max()) for V in stencil_blocks(net.get_params(), K, W)]
            if dead.size else [0.0]))
        held[name] = res["held_out"]
        out[f"{name}_points"] = int(len(keep))
        out[f"{name}_held_out_final"] = res["held_out"][-1][1]
        log(f"{name}: training {res['seconds']:.1f}s, final held-out {res['held_out'][-1][1]:.6f}")
        nets[name] = net
    _compare_judge(args, ctx, prm, nets, held, out, log, z, t)


def compare_architectures(args, ctx, prm, z, t, mean_li, log, data):
    """Sec. 7, Fig. 10: the progressive RPNN against two MLPs fed the whole descriptor at
    once, trained on the same pairs with the same minibatches, learning-rate schedule and
    step count, then judged on the same crop (all in FP32 for the judge, the plain form)."""
    import json
    import torch
    K, W = args.K, args.W
    out = dict(data)
    held = {}
    nets = {}
    for name, widths in ARCHS.items():
        if widths is None:
            net = ds.Net(ctx, K, W, 3)
            net.set_params(synth.init_params(K, W, 3, args.seed + 1, branch_scale=1 / math.sqrt(K),
                                             out_scale=0.01, out_bias=mean_li))
        else:
            net = ds.NetMLP(ctx, K, widths)
            net.set_params(synth.init_mlp([ds.STENCIL_N * K + 1] + widths, args.seed + 1,
                                          out_scale=0.01, out_bias=mean_li))
        ds.ds_net_set_train_precision(net.h, ds.DS_PREC_BF16 if args.train_precision == "bf16"
                                      else ds.DS_PREC_F32)
        opt = ds.ds_adam_create(net.h, args.lr)
        log(f"{name}: {net.n_params} parameters")
        res = train(net, opt, z, t, args.steps, args.batch, 0.25,
                    eval_every=max(1, args.steps // 20), log=log, lr=args.lr,
                    decay_at=tuple(args.decay_at))
        ds.ds_adam_destroy(opt)
        held[name] = res["held_out"]
        out[f"{name}_params"] = net.n_params
        out[f"{name}_train_seconds"] = res["seconds"]
        out[f"{name}_held_out_final"] = res["held_out"][-1][1]
        log(f"{name}: training {res['seconds']:.1f}s, final held-out {res['held_out'][-1][1]:.6f}")
        nets[name] = net
    _compare_judge(args, ctx, prm, nets, held, out, log, z, t)


def _compare_judge(args, ctx, prm, nets, held, out, log, z, t):
    """The judge of the comparisons: every network renders the same crop in FP32 (the plain
    form) against one path-traced reference; one JSON line with the held-out curves."""
    import json
    import torch
    K, W = args.K, args.W
    del z, t
    torch.cuda.empty_cache()
    if not args.no_judge:
        d = judge_density(args)
        amin, h0 = synth.unit_box(args.judge_n)
        Lj = min(16, int(math.ceil(math.log2(args.judge_n))) + 1)
        jc = ds.Cloud(ctx, d, args.sigma(args.n), amin, h0, Lj, K)
        del d
        light = synth.table1_lights()[args.light]
        c = args.crop
        co, cd = camera(args.width, args.height,
                        crop=((args.width - c) // 2, (args.height - c) // 2, c, c), seed=2)
        ref, _ = reference(ctx, jc, prm, light, co, cd, args.ref_spp, 11)
        for name, net in nets.items():
            img, _, direct, _ = ds.ds_render_rpnn(ctx.h, jc.h, net.h, ds.DS_PREC_F32, prm, light,
                                                  co, cd, args.crop_spp, 11, args.fallback_spp)
            l1, rmse = image_errors(img, ref)
            out[f"{name}_crop_rel_l1"] = l1
            out[f"{name}_crop_rmse"] = rmse
            log(f"{name}: crop {c}^2 rel L1 {l1:.4f}, RMSE {rmse:.5f}")
        jc.close()
    for name, net in nets.items():
        log(f"{name} held-out curve: " + ", ".join(f"({a}, {b:.3g})" for a, b in held[name]))
        net.close()
    out.update({"steps": args.steps, "batch": args.batch, "K": K, "W": W,
                "light": args.light, "crop": args.crop, "ref_spp": args.ref_spp,
                "judge_n": args.judge_n, "held_out": held})
    print(json.dumps(out), flush=True)
    _close(args, ctx)


def phase_study(args, ctx, log):
    """Fig. 3: the path tracer under five phase-function set-ups on the centred crop of the
    judge scene, front- and back-lit, each at --ref-spp samples per pixel: isotropic,
    Henyey-Greenstein (g 0.857), the full Lorenz-Mie function, the chopped one (thinner
    medium, chopped everywhere) and the chopped one with the full function
    for the first collision's direct term.  Reports time, mean pixel, the equal-time
    variance (render time x mean pixel variance of the mean, relative to the isotropic
    set-up) and the relative L1 against the full Lorenz-Mie image."""
    import json
    import torch
    albedo = 0.999
    _, p_lm, g_lm = synth.cloud_droplet_phase()
    full, chop = ds.Phase(ctx, p_lm), ds.Phase(ctx, p_lm, args.chop_deg)
    f = chop.removed
    d = judge_density(args)
    amin, h0 = synth.unit_box(args.judge_n)
    Lj = min(16, int(math.ceil(math.log2(args.judge_n))) + 1)
    cl = ds.Cloud(ctx, d, float(args.n), amin, h0, Lj, args.K)
    del d
    # with the chopped table the tracer traces the thinner medium itself
    setups = [("isotropic", ds.TracerParams(albedo, 0.0, 1.0)),
              ("hg_0.857", ds.TracerParams(albedo, 0.857, 1.0)),
              ("lm", ds.TracerParams(albedo, 0.0, 1.0, phase=full, phase_first=full)),
              ("lm_chopped", ds.TracerParams(albedo, 0.0, 1.0, phase=chop, phase_first=chop)),
              ("lm_chopped_full_first", ds.TracerParams(albedo, 0.0, 1.0, phase=chop,
                                                        phase_first=full))]
    c = args.crop
    co, cd = camera(args.width, args.height,
                    crop=((args.width - c) // 2, (args.height - c) // 2, c, c), seed=2)
    out = {"judge_n": args.judge_n, "crop": c, "spp": args.ref_spp, "albedo": albedo,
           "lm_mean_cos": g_lm, "chop_deg": args.chop_deg, "chop_removed": f}
    log(f"Lorenz-Mie mean cosine {g_lm:.4f}; chop at {args.chop_deg} deg removes {100 * f:.1f} %")
    try:
        for lname in ("front", "back"):
            light = synth.table1_lights()[lname]
            imgs, ttuv = {}, {}
            for name, prm in setups:
                torch.cuda.synchronize()
                t0 = time.time()
                m, v = reference(ctx, cl, prm, light, co, cd, args.ref_spp, 11)
                torch.cuda.synchronize()
                sec = time.time() - t0
                imgs[name] = m
                ttuv[name] = sec * float(v.mean())
                out[f"{lname}_{name}_seconds"] = sec
                out[f"{lname}_{name}_mean"] = float(m.mean())
            for name in imgs:
                rel = ttuv[name] / ttuv["isotropic"]
                l1, _ = image_errors(imgs[name], imgs["lm"])
                out[f"{lname}_{name}_equal_time_variance_rel"] = rel
                out[f"{lname}_{name}_rel_l1_vs_lm"] = l1
                log(f"{lname}-lit {name}: {out[f'{lname}_{name}_seconds']:.2f}s, mean pixel "
                    f"{out[f'{lname}_{name}_mean']:.5f}, equal-time variance x{rel:.1f} of "
                    f"isotropic, rel L1 against full LM {l1:.4f}")
    finally:
        cl.close()
        full.close()
        chop.close()
    print(json.dumps(out), flush=True)
    _close(args, ctx)


def judge_only(args, ctx, net, prm, log):
    """The judge part of main() for a given network: a full frame and the crop."""
    import json
    import torch
    K = net.K
    t0 = time.time()
    d = judge_density(args)
    amin, h0 = synth.unit_box(args.judge_n)
    Lj = min(16, int(math.ceil(math.log2(args.judge_n))) + 1)
    jc = ds.Cloud(ctx, d, args.sigma(args.n), amin, h0, Lj, K)
    del d
    log(f"judge cloud {args.judge_n}^3 built ({time.time() - t0:.1f}s)")
    light = synth.table1_lights()[args.light]
    o, dd = camera(args.width, args.height, seed=1)
    summary = {}
    quantize_on(ctx, net, jc)
    precs = (("bf16", ds.DS_PREC_BF16), ("fp8", ds.DS_PREC_FP8))
    for name, prec in precs:
        torch.cuda.synchronize()
        tf = time.time()
        img, _, direct, nfb = ds.ds_render_rpnn(ctx.h, jc.h, net.h, prec, prm, light, o, dd,
                                                args.frame_spp, 5, args.fallback_spp,
                                                count_fallback=True)
        torch.cuda.synchronize()
        summary[f"frame_ms_{name}"] = (time.time() - tf) * 1e3
        log(f"{args.width}x{args.height} frame {name}, {args.frame_spp} spp: "
            f"{summary[f'frame_ms_{name}']:.1f} ms, fallback samples {nfb}")
    cx0 = (args.width - args.crop) // 2
    cy0 = (args.height - args.crop) // 2
    js = {}
    if args.crop > 0:   # --crop 0 judges the frame and the light-set crop only
        co, cd = camera(args.width, args.height, crop=(cx0, cy0, args.crop, args.crop), seed=2)
        js = judge(ctx, jc, net, precs, prm, light, co, cd, args.crop_spp, args.ref_spp, 11,
                   args.fallback_spp, log=log)
    for name, j in js.items():
        for k in JUDGE_KEYS:
            summary[f"crop_{k}_{name}"] = j[k]
        log(f"crop {args.crop}^2 {name}: rel L1 {j['rel_l1']:.4f}, mean ratio "
            f"{j['mean_ratio']:.3f} (direct only "
            f"{j['rel_l1_direct_only']:.4f}), RMSE {j['rmse']:.5f}; reference noise "
            f"{j['ref_noise_rel']:.4f}; network {j['seconds_network']:.2f}s vs reference "
            f"{j['seconds_reference']:.2f}s ({args.ref_spp} spp); TTUV speedup "
            f"{j['ttuv_speedup']:.0f}x")
    if args.sun_sky:
        summary.update(judge_sun_sky(args, ctx, jc, net, prm, precs, log))
    if args.envmap:
        summary.update(judge_sun_sky(args, ctx, jc, net, prm, precs, log, kind="envmap"))
    summary.update({"judge_n": args.judge_n, "frame": [args.width, args.height],
                    "crop": args.crop, "crop_spp": args.crop_spp, "ref_spp": args.ref_spp,
                    "theta": args.load_theta})
    print(json.dumps(summary), flush=True)
    net.close()
    jc.close()
    _close(args, ctx)


if __name__ == "__main__":
    main()
