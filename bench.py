#!/usr/bin/env python3
"""Throughput of the radiance-prediction hot path on one MI355X.

One step = one prediction over the whole batch of shading points: the
hierarchical stencil gather from the mip pyramid plus the residual network, in
the fused BF16 kernel (the headline), replayed from a captured graph of the
autotuned launch.  Inputs are resident in HBM before timing starts.  The FP8
form (W x W layers on the FP8 matrix cores) is timed the same way and reported
beside it.

Default workload (paper-sized inference): seeded 512^3 fBm + Worley cloud,
sigma_max 512/unit, 10 mip levels, K = 10 stencil levels, 10 residual blocks of
width 200 plus 3 trailing layers, 2^20 shading points = primary hits of a
1024 x 1024 view, light from the side.  Also timed: the FP32 plain form (the
descriptor through HBM, one kernel per layer) on the same points, and the FP64
oracle on a bounded sample of them on the host cores.

    python bench.py [--steps K] [--warmup W] [--workload paper|tiny|batched] [--no-cpu]
                    [--no-fp8]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

METRIC = "shading points/s (stencil+RPNN) BF16/FP8 vs FP32 at stated rel. error; MFMA %"
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP8_TFLOPS = 5000.0

WORKLOADS = {
    "paper": dict(n=512, sigma=512.0, L=10, K=10, W=200, H=3, P=1 << 20, res=1024, worley=0.3,
                  seed_cloud=10, seed_pts=11, seed_theta=12,
                  name="paper-sized inference: 512^3 fBm+Worley cloud, 10 mip levels, K=10, "
                       "10 residual blocks x 200 + 3 layers, 2^20 primary hits of a 1024^2 view"),
    "tiny": dict(n=64, sigma=64.0, L=6, K=6, W=64, H=3, P=4096, res=64, worley=0.0,
                 seed_cloud=1, seed_pts=3, seed_theta=2,
                 name="tiny: 64^3 fBm cloud, 6 mip levels, K=6, 6 residual blocks x 64 + 3 layers, "
                      "4096 points"),
}


HERE = os.path.dirname(os.path.abspath(__file__))
PROFILES = os.path.join(HERE, "profiles")
KERNEL_SOURCES = ["fused.hip", "frame.h", "internal.h"]


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, "paper_1709_05418_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def short_kernel_name(k):
    """Kernel and its first two template arguments (tiles, waves): "k_fused_reg<13, 4, false,
    false>" -> "k_fused_reg<13,4>"."""
    k = k.replace(" ", "")
    if "<" in k:
        name, args = k.split("<", 1)
        k = name + "<" + ",".join(args.rstrip(">").split(",")[:2]) + ">"
    return k


def measured_traffic(kname):
    """(HBM bytes per launch, grid) of the fused BF16 kernel instantiation kname (as
    "k_fused_reg<13,8>"; a launch is its unclamped pass plus its clamped pass) from the
    committed counter summaries, or (None, "") when none covers it or the kernel sources
    changed since the counters were taken.  The persistent grid of a launch does not change
    the kernel's code; each summary states the grid it was taken at, returned beside the
    bytes."""
    import glob
    for f in sorted(glob.glob(os.path.join(PROFILES, "*bf16*_hbm_traffic.txt"))):
        vals = {}
        for ln in open(f):
            if ":" in ln and not ln.startswith("#"):
                k, v = ln.split(":", 1)
                vals[k.strip()] = v.strip()
        k = short_kernel_name(vals.get("kernel", ""))
        if k != kname or vals.get("kernel_sources_sha256") != kernel_sources_sha256():
            continue
        try:
            return int(vals["traffic_bytes_per_launch"]), vals.get("grid", "")
        except (KeyError, ValueError):
            return None, ""
    return None, ""


def cpu_model():
    """The host CPU's model name (first "model name" line of /proc/cpuinfo)."""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_rate(O, fn, n_points, threads, repeats=3):
    """Median over `repeats` runs of fn() (which evaluates n_points points) on `threads`
    host threads, as points/s; also the individual run times."""
    old = O.threads()
    O.set_threads(threads)
    try:
        times = []
        for _ in range(repeats):
            t0 = time.perf_counter()
            fn()
            times.append(time.perf_counter() - t0)
    finally:
        O.set_threads(old)
    return n_points / float(np.median(times)), times


def macs_per_point(K, W, H):
    return 226 * K * W + (K - 1) * W * W + K * W * W + (H - 1) * W * W + W


def fp8_macs_per_point(K, W, H):
    """MACs the FP8 form runs on the FP8 matrix cores: W1, W2 and the dense trailing
    layers (the descriptor layers stay BF16, the final W -> 1 layer FP32)."""
    return (K - 1) * W * W + K * W * W + (H - 1) * W * W


def theta_for(synth, K, W, H, seed):
    """He-uniform parameters with the residual branches scaled by 1/sqrt(K) and a live
    output unit, as in the parity tests (timing does not depend on the values)."""
    return synth.init_params(K, W, H, seed, branch_scale=1.0 / math.sqrt(K), out_scale=0.2,
                             out_bias=0.5)


BATCHED = dict(sizes=[128, 192, 256, 384, 512, 640, 768, 1024], seeds=list(range(100, 108)),
               point_seed=200, pts_seeds=list(range(300, 308)), K=10, W=200, H=3, seed_theta=12,
               name="batched uneven inference: 8 BF16 clouds 128^3..1024^3 (sigma_max = n/unit, "
                    "fBm+Worley), 10^4..2x10^6 points each (log-uniform), K=10, W=200, one "
                    "persistent launch replayed from a HIP graph (each cloud's points put in spatial order "
                    "on the device per step), autotuned variant")


def run_batched(args, log):
    """Batched uneven workload: one autotuned persistent launch over 8 clouds, the points
    of each cloud put in spatial order on the device first (inside the timed step),
    captured in a HIP graph and replayed; compared with the same plan in input order and
    with one ds_predict per cloud."""
    import torch
    import paper_1709_05418_amd as ds
    from paper_1709_05418_amd import synth
    cfg = BATCHED
    dev = torch.device("cuda:0")
    K, W, H = cfg["K"], cfg["W"], cfg["H"]
    rng = np.random.default_rng(cfg["point_seed"])
    counts = np.exp(rng.uniform(np.log(1e4), np.log(2e6), len(cfg["sizes"]))).astype(np.int64)
    ctx = ds.Context(0)
    clouds, pos, view, light = [], [], [], []
    t0 = time.time()
    for n, sd, ps, P in zip(cfg["sizes"], cfg["seeds"], cfg["pts_seeds"], counts):
        d = synth.cloud_density(n, sd, worley=0.3, device=dev, dtype=torch.bfloat16)
        amin, h0 = synth.unit_box(n)
        L = min(16, int(math.ceil(math.log2(n))) + 1)
        clouds.append(ds.Cloud(ctx, d, float(n), amin, h0, L, K))
        pos.append(synth.points_in_density_device(d, int(P), ps, amin, h0))
        view.append(torch.from_numpy(synth.uniform_dirs(int(P), ps + 1000)).to(dev))
        light.append(torch.from_numpy(synth.uniform_dirs(int(P), ps + 2000)).to(dev))
        del d
        torch.cuda.synchronize()
        log(f"cloud {n}^3: {int(P)} points, {L} levels, mean {clouds[-1].info['mean_mu_t']:.1f} "
            f"({time.time() - t0:.1f}s)")
    pos, view, light = torch.cat(pos), torch.cat(view), torch.cat(light)
    offsets = np.concatenate([[0], np.cumsum(counts)])
    N = int(offsets[-1])
    net = ds.Net(ctx, K, W, H)
    net.set_params(theta_for(synth, K, W, H, cfg["seed_theta"]))
    out = torch.empty(N, dtype=torch.float32, device=dev)
    order = {"input": ds.DS_ORDER_INPUT, "spatial": ds.DS_ORDER_SPATIAL}[args.batch_order]
    b = ds.ds_batch_create(ctx.h, net.h, [c.h for c in clouds], offsets)
    ds.ds_batch_set_order(b, order)
    ta = time.time()
    tuned = ds.ds_batch_autotune(b, ds.DS_PREC_BF16, pos, view, light, out, 2)
    log(f"autotune {time.time() - ta:.1f}s: {tuned}")
    ds.ds_batch_capture(b, ds.DS_PREC_BF16, pos, view, light, out)
    stream = torch.cuda.current_stream()

    def replay_timed(plan):
        for _ in range(args.warmup):
            ds.ds_batch_replay(plan)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        tw = time.perf_counter()
        for a, e in evs:
            a.record(stream)
            ds.ds_batch_replay(plan)
            e.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - tw
        return wall * 1e3 / args.steps, float(np.mean([a.elapsed_time(e) for a, e in evs]))
    ms_step, kernel_ms = replay_timed(b)
    # the same plan in the other point order
    other = None
    if not args.no_variants:
        b2 = ds.ds_batch_create(ctx.h, net.h, [c.h for c in clouds], offsets)
        ds.ds_batch_set_order(b2, ds.DS_ORDER_SPATIAL if order == ds.DS_ORDER_INPUT
                              else ds.DS_ORDER_INPUT)
        out2 = torch.empty_like(out)
        tuned2 = ds.ds_batch_autotune(b2, ds.DS_PREC_BF16, pos, view, light, out2, 2)
        ds.ds_batch_capture(b2, ds.DS_PREC_BF16, pos, view, light, out2)
        ms2, kms2 = replay_timed(b2)
        ds.ds_batch_destroy(b2)
        other = {"order": "input" if order == ds.DS_ORDER_SPATIAL else "spatial",
                 "ms_per_step": round(ms2, 4), "kernel_ms": round(kms2, 4), "autotuned": tuned2,
                 "identical_outputs": bool(torch.equal(out2, out))}
        log(f"batched, {other['order']} order: {ms2:.3f} ms ({kms2:.3f} ms events), {tuned2}")
    # the same points, one default ds_predict per cloud
    seq = torch.empty_like(out)
    def per_cloud():
        for c, (a, e) in zip(clouds, zip(offsets[:-1], offsets[1:])):
            ds.ds_predict(ctx.h, c.h, net.h, ds.DS_PREC_BF16, pos[a:e], view[a:e], light[a:e],
                          out=seq[a:e], want_pre=False, want_flags=False)
    per_cloud()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(args.steps):
        per_cloud()
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - ts) * 1e3 / args.steps
    same = bool(torch.equal(seq, out))
    # the FP8 form: calibrated on the 512^3 cloud's points, the same plan shape
    fp8 = None
    out8_keep = None
    if not args.no_fp8:
        ci = cfg["sizes"].index(512)
        a0, a1 = int(offsets[ci]), int(offsets[ci + 1])
        ds.ds_net_quantize(ctx.h, net.h, clouds[ci].h, ds.DS_PREC_FP8, pos[a0:a1], view[a0:a1],
                           light[a0:a1])
        out8 = torch.empty_like(out)
        b8 = ds.ds_batch_create(ctx.h, net.h, [c.h for c in clouds], offsets)
        ds.ds_batch_set_order(b8, order)
        tuned8 = ds.ds_batch_autotune(b8, ds.DS_PREC_FP8, pos, view, light, out8, 2)
        ds.ds_batch_capture(b8, ds.DS_PREC_FP8, pos, view, light, out8)
        ms8, kms8 = replay_timed(b8)
        ds.ds_batch_destroy(b8)
        out8_keep = out8
        fp8 = {"ms_per_step": round(ms8, 4), "value": round(N / (ms8 / 1e3), 1),
               "kernel_ms": round(kms8, 4), "speedup_over_bf16": round(ms_step / ms8, 3),
               "autotuned": tuned8}
        log(f"batched fp8 graph replay {ms8:.3f} ms ({kms8:.3f} ms events), {tuned8}")
    flop = 2.0 * macs_per_point(K, W, H) * N
    achieved = flop / (kernel_ms / 1e3) / 1e12
    log(f"batched graph replay {ms_step:.3f} ms ({kernel_ms:.3f} ms events), per-cloud "
        f"launches {ms_seq:.3f} ms, identical outputs {same}")
    # oracle on a strided sample of every cloud's points: parity of the BF16 (and FP8) batch
    # outputs, and the oracle's own rate (gather + network, pyramids excluded)
    cpu, parity = None, None
    if not args.no_cpu:
        sys.path.insert(0, HERE)
        import oracle as O
        theta64 = theta_for(synth, K, W, H, cfg["seed_theta"]).astype(np.float64)
        out_h = out.cpu().numpy()
        out8_h = out8_keep.cpu().numpy() if fp8 else None
        pos_h, view_h, light_h = pos.cpu().numpy(), view.cpu().numpy(), light.cpu().numpy()
        per = max(1, args.batch_cpu_sample // len(cfg["sizes"]))
        want, got, got8, n_pts = [], [], [], 0
        jobs = []
        for ci, (n, sd) in enumerate(zip(cfg["sizes"], cfg["seeds"])):
            a0, a1 = int(offsets[ci]), int(offsets[ci + 1])
            sel = np.unique(np.linspace(a0, a1 - 1, min(per, a1 - a0)).astype(np.int64))
            d = synth.cloud_density(n, sd, worley=0.3, device=dev, dtype=torch.bfloat16)
            bits = d.cpu().view(torch.int16).numpy().view(np.uint16)
            del d
            amin, h0 = synth.unit_box(n)
            L = min(16, int(math.ceil(math.log2(n))) + 1)
            grid = O.Grid(bits, float(n), amin, h0)
            tp = time.time()
            mean, _ = O.normalize(grid)
            pyr, dims, offs = O.pyramid(grid, mean, L)
            mips = O.default_mips(mean, h0, K, L)
            log(f"oracle pyramid {n}^3: {time.time() - tp:.1f}s")
            if list(mips) != list(clouds[ci].info["mip_of_level"]):
                log(f"cloud {n}^3: oracle and library mip maps differ, skipped")
                continue
            z, _ = O.gather(grid, pyr, dims, offs, mean, K, mips, pos_h[sel], view_h[sel],
                            light_h[sel])
            g, _ = O.forward(theta64, K, W, H, z)
            want.append(g)
            got.append(out_h[sel])
            if out8_h is not None:
                got8.append(out8_h[sel])
            n_pts += sel.size
            jobs.append((grid, pyr, dims, offs, mean, mips, sel))
        rl = lambda x, y: float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-30))
        want = np.concatenate(want)
        parity = {"sampled_points": n_pts, "rel_l2_bf16": rl(np.concatenate(got), want),
                  "rel_l2_fp8": rl(np.concatenate(got8), want) if got8 else None,
                  "tolerance_bf16": 2e-2, "tolerance_fp8": 5e-2}
        log(f"batched parity: {parity}")

        def oracle_points(frac=1):
            for grid, pyr, dims, offs, mean, mips, sel in jobs:
                sl = sel[::frac]
                z, _ = O.gather(grid, pyr, dims, offs, mean, K, mips, pos_h[sl], view_h[sl],
                                light_h[sl])
                O.forward(theta64, K, W, H, z)
        all_threads = O.threads()
        rate, runs = oracle_rate(O, oracle_points, n_pts, all_threads)
        n1 = sum(j[-1][::16].size for j in jobs)
        rate1, runs1 = oracle_rate(O, lambda: oracle_points(16), n1, 1)
        cpu = {"value": round(rate, 2), "unit": "shading points/s", "cores": all_threads,
               "kind": "oracle",
               "sample": f"{n_pts} of the {N} points (evenly strided within each cloud), FP64 "
                         f"gather + network, median of 3 runs "
                         f"({', '.join(f'{t:.2f}' for t in runs)} s); pyramids excluded",
               "single_thread": {"value": round(rate1, 2), "unit": "shading points/s",
                                 "sample": f"{n1} of those points, median of 3 runs "
                                           f"({', '.join(f'{t:.2f}' for t in runs1)} s)"},
               "cpu_model": cpu_model(), "nproc": os.cpu_count()}
        log(f"oracle: {rate:.1f} points/s on {all_threads} threads, {rate1:.1f} on 1 thread")
    line = {
        "metric": METRIC, "value": round(N / (ms_step / 1e3), 1), "unit": "shading points/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "points": N, "points_per_cloud": counts.tolist(),
                   "order": args.batch_order, "autotuned": tuned,
                   "per_cloud_launches_ms": round(ms_seq, 4), "batched_equals_per_cloud": same,
                   "other_order": other},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_BF16_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_BF16_TFLOPS, 4),
                     "traffic": None, "kernel": "fused prediction, autotuned variant",
                     "flop_per_point": 2 * macs_per_point(K, W, H), "points_per_launch": N},
        "cpu_baseline": cpu, "fp8": fp8, "parity": parity,
    }
    ds.ds_batch_destroy(b)
    net.close()
    for c in clouds:
        c.close()
    ctx.close()
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="paper", choices=sorted(WORKLOADS) + ["batched"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the FP64 oracle baseline")
    ap.add_argument("--cpu-sample", type=int, default=65536)
    ap.add_argument("--batch-cpu-sample", type=int, default=16384,
                    help="oracle sample of the batched workload, spread over its clouds")
    ap.add_argument("--fp32-steps", type=int, default=3, help="0 skips the FP32 plain form")
    ap.add_argument("--save-inputs", default=None, help="write the generated inputs to this .npz")
    ap.add_argument("--load-inputs", default=None,
                    help="read inputs written by --save-inputs instead of generating them "
                         "(keeps generator kernels out of profiled runs)")
    ap.add_argument("--no-fp8", action="store_true", help="skip the FP8 form")
    ap.add_argument("--batch-order", default="spatial", choices=["spatial", "input"],
                    help="point order of the batched plan (spatial: each cloud's points sorted "
                         "by a 32^3 grid cell on the device, inside the timed step)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the shuffled-order and front/back-light timings")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the default kernel variant instead of the autotuned one")
    ap.add_argument("--variant", default=None,
                    help="time this kernel variant, 'kind,waves,grid' (as ds_batch_set_config), "
                         "instead of the autotuned one (the FP8 form too, where it has one)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB elementwise copy kernel (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(shading points are independent: each GPU would take its own range of point tiles)",
              file=sys.stderr)
        sys.exit(2)

    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)
    if args.workload == "batched":
        return run_batched(args, log)

    import torch
    import paper_1709_05418_amd as ds
    from paper_1709_05418_amd import synth

    cfg = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    K, W, H, P = cfg["K"], cfg["W"], cfg["H"], cfg["P"]

    t0 = time.time()
    aabb_min, h0 = synth.unit_box(cfg["n"])
    if args.load_inputs:
        saved = np.load(args.load_inputs)
        density = torch.from_numpy(saved["density"]).to(dev)
        pos_np, view_np = saved["pos"], saved["view"]
    else:
        density = synth.cloud_density(cfg["n"], cfg["seed_cloud"], worley=cfg["worley"],
                                      device=dev)
        pos_np, view_np = synth.camera_hits(density, cfg["sigma"], cfg["res"], P,
                                            cfg["seed_pts"], aabb_min, h0, device=dev)
    if args.save_inputs:
        np.savez(args.save_inputs, density=density.cpu().numpy(), pos=pos_np, view=view_np)
    ctx = ds.Context(0)
    cloud = ds.Cloud(ctx, density, cfg["sigma"], aabb_min, h0, cfg["L"], K)
    light_np = np.broadcast_to(synth.table1_lights()["side"], (P, 3)).copy()
    pos = torch.from_numpy(pos_np).to(dev)
    view = torch.from_numpy(view_np).to(dev)
    light = torch.from_numpy(light_np).to(dev)
    theta = theta_for(synth, K, W, H, cfg["seed_theta"])
    net = ds.Net(ctx, K, W, H)
    net.set_params(theta)
    out = torch.empty(P, dtype=torch.float32, device=dev)
    flags = torch.empty(P, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    log(f"setup {time.time() - t0:.1f}s; cloud mean {cloud.info['mean_mu_t']:.3f}, "
        f"mips {cloud.info['mip_of_level']}")

    def run(prec, out_t, pre_t=None):
        ds.ds_predict(ctx.h, cloud.h, net.h, prec, pos, view, light, out=out_t, pre=pre_t,
                      flags=flags, want_pre=pre_t is not None)

    # ---------------------------------------------------------------- BF16 fused (timed)
    # the library's autotuner picks the kernel variant for this workload; the timed
    # step replays the captured launch
    stream = torch.cuda.current_stream()
    def timed(step):
        for _ in range(args.warmup):
            step()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for a, b in evs:
            a.record(stream)
            step()
            b.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        return wall * 1e3 / args.steps, float(np.mean([a.elapsed_time(b) for a, b in evs]))

    ms_default, _ = timed(lambda: run(ds.DS_PREC_BF16, out))
    log(f"bf16 fused, default variant: {ms_default:.3f} ms/step")
    batch = ds.ds_batch_create(ctx.h, net.h, [cloud.h], [0, P])
    tuned = {"kernel": ds.DS_KERNEL_REGISTER, "waves": 4, "grid": 0, "ms": None}
    if args.variant:
        kv, wv, gv = (int(x) for x in args.variant.split(","))
        ds.ds_batch_set_config(batch, kv, wv, gv)
        tuned = {"kernel": kv, "waves": wv, "grid": gv, "ms": None}
        log(f"fixed variant: {tuned}")
    elif not args.no_autotune:
        tuned = ds.ds_batch_autotune(batch, ds.DS_PREC_BF16, pos, view, light, out, 3)
        log(f"autotuned variant: {tuned}")
    ds.ds_batch_capture(batch, ds.DS_PREC_BF16, pos, view, light, out, None, flags)
    ms_step, avg_kernel_ms = timed(lambda: ds.ds_batch_replay(batch))
    value = P / (ms_step / 1e3)
    log(f"bf16 fused, graph replay of the tuned launch: {ms_step:.3f} ms/step (wall), kernel "
        f"{avg_kernel_ms:.3f} ms avg, {value:.3e} points/s")

    flop = 2.0 * macs_per_point(K, W, H) * P
    achieved = flop / (avg_kernel_ms / 1e3) / 1e12
    mt = (W + 15) // 16
    mt = next(v for v in (1, 2, 4, 8, 13, 16) if v >= mt)
    kname = {ds.DS_KERNEL_REGISTER: "k_fused_reg", ds.DS_KERNEL_PIPELINED: "k_fused",
             ds.DS_KERNEL_WIDE: "k_fused_wide",
             ds.DS_KERNEL_TEAMS: "k_fused_teams"}[tuned["kernel"]] + f"<{mt},{tuned['waves']}>"
    traffic, traffic_grid = measured_traffic(kname) if args.workload == "paper" else (None, "")
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_BF16_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_BF16_TFLOPS, 4),
                "traffic": traffic, "traffic_grid": traffic_grid or None,
                "kernel": kname + f" grid {tuned['grid'] or 'one workgroup per tile'} "
                                  "(BF16 MFMA, stencil gather fused)",
                "flop_per_point": 2 * macs_per_point(K, W, H), "points_per_launch": P}

    # ------------------------------------------------- same launch: point order, lights
    # the tuned BF16 launch on the same points in a random order (neighbouring lanes no
    # longer share cells: the worst case of the camera-ordered workload) and under the
    # front and back lights of the same view
    variants = None
    if not args.no_variants:
        variants = {}
        g = torch.Generator(device="cpu").manual_seed(cfg["seed_pts"] + 1)
        perm = torch.randperm(P, generator=g).to(dev)
        cases = [("shuffled_order", pos[perm].contiguous(), view[perm].contiguous(), light)]
        for lname in ("front", "back"):
            lt = torch.from_numpy(np.broadcast_to(synth.table1_lights()[lname], (P, 3)).copy())
            cases.append((f"{lname}_light", pos, view, lt.to(dev)))
        tv = ds.ds_batch_create(ctx.h, net.h, [cloud.h], [0, P])
        try:
            kv, wv, gv = tuned["kernel"], tuned["waves"], tuned["grid"]
            ds.ds_batch_set_config(tv, kv, wv, gv)
            out_v = torch.empty(P, dtype=torch.float32, device=dev)
            for name, pv, vv, lv in cases:
                ds.ds_batch_capture(tv, ds.DS_PREC_BF16, pv, vv, lv, out_v)
                msv, kmsv = timed(lambda: ds.ds_batch_replay(tv))
                variants[name] = {"ms_per_step": round(msv, 4), "kernel_ms": round(kmsv, 4),
                                  "value": round(P / (msv / 1e3), 1)}
                log(f"bf16 fused, {name}: {msv:.3f} ms/step, {P / (msv / 1e3):.3e} points/s")
        finally:
            ds.ds_batch_destroy(tv)

    # ---------------------------------------------------------------- FP8 form
    fp8 = None
    out8 = torch.empty(P, dtype=torch.float32, device=dev)
    if not args.no_fp8:
        cal = torch.arange(0, P, 16, device=dev)  # calibration: every 16th point
        ds.ds_net_quantize(ctx.h, net.h, cloud.h, ds.DS_PREC_FP8, pos[cal].contiguous(),
                           view[cal].contiguous(), light[cal].contiguous())
        batch8 = ds.ds_batch_create(ctx.h, net.h, [cloud.h], [0, P])
        tuned8 = {"kernel": ds.DS_KERNEL_REGISTER, "waves": 4, "grid": 0, "ms": None}
        if args.variant and tuned["kernel"] in (ds.DS_KERNEL_REGISTER, ds.DS_KERNEL_TEAMS):
            ds.ds_batch_set_config(batch8, tuned["kernel"], tuned["waves"], tuned["grid"])
            tuned8 = dict(tuned)
        elif not args.no_autotune:
            tuned8 = ds.ds_batch_autotune(batch8, ds.DS_PREC_FP8, pos, view, light, out8, 3)
        ds.ds_batch_capture(batch8, ds.DS_PREC_FP8, pos, view, light, out8)
        ms8, kms8 = timed(lambda: ds.ds_batch_replay(batch8))
        f16 = 2.0 * (macs_per_point(K, W, H) - fp8_macs_per_point(K, W, H)) * P
        f8 = 2.0 * fp8_macs_per_point(K, W, H) * P
        ideal_ms = (f16 / PEAK_BF16_TFLOPS + f8 / PEAK_FP8_TFLOPS) / 1e12 * 1e3
        fp8 = {"ms_per_step": round(ms8, 4), "value": round(P / (ms8 / 1e3), 1),
               "kernel_ms": round(kms8, 4), "speedup_over_bf16": round(ms_step / ms8, 3),
               "autotuned": tuned8,
               "roofline": {"bound": "mfma", "achieved": round((f16 + f8) / (kms8 / 1e3) / 1e12, 2),
                            "peak": round((f16 + f8) / (ideal_ms / 1e3) / 1e12, 1),
                            "unit": "TFLOP/s", "frac": round(ideal_ms / kms8, 4),
                            "peak_note": "time-weighted: BF16 layers at 2500, FP8 layers at "
                                         "5000 TFLOP/s"}}
        log(f"fp8 form, graph replay of the tuned launch: {ms8:.3f} ms/step, kernel "
            f"{kms8:.3f} ms, {P / (ms8 / 1e3):.3e} points/s, {tuned8}")
        ds.ds_batch_destroy(batch8)

    # ---------------------------------------------------------------- FP32 plain form
    out32 = torch.empty(P, dtype=torch.float32, device=dev)
    fp32 = None
    if args.fp32_steps > 0:
        run(ds.DS_PREC_F32, out32)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.fp32_steps):
            run(ds.DS_PREC_F32, out32)
        torch.cuda.synchronize()
        ms32 = (time.perf_counter() - t1) * 1e3 / args.fp32_steps
        log(f"fp32 plain: {ms32:.2f} ms/step, speedup of bf16 fused {ms32 / ms_step:.2f}x")
        fp32 = {"ms_per_step": round(ms32, 3), "value": P / (ms32 / 1e3),
                "speedup_bf16_over_fp32": round(ms32 / ms_step, 2)}

    if args.calib_copy:
        # plain elementwise copy of a known size: reads and writes 256 MiB each
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log("calibration copy: 3 x 256 MiB read + 256 MiB written")

    # ---------------------------------------------------------------- oracle baseline
    cpu = None
    parity = None
    if not args.no_cpu:
        sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
        import oracle as O
        S = min(args.cpu_sample, P)
        idx = np.linspace(0, P - 1, S).astype(np.int64)
        d_host = density.float().cpu().numpy()
        grid = O.Grid(d_host, cfg["sigma"], aabb_min, h0)
        tp = time.time()
        mean, _ = O.normalize(grid)
        pyr, dims, offs = O.pyramid(grid, mean, cfg["L"])
        mips = O.default_mips(mean, h0, K, cfg["L"])
        log(f"oracle pyramid {time.time() - tp:.1f}s (not part of the timed sample)")
        th64 = theta.astype(np.float64)
        g_ref = np.zeros(S)

        def oracle_points(sel, dst=None):
            for c0 in range(0, sel.size, 4096):
                sl = sel[c0:c0 + 4096]
                z, _ = O.gather(grid, pyr, dims, offs, mean, K, mips, pos_np[sl], view_np[sl],
                                light_np[sl])
                g, _ = O.forward(th64, K, W, H, z)
                if dst is not None:
                    dst[c0:c0 + sl.size] = g
        all_threads = O.threads()
        rate, runs = oracle_rate(O, lambda: oracle_points(idx, g_ref), S, all_threads)
        S1 = max(1, S // 32)
        idx1 = idx[:: max(1, S // S1)][:S1]
        rate1, runs1 = oracle_rate(O, lambda: oracle_points(idx1), idx1.size, 1)
        cpu = {"value": round(rate, 2), "unit": "shading points/s", "cores": all_threads,
               "kind": "oracle",
               "sample": f"{S} of the {P} shading points (evenly strided), FP64 gather + network, "
                         f"median of 3 runs ({', '.join(f'{t:.2f}' for t in runs)} s) on "
                         f"{all_threads} threads; pyramid build excluded",
               "single_thread": {"value": round(rate1, 2), "unit": "shading points/s",
                                 "sample": f"{idx1.size} of the same points, median of 3 runs "
                                           f"({', '.join(f'{t:.2f}' for t in runs1)} s)"},
               "cpu_model": cpu_model(), "nproc": os.cpu_count()}
        log(f"oracle: {rate:.1f} points/s on {all_threads} threads, {rate1:.1f} on 1 thread "
            f"({cpu['cpu_model']})")
        same_mips = list(mips) == list(cloud.info["mip_of_level"])
        g16 = out.cpu().numpy()[idx]
        g32 = out32.cpu().numpy()[idx] if fp32 else None
        rl = lambda a, b: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))
        g8 = out8.cpu().numpy()[idx] if fp8 else None
        parity = {"sampled_points": S, "same_mip_map": same_mips,
                  "rel_l2_bf16": rl(g16, g_ref) if same_mips else None,
                  "rel_l2_fp8": rl(g8, g_ref) if (same_mips and fp8) else None,
                  "rel_l2_fp32": rl(g32, g_ref) if (same_mips and fp32) else None,
                  "tolerance_bf16": 2e-2, "tolerance_fp8": 5e-2, "tolerance_fp32": 1e-5}
        log(f"parity on sample: {parity}")

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "shading points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "grid": cfg["n"], "mip_levels": cfg["L"], "K": K,
                   "W": W, "trailing_layers": H, "points": P, "precision": "bf16",
                   "light": "side"},
        "roofline": roofline, "cpu_baseline": cpu, "fp32_plain": fp32, "fp8": fp8,
        "parity": parity, "variants": variants,
        "kernel_ms": round(avg_kernel_ms, 4), "default_variant_ms": round(ms_default, 4),
        "autotuned": tuned,
    }
    ds.ds_batch_destroy(batch)
    net.close()
    cloud.close()
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
