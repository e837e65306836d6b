#!/usr/bin/env python3
"""Benchmark: training steps/s of one 3DGS rasterizer step on one MI355X.

A step is the whole hot path on one view: forward rasterization (preprocess,
compaction, depth sort, duplication, tile sort, ranges, blend), the L1 loss
gradient, the backward pass (blend backward, preprocess backward) and the
Adam update of all 59 parameters of every Gaussian.  Inputs are seeded
synthetic scenes resident in HBM before timing starts.

Variants: the backward pass fused with Adam (Sec. 3.3: the chain rule only for
the Gaussians with a gradient, kept in compact slots, and one streaming Adam
pass over every parameter) or followed by the separate Adam kernel; float32 or bfloat16 SH coefficients;
the Gaussians in z-order (the layout training keeps them in, re-sorted every
few thousand iterations; Sec. 3.3) or in the generator's random order.  The
first variant (default: fused, float32, z-ordered) gives the reported value;
all are listed, with the cost of the layout step.

Prints ONE JSON line.  Per-phase times come from HIP events recorded on the
stream the kernels are launched on; the dominant kernel's own duration comes
from events the library records around it (fgs_time_next_launch), and the
roofline block relates its algorithmic bytes to the 8 TB/s HBM peak.  The CPU
baseline times the FP64 oracle on a bounded sample of the same workload on
the host cores and extrapolates to one step.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synthetic as S  # noqa: E402

HBM_PEAK_GBS = 8000.0
PARAMS_PER_GAUSSIAN = 59


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c3", choices=sorted(S.WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 16-view batched step")
    ap.add_argument("--no-dynamic", action="store_true", help="skip the dynamic (4D) step")
    ap.add_argument("--cpu-budget-s", type=float, default=20.0)
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="HBM bytes per launch measured with rocprofv3 counters (optional)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run one elementwise kernel over this many MiB first (reference for counters)")
    ap.add_argument("--variants", default=",".join(VARIANTS),
                    help="comma-separated variants to time; the first is the reported value")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def algorithmic_bytes(n, n_touched, i_proc, pixels):
    """Bytes the method itself must move (float32 plain form)."""
    adam = n * PARAMS_PER_GAUSSIAN * 28            # read p, g, m, v; write p, m, v
    blend_bwd = n * 36 + i_proc * (4 + 48) + pixels * 28 + i_proc * 0  # clear, gather, per-pixel state
    pre_bwd = n * 36 + n_touched * (236 + 48) + n * 236   # accum, params+record (touched), grads
    return {"adam": adam, "bwd": blend_bwd + pre_bwd, "blend_bwd": blend_bwd, "pre_bwd": pre_bwd}


def source_digest(files) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2602_09999_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(path: str, kernel: str, workload: str):
    """HBM bytes per launch from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE, each scaled by a calibration kernel of known traffic), or None
    when missing or taken on a different version of the kernel's sources."""
    if not os.path.exists(path):
        return None
    try:
        ent = json.load(open(path))["kernels"][kernel][workload]
        if source_digest(ent["source"]) != ent["source_sha256_16"]:
            return None
        return float(ent["bytes_per_launch"])
    except (KeyError, ValueError, OSError, TypeError):
        return None


def cpu_baseline(workload: str, seed: int, budget_s: float):
    """FP64 oracle on a bounded sample of the workload, extrapolated to one step."""
    import oracle as O
    w = S.WORKLOADS[workload]
    threads = torch.get_num_threads()
    t_all = time.perf_counter()
    scene = S.make_scene(w.n, seed=seed)
    cam = S.workload_camera(workload)
    cx, cy = w.width // 2, w.height // 2
    crop = (cx - 16, cy - 16, cx + 16, cy + 16)
    dl = S.make_dl_dimage(32, 32, seed=1)
    r = O.render64(scene, cam, crop=crop, dl_dimage=dl)
    t_crop = r["seconds_compositing"]            # per-pixel compositing fwd+bwd of the crop only
    # per-Gaussian preprocess + its backward on a subset
    m = min(w.n, 200_000)
    sub = S.subset(scene, slice(0, m))
    rows = {k: (v.double().T.contiguous() if v.dim() == 2 else v.double()).requires_grad_(True)
            for k, v in sub.items()}
    t0 = time.perf_counter()
    pre = O.preprocess64(rows, cam)
    torch.autograd.backward([pre["mean2d"], pre["conic"], pre["opacity"], pre["rgb"]],
                            [torch.ones_like(pre["mean2d"]), torch.ones_like(pre["conic"]),
                             torch.ones_like(pre["opacity"]), torch.ones_like(pre["rgb"])])
    t_pre = (time.perf_counter() - t0) * (w.n / m)
    # Adam over a slice of the parameters
    k = 5_000_000
    p = torch.randn(k, dtype=torch.float64)
    t0 = time.perf_counter()
    O.adam64(p, p, torch.zeros_like(p), torch.zeros_like(p), 1, 1e-3)
    t_adam = (time.perf_counter() - t0) * (w.n * PARAMS_PER_GAUSSIAN / k)
    px = (crop[2] - crop[0]) * (crop[3] - crop[1])
    # the crop time is dominated by compositing; scale its pixel work to the frame
    t_blend = t_crop * (w.width * w.height / px)
    sec = t_blend + t_pre + t_adam
    log(f"cpu baseline: crop {t_crop:.1f}s (x{w.width * w.height / px:.0f} pixels), preprocess "
        f"{t_pre:.1f}s, adam {t_adam:.1f}s (extrapolated), sample wall {time.perf_counter() - t_all:.1f}s")
    return {"value": 1.0 / sec, "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 oracle: 32x32 central crop fwd+bwd (pixels scaled to {w.width}x{w.height}), "
                       f"preprocess fwd+bwd on {m} of {w.n} Gaussians, Adam on {k} of "
                       f"{w.n * PARAMS_PER_GAUSSIAN} parameters; extrapolated to one step"),
            "seconds_per_step_extrapolated": sec}


# name: (backward fused with Adam, SH element type, z-ordered layout, forward
# waits for the instance count on the host); the first is the headline.  The
# synchronisation-free forward sizes its launches by the instance capacity
# (set by the synchronised warm-up steps, with headroom) and reads the counts
# on the device; after the timed steps the overflow flag is checked.
VARIANTS = {
    "fused_f32": (True, torch.float32, True, False),
    "unfused_f32": (False, torch.float32, True, False),
    "fused_bf16sh": (True, torch.bfloat16, True, False),
    "unfused_bf16sh": (False, torch.bfloat16, True, False),
    "fused_f32_unordered": (True, torch.float32, False, False),
    "fused_f32_hostsync": (True, torch.float32, True, True),
}
ZORDER_EVERY = 5000  # iterations between z-order re-layouts (Sec. 3.3)
# the step each variant times live with the library's timing hook, and the kernel it is
TIMED = {True: ("adam_sparse", "k_adam_sparse"), False: ("adam", "k_adam")}


def fused_bytes(n, n_touched, sh_bf16):
    """Algorithmic bytes of the fused backward + Adam kernels.  'touched': the
    nine accumulators of every Gaussian and the 1-bit marks, and for each
    Gaussian with a gradient its record and parameters read and its 59
    gradients written.  'adam': read and write of p, m, v of every parameter
    (SH planes at 2 bytes per parameter when bfloat16), the marks once, and
    the gradients of the Gaussians that have one.  Slots and list entries are
    not counted (bookkeeping of this implementation)."""
    sh = 48 * (2 * 2 + 16) if sh_bf16 else 48 * 24
    per = 11 * 24 + sh
    touched = n * 36 + n // 4 + n_touched * (48 + 236 + 236)
    adam = n * per + n // 4 + n_touched * 236
    return {"touched": touched, "adam": adam}


def adam_bytes(n, sh_bf16):
    """Algorithmic bytes of the separate Adam kernel: read p, g, m, v; write p, m, v."""
    sh = 48 * (3 * 2 + 16 + 0) if sh_bf16 else 48 * 28
    return n * (11 * 28 + sh)


def run_variant(name, args, scene, cam, target, dev, w):
    import paper_2602_09999_amd as P
    from paper_2602_09999_amd import binding as B
    fused, shd, zorder, host_sync = VARIANTS[name]
    params = {k: v.to(dev) for k, v in scene.items()}
    for k in ("sh_dc", "sh_rest"):
        params[k] = params[k].to(shd).contiguous()
    rz = B.Rasterizer(cam, device=dev)
    opt = P.FusedAdam(params, S.ADAM_LR)
    zorder_ms = None
    if zorder:
        # the layout step of training (outside the timed region): parameters
        # and moments re-sorted in Morton order of the means
        B.apply_zorder(params, opt)  # first call warms up the kernels
        z0, z1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        z0.record()
        B.apply_zorder(params, opt)
        z1.record()
        torch.cuda.synchronize()
        zorder_ms = z0.elapsed_time(z1)
    stream = torch.cuda.current_stream()
    image = torch.empty(3, w.height, w.width, device=dev)
    t_final = torch.empty(w.height, w.width, device=dev)
    last = torch.empty(w.height, w.width, dtype=torch.int32, device=dev)
    dl = torch.empty_like(image)
    grads = None if fused else {k: torch.empty_like(v) for k, v in params.items()}
    step_name, kernel = TIMED[fused]

    def step(ev=None, kev=None, sync=True):
        if kev is not None:
            B.time_next_launch(step_name, kev[0], kev[1])
        if ev is not None:
            ev[0].record(stream)
        rz.forward(params, image, t_final, last, sync=sync)
        if ev is not None:
            ev[1].record(stream)
        B.l1_loss_backward(image, target, dl)
        if ev is not None:
            ev[2].record(stream)
        if fused:
            rz.backward_adam(params, image, last, dl, opt)
        else:
            rz.backward(params, image, last, dl, grads)
            if ev is not None:
                ev[3].record(stream)
            opt.step(grads)
        if ev is not None:
            if fused:
                ev[3].record(stream)
            ev[4].record(stream)

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    kevs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    for pair in kevs:  # torch creates events lazily: record each once so the hook can use it
        for e in pair:
            e.record(stream)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"{name}: warmup done; N_vis={rz.last_stats.get('n_visible')} I={rz.last_stats.get('n_instances')}")
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k], kevs[k], sync=host_sync)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if rz.overflowed():
        raise SystemExit(f"{name}: a timed step exceeded the instance capacity {rz.capacity}")
    ph = np.array([[evs[k][j].elapsed_time(evs[k][j + 1]) for j in range(4)] for k in range(args.steps)]).mean(0)
    kms = float(np.mean([kevs[k][0].elapsed_time(kevs[k][1]) for k in range(args.steps)]))
    ms_step = 1000.0 * elapsed / args.steps
    names = ("forward", "l1", "backward+adam", "-") if fused else ("forward", "l1", "backward", "adam")
    phases = {names[j]: float(ph[j]) for j in range(4) if names[j] != "-"}
    log(f"{name}: ms/step {ms_step:.3f}; " + " ".join(f"{k} {v:.3f}" for k, v in phases.items()) +
        f"; {kernel} {kms:.3f} ms")
    return {"steps": args.steps, "elapsed": elapsed, "ms_per_step": ms_step, "steps_per_s": args.steps / elapsed,
            "phase_ms": phases, "kernel": kernel, "kernel_ms": kms, "rz": rz, "params": params, "last": last,
            "fused": fused, "sh_bf16": shd == torch.bfloat16, "zorder": zorder, "zorder_ms": zorder_ms,
            "host_sync": host_sync}


BATCH_VIEWS, BATCH_N = 16, 1_500_000
DYN_STEPS, DYN_N = 8, 1_000_000


def batched_step_fn(br, params, opt, target, dl, grads, mode):
    from paper_2602_09999_amd import binding as B

    def step():
        images, _, _ = br.forward(params, mode=mode)
        B.l1_loss_backward(images, target, dl)
        br.backward(params, dl, grads)
        opt.step(grads)
    return step


def time_steps(step, steps, warmup):
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def run_batched(args, dev):
    """Several views per step: 1.5M Gaussians around the origin, 16 cameras on
    the radius-5 sphere with seeded uneven resolutions (640-1920 x 480-1080,
    f = width); tile size from the autotuner; the step timed eagerly and as a
    captured graph replayed (synchronisation-free forward, device step count)."""
    import paper_2602_09999_amd as P
    from paper_2602_09999_amd import _lib as L
    from paper_2602_09999_amd import binding as B
    from paper_2602_09999_amd.autotune import TileAutotuner
    scene = S.batch_scene(BATCH_N, seed=args.seed)
    cams = S.uniform_sphere_cameras(BATCH_VIEWS, seed=args.seed)
    params = {k: v.to(dev) for k, v in scene.items()}
    del scene
    tuner = TileAutotuner(reps=2)
    tile = tuner.choose(params, cams)
    tile_ms = next(iter(tuner.cache.values()))["ms"]
    st = B.default_settings(tile=tile)
    npix = sum(B.view_pixels(cams))
    target = torch.rand(3 * npix, generator=torch.Generator().manual_seed(args.seed)).to(dev)
    dl = torch.empty(3 * npix, device=dev)
    out = {"workload": f"{BATCH_N} Gaussians, {BATCH_VIEWS} views on a radius-5 sphere, "
                       f"{npix} pixels in all", "tile": tile, "autotune_ms_per_fwd_bwd": tile_ms}
    for mode_name, graph in (("eager", False), ("graph", True)):
        br = B.BatchRasterizer(cams, settings=st)
        opt = P.FusedAdam(params, S.ADAM_LR, device_step=graph)
        grads = {k: torch.empty_like(v) for k, v in params.items()}
        br.forward(params)
        br.ensure(BATCH_N, int(br.last_stats["n_instances"] * 1.3))
        out["instances"] = br.last_stats["n_instances"]
        step = batched_step_fn(br, params, opt, target, dl, grads, L.FGS_FORWARD_NO_SYNC if graph else 0)
        if graph:
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                step()
            torch.cuda.current_stream().wait_stream(side)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                step()
            sec = time_steps(g.replay, max(3, args.steps // 5), 1)
            if int(br.counters()[7].item()) != 0:
                raise RuntimeError("instance capacity exceeded during graph replay")
        else:
            sec = time_steps(step, max(3, args.steps // 5), 1)
        out[f"{mode_name}_ms_per_step"] = sec * 1e3
        out[f"{mode_name}_steps_per_s"] = 1.0 / sec
        out[f"{mode_name}_views_per_s"] = BATCH_VIEWS / sec
        log(f"batched {mode_name}: {sec * 1e3:.2f} ms per step of {BATCH_VIEWS} views (tile {tile})")
        del br, opt, grads
        torch.cuda.empty_cache()
    return out


def run_dynamic(args, dev):
    """Dynamic Gaussians: mean(t) = mu + v t + a t^2 (v ~ N(0, 0.1), a ~
    N(0, 0.02)), 1M Gaussians, 8 timesteps t = k/7 at 1280x720 (identity
    camera, f = 1000) in one batched step, bfloat16 SH; the backward yields the
    velocity and acceleration gradients, and Adam updates them too."""
    import paper_2602_09999_amd as P
    from paper_2602_09999_amd import binding as B
    scene = S.make_scene(DYN_N, seed=args.seed)
    scene.update(S.make_motion(DYN_N, seed=args.seed))
    params = {k: v.to(dev) for k, v in scene.items()}
    del scene
    for k in ("sh_dc", "sh_rest"):
        params[k] = params[k].bfloat16().contiguous()
    cam = S.identity_camera(1280, 720, 1000.0)
    times = S.timesteps(DYN_STEPS)
    br = B.BatchRasterizer([cam] * DYN_STEPS, times=times)
    lrs = dict(S.ADAM_LR, velocity=S.ADAM_LR["means"], accel=S.ADAM_LR["means"])
    opt = P.FusedAdam(params, lrs)
    npix = sum(B.view_pixels([cam] * DYN_STEPS))
    target = torch.rand(3 * npix, generator=torch.Generator().manual_seed(args.seed + 1)).to(dev)
    dl = torch.empty(3 * npix, device=dev)
    grads = {k: torch.empty_like(v) for k, v in params.items()}
    step = batched_step_fn(br, params, opt, target, dl, grads, 0)
    sec = time_steps(step, max(3, args.steps // 5), 2)
    log(f"dynamic: {sec * 1e3:.2f} ms per step of {DYN_STEPS} timesteps")
    return {"workload": f"{DYN_N} dynamic Gaussians, {DYN_STEPS} timesteps, 1280x720, bf16 SH",
            "ms_per_step": sec * 1e3, "steps_per_s": 1.0 / sec, "timesteps_per_s": DYN_STEPS / sec,
            "instances": br.last_stats["n_instances"]}


def workload_counts(r, w, dev):
    """Instance and gradient counts of a finished run (outside any timed region)."""
    rz, last = r["rz"], r["last"]
    lay = rz.layout()
    n = w.n
    tiles = lay.tiles_x * lay.tiles_y
    ranges = rz.view("ranges", 2 * tiles).view(torch.int32).view(tiles, 2)
    lp = torch.zeros(lay.tiles_y * 16, lay.tiles_x * 16, dtype=torch.int64, device=dev)
    lp[:w.height, :w.width] = last.long()
    walks = lp.view(lay.tiles_y, 16, lay.tiles_x, 16).amax(dim=(1, 3)).flatten()
    lens = (ranges[:, 1] - ranges[:, 0]).long()
    q = torch.tensor([0.5, 0.9, 0.99, 1.0], device=dev).double()
    log("tile walk p50/p90/p99/max", [int(x) for x in torch.quantile(walks.double(), q)],
        "list length p50/p90/p99/max", [int(x) for x in torch.quantile(lens.double(), q)],
        "tiles walking their whole list", int(((walks == lens) & (lens > 0)).sum()))
    accum = rz.view("accum", 9 * n, dtype=torch.float32).view(n, 9)
    return {"i_proc": int(walks.sum()), "n_touched": int((accum != 0).any(1).sum()),
            "visible": rz.last_stats.get("n_visible"), "instances": rz.last_stats.get("n_instances")}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    w = S.WORKLOADS[args.workload]
    log(f"workload {w.name}: {w.description}")
    scene = S.make_scene(w.n, seed=args.seed)
    cam = S.workload_camera(args.workload)
    dev = torch.device("cuda", 0)
    target = S.make_target(w.height, w.width, seed=args.seed).to(dev)
    if args.calibrate_copy_mib > 0:
        # a plain elementwise kernel (torch.neg) of known traffic: it reads and
        # writes exactly calibrate_copy_mib MiB, so HBM counters can be scaled
        src = torch.ones(args.calibrate_copy_mib << 18, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log(f"calibration kernel (neg): {args.calibrate_copy_mib} MiB read + {args.calibrate_copy_mib} MiB written")
        del src, dst
    names = [v for v in args.variants.split(",") if v]
    for v in names:
        if v not in VARIANTS:
            raise SystemExit(f"unknown variant {v}; choose from {', '.join(VARIANTS)}")
    head = names[0]
    results, counts = {}, None
    for v in names:
        r = run_variant(v, args, scene, cam, target, dev, w)
        if v == head:
            counts = workload_counts(r, w, dev)
        for k in ("rz", "params", "last"):
            r.pop(k)
        results[v] = r
        torch.cuda.empty_cache()
    hr = results[head]
    n, pixels = w.n, w.width * w.height
    bwd_blend = n * 36 + counts["i_proc"] * (4 + 48) + pixels * 28
    if hr["fused"]:
        fb = fused_bytes(n, counts["n_touched"], hr["sh_bf16"])
        kbytes = fb["adam"]
        bwd_bytes, bwd_ms = bwd_blend + fb["touched"] + fb["adam"], hr["phase_ms"]["backward+adam"]
    else:
        kbytes = adam_bytes(n, hr["sh_bf16"])
        bwd_bytes = bwd_blend + algorithmic_bytes(n, counts["n_touched"], counts["i_proc"], pixels)["pre_bwd"]
        bwd_ms = hr["phase_ms"]["backward"]
    k_gbs = kbytes / (hr["kernel_ms"] * 1e-3) / 1e9
    bwd_gbs = bwd_bytes / (bwd_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.traffic_json, hr["kernel"], args.workload)
    variants = {}
    for v, r in results.items():
        kb = fused_bytes(n, counts["n_touched"], r["sh_bf16"])["adam"] if r["fused"] else adam_bytes(n, r["sh_bf16"])
        variants[v] = {"steps_per_s": r["steps_per_s"], "ms_per_step": r["ms_per_step"], "phase_ms": r["phase_ms"],
                       "sh": "bf16" if r["sh_bf16"] else "f32", "backward_fused_with_adam": r["fused"],
                       "zorder_layout": r["zorder"], "forward_host_sync": r["host_sync"],
                       "timed_kernel": {"name": r["kernel"], "avg_launch_ms": r["kernel_ms"],
                                        "algorithmic_bytes": kb,
                                        "GB_per_s": kb / (r["kernel_ms"] * 1e-3) / 1e9}}
    out = {
        "metric": "train steps/s (fwd+bwd+Adam) at 3M Gaussians 1600x1060; bwd HBM GB/s",
        "value": hr["steps_per_s"],
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hr["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded scene, random uniform target)",
        "config": {"workload": f"{w.name}: {w.description}", "gaussians": n, "width": w.width,
                   "height": w.height, "tile": 16, "sh_degree": 3, "seed": args.seed, "variant": head,
                   "forward_host_sync": hr["host_sync"],
                   "visible": counts["visible"], "instances": counts["instances"],
                   "instances_walked": counts["i_proc"], "gaussians_with_gradient": counts["n_touched"]},
        "roofline": {"bound": "hbm", "kernel": hr["kernel"], "achieved": k_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": k_gbs / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes": kbytes, "avg_launch_ms": hr["kernel_ms"]},
        "bwd_hbm": {"achieved": bwd_gbs, "unit": "GB/s", "frac": bwd_gbs / HBM_PEAK_GBS,
                    "algorithmic_bytes": bwd_bytes, "ms": bwd_ms,
                    "covers": "blend backward + " + ("preprocess backward fused with Adam (both kernels)"
                                                     if hr["fused"] else "preprocess backward")},
        "phase_ms": hr["phase_ms"],
        "zorder": None if hr["zorder_ms"] is None else {
            "layout_ms": hr["zorder_ms"], "every_iterations": ZORDER_EVERY,
            "amortized_ms_per_step": hr["zorder_ms"] / ZORDER_EVERY,
            "covers": "Morton permutation of the means + gather of all parameters and both Adam moments"},
        "variants": variants,
    }
    if not args.no_batched:
        out["batched"] = run_batched(args, dev)
        torch.cuda.empty_cache()
    if not args.no_dynamic:
        out["dynamic"] = run_dynamic(args, dev)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload, args.seed, args.cpu_budget_s)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
