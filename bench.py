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
    ap.add_argument("--batched-tile", type=int, default=0, choices=[0, 8, 16, 32],
                    help="tile size of the batched step (0: the autotuner's choice of tile, schedule and sort block)")
    ap.add_argument("--batched-schedule", default="grid", choices=["grid", "queue"],
                    help="blend schedule of the batched step with --batched-tile: one workgroup per tile, or "
                         "persistent waves over per-XCD tile queues")
    ap.add_argument("--batched-sort-block", type=int, default=4096, choices=[4096, 8192],
                    help="pairs per block of the batched step's tile sort with --batched-tile")
    ap.add_argument("--form", default="step", choices=["step", "batched", "dynamic", "conditional"],
                    help="step: the full report; otherwise time only that form and print its block "
                         "(for kernel traces of one form)")
    ap.add_argument("--dist-steps", type=int, default=200,
                    help="steps timed one by one (events around each) for the median and p10/p90")
    ap.add_argument("--split-reps", type=int, default=3,
                    help="steps per stage timed with the library's launch hook (per-kernel split)")
    ap.add_argument("--extra-workloads", default="c2",
                    help="comma-separated further workloads timed with the headline variant")
    ap.add_argument("--no-oracle-error", action="store_true",
                    help="skip the FP64-oracle error statement of the crops (part of the CPU baseline leg)")
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


# 64x64 windows of the full-size workloads where the FP64 oracle is run: the
# image centre and the bottom edge (at 1600x1060 a partial tile row: 1060 =
# 66 * 16 + 4).  The corner [0, 64)^2 of these scenes holds no Gaussian (the
# projected means start about 200 pixels in), so it would time nothing.
CROPS = {"c2": {"centre": (608, 328, 672, 392), "edge": (1076, 656, 1140, 720)},
         "c3": {"centre": (768, 498, 832, 562), "edge": (1336, 996, 1400, 1060)}}
SH_NAMES = ("sh_dc", "sh_rest")


def bf16_rounded(scene):
    """The scene with its SH coefficients rounded to bfloat16 (kept float32):
    the precision form's inputs as the oracle consumes them."""
    out = dict(scene)
    for k in SH_NAMES:
        out[k] = scene[k].bfloat16().float()
    return out


def crop_upstream(crop, seed):
    x0, y0, x1, y1 = crop
    return S.make_dl_dimage(y1 - y0, x1 - x0, seed=seed)


# wave64 VALU instructions the chip can issue per second: 256 CUs x 4 SIMDs,
# one FP32 wave instruction per 4 cycles (16 lanes per cycle), 2.4 GHz
VALU_WAVE_INSTS_PER_S = 256 * 4 / 4 * 2.4e9


def measured_counters(path: str, kernel: str, workload: str):
    """Instruction and atomic counts per launch from the committed counter
    summary, or None when missing or taken on other kernel sources."""
    if not os.path.exists(path):
        return None
    try:
        ent = json.load(open(path))["kernels"][kernel][workload]
        if source_digest(ent["source"]) != ent["source_sha256_16"]:
            return None
        return {k: float(ent[k]) for k in ("valu_insts_per_launch", "atomics_per_launch") if k in ent}
    except (KeyError, ValueError, OSError, TypeError):
        return None


def cpu_baseline(workload: str, seed: int, scene, with_bf16: bool):
    """The FP64 oracle on the host cores, timed on a bounded sample of the
    workload and extrapolated to one step: forward + backward of the 64x64
    centre and edge crops (compositing seconds per pixel, scaled to the
    frame), the preprocess forward + backward on a subset of the Gaussians,
    Adam on a slice of the parameters.  The crop renders (also of the
    bfloat16-rounded scene when with_bf16) are returned for the error
    statement of the GPU results."""
    import oracle as O
    w = S.WORKLOADS[workload]
    threads = torch.get_num_threads()
    t_all = time.perf_counter()
    cam = S.workload_camera(workload)
    refs, t_comp, px, t_crops = {}, 0.0, 0, 0.0
    for where, crop in CROPS[workload].items():
        for sh in (("f32", "bf16") if with_bf16 else ("f32",)):
            sc = scene if sh == "f32" else bf16_rounded(scene)
            t0 = time.perf_counter()
            r = O.render64(sc, cam, crop=crop, dl_dimage=crop_upstream(crop, 7), mask_borderline=True)
            if sh == "f32":
                t_crops += time.perf_counter() - t0
                t_comp += r["seconds_compositing"]
                px += (crop[2] - crop[0]) * (crop[3] - crop[1])
            refs[(where, sh)] = {k: r[k] for k in ("image", "t_final", "borderline", "dl_used", "grads")}
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
    frame = w.width * w.height
    t_blend = t_comp / px * frame   # per-pixel compositing (forward + backward) scaled to the frame
    sec = t_blend + t_pre + t_adam
    log(f"cpu baseline ({threads} threads, os.cpu_count() {os.cpu_count()}): crops {t_crops:.1f}s "
        f"(compositing {t_comp:.2f}s for {px} pixels), per-frame compositing {t_blend:.1f}s, preprocess "
        f"{t_pre:.1f}s, adam {t_adam:.1f}s (extrapolated), sample wall {time.perf_counter() - t_all:.1f}s")
    base = {"value": 1.0 / sec, "unit": "steps/s", "cores": threads, "os_cpu_count": os.cpu_count(),
            "kind": "oracle",
            "sample": (f"FP64 oracle: forward + backward of the 64x64 centre and edge crops "
                       f"({', '.join(str(c) for c in CROPS[workload].values())}), compositing time per pixel "
                       f"scaled to {w.width}x{w.height}; preprocess forward + backward on {m} of {w.n} "
                       f"Gaussians; Adam on {k} of {w.n * PARAMS_PER_GAUSSIAN} parameters; extrapolated to one "
                       f"step (label: extrapolated)"),
            "seconds_per_step_extrapolated": sec, "seconds_per_pixel_compositing": t_comp / px,
            "crop_seconds_total": t_crops}
    return base, refs


def err_stats(got: torch.Tensor, ref: torch.Tensor, mask=None):
    """max abs, max relative and RMS of got - ref.  The relative error divides
    by max(|ref|, the RMS of the nonzero reference entries), as the parity
    tests' elementwise bound does (a sum that nearly cancels has no meaningful
    relative error of its own)."""
    d = (got.double() - ref.double()).abs()
    r = ref.double().abs()
    if mask is not None:
        d, r = d[..., mask], r[..., mask]
    if d.numel() == 0:
        return {"max_abs": 0.0, "max_rel": 0.0, "rms": 0.0}
    live = r[r != 0]
    rms_ref = float(torch.sqrt((live ** 2).mean())) if live.numel() else 0.0
    rel = d / torch.clamp(r, min=max(rms_ref, 1e-300))
    return {"max_abs": float(d.max()), "max_rel": float(rel.max()), "rms": float(torch.sqrt((d ** 2).mean()))}


def bf16_ulps(got: torch.Tensor, ref: torch.Tensor):
    """Largest distance of bfloat16-stored values from the bfloat16 rounding of
    the float64 reference, in units of the reference's bfloat16 ulp."""
    r = ref.double()
    rb = r.to(torch.bfloat16).double()
    e = torch.floor(torch.log2(torch.clamp(r.abs(), min=1e-38)))
    ulp = torch.pow(2.0, e - 7)
    return {"max_bf16_ulps": float(((got.double() - rb).abs() / ulp).max())}


def update_error_beyond_rounding(p_gpu: torch.Tensor, p0: torch.Tensor, p_ref: torch.Tensor):
    """The float32 update's error beyond the rounding of the stored parameter:
    max(0, |p_gpu - p_ref| - ulp(p_ref) / 2) relative to max(|update|, the
    RMS of the nonzero updates), p_ref the float64 reference.  An update far
    smaller than the parameter is resolved only to the parameter's ulp, which
    no implementation can beat; what is left is the update's own error."""
    r = p_ref.double()
    upd = r - p0.double()
    half_ulp = 0.5 * torch.pow(2.0, torch.floor(torch.log2(torch.clamp(r.abs(), min=1e-38))) - 23)
    excess = torch.clamp((p_gpu.double() - r).abs() - half_ulp, min=0.0)
    live = upd[upd != 0]
    rms = float(torch.sqrt((live ** 2).mean())) if live.numel() else 0.0
    return float((excess / torch.clamp(upd.abs(), min=max(rms, 1e-300))).max())


def unpermute(t: torch.Tensor, perm: torch.Tensor) -> torch.Tensor:
    """Gaussian axis (last) back from z-order: out[..., perm[i]] = t[..., i]."""
    out = torch.empty_like(t)
    out[..., perm.long()] = t
    return out


def oracle_errors(refs, scene, workload: str, dev, with_bf16: bool):
    """The error of each result of the benchmark's step against the FP64
    oracle on the crops, for float32 and bfloat16 SH: the parameters in
    z-order, the forward without host synchronisation, then (a) the
    gradients of the separate backward and (b) the parameters after the
    backward fused with Adam (seeded moments, step 3, against adam64 of the
    oracle gradients).  Pixels with a borderline decision are left out of
    the image statistics (their count is given); the relative error divides
    by max(|reference|, its RMS)."""
    import oracle as O
    import paper_2602_09999_amd as P
    from paper_2602_09999_amd import binding as B
    cam = S.workload_camera(workload)
    out = {}
    for sh in (("f32", "bf16") if with_bf16 else ("f32",)):
        shd = torch.float32 if sh == "f32" else torch.bfloat16
        params = {k: v.to(dev) for k, v in scene.items()}
        for k in SH_NAMES:
            params[k] = params[k].to(shd).contiguous()
        perm = B.apply_zorder(params)
        rz = B.Rasterizer(cam, device=dev)
        rz.forward(params)
        image, t_final, last = rz.forward(params, sync=False)
        torch.cuda.synchronize()
        res = {}
        for where, crop in CROPS[workload].items():
            ref = refs[(where, sh)]
            x0, y0, x1, y1 = crop
            ok = ~ref["borderline"]
            e = {"borderline_pixels_excluded": int((~ok).sum()), "pixels": int(ok.numel())}
            e["image"] = err_stats(image[:, y0:y1, x0:x1].cpu(), ref["image"], ok)
            e["t_final"] = err_stats(t_final[y0:y1, x0:x1].cpu(), ref["t_final"], ok)
            dl = torch.zeros(3, cam.height, cam.width, device=dev)
            dl[:, y0:y1, x0:x1] = ref["dl_used"].float().to(dev)
            grads = rz.backward(params, image, last, dl)
            e["gradients"] = {k: err_stats(unpermute(grads[k].float(), perm).cpu(), ref["grads"][k])
                              for k in B.PARAM_NAMES}
            scales = {}
            for k, g in ref["grads"].items():
                live = g[g != 0]
                scales[k] = float(torch.sqrt((live ** 2).mean())) if live.numel() else 1e-6
            m0, v0 = S.make_adam_state({k: tuple(v.shape) for k, v in scene.items()}, scales, seed=3)
            pc = {k: v.clone() for k, v in params.items()}
            opt = P.FusedAdam(pc, S.ADAM_LR)
            inv = torch.argsort(perm.long().cpu())
            for k in pc:  # the moments in z-order, like the parameters
                opt.exp_avg[k].copy_(m0[k][..., perm.long().cpu()].to(dev))
                opt.exp_avg_sq[k].copy_(v0[k][..., perm.long().cpu()].to(dev))
            opt.t = 2
            rz.backward_adam(pc, image, last, dl, opt)
            torch.cuda.synchronize()
            upd = {}
            for k in B.PARAM_NAMES:
                p0 = params[k].float().cpu()[..., inv]
                p_ref, _, _ = O.adam64(p0, ref["grads"][k], m0[k], v0[k], 3, S.ADAM_LR[k])
                p_gpu = pc[k].float().cpu()[..., inv]
                if pc[k].dtype == torch.bfloat16:
                    upd[k] = bf16_ulps(p_gpu, p_ref)  # stored in bfloat16: the step is rounded to it
                else:
                    # the update of every parameter, and its error beyond the float32 rounding of the parameter
                    upd[k] = dict(err_stats(p_gpu - p0, p_ref - p0.double()),
                                  max_rel_beyond_rounding=update_error_beyond_rounding(p_gpu, p0, p_ref))
            e["fused_adam_update"] = upd
            res[where] = e
            f32u = [v["max_rel_beyond_rounding"] for v in upd.values() if "max_rel_beyond_rounding" in v]
            bf16u = [v["max_bf16_ulps"] for v in upd.values() if "max_bf16_ulps" in v]
            log(f"oracle error {sh} {where}: image max abs {e['image']['max_abs']:.2e} "
                f"({e['borderline_pixels_excluded']} borderline px), worst gradient max rel "
                f"{max(v['max_rel'] for v in e['gradients'].values()):.2e}, float32 updates max rel "
                f"{max(f32u):.2e} beyond the parameters' rounding"
                + (f", bfloat16 parameters within {max(bf16u):.0f} bf16 ulp" if bf16u else ""))
        out[sh] = res
        del params, rz
        torch.cuda.empty_cache()
    return out


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

    def step(ev=None, kev=None, sync=True, hook=None):
        if kev is not None:
            B.time_next_launch(hook or step_name, kev[0], kev[1])
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
    # distribution: steps timed one by one with events on the launch stream
    dist = None
    if args.dist_steps > 0:
        dev_ = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.dist_steps)]
        for k in range(args.dist_steps):
            step(dev_[k], sync=host_sync)
        torch.cuda.synchronize()
        per = np.array([dev_[k][0].elapsed_time(dev_[k][4]) for k in range(args.dist_steps)])
        dist = {"steps": args.dist_steps, "median": float(np.median(per)), "p10": float(np.percentile(per, 10)),
                "p90": float(np.percentile(per, 90)), "mean": float(per.mean()),
                "steps_per_s_at_median": 1000.0 / float(np.median(per))}
    # per-stage split: the library records events around one stage's launches
    split = {}
    stages = ["preprocess", "duplicate", "tile_sort", "blend_forward", "blend_backward"]
    stages += ["touched_gradients", "adam_sparse"] if fused else ["preprocess_backward", "adam"]
    sev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.split_reps)]
    for pair in sev:
        for e in pair:
            e.record(stream)
    for st_name in stages if args.split_reps > 0 else ():
        for k in range(args.split_reps):
            step(kev=sev[k], sync=host_sync, hook=st_name)
        torch.cuda.synchronize()
        split[st_name] = float(np.mean([sev[k][0].elapsed_time(sev[k][1]) for k in range(args.split_reps)]))
    if rz.overflowed():
        raise SystemExit(f"{name}: a step exceeded the instance capacity {rz.capacity}")
    names = ("forward", "l1", "backward+adam", "-") if fused else ("forward", "l1", "backward", "adam")
    phases = {names[j]: float(ph[j]) for j in range(4) if names[j] != "-"}
    log(f"{name}: ms/step {ms_step:.3f}; " + " ".join(f"{k} {v:.3f}" for k, v in phases.items()) +
        f"; {kernel} {kms:.3f} ms" + (f"; {dist['steps']} steps median {dist['median']:.3f} p10 {dist['p10']:.3f} "
                                      f"p90 {dist['p90']:.3f} ms" if dist else ""))
    if split:
        log(f"{name}: stage split (ms) " + " ".join(f"{k} {v:.3f}" for k, v in split.items()))
    return {"steps": args.steps, "elapsed": elapsed, "ms_per_step": ms_step, "steps_per_s": args.steps / elapsed,
            "phase_ms": phases, "kernel": kernel, "kernel_ms": kms, "rz": rz, "params": params, "last": last,
            "step_ms": dist, "stage_ms": split,
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


def adam_roofline(step, params, sh_bf16_names=()):
    """Duration of the separate Adam kernel inside one more eager step
    (library launch hook) against its algorithmic bytes: read p, g, m, v and
    write p, m, v of every parameter (bfloat16 p and g where stored so)."""
    from paper_2602_09999_amd import binding as B
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for x in e:
        x.record()
    B.time_next_launch("adam", e[0], e[1])
    step()
    torch.cuda.synchronize()
    ms = e[0].elapsed_time(e[1])
    nbytes = 0
    for k, v in params.items():
        w = v.element_size()
        nbytes += v.numel() * (3 * w + 16)  # p, g, p' at the parameter's width; m, v, m', v' float32
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": "k_adam", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "algorithmic_bytes": nbytes, "avg_launch_ms": ms}


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
    f = width); tile size, blend schedule and sort block from the autotuner
    (or --batched-tile and its options); the step timed eagerly and as a
    captured graph replayed (synchronisation-free forward, device step count)."""
    import paper_2602_09999_amd as P
    from paper_2602_09999_amd import _lib as L
    from paper_2602_09999_amd import binding as B
    from paper_2602_09999_amd.autotune import Autotuner, settings_for
    scene = S.batch_scene(BATCH_N, seed=args.seed)
    cams = S.uniform_sphere_cameras(BATCH_VIEWS, seed=args.seed)
    params = {k: v.to(dev) for k, v in scene.items()}
    del scene
    if args.batched_tile:
        config = {"tile": args.batched_tile, "schedule": args.batched_schedule, "sort_block": args.batched_sort_block}
        tune_ms = None
    else:
        tuner = Autotuner(reps=2)
        config = tuner.choose(params, cams)
        tune_ms = next(iter(tuner.cache.values()))["ms"]
    tile = config["tile"]
    st = settings_for(config)
    npix = sum(B.view_pixels(cams))
    target = torch.rand(3 * npix, generator=torch.Generator().manual_seed(args.seed)).to(dev)
    dl = torch.empty(3 * npix, device=dev)
    out = {"workload": f"{BATCH_N} Gaussians, {BATCH_VIEWS} views on a radius-5 sphere, "
                       f"{npix} pixels in all", "tile": tile, "schedule": config["schedule"],
           "sort_block": config["sort_block"], "autotune_ms_per_fwd_bwd": tune_ms}
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
        if not graph:
            out["roofline"] = adam_roofline(step, params)
        out[f"{mode_name}_ms_per_step"] = sec * 1e3
        out[f"{mode_name}_steps_per_s"] = 1.0 / sec
        out[f"{mode_name}_views_per_s"] = BATCH_VIEWS / sec
        log(f"batched {mode_name}: {sec * 1e3:.2f} ms per step of {BATCH_VIEWS} views (tile {tile}, "
            f"{config['schedule']} schedule, sort blocks of {config['sort_block']})")
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
    roof = adam_roofline(step, params)
    log(f"dynamic: {sec * 1e3:.2f} ms per step of {DYN_STEPS} timesteps; k_adam {roof['avg_launch_ms']:.3f} ms "
        f"({roof['frac']:.2f} of HBM peak)")
    return {"workload": f"{DYN_N} dynamic Gaussians, {DYN_STEPS} timesteps, 1280x720, bf16 SH",
            "ms_per_step": sec * 1e3, "steps_per_s": 1.0 / sec, "timesteps_per_s": DYN_STEPS / sec,
            "instances": br.last_stats["n_instances"], "roofline": roof}


def run_dynamic_conditional(args, dev):
    """Conditional 4D Gaussians (Sec. 3.4) at the dynamic workload's shape: 1M
    Gaussians with a time mean, a temporal scale and a right quaternion, 8
    timesteps t = k/7 at 1280x720 rendered as their conditional 3D Gaussians,
    bfloat16 SH; the backward yields the 4D parameters' gradients and Adam
    updates all of them."""
    import paper_2602_09999_amd as P
    from paper_2602_09999_amd import binding as B
    scene = S.make_scene(DYN_N, seed=args.seed)
    scene.update(S.make_cond4d(scene, seed=args.seed))
    params = {k: v.to(dev) for k, v in scene.items()}
    del scene
    for k in ("sh_dc", "sh_rest"):
        params[k] = params[k].bfloat16().contiguous()
    cam = S.identity_camera(1280, 720, 1000.0)
    times = S.timesteps(DYN_STEPS)
    br = B.BatchRasterizer([cam] * DYN_STEPS, times=times)
    lrs = dict(S.ADAM_LR, mean_t=S.ADAM_LR["means"], log_scale_t=S.ADAM_LR["log_scales"], quats_r=S.ADAM_LR["quats"])
    opt = P.FusedAdam(params, lrs)
    npix = sum(B.view_pixels([cam] * DYN_STEPS))
    target = torch.rand(3 * npix, generator=torch.Generator().manual_seed(args.seed + 2)).to(dev)
    dl = torch.empty(3 * npix, device=dev)
    grads = {k: torch.empty_like(v) for k, v in params.items()}
    step = batched_step_fn(br, params, opt, target, dl, grads, 0)
    sec = time_steps(step, max(3, args.steps // 5), 2)
    roof = adam_roofline(step, params)
    log(f"dynamic (conditional 4D): {sec * 1e3:.2f} ms per step of {DYN_STEPS} timesteps; k_adam "
        f"{roof['avg_launch_ms']:.3f} ms ({roof['frac']:.2f} of HBM peak)")
    return {"workload": f"{DYN_N} conditional 4D Gaussians, {DYN_STEPS} timesteps, 1280x720, bf16 SH",
            "ms_per_step": sec * 1e3, "steps_per_s": 1.0 / sec, "timesteps_per_s": DYN_STEPS / sec,
            "instances": br.last_stats["n_instances"], "roofline": roof}


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
    if args.form != "step":
        dev = torch.device("cuda", 0)
        run = {"batched": run_batched, "dynamic": run_dynamic, "conditional": run_dynamic_conditional}[args.form]
        print(json.dumps({"form": args.form, args.form: run(args, dev)}))
        return
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
    # the backward rasterizer alone (blend backward + preprocess backward, no
    # Adam): the separate backward phase of an unfused variant
    bwd_r = None
    unf = next((v for v in results if not results[v]["fused"]), None)
    if unf is not None:
        ru = results[unf]
        b_blend = bwd_blend
        b_pre = algorithmic_bytes(n, counts["n_touched"], counts["i_proc"], pixels)["pre_bwd"]
        if ru["sh_bf16"]:
            b_pre -= n * 48 * 2  # bfloat16 SH gradients: 2 instead of 4 bytes
        ms_b = ru["phase_ms"]["backward"]
        bwd_r = {"variant": unf, "algorithmic_bytes": b_blend + b_pre, "ms": ms_b,
                 "achieved": (b_blend + b_pre) / (ms_b * 1e-3) / 1e9, "unit": "GB/s",
                 "frac": (b_blend + b_pre) / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS,
                 "covers": "accumulator clear + k_blend_bwd + k_preprocess_bwd (the separate backward call)",
                 "kernels": {}}
        for st_name, kb in (("blend_backward", b_blend), ("preprocess_backward", b_pre)):
            t = ru["stage_ms"].get(st_name)
            if t:
                bwd_r["kernels"][st_name] = {"ms": t, "algorithmic_bytes": kb, "GB_per_s": kb / (t * 1e-3) / 1e9,
                                             "hbm_frac": kb / (t * 1e-3) / 1e9 / HBM_PEAK_GBS}
        # the blend backward is bound by instruction issue and atomics, not HBM
        cnt = measured_counters(args.traffic_json, "k_blend_bwd<16>", args.workload)
        t = ru["stage_ms"].get("blend_backward")
        if cnt and t and "blend_backward" in bwd_r["kernels"]:
            kk = bwd_r["kernels"]["blend_backward"]
            if cnt.get("valu_insts_per_launch"):
                peak = VALU_WAVE_INSTS_PER_S
                kk["valu"] = {"insts_per_launch": cnt["valu_insts_per_launch"],
                              "achieved_insts_per_s": cnt["valu_insts_per_launch"] / (t * 1e-3),
                              "peak_insts_per_s": peak,
                              "frac": cnt["valu_insts_per_launch"] / (t * 1e-3) / peak}
            if cnt.get("atomics_per_launch"):
                kk["atomics"] = {"per_launch": cnt["atomics_per_launch"],
                                 "per_s": cnt["atomics_per_launch"] / (t * 1e-3)}
    variants = {}
    for v, r in results.items():
        kb = fused_bytes(n, counts["n_touched"], r["sh_bf16"])["adam"] if r["fused"] else adam_bytes(n, r["sh_bf16"])
        variants[v] = {"steps_per_s": r["steps_per_s"], "ms_per_step": r["ms_per_step"], "phase_ms": r["phase_ms"],
                       "sh": "bf16" if r["sh_bf16"] else "f32", "backward_fused_with_adam": r["fused"],
                       "zorder_layout": r["zorder"], "forward_host_sync": r["host_sync"],
                       "timed_kernel": {"name": r["kernel"], "avg_launch_ms": r["kernel_ms"],
                                        "algorithmic_bytes": kb,
                                        "GB_per_s": kb / (r["kernel_ms"] * 1e-3) / 1e9},
                       "step_ms": r["step_ms"], "stage_ms": r["stage_ms"]}
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
        "step_ms": hr["step_ms"],
        "bwd_rasterizer": bwd_r,
        "phase_ms": hr["phase_ms"],
        "stage_ms": hr["stage_ms"],
        "zorder": None if hr["zorder_ms"] is None else {
            "layout_ms": hr["zorder_ms"], "every_iterations": ZORDER_EVERY,
            "amortized_ms_per_step": hr["zorder_ms"] / ZORDER_EVERY,
            "covers": "Morton permutation of the means + gather of all parameters and both Adam moments"},
        "variants": variants,
    }
    extra = {}
    for wl in [x for x in args.extra_workloads.split(",") if x and x != args.workload]:
        if wl not in S.WORKLOADS:
            raise SystemExit(f"unknown workload {wl}")
        we = S.WORKLOADS[wl]
        sc_e = S.make_scene(we.n, seed=args.seed)
        tg_e = S.make_target(we.height, we.width, seed=args.seed).to(dev)
        re = run_variant(head, argparse.Namespace(**dict(vars(args), split_reps=0)), sc_e,
                         S.workload_camera(wl), tg_e, dev, we)
        ce = workload_counts(re, we, dev)
        kb = (fused_bytes(we.n, ce["n_touched"], re["sh_bf16"])["adam"] if re["fused"]
              else adam_bytes(we.n, re["sh_bf16"]))
        extra[wl] = {"workload": we.description, "variant": head, "steps_per_s": re["steps_per_s"],
                     "ms_per_step": re["ms_per_step"], "step_ms": re["step_ms"], "phase_ms": re["phase_ms"],
                     "visible": ce["visible"], "instances": ce["instances"], "instances_walked": ce["i_proc"],
                     "roofline": {"bound": "hbm", "kernel": re["kernel"],
                                  "achieved": kb / (re["kernel_ms"] * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                                  "unit": "GB/s", "frac": kb / (re["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                  "algorithmic_bytes": kb, "avg_launch_ms": re["kernel_ms"]}}
        del sc_e, tg_e, re
        torch.cuda.empty_cache()
    if extra:
        out["other_workloads"] = extra
    if not args.no_batched:
        out["batched"] = run_batched(args, dev)
        torch.cuda.empty_cache()
    if not args.no_dynamic:
        out["dynamic"] = run_dynamic(args, dev)
        torch.cuda.empty_cache()
        out["dynamic_conditional"] = run_dynamic_conditional(args, dev)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        with_bf16 = any(results[v]["sh_bf16"] for v in results)
        out["cpu_baseline"], refs = cpu_baseline(args.workload, args.seed, scene, with_bf16)
        if not args.no_oracle_error:
            # the GPU results on the crops the oracle just rendered
            out["oracle_error"] = {
                "covers": (f"64x64 crops {CROPS[args.workload]} of the {args.workload} frame; per SH form: "
                           "image and T (borderline pixels excluded), the gradients of the separate backward, "
                           "and the parameter update of the backward fused with Adam; z-ordered layout, "
                           "forward without host synchronisation (the timed configuration)"),
                "results": oracle_errors(refs, scene, args.workload, dev, with_bf16)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
