#!/usr/bin/env python3
"""Throughput of the per-frame stitching path on one MI355X.

Workload (default): four 1920x1080 RGB uint8 cameras -> 6400x1080 panorama, 6 pyramid
levels, a 30-frame sequence with per-frame noise and fixed homographies.  One step
stitches the whole 30-frame sequence (30 stitch_frame calls: fused warp + Laplacian
pyramids + seam-weight pyramids + blend + collapse per frame) with every input
already resident in HBM and a distinct output buffer per frame.

Prints ONE JSON line: panorama Mpx/s for the step, the HBM roofline of the dominant
kernel (algorithmic bytes per launch / average launch time from HIP events recorded
between launches inside the timed region), and the CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

import numpy as np  # noqa: E402
import torch  # noqa: E402

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
METRIC = "panorama Mpx/s (warp+multi-band blend), batched/FP16 vs plain, % HBM roofline"


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--frames", type=int, default=30, help="frames per step (the sequence length)")
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c4"])
    ap.add_argument("--storage", default="f32", choices=["f32", "f16"])
    ap.add_argument("--forms", default="f16,batched_f32,batched_f16",
                    help="extra forms timed after the headline (comma list or 'none')")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-events", action="store_true",
                    help="time the step without per-launch events (roofline then omitted)")
    return ap.parse_args()


def rig_for(name):
    import workloads as wl
    return {"c1": wl.rig_c1, "c2": wl.rig_c2, "c4": wl.rig_c4}[name]()


def workload_name(rig, frames):
    fw, fh = rig.frame_sizes[0]
    return (f"{rig.name}: {rig.n}x{fw}x{fh} RGB u8 -> {rig.canvas_w}x{rig.canvas_h} canvas, "
            f"{rig.levels} levels, {frames}-frame sequence")


def source_pixels_in(rig, i, roi):
    """Source pixels of camera i whose canvas position lies inside roi (x, y, w, h)."""
    (w, h), H = rig.frame_sizes[i], rig.H[i]
    n = 0
    for y0 in range(0, h, 256):
        ys, xs = np.mgrid[y0:min(h, y0 + 256), 0:w].astype(np.float64)
        z = H[2, 0] * xs + H[2, 1] * ys + H[2, 2]
        X = (H[0, 0] * xs + H[0, 1] * ys + H[0, 2]) / z
        Y = (H[1, 0] * xs + H[1, 1] * ys + H[1, 2]) / z
        n += int(np.count_nonzero((X >= roi[0] - 1) & (X < roi[0] + roi[2]) & (Y >= roi[1] - 1)
                                  & (Y < roi[1] + roi[3])))
    return n


def algorithmic_bytes(plan, rig, s, keep_r0=False):
    """Compulsory HBM bytes per launch of each kernel kind, from the plan's stored regions
    (G and weight levels on each camera's ROI, Laplacian bands on the seam-weight support,
    R levels on the whole canvas), s = bytes per stored sample."""
    L, n = rig.levels, rig.n
    area = lambda r: r[2] * r[3]
    reg = [[plan.regions(i, k) for k in range(L)] for i in range(n)]
    dims = [((rig.canvas_h + (1 << k) - 1) >> k, (rig.canvas_w + (1 << k) - 1) >> k) for k in range(L)]
    C = [a * b for a, b in dims]
    out = {}
    if L > 1:
        b0 = 0
        for i in range(n):
            roi0, band0 = reg[i][0]
            roi1, _ = reg[i][1]
            if area(roi0) == 0:
                continue
            b0 += 3 * source_pixels_in(rig, i, roi0) + area(roi0)          # frame + u8 weights
            b0 += 3 * s * area(band0) + 4 * s * area(roi1)                   # L_0; G_1 and Gm_1
        out["warp_level0_pass"] = [b0]
        lv = []
        for k in range(1, L - 1):
            b = 0
            for i in range(n):
                roi, band = reg[i][k]
                roi1, _ = reg[i][k + 1]
                b += 4 * s * area(roi) + 3 * s * area(band) + 4 * s * area(roi1)
            lv.append(b)
        if lv:
            out["level_pass"] = lv
        mids = []
        for k in range(L - 1, -1, -1):
            bands = sum(area(reg[i][k][1]) for i in range(n))
            wbytes = 1 if k == 0 else s
            b = (3 * s + wbytes) * bands
            if k + 1 < L:
                b += 3 * s * C[k + 1]
            if k == 0:
                b += 3 * C[0] + (3 * s * C[0] if keep_r0 else 0)
                out["blend_level0"] = [b]
            elif k == L - 1:
                out["blend_top"] = [b + 3 * s * C[k]]
            else:
                mids.append(b + 3 * s * C[k])
        if mids:
            out["blend_middle"] = mids
    return out


def make_frames(rig, nframes, device):
    import workloads as wl
    return wl.render_rig_sequence(rig, range(nframes), device)


def time_form(rig, frames, storage, steps, warmup, kernel_events=True):
    import paper_1810_03988_amd as P
    dev = frames[0][0].device
    plan = P.Plan(rig.frame_sizes, rig.H, rig.masks(), rig.canvas_w, rig.canvas_h, rig.levels, storage=storage,
                  device=dev)
    panos = [torch.empty((rig.canvas_h, rig.canvas_w, 3), dtype=torch.uint8, device=dev) for _ in frames]
    args = [plan.frame_args(f, p) for f, p in zip(frames, panos)]
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream

    def step():
        for a in args:
            plan.frame_raw(a, sh)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    if kernel_events:
        plan.set_timing(True)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(steps):
        step()
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    timing = plan.read_timing() if kernel_events else {}
    plan.set_timing(False)
    return plan, ms, timing, panos


def time_batched(rig, frames, storage, steps, warmup, tune_cache=None):
    """All frames of the sequence as jobs of one batch (one plan per job), captured once
    into a HIP graph and replayed per step."""
    import paper_1810_03988_amd as P
    dev = frames[0][0].device
    plans = [P.Plan(rig.frame_sizes, rig.H, rig.masks(), rig.canvas_w, rig.canvas_h, rig.levels, storage=storage,
                    device=dev) for _ in frames]
    panos = [torch.empty((rig.canvas_h, rig.canvas_w, 3), dtype=torch.uint8, device=dev) for _ in frames]
    batch = P.Batch(plans, device=dev)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        cfg = batch.autotune(frames, panos, stream=stream, cache_path=tune_cache)
        args = batch.args(frames, panos)
        sh = stream.cuda_stream
        for _ in range(warmup):
            batch.run_raw(args, sh)
        stream.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(steps):
            batch.run_raw(args, sh)
        t1.record(stream)
        stream.synchronize()
    ms = t0.elapsed_time(t1) / steps
    return ms, cfg, batch, panos


def kernel_table(plan, rig, timing, steps, s):
    alg = algorithmic_bytes(plan, rig, s)
    table = {}
    for kind, (tot_ms, launches) in timing.items():
        per_launch = alg.get(kind)
        if not per_launch:
            continue
        # every frame launches each level once: average the per-launch bytes the same way
        avg_bytes = float(np.mean(per_launch))
        avg_s = tot_ms / launches / 1e3
        gbs = avg_bytes / avg_s / 1e9
        table[kind] = {"launches_per_step": launches // steps, "avg_us": round(avg_s * 1e6, 3),
                       "alg_bytes_per_launch": int(avg_bytes), "achieved_GBs": round(gbs, 1),
                       "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                       "ms_per_step": round(tot_ms / steps, 4)}
    return table


def cpu_baseline(rig, frames0):
    """The oracle as it stands, on a bounded sample: the full-height column window
    [1248, 1888) of frame 0 (spans the first seam), all levels through their cones."""
    import oracle
    fr = [f.cpu().numpy() for f in frames0]
    x0, x1 = 1248, 1888
    if rig.canvas_w < x1:
        x0, x1 = 0, rig.canvas_w
    so = oracle.StitchOracle(fr, rig.H, rig.masks(), rig.canvas_w, rig.canvas_h, rig.levels)
    t = time.perf_counter()
    so.panorama(np.arange(rig.canvas_h), np.arange(x0, x1))
    dt = time.perf_counter() - t
    px = rig.canvas_h * (x1 - x0)
    return {"value": round(px / dt / 1e6, 5), "unit": "Mpx/s", "cores": 1, "kind": "oracle",
            "sample": f"frame 0, canvas columns [{x0},{x1}) x all {rig.canvas_h} rows ({px / 1e6:.3f} Mpx) "
                      f"through every level, FP64 numpy, one thread, {dt:.1f} s",
            "cpu": platform.processor() or platform.machine(), "numpy": np.__version__}


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py: this build measures one GPU; --gpus {a.gpus} is not supported "
              "(independent frames and jobs would shard round-robin across GPUs with no exchange)",
              file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    rig = rig_for(a.config)
    t = time.perf_counter()
    frames = make_frames(rig, a.frames, "cuda")
    torch.cuda.synchronize()
    print(f"# generated {a.frames} x {rig.n} frames in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    s = 2 if a.storage == "f16" else 4
    plan, ms, timing, _ = time_form(rig, frames, a.storage, a.steps, a.warmup, not a.no_kernel_events)
    ms_plain = time_form(rig, frames, a.storage, a.steps, a.warmup, False)[1] if timing else ms
    px_per_step = rig.canvas_w * rig.canvas_h * a.frames
    value = px_per_step / (ms / 1e3) / 1e6
    print(f"# {a.storage}: {ms:.3f} ms/step, {value:.0f} Mpx/s", file=sys.stderr, flush=True)
    kernels = kernel_table(plan, rig, timing, a.steps, s) if timing else {}
    for k, v in kernels.items():
        print(f"#   {k:18s} {v['avg_us']:9.2f} us/launch x{v['launches_per_step']:4d}  "
              f"{v['alg_bytes_per_launch'] / 1e6:8.2f} MB  {v['achieved_GBs']:8.1f} GB/s", file=sys.stderr, flush=True)
    roof = None
    if kernels:
        dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
        kd = kernels[dom]
        roof = {"bound": "hbm", "achieved": kd["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(kd["achieved_GBs"] / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom}
    forms = {f"plain_{a.storage}": {"Mpx_s": round(value, 1), "ms_per_step": round(ms, 4),
                                    "ms_per_step_without_launch_events": round(ms_plain, 4)}}
    for form in [f for f in a.forms.split(",") if f and f != "none" and f != a.storage]:
        if form.startswith("batched_"):
            st = form.split("_", 1)[1]
            bms, cfg, _b, _p = time_batched(rig, frames, st, a.steps, a.warmup,
                                            tune_cache=os.environ.get("STITCH_TUNE_CACHE"))
            bval = px_per_step / (bms / 1e3) / 1e6
            forms[form] = {"Mpx_s": round(bval, 1), "ms_per_step": round(bms, 4),
                           "wg_per_cu_by_level": cfg[:rig.levels - 1],
                           "how": f"{a.frames} jobs (one per frame) in one batch, one HIP graph replay per step"}
            print(f"# {form}: {bms:.3f} ms/step, {bval:.0f} Mpx/s (tuned wg/CU {cfg[:rig.levels - 1]})",
                  file=sys.stderr, flush=True)
            del _b, _p
            continue
        fplan, fms, ftim, _panos = time_form(rig, frames, form, a.steps, a.warmup, True)
        fval = px_per_step / (fms / 1e3) / 1e6
        fk = kernel_table(fplan, rig, ftim, a.steps, 2 if form == "f16" else 4)
        forms[f"plain_{form}"] = {"Mpx_s": round(fval, 1), "ms_per_step": round(fms, 4),
                                  "kernels": fk}
        print(f"# {form}: {fms:.3f} ms/step, {fval:.0f} Mpx/s", file=sys.stderr, flush=True)
    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(rig, frames[0])
        print(f"# cpu oracle: {cpu['value']} Mpx/s", file=sys.stderr, flush=True)
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mpx/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if a.storage == "f32" else "f32 (f16 storage)", "data": "synthetic",
        "config": {"workload": workload_name(rig, a.frames), "form": f"plain, {a.storage} storage, one "
                   "stitch_frame per frame", "frames_per_step": a.frames, "cameras": rig.n,
                   "canvas": [rig.canvas_w, rig.canvas_h], "levels": rig.levels},
        "roofline": roof, "cpu_baseline": cpu, "kernels": kernels, "forms": forms,
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
