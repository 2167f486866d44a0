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
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3", "c4", "c5"],
                    help="c3 (default): 64 jobs of 2-6 cameras, one frame set each, batched against one by one; "
                         "c2/c4: one rig's frame sequence; c5: the adjoint's refinement report over 16 pairs")
    ap.add_argument("--jobs", type=int, default=64, help="jobs of the c3 batch")
    ap.add_argument("--profile-form", choices=["f16", "f32"],
                    help="c3 under a profiler: only the batched form of this storage, one sequence (no groups), "
                         "no plain forms, no CPU baseline")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16"])
    ap.add_argument("--form", default="batched", choices=["batched", "plain"],
                    help="the headline form: all frames of the step as one batch, or one stitch_frame per frame")
    ap.add_argument("--forms", default="batched_graph_f16,plain_f32,plain_f16,pipe_f32,lorb,register",
                    help="extra forms timed after the headline (comma list of batched_graph_<s> / plain_<s> / "
                         "pipe_<s>, the last end to end through PCIe, lorb (the feature-extraction front "
                         "end on the same frames), register (L-ORB, matching and PROSAC of the rig's "
                         "neighbouring pairs), or 'none')")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-events", action="store_true",
                    help="time the step without per-launch events (roofline then omitted)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the forms, run a plain float32 copy kernel (y = -x) over this many MiB, "
                         "three times: the reference for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE")
    ap.add_argument("--precision", action="store_true",
                    help="instead of timing: error of the FP32- and FP16-storage paths against the FP64 "
                         "oracle per level (on windows through their dependency cones) and on the uint8 "
                         "output, and FP16 against FP32 on the whole canvas; prints one JSON line")
    ap.add_argument("--windows", type=int, default=8, help="oracle windows for --precision")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print the HBM traffic summary of two rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE) "
                         "taken with --copy-calibration-mib 512, then exit")
    ap.add_argument("--rocprof-summary", metavar="DIR",
                    help="summarise the rocprofv3 CSV output under DIR (kernel stats and counters per "
                         "kernel) and exit; needs no GPU")
    return ap.parse_args()


# rocprofv3 kernel names of the path -> the kinds this script reports
KERNEL_KINDS = {
    "k_pyr<float, true, true>": "warp_level0_pass (f32)", "k_pyr<float, true, false>": "level_pass (f32)",
    "k_pyr<_Float16, true, true>": "warp_level0_pass (f16)", "k_pyr<_Float16, true, false>": "level_pass (f16)",
    "k_blend<float, true, true>": "blend_level0 (f32)", "k_blend<float, false, true>": "blend_middle/top (f32)",
    "k_blend<_Float16, true, true>": "blend_level0 (f16)", "k_blend<_Float16, false, true>": "blend_middle/top (f16)",
    "k_blend<float, true, false>": "blend_level0, batched (f32)",
    "k_blend<float, false, false>": "blend_middle/top, batched (f32)",
    "k_blend<_Float16, true, false>": "blend_level0, batched (f16)",
    "k_blend<_Float16, false, false>": "blend_middle/top, batched (f16)",
    "k_lorb_clear": "L-ORB clear", "k_lorb_detect": "L-ORB detect (FAST, R, suppression)",
    "k_lorb_select": "L-ORB select (histogram threshold)", "k_lorb_rank": "L-ORB rank",
    "k_lorb_brief": "L-ORB BRIEF",
    "k_lsh_keys": "LSH keys", "k_lsh_match": "LSH matching", "k_prosac_prepare": "PROSAC order + growth",
    "k_prosac_hyp": "PROSAC hypotheses", "k_prosac_final": "PROSAC best + refit",
    "k_lsh_keys_multi": "LSH keys, all pairs", "k_lsh_match_multi": "LSH matching, all pairs",
    "k_prosac_prepare_multi": "PROSAC order + growth, all pairs", "k_prosac_hyp_multi": "PROSAC hyps, all pairs",
    "k_prosac_final_multi": "PROSAC best + refit, all pairs",
}
COPY_KERNEL_HINT = "neg"


def _short_kernel(name: str) -> str:
    import re
    name = name.replace("(anonymous namespace)::", "")
    m = re.search(r"(k_[a-z_]+)<([^()]*)>", name)
    if m:
        return m.group(1) + "<" + m.group(2) + ">"
    # mangled names (as some rocprofv3 builds report them): this library's kernels
    m = re.search(r"\d+(k_[a-z_]+?)I(DF16_|f)Lb([01])ELb([01])E", name)
    if m:
        t = "_Float16" if m.group(2) == "DF16_" else "float"
        b = lambda v: "true" if v == "1" else "false"
        return f"{m.group(1)}<{t}, {b(m.group(3))}, {b(m.group(4))}>"
    m = re.search(r"_GLOBAL__N_1\d+(k_[a-z0-9_]+?)E", name)
    if m:
        return m.group(1)
    return name.split("(")[0][-90:]


def rocprof_summary(root: str) -> None:
    """Per-kernel figures from rocprofv3 CSV files: average durations from the kernel
    trace, and per-dispatch averages of every collected counter.  FETCH_SIZE / WRITE_SIZE
    (KiB per dispatch) are also scaled by what they read for the calibration copy kernel
    (y = -x over a known number of bytes), when it is in the same run."""
    import csv
    import glob
    from collections import defaultdict
    files = sorted(glob.glob(os.path.join(root, "**", "*.csv"), recursive=True))
    for f in files:
        if f.endswith("kernel_trace.csv"):
            dur = defaultdict(list)
            with open(f) as fh:
                for row in csv.DictReader(fh):
                    dur[_short_kernel(row["Kernel_Name"])].append(
                        (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1e3)
            print(f"## kernel trace ({os.path.relpath(f, root)}): average duration per kernel")
            print(f"{'kernel':44s} {'kind':34s} {'calls':>6s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s}")
            for k, v in sorted(dur.items(), key=lambda kv: -sum(kv[1])):
                print(f"{k:44s} {KERNEL_KINDS.get(k, ''):34s} {len(v):6d} {np.mean(v):9.2f} {np.min(v):9.2f} "
                      f"{np.max(v):9.2f}")
        elif f.endswith("counter_collection.csv"):
            agg = defaultdict(lambda: defaultdict(float))
            disp = defaultdict(set)
            with open(f) as fh:
                for row in csv.DictReader(fh):
                    k = _short_kernel(row["Kernel_Name"])
                    agg[k][row["Counter_Name"]] += float(row["Counter_Value"])
                    disp[k].add(row["Dispatch_Id"])
            print(f"## counters ({os.path.relpath(f, root)}): average per dispatch")
            copy = [k for k in agg if COPY_KERNEL_HINT in k]
            for k, d in sorted(agg.items()):
                n = max(1, len(disp[k]))
                print(f"{k:44s} {KERNEL_KINDS.get(k, ''):34s} n={n:5d} " +
                      " ".join(f"{c}={v / n:.6g}" for c, v in sorted(d.items())))
            if copy:
                k = copy[0]
                n = max(1, len(disp[k]))
                print(f"# calibration kernel: {k} ({n} dispatches)")
                for c, v in sorted(agg[k].items()):
                    print(f"#   {c} reads {v / n:.6g} KiB per dispatch")
        elif f.endswith("kernel_stats.csv"):
            print(f"## kernel stats ({os.path.relpath(f, root)})")
            with open(f) as fh:
                for row in csv.DictReader(fh):
                    print(f"{_short_kernel(row['Name']):44s} calls={row['Calls']:>6s} "
                          f"avg_ns={float(row['AverageNs']):12.1f} total_ns={float(row['TotalDurationNs']):14.1f} "
                          f"pct={float(row['Percentage']):6.2f}")


def traffic_summary(fetch_dir: str, write_dir: str) -> None:
    """The body of a profiles/hbm_traffic_*.txt file from two rocprofv3 counter runs of the
    same command (FETCH_SIZE in one, WRITE_SIZE in the other, each with the calibration copy
    kernel): the source hash the figures belong to, the calibration, the raw per-dispatch
    averages, and one line per kernel: traffic <kind> <kernel> <HBM bytes per dispatch>."""
    import csv
    import glob
    from collections import defaultdict
    raw = defaultdict(dict)
    scale = {}
    for ctr, root in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        agg, disp = defaultdict(float), defaultdict(set)
        for f in glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for row in csv.DictReader(fh):
                    if row["Counter_Name"] != ctr:
                        continue
                    k = _short_kernel(row["Kernel_Name"])
                    agg[k] += float(row["Counter_Value"])
                    disp[k].add(row["Dispatch_Id"])
        copy = [k for k in agg if COPY_KERNEL_HINT in k]
        if not copy:
            raise SystemExit(f"no calibration kernel in {root}")
        c = agg[copy[0]] / len(disp[copy[0]])
        scale[ctr] = (c, COPY_MIB * 1024 / c)
        for k in agg:
            if COPY_KERNEL_HINT not in k:
                raw[k][ctr] = (agg[k] / len(disp[k]), len(disp[k]))
    print(f"# source sha256: {source_hash()}   (code of kernels.hip + stitch_api.cpp: comments and whitespace "
          f"removed, see bench.source_hash)")
    print(f"# Calibration: the copy kernel y = -x over {COPY_MIB} MiB float32 reads and writes {COPY_MIB * 1024} KiB "
          f"per dispatch;")
    print(f"#   FETCH_SIZE reads {scale['FETCH_SIZE'][0]:.0f} KiB, WRITE_SIZE reads {scale['WRITE_SIZE'][0]:.0f} KiB "
          f"for it")
    print(f"# scale factors: FETCH_SIZE x {scale['FETCH_SIZE'][1]:.3f}, WRITE_SIZE x {scale['WRITE_SIZE'][1]:.3f}")
    print("#")
    print("# raw counters (KiB per dispatch, averaged over the dispatches of each kernel):")
    for k in sorted(raw):
        f_, w_ = raw[k].get("FETCH_SIZE", (0.0, 0)), raw[k].get("WRITE_SIZE", (0.0, 0))
        print(f"#   {k:34s} {KERNEL_KINDS.get(k, ''):34s} n={f_[1]:4d} FETCH_SIZE={f_[0]:.6g} WRITE_SIZE={w_[0]:.6g}")
    print("#")
    print("# scaled HBM bytes per dispatch (x 1024):")
    for k in sorted(raw):
        kind = KERNEL_KINDS.get(k, "").split(" (")[0].split(",")[0]
        if not kind or "FETCH_SIZE" not in raw[k] or "WRITE_SIZE" not in raw[k]:
            continue
        b = (raw[k]["FETCH_SIZE"][0] * scale["FETCH_SIZE"][1] + raw[k]["WRITE_SIZE"][0] * scale["WRITE_SIZE"][1]) * 1024
        print(f"traffic {kind:18s} {k:34s} {int(round(b))}")


COPY_MIB = 512


def _window_list(rig, n, win):
    """Level-0 window origins: seam columns, canvas corners and edges, interior points."""
    W, H = rig.canvas_w, rig.canvas_h
    cand = [(H // 2 - win // 2, x - win // 2) for x in rig.seams]
    cand += [(0, 0), (H - win, W - win), (0, W - win), (H - win, 0), (H // 3, W // 5), (2 * H // 3, 3 * W // 5),
             (H // 2, W // 2 + 7), (5, W // 3)]
    out = []
    for y, x in cand:
        y, x = min(max(y, 0), H - win), min(max(x, 0), W - win)
        if (y, x) not in out:
            out.append((y, x))
    return out[:n]


def precision_report(rig, nwin: int = 8, win: int = 32, full: bool = False) -> dict:
    """Max / mean |delta| of R_k and of every stored band L_k against the FP64 oracle, per
    level, for FP32 and FP16 storage; uint8 output |delta| histograms against the oracle
    (on the windows) and of FP16 against FP32 (whole canvas)."""
    import oracle
    import paper_1810_03988_amd as P
    import workloads as wl
    frames_d = wl.render_rig_frames(rig, frame=0, device="cuda")
    frames = [f.cpu().numpy() for f in frames_d]
    masks = rig.masks()
    so = oracle.StitchOracle(frames, rig.H, masks, rig.canvas_w, rig.canvas_h, rig.levels)
    L = rig.levels
    wins = [(0, 0)] if full else _window_list(rig, nwin, win)
    wsz = (rig.canvas_h, rig.canvas_w) if full else (win, win)

    def level_window(k, y, x):
        hk, wk = so.dims[k]
        r0, c0 = y >> k, x >> k
        r1 = min(hk, -(-(y + wsz[0]) // (1 << k)))
        c1 = min(wk, -(-(x + wsz[1]) // (1 << k)))
        return np.arange(r0, r1), np.arange(c0, c1)

    # oracle values on the windows, once
    want_R = [[None] * len(wins) for _ in range(L)]
    want_L = [[[None] * len(wins) for _ in range(L)] for _ in range(rig.n)]
    want_u8 = []
    plan32 = P.Plan(rig.frame_sizes, rig.H, masks, rig.canvas_w, rig.canvas_h, L, storage="f32", keep_r0=True)
    bands = [[plan32.regions(i, k)[1] for k in range(L)] for i in range(rig.n)]
    t = time.perf_counter()
    for j, (y, x) in enumerate(wins):
        for k in range(L):
            rows, cols = level_window(k, y, x)
            want_R[k][j] = so.R(k, rows, cols)
            for i in range(rig.n):
                bx, by, bw, bh = bands[i][k]
                rr = rows[(rows >= by) & (rows < by + bh)]
                cc = cols[(cols >= bx) & (cols < bx + bw)]
                if len(rr) and len(cc):
                    want_L[i][k][j] = (rr, cc, so.Lap(i, k, rr, cc))
        want_u8.append(oracle.quantise(want_R[0][j]))          # HWC uint8
        so.clear()
    oracle_s = time.perf_counter() - t

    def hist(d):
        v, c = np.unique(np.abs(d.astype(np.int64)), return_counts=True)
        return {int(a): int(b) for a, b in zip(v, c)}

    report = {"workload": workload_name(rig, 1), "windows": [list(w) for w in wins], "window": list(wsz),
              "oracle_seconds": round(oracle_s, 1)}
    panos = {}
    for storage in ("f32", "f16"):
        plan = plan32 if storage == "f32" else P.Plan(rig.frame_sizes, rig.H, masks, rig.canvas_w, rig.canvas_h, L,
                                                      storage="f16", keep_r0=True)
        pano = plan.frame(frames_d)
        torch.cuda.synchronize()
        panos[storage] = pano.cpu().numpy()
        levels = []
        for k in range(L):
            r, _ = plan.view("r", 0, k)
            if r is None:
                continue
            r = r.float().cpu().numpy()
            dR = np.concatenate([np.abs(r[:, rows[:, None], cols[None, :]] - want_R[k][j]).ravel()
                                 for j, (rows, cols) in enumerate(level_window(k, y, x) for y, x in wins)])
            dL = []
            for i in range(rig.n):
                lap, (ox, oy) = plan.view("lap", i, k)
                if lap is None:
                    continue
                lap = lap.float().cpu().numpy()
                for j in range(len(wins)):
                    if want_L[i][k][j] is None:
                        continue
                    rr, cc, wv = want_L[i][k][j]
                    dL.append(np.abs(lap[:, rr[:, None] - oy, cc[None, :] - ox] - wv).ravel())
            dL = np.concatenate(dL) if dL else np.zeros(1)
            levels.append({"k": k, "R_max": float(dR.max()), "R_mean": float(dR.mean()),
                           "L_max": float(dL.max()), "L_mean": float(dL.mean()), "R_samples": int(dR.size),
                           "L_samples": int(dL.size)})
        got_u8 = np.concatenate([panos[storage][y:y + wsz[0], x:x + wsz[1]].ravel() for y, x in wins])   # HWC
        want = np.concatenate([w_.ravel() for w_ in want_u8])
        h = hist(got_u8.astype(np.int64) - want)
        report[storage] = {"levels": levels, "u8_vs_oracle_hist": h,
                           "u8_vs_oracle_frac_off": float(1.0 - h.get(0, 0) / want.size)}
        del plan
    h = hist(panos["f16"].astype(np.int64) - panos["f32"])
    report["f16_vs_f32_u8_hist_full_canvas"] = h
    report["f16_vs_f32_u8_frac_off"] = float(1.0 - h.get(0, 0) / panos["f32"].size)
    return report


def copy_calibration(mib: int) -> None:
    """A plain streaming kernel of known traffic: y = -x over mib MiB of float32, three
    dispatches (each reads and writes mib MiB)."""
    n = mib * (1 << 20) // 4
    x = torch.rand(n, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    print(f"# copy calibration: 3 x y = -x over {mib} MiB float32", file=sys.stderr, flush=True)


def rig_for(name):
    import workloads as wl
    return {"c1": wl.rig_c1, "c2": wl.rig_c2, "c4": wl.rig_c4}[name]()


def workload_name(rig, frames):
    fw, fh = rig.frame_sizes[0]
    return (f"{rig.name}: {rig.n}x{fw}x{fh} RGB u8 -> {rig.canvas_w}x{rig.canvas_h} canvas, "
            f"{rig.levels} levels, {frames}-frame sequence")


_SRC_PX = {}


def source_pixels_in(rig, i, roi):
    """Source pixels of camera i whose canvas position lies inside roi (x, y, w, h)."""
    key = (rig.name, i, tuple(roi))
    if key not in _SRC_PX:
        _SRC_PX[key] = _source_pixels_in(rig, i, roi)
    return _SRC_PX[key]


def _source_pixels_in(rig, i, roi):
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


def phase_bytes(plan, rig, s, keep_r0=False):
    """Compulsory HBM bytes of each launch of one frame, from the plan's stored regions (G
    and weight levels on each camera's ROI, Laplacian bands on the seam-weight support, R
    levels on the whole canvas), s = bytes per stored sample.  Keys: "pyr0" (warp + level-0
    pass), "pyr<k>" (pass from level k), "blend<k>" (blend of level k)."""
    L, n = rig.levels, rig.n
    area = lambda r: r[2] * r[3]
    reg = [[plan.regions(i, k) for k in range(L)] for i in range(n)]
    dims = [((rig.canvas_h + (1 << k) - 1) >> k, (rig.canvas_w + (1 << k) - 1) >> k) for k in range(L)]
    C = [a * b for a, b in dims]
    out = {}
    if L < 2:
        return out
    b0 = 0
    for i in range(n):
        roi0, band0 = reg[i][0]
        roi1, _ = reg[i][1]
        if area(roi0) == 0:
            continue
        b0 += 3 * source_pixels_in(rig, i, roi0) + area(roi0)          # frame + u8 weights
        b0 += 3 * s * area(band0) + 4 * s * area(roi1)                   # L_0; G_1 and Gm_1
    out["pyr0"] = b0
    for k in range(1, L - 1):
        b = 0
        for i in range(n):
            roi, band = reg[i][k]
            roi1, _ = reg[i][k + 1]
            b += 4 * s * area(roi) + 3 * s * area(band) + 4 * s * area(roi1)
        out[f"pyr{k}"] = b
    for k in range(L - 1, -1, -1):
        bands = sum(area(reg[i][k][1]) for i in range(n))
        b = (3 * s + (1 if k == 0 else s)) * bands
        if k + 1 < L:
            b += 3 * s * C[k + 1]
        b += 3 * C[0] + (3 * s * C[0] if keep_r0 else 0) if k == 0 else 3 * s * C[k]
        out[f"blend{k}"] = b
    return out


# launch kinds of the plain form's event timing -> the phases each covers
PLAIN_KINDS = {"warp_level0_pass": lambda L: ["pyr0"],
               "level_pass": lambda L: [f"pyr{k}" for k in range(1, L - 1)],
               "blend_level0": lambda L: ["blend0"],
               "blend_middle": lambda L: [f"blend{k}" for k in range(L - 2, 0, -1)],
               "blend_top": lambda L: [f"blend{L - 1}"]}


def phase_name(key):
    """Batch timing kind -> readable phase name."""
    what, k = key
    if what == "pyr":
        return "warp_level0_pass" if k == 0 else f"level_pass_{k}"
    return f"blend_level{k}"


def source_hash() -> str:
    """SHA-256 over the code that decides what a launch does: the kernels and the planner
    (regions, tiles, tables), with comments and whitespace removed (neither source holds a
    comment marker inside a string literal)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in ("kernels.hip", "stitch_api.cpp"):
        text = (ROOT / "paper_1810_03988_amd" / "csrc" / name).read_text()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def profiled_traffic(config: str, form: str, storage: str, kind: str):
    """HBM bytes per launch of one kernel kind from the committed rocprofv3 counter summary
    of this workload (FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel calibration), or
    None when there is none or the kernel or planner source has changed since it was taken."""
    import hashlib
    import re
    f = ROOT / "profiles" / f"hbm_traffic_{config}_{form}_{storage}.txt"
    if not f.exists():
        return None
    text = f.read_text()
    m = re.search(r"source sha256: ([0-9a-f]{64})", text)
    if not m or source_hash() != m.group(1):
        return None
    m = re.search(rf"^traffic {re.escape(kind)}\s+.*?\s(\d+)$", text, re.M)
    return int(m.group(1)) if m else None


def profiled_counters(config: str, form: str, storage: str, kernel: str):
    """The derived per-CU figures (VALU_busy, TD_busy, ...) of one kernel from the committed
    rocprofv3 counter summary of this workload, or None when there is none or the kernel or
    planner source has changed since it was taken."""
    import re
    f = ROOT / "profiles" / f"counters_{config}_{form}_{storage}.txt"
    if not f.exists():
        return None
    text = f.read_text()
    m = re.search(r"source sha256: ([0-9a-f]{64})", text)
    if not m or source_hash() != m.group(1):
        return None
    m = re.search(rf"^{re.escape(kernel)}\n(?:  raw .*\n)?  derived (.*)$", text, re.M)
    if not m:
        return None
    return {k: float(v) for k, v in re.findall(r"([\w/]+)=([0-9.eE+-]+)", m.group(1))}


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


def time_pipe(rig, frames, storage, steps, warmup, depth=3):
    """End to end through the pipelined sequence form: the step's frame sets start in
    pinned host memory and its panoramas end there (PCIe both ways, overlapped with the
    stitching on separate streams).  Wall-clock ms per step."""
    import paper_1810_03988_amd as P
    plan = P.Plan(rig.frame_sizes, rig.H, rig.masks(), rig.canvas_w, rig.canvas_h, rig.levels, storage=storage)
    host = [[f.cpu().pin_memory() for f in fs] for fs in frames]
    panos = [torch.empty((rig.canvas_h, rig.canvas_w, 3), dtype=torch.uint8, pin_memory=True) for _ in frames]
    pipe = P.Pipe(plan, depth)
    for _ in range(warmup):
        pipe.run(host, panos)
    t0 = time.perf_counter()
    for _ in range(steps):
        pipe.run(host, panos)
    ms = (time.perf_counter() - t0) * 1e3 / steps
    pipe.close()
    in_bytes = sum(f.numel() for fs in host for f in fs)
    out_bytes = sum(p.numel() for p in panos)
    return ms, in_bytes, out_bytes


def time_lorb(rig, frames, steps, warmup, n_max=500, nd=256):
    """L-ORB feature extraction (Alg. 1-2) of every camera of a frame set in its pre-aligned
    overlap areas, frames already in HBM: one stitch_lorb call per camera, timed (a) on one
    stream, (b) on one stream with per-launch events (kernel table), (c) with each camera on
    its own stream (default priority), as the paper runs L-ORB on stream queues."""
    import paper_1810_03988_amd as P
    from paper_1810_03988_amd import stitch as S
    import workloads as wl
    areas = P.detection_areas(rig.frame_sizes, rig.H, rig.canvas_w, rig.canvas_h)   # Alg. 2 step 1
    pattern = torch.from_numpy(wl.brief_pattern(nd)).cuda()
    cams = [i for i in range(rig.n) if areas[i]]
    lorbs = {i: P.Lorb(*rig.frame_sizes[i], areas[i], n_max=n_max, nd=nd) for i in cams}
    main = torch.cuda.current_stream()
    streams = {i: torch.cuda.Stream() for i in cams}

    def step(t, per_camera_streams=False):
        for i in cams:
            h = streams[i].cuda_stream if per_camera_streams else main.cuda_stream
            lorbs[i].run_raw(frames[t % len(frames)][i], pattern, h)

    def timed(per_camera_streams):
        for t in range(warmup):
            step(t, per_camera_streams)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(main)
        if per_camera_streams:
            for st in streams.values():
                st.wait_event(e0)
        for t in range(steps):
            step(t, per_camera_streams)
        if per_camera_streams:
            for st in streams.values():
                ev = torch.cuda.Event()
                ev.record(st)
                main.wait_event(ev)
        e1.record(main)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms_one = timed(False)
    ms_multi = timed(True)
    # every camera of the frame set in one stitch_lorb_multi call
    lset = P.LorbSet([rig.frame_sizes[i] for i in cams], [areas[i] for i in cams], n_max=n_max, nd=nd)

    def step_set(t):
        lset.run_raw([frames[t % len(frames)][i] for i in cams], pattern, main.cuda_stream)

    def timed_set():
        for t in range(warmup):
            step_set(t)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(main)
        for t in range(steps):
            step_set(t)
        e1.record(main)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms_set = timed_set()
    # the same call captured once per frame set of the cycle and replayed from HIP graphs
    graphs = []
    side = torch.cuda.Stream()
    side.wait_stream(main)
    for t in range(min(len(frames), warmup + steps)):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            lset.run_raw([frames[t][i] for i in cams], pattern, side.cuda_stream)
        graphs.append(g)
    torch.cuda.synchronize()
    for t in range(warmup):
        graphs[t % len(graphs)].replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(main)
    for t in range(steps):
        graphs[t % len(graphs)].replay()
    e1.record(main)
    torch.cuda.synchronize()
    ms_graph = e0.elapsed_time(e1) / steps
    del graphs
    S.lorb_set_timing(True)
    ms_events = timed_set()
    tim = S.lorb_read_timing()
    S.lorb_set_timing(False)
    px = {i: sum(_scanned(r, *rig.frame_sizes[i]) for r in areas[i]) for i in cams}
    counts = {i: lorbs[i].counts.cpu().tolist() for i in cams}
    kernels = {}
    for k, (tot, n) in tim.items():
        if n:
            kernels[k] = {"avg_us": round(tot / n * 1e3, 2), "launches_per_step": 1,
                          "ms_per_step": round(tot / n, 4)}
    # detection reads each scanned sample's 3 bytes once (halo re-reads are not algorithmic)
    det_bytes = 3 * sum(px.values())
    kd = kernels["detect"]
    kd["alg_bytes_per_launch"] = int(det_bytes)
    kd["achieved_GBs"] = round(det_bytes / (kd["avg_us"] * 1e-6) / 1e9, 1)
    return {"ms_one_stream": ms_one, "ms_per_camera_streams": ms_multi, "ms_with_launch_events": ms_events,
            "ms_one_call": ms_set, "ms_graph": ms_graph,
            "px": sum(px.values()), "areas": areas, "counts": counts, "kernels": kernels}


def time_register(rig, frames, steps, warmup, n_max=500, nd=256, nhyp=1024):
    """Registration of a rig (Alg. 3, Alg. 4 steps 2-5): L-ORB of every camera in its overlap
    areas, then for each pair of neighbouring cameras multi-probe LSH matching of the facing
    areas and PROSAC to the map between their frames; one stream, frames in HBM.  Timed as
    the whole chain and as matching + PROSAC alone; accuracy against the rig's true maps."""
    import paper_1810_03988_amd as P
    import workloads as wl
    areas = P.detection_areas(rig.frame_sizes, rig.H, rig.canvas_w, rig.canvas_h)   # Alg. 2 step 1
    pattern = torch.from_numpy(wl.brief_pattern(nd)).cuda()
    cams = [i for i in range(rig.n) if areas[i]]
    lset = P.LorbSet([rig.frame_sizes[i] for i in cams], [areas[i] for i in cams], n_max=n_max, nd=nd)
    first = {}                                      # camera -> its first area's index in the set
    for i in cams:
        first[i] = sum(len(areas[j]) for j in cams if j < i)
    pos = np.random.default_rng(42).integers(0, nd, (6, 14))
    uni = torch.from_numpy(np.random.default_rng(7).random((nhyp, 4))).cuda()
    pairs = [i for i in range(rig.n - 1) if areas[i] and areas[i + 1]]
    matchers = {i: P.Matcher(n_max, n_max, nd, pos, nd // 4) for i in pairs}
    prosacs = {i: P.Prosac(n_max, n_max, nhyp, 200000.0, 3.0) for i in pairs}
    mset = P.MatcherSet([(n_max, n_max)] * len(pairs), nd, pos, nd // 4)
    pset = P.ProsacSet([(n_max, n_max)] * len(pairs), nhyp, 200000.0, 3.0)
    h = torch.cuda.current_stream().cuda_stream

    def feats(i):
        za, zb = first[i] + len(areas[i]) - 1, first[i + 1]
        return (lset.points[za], lset.descriptors[za], lset.counts[za:za + 1],
                lset.points[zb], lset.descriptors[zb], lset.counts[zb:zb + 1])

    ins = [feats(i) for i in pairs]                 # views of the L-ORB set's outputs
    m_in = [(da, ca, db, cb) for pa, da, ca, pb, db, cb in ins]
    p_in = [(pa, pb, mset.match[p], mset.dist[p], ca, uni) for p, (pa, da, ca, pb, db, cb) in enumerate(ins)]

    def match_prosac():
        for i in pairs:
            pa, da, ca, pb, db, cb = feats(i)
            matchers[i].run_raw(da, ca, db, cb, h)
            prosacs[i].run_raw(pa, pb, matchers[i].match, matchers[i].dist, ca, uni, h)

    def match_prosac_one_call(handle=None):
        mset.run_raw(m_in, h if handle is None else handle)
        pset.run_raw(p_in, h if handle is None else handle)

    def chain(t, handle=None):
        lset.run_raw([frames[t % len(frames)][c] for c in cams], pattern, h if handle is None else handle)
        match_prosac_one_call(handle)

    def timed(fn):
        for t in range(warmup):
            fn(t)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for t in range(steps):
            fn(t)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms_chain = timed(chain)
    chain(0)                                        # features and maps of frame set 0
    torch.cuda.synchronize()
    ms_one = timed(lambda t: match_prosac_one_call())
    ms_mp = timed(lambda t: match_prosac())
    # the pairs are independent (own workspaces and outputs): one stream per pair
    main = torch.cuda.current_stream()
    pstreams = {i: torch.cuda.Stream() for i in pairs}

    def match_prosac_streams(t):
        ev0 = torch.cuda.Event()
        ev0.record(main)
        for i in pairs:
            st = pstreams[i]
            st.wait_event(ev0)
            pa, da, ca, pb, db, cb = feats(i)
            matchers[i].run_raw(da, ca, db, cb, st.cuda_stream)
            prosacs[i].run_raw(pa, pb, matchers[i].match, matchers[i].dist, ca, uni, st.cuda_stream)
            ev = torch.cuda.Event()
            ev.record(st)
            main.wait_event(ev)

    ms_mp_streams = timed(match_prosac_streams)
    # the whole chain captured once per frame set of the cycle and replayed from HIP graphs
    # (every call of it takes its tables as launch arguments)
    graphs = []
    side = torch.cuda.Stream()
    side.wait_stream(main)
    for t in range(min(len(frames), warmup + steps)):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            chain(t, side.cuda_stream)
        graphs.append(g)
    torch.cuda.synchronize()
    ms_graph = timed(lambda t: graphs[t % len(graphs)].replay())
    del graphs
    chain(0)                                        # frame set 0 again, as the per-pair calls saw it
    torch.cuda.synchronize()
    res = []
    for p, i in enumerate(pairs):
        H = pset.H[p].cpu().numpy().reshape(3, 3)
        H_true = np.linalg.inv(np.asarray(rig.H[i + 1])) @ np.asarray(rig.H[i])
        x0, y0, w, hh = areas[i][-1]
        err = 0.0
        for (x, y) in [(x0, y0), (x0 + w, y0), (x0, y0 + hh), (x0 + w, y0 + hh)]:
            a = H @ np.array([x, y, 1.0])
            b = H_true @ np.array([x, y, 1.0])
            err = max(err, float(np.hypot(*(a[:2] / a[2] - b[:2] / b[2]))))
        res.append({"pair": [i, i + 1], "matches": int((mset.match[p] >= 0).sum()),
                    "inliers": int(pset.inliers[p]), "max_corner_error_px": round(err, 3),
                    "same_as_per_pair_calls": bool(torch.equal(pset.H[p], prosacs[i].H) and
                                                   torch.equal(mset.match[p], matchers[i].match))})
    return {"ms_chain": ms_chain, "ms_chain_graph": ms_graph, "ms_match_prosac_one_call": ms_one,
            "ms_match_prosac": ms_mp,
            "ms_match_prosac_streams": ms_mp_streams,
            "pairs": res, "nhyp": nhyp,
            "features": (feats, pos, uni)}


def register_cpu_baseline(rig, frames0, feats, pos, uni, nd=256):
    """The registration oracle (matching and PROSAC, Python loops, one thread) on the first
    pair's features as the GPU found them: seconds per pair."""
    from oracle import register_oracle as ro
    pa, da, ca, pb, db, cb = feats(0)
    na, nb = int(ca[0]), int(cb[0])
    dah, dbh = da.cpu().numpy().view(np.uint32)[:na], db.cpu().numpy().view(np.uint32)[:nb]
    t = time.perf_counter()
    idx, dist = ro.lsh_match(dah, dbh, pos, nd // 4)
    ro.prosac(pa.cpu().numpy()[:na], pb.cpu().numpy(), idx, dist, uni.cpu().numpy(), 200000.0, 3.0)
    dt = time.perf_counter() - t
    return {"value": round(1.0 / dt, 4), "unit": "pairs/s (matching + PROSAC)", "cores": 1, "kind": "oracle",
            "sample": f"pair 0-1 of frame set 0, {na} x {nb} features, {len(uni)} hypotheses, {dt:.1f} s"}


def _scanned(rect, w, h, margin=17):
    """Samples of a detection area that are scanned: those 17 or more from every frame
    edge (the descriptor support)."""
    x0, y0, rw, rh = rect
    cw = min(x0 + rw, w - margin) - max(x0, margin)
    ch = min(y0 + rh, h - margin) - max(y0, margin)
    return max(0, cw) * max(0, ch)


def lorb_cpu_baseline(rig, frames0, n_max=500, nd=256):
    """The L-ORB oracle on one detection area of camera 0 (exact integer numpy and Python
    loops, one thread): area samples per second."""
    import oracle
    from oracle import lorb_oracle as lo
    import workloads as wl
    area = oracle.detection_areas(rig.frame_sizes, rig.H, rig.canvas_w, rig.canvas_h)[0][0]
    w, h = rig.frame_sizes[0]
    frame = frames0[0].cpu().numpy()
    t = time.perf_counter()
    lo.lorb(frame, [area], 20, 0, n_max, wl.brief_pattern(nd))
    dt = time.perf_counter() - t
    px = _scanned(area, w, h)
    return {"value": round(px / dt / 1e6, 5), "unit": "Mpx/s (detection-area samples)", "cores": 1,
            "kind": "oracle", "sample": f"camera 0, area {tuple(area)}: {px} samples scanned, frame 0, {dt:.1f} s"}


def time_batched(rig, frames, storage, steps, warmup, tune_cache=None, kernel_events=True):
    """All frames of the sequence as jobs of one batch (one plan per job).  Timed twice on
    one stream: with per-launch HIP events (launches issued directly, an event after each)
    and as HIP graph replays (one capture, one replay per step)."""
    import paper_1810_03988_amd as P
    dev = frames[0][0].device
    plans = [P.Plan(rig.frame_sizes, rig.H, rig.masks(), rig.canvas_w, rig.canvas_h, rig.levels, storage=storage,
                    device=dev) for _ in frames]
    panos = [torch.empty((rig.canvas_h, rig.canvas_w, 3), dtype=torch.uint8, device=dev) for _ in frames]
    batch = P.Batch(plans, device=dev)
    stream = torch.cuda.Stream()
    res = {}
    with torch.cuda.stream(stream):
        cfg = batch.autotune(frames, panos, stream=stream, cache_path=tune_cache)
        args = batch.args(frames, panos)
        sh = stream.cuda_stream
        for mode in (["events"] if kernel_events else []) + ["graph"]:
            batch.set_timing(mode == "events")
            for _ in range(warmup):
                batch.run_raw(args, sh)
            stream.synchronize()
            batch.set_timing(mode == "events")    # clears the warm-up's events
            t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0.record(stream)
            for _ in range(steps):
                batch.run_raw(args, sh)
            t1.record(stream)
            stream.synchronize()
            res[mode] = (t0.elapsed_time(t1) / steps, batch.read_timing() if mode == "events" else {})
        batch.set_timing(False)
    return res, cfg, plans[0], batch, panos


def run_c5(a):
    """The differentiation workload: 16 pairs of 1280x720 frames (20 % overlap, 2304x720
    canvas, 3 levels), frame B's corners off the truth by U[-3, 3] px; 50 Adam steps on the
    pair loss (lr 1e-3 on the normalised corners), each gradient through
    stitch_frame_backward.  Reports the mean corner error at steps 0/10/25/50 per pair and
    over the pairs, and the time of one loss + gradient evaluation."""
    import paper_1810_03988_amd as P
    import workloads as wl
    pairs = wl.rig_c5_pairs(16)
    out, errs = [], {0: [], 10: [], 25: [], 50: []}
    t_eval = []
    for r in pairs:
        w, h = r.frame_sizes[1]
        fr = [f.permute(2, 0, 1).float().div(255.0).contiguous().cuda() for f in wl.render_rig_frames(r)]
        c = np.c_[[[0, 0], [w - 1, 0], [w - 1, h - 1], [0, h - 1]], np.ones(4)] @ np.asarray(r.H[1]).T
        qt = (c[:, :2] / c[:, 2:]).ravel()
        g = P.Grad(r.frame_sizes, r.masks(), r.canvas_w, r.canvas_h, r.levels)
        q0 = qt + r.extra["corner_noise"]
        # one timed loss + gradient at the start point (freeze, forward, upstream, VJP, chain rule)
        for rep in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            Hb = P.corners_to_h(q0, w, h)
            g.freeze([np.eye(3), Hb])
            q = torch.tensor(q0, dtype=torch.float64, requires_grad=True)
            P.StitchPairLoss.apply(fr[0], fr[1], q, g, np.eye(3)).backward()
            torch.cuda.synchronize()
            if rep:
                t_eval.append((time.perf_counter() - t) * 1e3)
        _, log = P.refine_pair(g, fr[0], fr[1], np.eye(3), q0, steps=50, q_true=qt)
        row = {"pair": r.name, "yaw_deg": round(r.extra["yaw_deg"], 4)}
        for k in errs:
            errs[k].append(log[k][1])
            row[f"corner_err_px_step{k}"] = round(log[k][1], 4)
            row[f"loss_step{k}"] = float(f"{log[k][0]:.6e}")
        out.append(row)
        print(f"# {r.name}: " + ", ".join(f"step {k}: {log[k][1]:.3f} px" for k in errs), file=sys.stderr, flush=True)
        g.close()
    line = {"report": "C5 registration refinement through the adjoint", "pairs": len(pairs),
            "mean_corner_err_px": {f"step{k}": round(float(np.mean(v)), 4) for k, v in errs.items()},
            "pairs_improved_at_step50": int(sum(e50 < e0 for e0, e50 in zip(errs[0], errs[50]))),
            "ms_per_loss_and_gradient": round(float(np.median(t_eval)), 3),
            "how": "freeze, forward (FP64 full canvas), upstream terms, stitch_frame_backward, corner chain rule; "
                   "host round trips included", "per_pair": out, "device": torch.cuda.get_device_name(0)}
    print(json.dumps(line), flush=True)


def cpu_model() -> str:
    try:
        for line in Path("/proc/cpuinfo").read_text().splitlines():
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def _oracle_strip(unit):
    """One cpu_baseline unit: the oracle (FP64 numpy, as it stands) on a full-height column
    strip of a job's canvas, evaluated through the strip's dependency cones (ROI mode).
    Returns (canvas samples, seconds)."""
    import oracle
    rig, frames, x0, x1 = unit
    t = time.perf_counter()
    so = oracle.StitchOracle(frames, rig.H, rig.masks(), rig.canvas_w, rig.canvas_h, rig.levels)
    so.panorama(np.arange(rig.canvas_h), np.arange(x0, x1))
    return (x1 - x0) * rig.canvas_h, time.perf_counter() - t


def c3_cpu_baseline(rigs, frames, single_units=4, strip=256):
    """The oracle on the batching workload's own jobs: units are full-height strips of
    `strip` columns centred on each job's first seam.  Timed in one process on the first
    `single_units` jobs, then over a process pool of every usable core (at most 16, the
    box's CPU share) on two units per worker.  value = the pool's canvas Mpx/s."""
    import multiprocessing as mp

    def unit(j):
        r = rigs[j]
        c = r.seams[0] if r.seams else r.canvas_w // 2
        x0 = max(0, min(r.canvas_w - strip, c - strip // 2))
        return (r, [f.cpu().numpy() for f in frames[j]], x0, min(r.canvas_w, x0 + strip))

    px = dt = 0.0
    for j in range(min(single_units, len(rigs))):
        n, t = _oracle_strip(unit(j))
        px, dt = px + n, dt + t
    single = px / dt / 1e6
    workers = max(1, min(len(os.sched_getaffinity(0)), 16))
    units = [unit(j % len(rigs)) for j in range(2 * workers)]
    ctx = mp.get_context("spawn")
    t = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_strip, units, chunksize=1)
    wall = time.perf_counter() - t
    ppx = sum(n for n, _ in res)
    return {"value": round(ppx / wall / 1e6, 5), "unit": "Mpx/s", "cores": workers, "kind": "oracle",
            "sample": f"full-height {strip}-column strips of the jobs' canvases centred on each job's first seam, "
                      f"through every level (FP64 numpy oracle in ROI mode): {len(units)} strips of jobs "
                      f"0-{len(units) - 1} ({ppx / 1e6:.2f} Mpx) over a pool of {workers} processes in "
                      f"{wall:.1f} s wall (process start included)",
            "single_process": {"value": round(single, 5), "cores": 1,
                               "sample": f"strips of jobs 0-{min(single_units, len(rigs)) - 1} "
                                         f"({px / 1e6:.2f} Mpx) in {dt:.1f} s"},
            "cpu": cpu_model(), "logical_cpus_visible": os.cpu_count(), "numpy": np.__version__}


def time_graph_and_events(batch, bargs, stream, steps, warmup, events=True):
    """A batch timed as HIP graph replays (one per step) and, separately, launched eagerly
    with a HIP event after every launch (the per-kernel table)."""
    sh = stream.cuda_stream
    out = {}
    for mode in ["graph"] + (["events"] if events else []):
        batch.set_timing(mode == "events")
        for _ in range(warmup):
            batch.run_raw(bargs, sh)
        stream.synchronize()
        batch.set_timing(mode == "events")    # clears the warm-up's events
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(steps):
            batch.run_raw(bargs, sh)
        t1.record(stream)
        stream.synchronize()
        out[mode] = (t0.elapsed_time(t1) / steps, batch.read_timing() if mode == "events" else {})
    batch.set_timing(False)
    return out


def run_c3(a):
    """The batching workload (the largest single-GPU configuration): njobs stitch jobs of
    2-6 cameras at 640x480 .. 3840x2160 and 4-7 levels, one frame set each.  Forms: the
    batch (one launch per level over all jobs, captured into a HIP graph, autotuned tiles)
    in FP16 and FP32 storage, and the same jobs stitched one by one (one stitch_frame per
    job, eager launches, the planner's default tiles).  value = batched FP16."""
    import paper_1810_03988_amd as P
    import workloads as wl
    rigs = wl.rig_c3_jobs(a.jobs)
    t = time.perf_counter()
    frames = [wl.render_rig_frames(r, 0, "cuda") for r in rigs]
    torch.cuda.synchronize()
    px = sum(r.canvas_pixels() for r in rigs)
    in_px = sum(w * h for r in rigs for (w, h) in r.frame_sizes)
    print(f"# {len(rigs)} jobs rendered in {time.perf_counter() - t:.1f} s: {px / 1e6:.1f} Mpx canvas, "
          f"{in_px / 1e6:.1f} Mpx input", file=sys.stderr, flush=True)
    stream = torch.cuda.Stream()
    sh = stream.cuda_stream
    tune = os.environ.get("STITCH_TUNE_CACHE")
    forms, ref_panos, tables, configs, plans0 = {}, {}, {}, {}, {}
    mpx = lambda ms_: round(px / (ms_ / 1e3) / 1e6, 1)
    prof = a.profile_form
    for st in ((prof,) if prof else ("f16", "f32")):
        t = time.perf_counter()
        plans = [P.Plan(r.frame_sizes, r.H, r.masks(), r.canvas_w, r.canvas_h, r.levels, storage=st) for r in rigs]
        panos = [torch.empty((r.canvas_h, r.canvas_w, 3), dtype=torch.uint8, device="cuda") for r in rigs]
        one = [torch.empty_like(p) for p in panos]
        torch.cuda.synchronize()
        print(f"# {st}: {len(plans)} plans in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
        args = [p.frame_args(f, o) for p, f, o in zip(plans, frames, one)]

        def one_by_one():
            for p, ar in zip(plans, args):
                p.frame_raw(ar, sh)

        with torch.cuda.stream(stream):
            ms1 = float("nan")
            if not prof:
                for _ in range(a.warmup):
                    one_by_one()
                stream.synchronize()
                t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                t0.record(stream)
                for _ in range(a.steps):
                    one_by_one()
                t1.record(stream)
                stream.synchronize()
                ms1 = t0.elapsed_time(t1) / a.steps
                forms[f"plain_{st}"] = {"Mpx_s": mpx(ms1), "ms_per_step": round(ms1, 4),
                                        "how": "one stitch_frame per job, eager launches, default tiles"}
                print(f"# plain_{st}: {ms1:.3f} ms/step, {mpx(ms1):.0f} Mpx/s", file=sys.stderr, flush=True)
            batch = P.Batch(plans)
            cfg = batch.autotune(frames, panos, stream=stream, cache_path=tune)
            bargs = batch.args(frames, panos)
            # the schedule: one sequence, or the jobs as groups pipelined over two streams
            # (the warp pass of one group under the memory-bound passes of the previous)
            # (persistent grids hold every compute unit until they end, so the grouped schedule
            # is also tried with one workgroup per tile, which lets the two streams' kernels share
            # the compute units)
            by_groups = {}
            tuned_wg = list(cfg["wg_per_cu"])
            for G in [g for g in (1, 2, 3, 4) if g <= len(rigs) and (not prof or g == 1)]:
                for per_tile in ((False, True) if G > 1 else (False,)):
                    batch.set_groups(G)
                    batch.set_config([-1] * len(tuned_wg) if per_tile else tuned_wg, [0] * len(tuned_wg))
                    key = f"{G}{'/per-tile' if per_tile else ''}"
                    by_groups[key] = round(time_graph_and_events(batch, bargs, stream, max(3, a.steps // 2), 2,
                                                                 events=False)["graph"][0], 4)
            best_g = min(by_groups, key=by_groups.get)
            G_best, per_tile_best = int(best_g.split("/")[0]), best_g.endswith("per-tile")
            batch.set_groups(G_best)
            batch.set_config([-1] * len(tuned_wg) if per_tile_best else tuned_wg, [0] * len(tuned_wg))
            print(f"# {st} batched graph ms by groups: {by_groups} -> {best_g}", file=sys.stderr, flush=True)
            res = time_graph_and_events(batch, bargs, stream, a.steps, a.warmup, events=not a.no_kernel_events)
        torch.cuda.synchronize()
        same = None if prof else all(torch.equal(x, y) for x, y in zip(panos, one))
        ms = res["graph"][0]
        forms[f"batched_graph_{st}"] = {
            "Mpx_s": mpx(ms), "ms_per_step": round(ms, 4), "how": "one HIP graph replay per step",
            "speedup_vs_one_by_one": round(ms1 / ms, 3), "equals_one_by_one_bitwise": same,
            "groups": best_g, "ms_per_step_by_groups": by_groups,
            "tuned": {k: v[:max(r.levels for r in rigs) - 1] for k, v in cfg.items()}}
        if "events" in res:
            forms[f"batched_graph_{st}"]["ms_per_step_eager_with_launch_events"] = round(res["events"][0], 4)
            s_b = 2 if st == "f16" else 4
            tables[st] = c3_kernel_table(plans, rigs, res["events"][1], a.steps, s_b)
            forms[f"batched_graph_{st}"]["kernels"] = tables[st]
        print(f"# batched_graph_{st}: {ms:.3f} ms/step, {mpx(ms):.0f} Mpx/s, x{ms1 / ms:.2f} vs one by one, "
              f"bitwise equal: {same}", file=sys.stderr, flush=True)
        for k, v in tables.get(st, {}).items():
            print(f"#   {k:18s} {v['avg_us']:9.2f} us/launch  {v['alg_bytes_per_launch'] / 1e6:9.2f} MB  "
                  f"{v['achieved_GBs']:8.1f} GB/s", file=sys.stderr, flush=True)
        del batch, plans, panos, one, args
        torch.cuda.empty_cache()
    if prof:
        if a.copy_calibration_mib > 0:
            copy_calibration(a.copy_calibration_mib)
        print(json.dumps({"profile_form": prof, "forms": forms}), flush=True)
        return
    head = forms["batched_graph_f16"]
    roof = None
    if "f16" in tables:
        kt = tables["f16"]
        dom = max(kt, key=lambda k: kt[k]["ms_per_step"])
        kd = kt[dom]
        roof = {"bound": "hbm", "achieved": kd["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(kd["achieved_GBs"] / HBM_PEAK_GBS, 4),
                "traffic": profiled_traffic("c3", "batched", "f16", dom), "kernel": dom,
                "alg_bytes": kd["alg_bytes_per_launch"], "avg_us": kd["avg_us"],
                "step_alg_bytes": int(sum(v["alg_bytes_per_launch"] * v["launches_per_step"] for v in kt.values())),
                "step_frac": round(sum(v["alg_bytes_per_launch"] * v["launches_per_step"] for v in kt.values())
                                   / (head["ms_per_step"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        # what holds the kernel under the HBM roof: its vector-ALU busy fraction from the
        # committed counter summary (1.0: every SIMD issues a VALU instruction every 4 cycles)
        kname = next((k for want in (f"{dom}, batched (f16)", f"{dom} (f16)")
                      for k, v in KERNEL_KINDS.items() if v == want), None)
        ctr = profiled_counters("c3", "batched", "f16", kname) if kname else None
        roof["valu_busy"] = ctr.get("VALU_busy") if ctr else None
    if a.copy_calibration_mib > 0:
        copy_calibration(a.copy_calibration_mib)
    cpu = None
    if not a.no_cpu_baseline:
        cpu = c3_cpu_baseline(rigs, frames)
        print(f"# cpu oracle: {cpu['value']} Mpx/s on {cpu['cores']} processes, "
              f"{cpu['single_process']['value']} Mpx/s on one", file=sys.stderr, flush=True)
    cams = [r.n for r in rigs]
    line = {
        "metric": METRIC, "value": head["Mpx_s"], "unit": "Mpx/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (f16 storage)", "data": "synthetic",
        "config": {"workload": f"C3: {len(rigs)} stitch jobs of {min(cams)}-{max(cams)} cameras at 640x480 to "
                               f"3840x2160, 4-7 levels, {px / 1e6:.1f} Mpx of canvas and {in_px / 1e6:.1f} Mpx "
                               f"of input per step, one frame set per job",
                   "form": "batched, FP16 storage: one launch per pyramid level and per blend level over all "
                           "jobs (or over each of a few job groups, the warp pass of one group overlapping the "
                           "later passes of the previous on a second stream), captured into one HIP graph (one "
                           "replay per step), autotuned tiles",
                   "jobs": len(rigs)},
        "batched_f16_vs_plain_f32": round(forms["plain_f32"]["ms_per_step"] / head["ms_per_step"], 3),
        "roofline": roof, "cpu_baseline": cpu, "forms": forms, "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(line), flush=True)


def c3_kernel_table(plans, rigs, timing, steps, s):
    """Batched form on the jobs: per launch kind, average launch time and the algorithmic
    bytes of the jobs that launch covers (each job's phase bytes from its own regions)."""
    per_job = [phase_bytes(p, r, s) for p, r in zip(plans, rigs)]
    table = {}
    for key, (tot_ms, launches) in sorted(timing.items()):
        pk = f"{key[0]}{key[1]}"
        nbytes = sum(b.get(pk, 0) for b in per_job)
        if nbytes:
            table[phase_name(key)] = _row(tot_ms, launches, steps, nbytes)
    return table


def _row(tot_ms, launches, steps, nbytes):
    avg_s = tot_ms / launches / 1e3
    gbs = nbytes / avg_s / 1e9
    return {"launches_per_step": launches // steps, "avg_us": round(avg_s * 1e6, 3),
            "alg_bytes_per_launch": int(nbytes), "achieved_GBs": round(gbs, 1),
            "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4), "ms_per_step": round(tot_ms / steps, 4)}


def kernel_table(plan, rig, timing, steps, s):
    """Plain form: per launch kind, average launch time and bytes (the kind's phases of a
    frame averaged the same way as its launches)."""
    ph = phase_bytes(plan, rig, s)
    table = {}
    for kind, (tot_ms, launches) in timing.items():
        keys = PLAIN_KINDS.get(kind, lambda L: [])(rig.levels)
        if not keys:
            continue
        table[kind] = _row(tot_ms, launches, steps, float(np.mean([ph[k] for k in keys])))
    return table


def batch_kernel_table(plan, rig, timing, steps, s, njobs):
    """Batched form: one launch per phase per step covering all njobs frames."""
    ph = phase_bytes(plan, rig, s)
    table = {}
    for key, (tot_ms, launches) in sorted(timing.items()):
        name = phase_name(key)
        pk = f"{key[0]}{key[1]}"
        if pk in ph:
            table[name] = _row(tot_ms, launches, steps, njobs * ph[pk])
    return table


def cpu_baseline(rig, frames0):
    """The oracle as it stands, on a bounded sample: the full-height column window
    [1248, 3168) of frame 0 (spans the first seam), all levels through their cones."""
    import oracle
    fr = [f.cpu().numpy() for f in frames0]
    x0, x1 = 1248, 3168
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
    if a.traffic_summary:
        traffic_summary(*a.traffic_summary)
        return
    if a.rocprof_summary:
        rocprof_summary(a.rocprof_summary)
        return
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py: measures one GPU; --gpus {a.gpus} is not supported "
              "(independent frames and jobs would shard round-robin across GPUs with no exchange)",
              file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if a.config == "c3":
        run_c3(a)
        return
    if a.config == "c5":
        run_c5(a)
        return
    rig = rig_for(a.config)
    if a.precision:
        print(json.dumps(precision_report(rig, a.windows, full=a.config == "c1")), flush=True)
        return
    t = time.perf_counter()
    frames = make_frames(rig, a.frames, "cuda")
    torch.cuda.synchronize()
    print(f"# generated {a.frames} x {rig.n} frames in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    s = 2 if a.storage == "f16" else 4
    px_per_step = rig.canvas_w * rig.canvas_h * a.frames
    mpx = lambda ms_: round(px_per_step / (ms_ / 1e3) / 1e6, 1)
    tune = os.environ.get("STITCH_TUNE_CACHE")
    forms = {}
    events = not a.no_kernel_events
    if a.form == "batched":
        res, cfg, plan0, _b, _p = time_batched(rig, frames, a.storage, a.steps, a.warmup, tune, events)
        ms = res["events"][0] if events else res["graph"][0]
        kernels = batch_kernel_table(plan0, rig, res["events"][1], a.steps, s, a.frames) if events else {}
        forms[f"batched_{a.storage}"] = {"Mpx_s": mpx(ms), "ms_per_step": round(ms, 4),
                                         "how": "launches issued directly, an event after each"}
        forms[f"batched_graph_{a.storage}"] = {"Mpx_s": mpx(res["graph"][0]),
                                               "ms_per_step": round(res["graph"][0], 4),
                                               "how": "one HIP graph replay per step"}
        form_desc = (f"batched, {a.storage} storage: the {a.frames} frames as {a.frames} jobs of one batch, one "
                     f"launch per pyramid level and per blend level (tuned workgroups/CU {cfg['wg_per_cu'][:rig.levels - 1]}, tile rows {cfg['tile_rows'][:rig.levels - 1]})")
        del _b, _p
    else:
        plan0, ms, timing, _ = time_form(rig, frames, a.storage, a.steps, a.warmup, events)
        kernels = kernel_table(plan0, rig, timing, a.steps, s) if events else {}
        forms[f"plain_{a.storage}"] = {"Mpx_s": mpx(ms), "ms_per_step": round(ms, 4)}
        form_desc = f"plain, {a.storage} storage, one stitch_frame per frame"
    value = px_per_step / (ms / 1e3) / 1e6
    print(f"# {a.form} {a.storage}: {ms:.3f} ms/step, {value:.0f} Mpx/s", file=sys.stderr, flush=True)
    for k, v in kernels.items():
        print(f"#   {k:18s} {v['avg_us']:9.2f} us/launch x{v['launches_per_step']:4d}  "
              f"{v['alg_bytes_per_launch'] / 1e6:9.2f} MB  {v['achieved_GBs']:8.1f} GB/s", file=sys.stderr, flush=True)
    roof = None
    if kernels:
        dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
        kd = kernels[dom]
        roof = {"bound": "hbm", "achieved": kd["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(kd["achieved_GBs"] / HBM_PEAK_GBS, 4),
                "traffic": profiled_traffic(a.config, a.form, a.storage, dom), "kernel": dom,
                "alg_bytes": kd["alg_bytes_per_launch"], "avg_us": kd["avg_us"]}
    for form in [f for f in a.forms.split(",") if f and f != "none"]:
        kind, st = form.rsplit("_", 1) if "_" in form else (form, "")
        if (kind == a.form and st == a.storage) or (kind == "batched_graph" and a.form == "batched" and
                                                    st == a.storage):
            continue
        if form == "register":
            G = time_register(rig, frames, a.steps, a.warmup)
            feats, pos, uni = G.pop("features")
            forms["register"] = {
                "ms_per_rig_registration": round(G["ms_chain"], 4),
                "ms_per_rig_registration_graph_replay": round(G["ms_chain_graph"], 4),
                "ms_match_prosac_all_pairs_one_call_per_stage": round(G["ms_match_prosac_one_call"], 4),
                "ms_match_prosac_all_pairs_per_pair_calls": round(G["ms_match_prosac"], 4),
                "ms_match_prosac_all_pairs_stream_per_pair": round(G["ms_match_prosac_streams"], 4),
                "how": "L-ORB of every camera in its overlap areas (one stitch_lorb_multi call), then every "
                       "neighbouring pair's multi-probe LSH matching (6 tables x 14 bits, distance <= 64; one "
                       "stitch_lsh_match_multi call) and PROSAC (1024 hypotheses, T_N 2e5, eps 3 px, "
                       "least-squares refit; one stitch_prosac_multi call); one stream, frames in HBM",
                "pairs": G["pairs"], "nhyp": G["nhyp"]}
            if not a.no_cpu_baseline:
                forms["register"]["cpu_baseline"] = register_cpu_baseline(rig, frames[0], feats, pos, uni)
            print(f"# register: {json.dumps(forms['register'])}", file=sys.stderr, flush=True)
            continue
        if form == "lorb":
            L = time_lorb(rig, frames, a.steps, a.warmup)
            lms, lpx = L["ms_one_call"], L["px"]
            kd = L["kernels"]["detect"]
            forms["lorb"] = {
                "ms_per_frame_set": round(lms, 4), "frame_sets_per_s": round(1e3 / lms, 1),
                "area_Mpx_s": round(lpx / (lms / 1e3) / 1e6, 1), "area_px_per_frame_set": lpx,
                "ms_per_frame_set_with_launch_events": round(L["ms_with_launch_events"], 4),
                "ms_per_frame_set_graph_replay": round(L["ms_graph"], 4),
                "area_Mpx_s_graph_replay": round(lpx / (L["ms_graph"] / 1e3) / 1e6, 1),
                "ms_per_frame_set_call_per_camera": round(L["ms_one_stream"], 4),
                "ms_per_frame_set_call_per_camera_own_streams": round(L["ms_per_camera_streams"], 4),
                "how": "L-ORB (Alg. 1-2) of every camera in its overlap areas, tf 20, t 0, 500 points, "
                       "256 pairs; frames in HBM; all cameras in one stitch_lorb_multi call (the "
                       "form's headline and kernel table), the same call replayed from HIP graphs, "
                       "and one stitch_lorb per camera on one stream or on a stream each",
                "kernels": L["kernels"],
                "roofline": {"bound": "hbm", "kernel": "detect", "achieved": kd["achieved_GBs"],
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(kd["achieved_GBs"] / HBM_PEAK_GBS, 4), "traffic": None,
                             "alg_bytes": kd["alg_bytes_per_launch"], "avg_us": kd["avg_us"]},
                "areas": L["areas"], "points_kept": L["counts"]}
            if not a.no_cpu_baseline:
                forms["lorb"]["cpu_baseline"] = lorb_cpu_baseline(rig, frames[0])
            print(f"# lorb: {json.dumps({k: v for k, v in forms['lorb'].items() if k not in ('areas',)})}",
                  file=sys.stderr, flush=True)
            continue
        if kind == "pipe":
            pms, in_b, out_b = time_pipe(rig, frames, st, a.steps, a.warmup)
            forms[f"pipe_{st}"] = {"Mpx_s": mpx(pms), "ms_per_step": round(pms, 4),
                                   "how": "end to end: pinned host frames in, host panoramas out, uploads, "
                                          "stitch_frame and downloads on three streams (3 slots); wall clock",
                                   "pcie_bytes_per_step": [in_b, out_b],
                                   "pcie_GBs": round((in_b + out_b) / (pms / 1e3) / 1e9, 1)}
        elif kind in ("batched", "batched_graph"):
            res, cfg, _pl, _b, _p = time_batched(rig, frames, st, a.steps, a.warmup, tune, False)
            forms[f"batched_graph_{st}"] = {"Mpx_s": mpx(res["graph"][0]), "ms_per_step": round(res["graph"][0], 4),
                                            "how": "one HIP graph replay per step"}
            del _b, _p, _pl
        else:
            fplan, fms, ftim, _panos = time_form(rig, frames, st, a.steps, a.warmup, True)
            fms_plain = time_form(rig, frames, st, a.steps, a.warmup, False)[1]
            forms[f"plain_{st}"] = {"Mpx_s": mpx(fms), "ms_per_step": round(fms, 4),
                                    "ms_per_step_without_launch_events": round(fms_plain, 4),
                                    "Mpx_s_without_launch_events": mpx(fms_plain),
                                    "kernels": kernel_table(fplan, rig, ftim, a.steps, 2 if st == "f16" else 4)}
            del fplan, _panos
        print(f"# {form}: {json.dumps({k: v for k, v in list(forms.items())[-1][1].items() if k != 'kernels'})}",
              file=sys.stderr, flush=True)
    if a.copy_calibration_mib > 0:
        copy_calibration(a.copy_calibration_mib)
    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(rig, frames[0])
        print(f"# cpu oracle: {cpu['value']} Mpx/s", file=sys.stderr, flush=True)
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mpx/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if a.storage == "f32" else "f32 (f16 storage)", "data": "synthetic",
        "config": {"workload": workload_name(rig, a.frames), "form": form_desc, "frames_per_step": a.frames,
                   "cameras": rig.n,
                   "canvas": [rig.canvas_w, rig.canvas_h], "levels": rig.levels},
        "roofline": roof, "cpu_baseline": cpu, "kernels": kernels, "forms": forms,
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
