"""Benchmark of the FRKC2 superstep on one MI355X.

One step = the whole hot path on the 3D variable-coefficient diffusion
workload: u_t = div(D grad u) on 256^3 interior nodes (FP64, 7-point flux
stencil, lognormal D, Dirichlet zero, seeded Gaussian-blob u0), FRKC2 with
s = 100 stages, 10 supersteps: stepsizes (cached), Gershgorin bound and
stability check, 1000 fused stage kernels, the final ||Im W^L|| / ||W^L||
diagnostic and the L2 norm of the result.

Prints one JSON line: grid-point-stage updates per second, the roofline of
the dominant kernel (the interior stage pass) and the CPU oracle timed on a
bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 vector
S_STAGES = 100
SUPERSTEPS = 10
NU = 0.01
CFL = 0.9


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


# Sources that define the dominant kernel of each tile shape (k = 1: the plane kernel).
KERNEL_SOURCES = {1: ("stage.hip", "plane_tile.h"), 2: ("tblock.hip",), 3: ("tblock.hip",),
                  4: ("tb3d.hip", "tb3d_tile.h"), 5: ("tb3d.hip", "tb3d_tile.h")}
COMMON_SOURCES = ("device_common.h", "internal.h")
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic_stage3d_256.json")


def kernel_sources_sha256(k, tile):
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[1 if k == 1 else tile] + COMMON_SOURCES:
        with open(os.path.join(ROOT, "paper_1702_03818_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(k, tile, zchunk):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources and launch configuration."""
    if not os.path.exists(TRAFFIC_JSON):
        return None, "no counter summary"
    with open(TRAFFIC_JSON) as f:
        t = json.load(f)
    if t.get("sources_sha256") != kernel_sources_sha256(k, tile):
        return None, "counters were taken on different kernel sources"
    if t.get("config") != {"tblock": k, "tile": tile, "zchunk": zchunk}:
        return None, "counters were taken in another launch configuration (%s)" % t.get("config")
    return t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"], t.get("note", "")


def kernel_pattern(k, tile):
    """Name fragment rocprofv3 prints for the interior-pass kernel of the 3D workload."""
    if k == 1:
        return "plane_stage<1, 1, 3, 64, 4, false, false>"
    if tile in (4, 5):
        # both march directions (the last template argument)
        return "tb3d_stage<1, 1, %d, false, false, false, false, %d, " % (k, 64 if tile == 4 else 32)
    shape = {1: "64, 16, 1", 2: "64, 16, 2", 3: "64, 8, %d" % (4 if k == 2 else 3)}[tile]
    return "tb_stage<1, 1, 3, %s, %d, false, false>" % (shape, k)


def _csv_rows(directory, suffix):
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit("no *%s under %s" % (suffix, directory))
    rows = []
    for fn in files:
        with open(fn) as f:
            rows.extend(csv.DictReader(f))
    return rows


def _short(name):
    return name.replace("frkc2::(anonymous namespace)::", "")


def summarize_trace(directory, command, k, tile, out_md, pattern=None, title=None, note=None,
                    by_kernel=False):
    """Per-(kernel, grid) durations from a rocprofv3 --kernel-trace run, as markdown (per
    kernel over all grid sizes with by_kernel)."""
    groups = {}
    for r in _csv_rows(directory, "kernel_trace.csv"):
        grid = int(r["Grid_Size"]) if "Grid_Size" in r else (
            int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]))
        key = (r["Kernel_Name"], "various" if by_kernel else grid)
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
        groups.setdefault(key, []).append(d)
    total = sum(sum(v) for v in groups.values())
    pat = pattern or kernel_pattern(k, tile)
    dom = max((key for key in groups if pat in key[0]), key=lambda kk: len(groups[kk]))
    # every kernel the pattern names at that grid size (e.g. both march directions)
    dom_d = [d for key in groups if pat in key[0] and key[1] == dom[1] for d in groups[key]]
    dom_names = sorted({_short(key[0]) for key in groups if pat in key[0] and key[1] == dom[1]})
    what = ("Dominant kernel (interior pass, k = %d, tile %d)" % (k, tile)) if pattern is None \
        else "Kernel"
    lines = ["# Kernel trace: %s" % (title or "3D variable-D 256^3, s = 100 (bench step)"), "",
             "Command (from /tmp, with the repository as the working copy):", "",
             "    " + command, ""] + ([note, ""] if note else []) + [
             "Durations per (kernel, grid size in threads) from rocprofv3 `kernel_trace.csv`, "
             "microseconds%s." % (", over all grid sizes of a kernel" if by_kernel else ""), "",
             "%s: %s at grid %s: %d launches, average %.2f us." % (
                 what, " and ".join("`%s`" % n for n in dom_names), dom[1], len(dom_d),
                 sum(dom_d) / len(dom_d)), "",
             "| Kernel | grid | calls | total ms | average us | min us | max us | % |",
             "|---|---|---|---|---|---|---|---|"]
    for key, v in sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:25]:
        lines.append("| `%s` | %s | %d | %.2f | %.2f | %.2f | %.2f | %.2f |" % (
            _short(key[0]), key[1], len(v), sum(v) * 1e-3, sum(v) / len(v), min(v), max(v),
            100 * sum(v) / total))
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return sum(dom_d) / len(dom_d)


def summarize_counters(fetch_dir, write_dir, fetch_cmd, write_cmd, k, tile, zchunk, out_md):
    """HBM traffic of the dominant kernel from FETCH_SIZE / WRITE_SIZE runs, calibrated on the
    bench's 1 GiB device copies (the six largest copy dispatches of each run)."""
    per = {}
    for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        groups, copies = {}, []
        for r in _csv_rows(d, "counter_collection.csv"):
            if r["Counter_Name"] != name:
                continue
            v = float(r["Counter_Value"])
            if "copyBuffer" in r["Kernel_Name"]:
                copies.append(v)
            groups.setdefault((r["Kernel_Name"], int(r["Grid_Size"])), []).append(v)
        copies = sorted(copies)[-6:]
        scale = (1 << 30) / (1024.0 * sum(copies) / len(copies))
        per[name] = (groups, scale)
    pat = kernel_pattern(k, tile)
    fg, fs = per["FETCH_SIZE"]
    wg, ws = per["WRITE_SIZE"]
    dom = max((key for key in fg if pat in key[0]), key=lambda kk: len(fg[kk]))
    keys = [key for key in fg if pat in key[0] and key[1] == dom[1]]
    fv_all = [v for key in keys for v in fg[key]]
    wv_all = [v for key in keys for v in wg.get(key, [])]
    fetch = 1024.0 * fs * sum(fv_all) / len(fv_all)
    write = 1024.0 * ws * sum(wv_all) / len(wv_all)
    n = 256 ** 3
    alg = 40 * n
    t = {"kernel": " and ".join(sorted(_short(key[0]) for key in keys)), "grid": dom[1],
         "workload": "3D var-D 256^3, s = 100, k = %d (interior passes)" % k,
         "config": {"tblock": k, "tile": tile, "zchunk": zchunk},
         "sources_sha256": kernel_sources_sha256(k, tile),
         "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
         "algorithmic_bytes_per_launch": alg, "fetch_scale": fs, "write_scale": ws,
         "note": "FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by the ratio of the exact "
                 "bytes of the bench's 1 GiB device copies to what the same counters read for "
                 "them", "commands": [fetch_cmd, write_cmd]}
    with open(TRAFFIC_JSON, "w") as f:
        json.dump(t, f, indent=1)
    lines = ["# HBM traffic counters: 3D variable-D interior pass, 256^3, s = 100", "",
             "Commands (from /tmp, with the repository as the working copy):", "",
             "    " + fetch_cmd, "    " + write_cmd, "",
             "Copy calibration: FETCH_SIZE scaled by %.4f, WRITE_SIZE by %.4f (exact bytes of "
             "the bench's 1 GiB device copies over what the counters read for them)." % (fs, ws),
             "",
             "| Kernel | grid | dispatches | FETCH KiB/disp | WRITE KiB/disp | read MB | write MB |",
             "|---|---|---|---|---|---|---|"]
    for key in sorted(fg, key=lambda kk: -len(fg[kk]) * sum(fg[kk]))[:12]:
        fv = sum(fg[key]) / len(fg[key])
        wv = sum(wg.get(key, [0.0])) / max(1, len(wg.get(key, [])))
        lines.append("| `%s` | %d | %d | %.1f | %.1f | %.1f | %.1f |" % (
            _short(key[0]), key[1], len(fg[key]), fv, wv, fv * 1024 * fs / 1e6,
            wv * 1024 * ws / 1e6))
    lines += ["", "Dominant kernel %s (grid %d): %.1f MB read and %.1f MB written per launch; "
              "algorithmic %.1f MB read (16 B complex W + 8 B D per point) and %.1f MB written "
              "(16 B per point), so %.3f x the algorithmic bytes." % (
                  " and ".join("`%s`" % _short(key[0]) for key in sorted(keys)), dom[1],
                  fetch / 1e6, write / 1e6, 24 * n / 1e6, 16 * n / 1e6,
                  (fetch + write) / alg)]
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return t


SQ_DERIVED_NOTE = (
    "Counters are summed over the GPU per dispatch and averaged over the dispatches of the "
    "kernel. SQ_BUSY_CU_CYCLES counts cycles summed over CUs; SQ_ACTIVE_INST_VALU and the "
    "wait counters count 4-cycle units per wavefront; the LDS bandwidth counters count "
    "64-byte units. Derived: VALU busy per SIMD = 4 ACTIVE_INST_VALU / (4 BUSY_CU_CYCLES); "
    "LDS bytes per CU-cycle = 64 (LOAD_BANDWIDTH + STORE_BANDWIDTH) / BUSY_CU_CYCLES against "
    "128 per cycle; FP64 share = (ADD + MUL + FMA F64) / INSTS_VALU.")


def summarize_sq(dirs, pattern, commands, title, out_md):
    """SQ counters of one kernel from rocprofv3 --pmc runs (one directory per pass)."""
    vals, grid, name = {}, None, None
    for d in dirs:
        per = {}
        for r in _csv_rows(d, "counter_collection.csv"):
            if pattern not in r["Kernel_Name"]:
                continue
            key = (r["Kernel_Name"], int(r["Grid_Size"]))
            per.setdefault(key, {}).setdefault(r["Counter_Name"], []).append(
                float(r["Counter_Value"]))
        if not per:
            raise SystemExit("no dispatch of %s under %s" % (pattern, d))
        key = max(per, key=lambda k: len(next(iter(per[k].values()))))
        grid = key[1]
        keys = sorted(k for k in per if k[1] == grid)   # e.g. both march directions
        name = " and ".join(k[0] for k in keys)
        for c in per[key]:
            v = [x for k in keys for x in per[k].get(c, [])]
            vals[c] = sum(v) / len(v)
    g = vals.get
    derived = {}
    if g("SQ_BUSY_CU_CYCLES"):
        bc = g("SQ_BUSY_CU_CYCLES")
        if g("SQ_ACTIVE_INST_VALU") is not None:
            derived["VALU busy per SIMD"] = g("SQ_ACTIVE_INST_VALU") / bc
        if g("SQ_INSTS_LDS_LOAD_BANDWIDTH") is not None:
            lb = 64 * (g("SQ_INSTS_LDS_LOAD_BANDWIDTH") + g("SQ_INSTS_LDS_STORE_BANDWIDTH", 0.0))
            derived["LDS bytes per CU-cycle (of 128)"] = lb / bc
        if g("SQ_LDS_BANK_CONFLICT") is not None:
            derived["LDS bank-conflict cycles per CU-cycle"] = g("SQ_LDS_BANK_CONFLICT") / bc
    if g("SQ_INSTS_VALU") and g("SQ_INSTS_VALU_FMA_F64") is not None:
        derived["FP64 share of VALU instructions"] = (
            g("SQ_INSTS_VALU_FMA_F64") + g("SQ_INSTS_VALU_ADD_F64") + g("SQ_INSTS_VALU_MUL_F64")) / g(
            "SQ_INSTS_VALU")
    if g("SQ_WAVES") and g("SQ_INSTS_VALU"):
        derived["VALU instructions per wavefront"] = g("SQ_INSTS_VALU") / g("SQ_WAVES")
        if g("SQ_INSTS_SALU") is not None:
            derived["SALU instructions per wavefront"] = g("SQ_INSTS_SALU") / g("SQ_WAVES")
        if g("SQ_INSTS_LDS") is not None:
            derived["LDS instructions per wavefront"] = g("SQ_INSTS_LDS") / g("SQ_WAVES")
    if g("SQ_WAVE_CYCLES") and g("SQ_WAIT_INST_LDS") is not None:
        derived["share of wave time waiting to issue LDS"] = g("SQ_WAIT_INST_LDS") / g("SQ_WAVE_CYCLES")
    lines = ["# SQ counters: %s" % title, "",
             "Commands (from /tmp, with the repository as the working copy), one per counter pass:",
             ""] + ["    " + c for c in commands] + [
             "", "Kernels (dispatches of all averaged) `%s`, grid %d threads." % (_short(name).replace(" and ", "` and `"), grid), "",
             "| Counter | per dispatch |", "|---|---|"]
    for c in sorted(vals):
        lines.append("| %s | %.4g |" % (c, vals[c]))
    lines += ["", "| Derived | value |", "|---|---|"]
    for k, v in derived.items():
        lines.append("| %s | %.3f |" % (k, v))
    lines += ["", SQ_DERIVED_NOTE]
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return vals, derived


def kernel_name(k, tile):
    """The dominant kernel of a superstep at fused depth k and tile shape (option numbering)."""
    if k == 1:
        return "plane_stage<VARCOEF, Dirichlet, 3D, 64x4>"
    if tile in (4, 5):
        return ("tb3d_stage<VARCOEF, Dirichlet, K=%d> (%d-column output rows, halo wavefronts)"
                % (k, 64 if tile == 4 else 32))
    return "tb_stage<VARCOEF, Dirichlet, 3D, shape %d, K=%d>" % (tile, k)


def pass_schedule(s, k, supported=(2, 3)):
    """Stages per HBM pass for one superstep, as the library schedules them (3D)."""
    out, l = [], 0
    while l < s:
        kk = k if (k >= 2 and s - l >= k) else 1
        if kk >= 3 and s - l - kk == 1 and (kk - 1) in supported:
            kk -= 1
        if kk == 1 and k > 2 and s - l >= 2 and (s - l) in supported:
            kk = s - l
        if l == 0 and kk == s:
            kk = s - 1
            while kk >= 2 and kk not in supported:
                kk -= 1
        out.append(kk)
        l += kk
    return out


def cpu_baseline(prob, T, c_lib, min_seconds=8.0, max_supersteps=4):
    """The oracle (plain C stage loops, OpenMP over points) timed on the host cores, at all
    cores and at one thread, on a bounded sample of each configuration (about 40 s of CPU
    work in all). The headline value is the 256^3 variable-D workload at all cores:
    consecutive supersteps (s = 100) until about min_seconds. Per configuration the sample is
    stated next to it; rates are grid-point-stage updates per second (the adjoint: forward
    point-stages whose reverse sweep, stage recompute included, completes per second)."""
    from oracle import frkc2_coeffs as ocoeffs
    from oracle import stage as ostage
    from paper_1702_03818_amd import workloads as wl
    all_cores = ostage.threads()
    c = ocoeffs(S_STAGES, NU)

    def timed(fn):
        t0 = time.perf_counter()
        fn()
        return time.perf_counter() - t0

    def both(fn, work_all, work_one, fn_one=None):
        out = {}
        for name, nthr, f, work in (("all_cores", all_cores, fn, work_all),
                                    ("one_thread", 1, fn_one or fn, work_one)):
            ostage.set_threads(nthr)
            dt = timed(f)
            out[name] = {"threads": nthr, "seconds": dt, "value": work / dt}
        ostage.set_threads(all_cores)
        return out

    # C2 headline: whole supersteps at all cores
    w = prob.w0
    n = 0
    t0 = time.perf_counter()
    while True:
        w = ostage.superstep(prob, w, T * c.a_re, T * c.a_im)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds or n >= max_supersteps:
            break
    ups = prob.npoints * S_STAGES * n / dt
    cfg = {}
    # C2 at one thread: the first 5 stages of a superstep on the full grid
    ostage.set_threads(1)
    d1 = timed(lambda: ostage.superstep(prob, prob.w0, T * c.a_re[:5], T * c.a_im[:5]))
    ostage.set_threads(all_cores)
    cfg["C2_diffusion3d_256"] = {
        "all_cores": {"threads": all_cores, "seconds": dt, "value": ups,
                      "sample": "%d whole supersteps (s = 100)" % n},
        "one_thread": {"threads": 1, "seconds": d1, "value": prob.npoints * 5 / d1,
                       "sample": "the first 5 stages of one superstep, full grid"}}
    # C1: the whole 1D heat run (20 supersteps of s = 16 on 1024 points), median of 3
    p1 = wl.heat1d()
    c16 = ocoeffs(16, NU)
    T1 = CFL * c16.beta_bar / (4.0 / (p1.h * p1.h))

    def heat():
        ts = []
        for _ in range(3):
            ts.append(timed(lambda: ostage.run(p1, 16, 20, T=T1, coeffs=c16)))
        return sorted(ts)[1]
    r = {}
    for name, nthr in (("all_cores", all_cores), ("one_thread", 1)):
        ostage.set_threads(nthr)
        sec = heat()
        r[name] = {"threads": nthr, "seconds": sec, "ms": sec * 1e3,
                   "value": p1.npoints * 16 * 20 / sec}
    ostage.set_threads(all_cores)
    r["sample"] = "the whole run (20 supersteps, s = 16, 1024 points), median of 3"
    cfg["C1_heat1d_1024"] = r
    # C3: the first 5 stages of one s = 400 superstep of the 4096^2 porous medium
    p3 = wl.porous2d()
    c400 = ocoeffs(400, NU)
    T3 = 0.002 * c400.beta_bar / ostage.rho_bound(p3, p3.w0)
    r = both(lambda: ostage.superstep(p3, p3.w0, T3 * c400.a_re[:5], T3 * c400.a_im[:5]),
             p3.npoints * 5, p3.npoints * 5)
    r["sample"] = "the first 5 stages of one s = 400 superstep, full 4096^2 grid"
    cfg["C3_porous2d_4096"] = r
    del p3
    # C4: whole supersteps of sampled problems of the 512-problem batch
    batch = wl.batched()
    sample_all = batch[::32]
    sample_one = batch[::128]

    def run_batch(sample):
        def f():
            for p, s in sample:
                cs = ocoeffs(s, NU)
                Tb = CFL * cs.beta_bar / ostage.rho_bound(p)
                ostage.superstep(p, p.w0, Tb * cs.a_re, Tb * cs.a_im)
        return f
    for p, s in sample_all:   # stepsizes and bounds outside the timed region
        ocoeffs(s, NU)
    r = both(run_batch(sample_all), sum(p.npoints * s for p, s in sample_all),
             sum(p.npoints * s for p, s in sample_one), run_batch(sample_one))
    r["sample"] = ("one superstep of every 32nd problem (%d problems) at all cores, of every "
                   "128th (%d) at one thread" % (len(sample_all), len(sample_one)))
    cfg["C4_batched_512"] = r
    del batch
    # C5: the adjoint of one superstep of the 128^3 problem (s = 64; one thread: 16 stages)
    p5, target = wl.adjoint3d()
    c64 = ocoeffs(64, NU)
    T5 = CFL * c64.beta_bar / ostage.rho_bound(p5)
    lam = 2 * (p5.w0.reshape(-1) - target.reshape(-1))

    def adj(k):
        return lambda: ostage.adjoint(p5, p5.w0, lam, T5 * c64.a_re[:k], T5 * c64.a_im[:k],
                                      grad_logD=np.zeros(p5.npoints))
    r = both(adj(64), p5.npoints * 64, p5.npoints * 16, adj(16))
    r["sample"] = ("the adjoint of one superstep (forward recompute with the stage store, then "
                   "the reverse stages and the log-D gradient): s = 64 at all cores, the first "
                   "16 stages at one thread")
    cfg["C5_adjoint3d_128"] = r
    return {"value": ups, "unit": "grid-point-stage updates/s", "cores": all_cores,
            "kind": "oracle",
            "sample": "%d consecutive supersteps (s=100) of the same 256^3 variable-D problem, "
                      "%.1f s" % (n, dt),
            "configs": cfg,
            "heat1d": {"cpu_ms": cfg["C1_heat1d_1024"]["all_cores"]["ms"],
                       "value": cfg["C1_heat1d_1024"]["all_cores"]["value"],
                       "sample": cfg["C1_heat1d_1024"]["sample"]}}


def batched_leg(F, wl, torch, reps=5):
    """512 independent 2D/3D variable-D problems (uneven sizes and s), one superstep each:
    one graph launch vs the plain path called problem by problem."""
    log("generating the 512-problem batch")
    probs = wl.batched()
    ws_list, D_list, T_list, s_list, grids = [], [], [], [], []
    for p, s in probs:
        w = torch.tensor(p.w0.reshape(-1), dtype=torch.float64, device="cuda")
        D = torch.tensor(p.D.reshape(-1), dtype=torch.float64, device="cuda")
        _, _, info, _ = F.frkc2_coeffs(s, NU)
        T_list.append(CFL * info["beta_bar"] / F.frkc2_rho_bound(p, None, D))
        ws_list.append(w)
        D_list.append(D)
        s_list.append(s)
        grids.append(p)
    work = sum(p.npoints * s for p, s in probs)
    # the built-in launch configuration (the library's timing autotuner is switched off)
    k3, cols3, k2 = F.frkc2_batched_config(grids, s_list)
    log("batched configuration: k3=%d cols=%d k2=%d (built-in)" % (k3, cols3, k2))
    args = F.BatchedArgs(grids, ws_list, D_list, T_list, s_list)
    F.frkc2_step_batched(args)          # builds and captures the graph
    for _ in range(2):                  # and runs until the clocks have settled
        F.frkc2_step_batched(args)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        F.frkc2_step_batched(args)
    e1.record()
    torch.cuda.synchronize()
    t_b = e0.elapsed_time(e1) / reps
    log("batched: %.2f ms per round" % t_b)
    # plain path, problem after problem
    def plain():
        for p, w, D, T, s in zip(grids, ws_list, D_list, T_list, s_list):
            F.frkc2_step(p, w, D, T=T, s=s, nsteps=1)
    plain()
    torch.cuda.synchronize()
    e0.record()
    plain()
    e1.record()
    torch.cuda.synchronize()
    t_p = e0.elapsed_time(e1)
    log("plain sequential: %.2f ms per round" % t_p)
    F.frkc2_batched_release()
    return {"problems": len(probs), "points": int(sum(p.npoints for p, _ in probs)),
            "point_stages": int(work), "ms_per_round": t_b, "value": work / (t_b * 1e-3),
            "unit": "grid-point-stage updates/s",
            "plain_sequential_ms": t_p, "plain_sequential_value": work / (t_p * 1e-3),
            "speedup_vs_plain": t_p / t_b,
            "config": {"k3": k3, "cols3": cols3, "k2": k2, "source": "built-in"}}


def heat1d_leg(F, wl, torch, reps=10):
    """1D heat equation, 1024 points periodic, s = 16, 20 supersteps with T = 0.9 betabar / rho
    (rho = 4/h^2, exact for the periodic Laplacian): the whole run fits in LDS, so it is
    timed as a latency figure (median of reps runs), not against the HBM roofline."""
    p = wl.heat1d()
    s, nsup = 16, 20
    _, _, info16, _ = F.frkc2_coeffs(s, NU)
    T = CFL * info16["beta_bar"] / (4.0 / (p.h * p.h))
    w0 = torch.tensor(p.w0.reshape(-1), dtype=torch.float64, device="cuda")
    w = w0.clone()
    F.frkc2_step(p, w, None, T=T, s=s, nsteps=nsup)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        w.copy_(w0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        F.frkc2_step(p, w, None, T=T, s=s, nsteps=nsup)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = sorted(times)[len(times) // 2]
    work = p.npoints * s * nsup
    return {"grid": [p.npoints], "s": s, "supersteps": nsup, "T": T, "gpu_ms": ms,
            "value": work / (ms * 1e-3), "unit": "grid-point-stage updates/s"}


def porous2d_leg(F, wl, torch, nsup=5):
    """2D porous-medium equation u_t = div(u^2 grad u), 4096^2 periodic, s = 400, 5 supersteps
    with T = cfl betabar / rho of the current state at cfl = 0.002 (the complex stages of the
    nonlinear operator are stable there), launch configuration from the library's autotuner.
    Algorithmic bytes: 32 per point and pass (complex W in and out)."""
    p = wl.porous2d()
    s = 400
    w0 = torch.tensor(p.w0.reshape(-1), dtype=torch.float64, device="cuda")
    w = w0.clone()
    tune = F.frkc2_autotune(p, w, None, s=s, nu=NU, reps=1)
    w.copy_(w0)
    F.frkc2_step(p, w, None, cfl=0.002, s=s, nsteps=1)
    torch.cuda.synchronize()
    w.copy_(w0)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    F.frkc2_step(p, w, None, cfl=0.002, s=s, nsteps=nsup)
    e1.record()
    torch.cuda.synchronize()
    F.frkc2_set_option(F.OPT_CLEAR_TUNED, 0)
    ms = e0.elapsed_time(e1) / nsup
    k = max(1, tune["tblock"])
    npass = -(-s // k)
    gbs = 32.0 * p.npoints * npass / (ms * 1e-3) / 1e9
    log("porous 2D: %.3f ms per superstep (k=%d tile=%d)" % (ms, tune["tblock"], tune["tile"]))
    return {"grid": [4096, 4096], "s": s, "supersteps": nsup, "cfl": 0.002,
            "ms_per_superstep": ms, "value": p.npoints * s / (ms * 1e-3),
            "unit": "grid-point-stage updates/s", "stages_per_pass": tune["tblock"],
            "tile": tune["tile"], "bytes_per_point_per_pass": 32, "achieved_gbs": gbs,
            "frac": gbs / HBM_PEAK_GBS,
            "bound": "valu (FP64 issue; frac is the HBM fraction, not this pass's roofline)"}


def adaptive_leg(F, wl, torch, prob, D, rho, info):
    """Error-controlled integration on the 256^3 workload: the same span as one benchmark
    step (10 supersteps at T = 0.9 betabar(100) / rho), tol = 1e-3, first trial T = that T.
    Updates/s counts the stages of every attempt (rejected ones included)."""
    T = CFL * info["beta_bar"] / rho
    span = SUPERSTEPS * T
    w0 = torch.tensor(prob.w0.reshape(-1), dtype=torch.float64, device="cuda")
    w = w0.clone()
    F.frkc2_integrate(prob, w, D, t_span=span, T0=T, tol=1e-3)      # warm-up, coefficients
    torch.cuda.synchronize()
    w.copy_(w0)
    t0 = time.perf_counter()
    st, trace = F.frkc2_integrate(prob, w, D, t_span=span, T0=T, tol=1e-3, trace_cap=4096)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n = prob.npoints
    log("adaptive: %d attempts (%d rejected), %d stages, %.1f ms" % (
        st["attempts"], st["rejected"], st["stages"], dt * 1e3))
    return {"t_span": span, "tol": 1e-3, "attempts": st["attempts"], "accepted": st["accepted"],
            "rejected": st["rejected"], "stages": st["stages"],
            "s_used": sorted(set(int(v) for v in trace[:, 2])), "wall_ms": dt * 1e3,
            "value": n * st["stages"] / dt, "unit": "grid-point-stage updates/s (all attempts)",
            "fixed_step_stages": S_STAGES * SUPERSTEPS}


def brusselator_throughput(F, wl, torch):
    """2048^2 Brusselator supersteps (s = 100, T = 0.9 betabar / rho of the current state), the
    default passes of 4 fused stages and one stage per pass: 10 timed after 20 warm-up ones."""
    big = wl.brusselator(2048)
    n = big.npoints

    def superstep_ms(depth):
        F.frkc2_set_option(F.OPT_TBLOCK, depth)
        try:
            w = torch.tensor(big.w0.reshape(-1), dtype=torch.float64, device="cuda")
            # warm-up long enough for the clocks to settle after the host-side set-up (the
            # first few supersteps after an idle gap run up to 20 % slower)
            F.frkc2_step(big, w, None, cfl=CFL, s=S_STAGES, nsteps=20)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            F.frkc2_step(big, w, None, cfl=CFL, s=S_STAGES, nsteps=10)
            e1.record()
            torch.cuda.synchronize()
        finally:
            F.frkc2_set_option(F.OPT_TBLOCK, 0)
        return e0.elapsed_time(e1) / 10

    ms = superstep_ms(0)        # the default: passes of 4 fused stages
    ms1 = superstep_ms(1)       # one stage per pass, for comparison
    # 64 B per point and pass (two complex values in and out), 4 stages per pass
    thr = {"grid": [2048, 2048], "s": S_STAGES, "stages_per_pass": 4, "ms_per_superstep": ms,
           "value": n * S_STAGES / (ms * 1e-3), "unit": "grid-point-stage updates/s (2 species)",
           "bytes_per_point_stage": 16,
           "achieved_gbs": 16 * n * S_STAGES / (ms * 1e-3) / 1e9,
           "one_stage_passes": {"ms_per_superstep": ms1, "value": n * S_STAGES / (ms1 * 1e-3)}}
    return thr


def brusselator_leg(F, wl, torch):
    """The paper's two-species Brusselator (Sec. 3.1). Throughput: 10 supersteps (s = 100,
    T = 0.9 betabar / rho of the current state) on a 2048^2 grid. Accuracy: error-controlled
    runs on the paper's 200^2 grid from its initial data to t = 1 at several tolerances, with
    the accepted steps, the stages and the max error against a tol = 1e-8 run (the paper's
    steps-to-error comparison, FRKC2 alone)."""
    thr = brusselator_throughput(F, wl, torch)
    p = wl.brusselator(200)
    runs = []
    ref = torch.tensor(p.w0.reshape(-1), dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    st_ref, _ = F.frkc2_integrate(p, ref, None, t_span=1.0, T0=1e-4, tol=1e-8, max_attempts=200000)
    ref_s = time.perf_counter() - t0
    for tol in (1e-3, 1e-4, 1e-5, 1e-6):
        w = torch.tensor(p.w0.reshape(-1), dtype=torch.float64, device="cuda")
        t0 = time.perf_counter()
        st, _ = F.frkc2_integrate(p, w, None, t_span=1.0, T0=1e-4, tol=tol, max_attempts=200000)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        err = float(torch.max(torch.abs(w - ref)))
        runs.append({"tol": tol, "accepted": st["accepted"], "rejected": st["rejected"],
                     "stages": st["stages"], "max_error": err, "wall_ms": dt * 1e3})
        log("brusselator tol %.0e: %d steps, %d stages, error %.2e" % (tol, st["accepted"],
                                                                     st["stages"], err))
    return {"throughput": thr, "t_end": 1.0, "reference": {"tol": 1e-8, "accepted": st_ref["accepted"],
                                                          "stages": st_ref["stages"],
                                                          "wall_s": ref_s},
            "steps_to_error": runs}


def fourth_order_leg(F, wl, torch, steps=(10, 20, 40, 80, 160, 320), m_ref=2560):
    """Steps to error on the Brusselator (Sec. 3.1 problem, 200^2, t = 0 .. 1): fixed-step
    FRKC4s (the split fourth-order scheme of Sec. 4.1, nsub = 4 reaction substeps) against
    fixed-step FRKC2 with the same number of steps. Each run uses the smallest stage count
    whose extent covers its step (FRKC4s: (T/4) rho_A <= 0.9 betabar_4(s), rho_A = 8 d / h^2;
    FRKC2: T rho <= 0.7 betabar(s) with rho the Gershgorin bound of the initial state).
    Errors are max norms against FRKC4s with m_ref steps (a self-convergence reference)."""
    p = wl.brusselator(200)
    rho_a = 8 * p.d_const / (p.h * p.h)
    w0 = torch.tensor(p.w0.reshape(-1), dtype=torch.float64, device="cuda")
    rho2 = F.frkc2_rho_bound(p, w0, None)

    def s4_for(T):
        s = 4
        while F.frkc4_coeffs(s, NU)[2]["beta_bar"] * 0.9 < 0.25 * T * rho_a:
            s += 4
        return s

    def s2_for(T):
        s = 2
        while F.frkc2_coeffs(s, NU)[2]["beta_bar"] * 0.7 < T * rho2:
            s += 2
        return s

    def run4(m):
        T = 1.0 / m
        s = s4_for(T)
        w = w0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F.frkc4s_step(p, w, T, s, nsub=4, nu=NU, nsteps=m)
        torch.cuda.synchronize()
        return w, s, time.perf_counter() - t0

    ref, s_ref, t_ref = run4(m_ref)
    out = {"grid": [200, 200], "t_end": 1.0, "nsub": 4,
           "reference": {"scheme": "FRKC4s", "steps": m_ref, "s": s_ref, "wall_s": t_ref},
           "frkc4s": [], "frkc2": []}
    for m in steps:
        w, s, dt = run4(m)
        err = float(torch.max(torch.abs(w - ref)))
        out["frkc4s"].append({"steps": m, "s": s, "diffusion_stages": m * 4 * s,
                              "max_error": err, "wall_ms": dt * 1e3})
        T = 1.0 / m
        s2 = s2_for(T)
        w = w0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F.frkc2_step(p, w, None, T=T, s=s2, nsteps=m)
        torch.cuda.synchronize()
        dt2 = time.perf_counter() - t0
        err2 = float(torch.max(torch.abs(w - ref)))
        out["frkc2"].append({"steps": m, "s": s2, "stages": m * s2, "max_error": err2,
                             "wall_ms": dt2 * 1e3})
        log("fourth order: %d steps: FRKC4s s=%d error %.2e; FRKC2 s=%d error %.2e"
            % (m, s, err, s2, err2))
    e = [r["max_error"] for r in out["frkc4s"]]
    out["frkc4s_order"] = [float(np.log2(e[i] / e[i + 1])) for i in range(len(e) - 1)]
    e2 = [r["max_error"] for r in out["frkc2"]]
    out["frkc2_order"] = [float(np.log2(e2[i] / e2[i + 1])) for i in range(len(e2) - 1)]
    return out


def adjoint_leg(F, wl, torch, reps=3):
    """3D 128^3 variable D, s = 64, 8 supersteps, J = sum (w - target)^2: forward alone
    and forward + adjoint through the autograd function."""
    from paper_1702_03818_amd.autograd import _want_store, superstep_fn
    log("generating the adjoint workload")
    p, target = wl.adjoint3d()
    s, nsteps = 64, 8
    u0 = torch.tensor(p.w0.reshape(-1), dtype=torch.float64, device="cuda")
    logD = torch.tensor(np.log(p.D.reshape(-1)), dtype=torch.float64, device="cuda")
    tgt = torch.tensor(target.reshape(-1), dtype=torch.float64, device="cuda")
    D = torch.exp(logD)
    _, _, info, _ = F.frkc2_coeffs(s, NU)
    T = CFL * info["beta_bar"] / F.frkc2_rho_bound(p, None, D)

    def fwd():
        w = u0.clone()
        F.frkc2_step(p, w, D, T=T, s=s, nsteps=nsteps)
        return w

    def fwd_bwd(store):
        u = u0.clone().requires_grad_(True)
        ld = logD.clone().requires_grad_(True)
        J = ((superstep_fn(u, ld, p, T, s, nsteps, store_stages=store) - tgt) ** 2).sum()
        J.backward()
        return J

    # the autograd function's automatic choice (the stage store when it fits a quarter of the
    # free memory, as it does here: 8 x 64 x 128^3 complex states, 17.2 GB), then the
    # per-superstep checkpoints that recompute the stages in the backward
    res = {"stage_store": _want_store(p, s, nsteps, u0.device)}
    for name, fn in (("forward", fwd), ("forward_backward", lambda: fwd_bwd(None)),
                     ("forward_backward_checkpoints", lambda: fwd_bwd(False))):
        fn()
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        res[name + "_ms"] = e0.elapsed_time(e1) / reps
    work = p.npoints * s * nsteps
    res.update({"grid": [128] * 3, "s": s, "supersteps": nsteps, "forward_point_stages": work,
                "value_forward": work / (res["forward_ms"] * 1e-3),
                "value_forward_backward": work / (res["forward_backward_ms"] * 1e-3),
                "unit": "forward grid-point-stage updates/s",
                "backward_over_forward": res["forward_backward_ms"] / res["forward_ms"]})
    log("adjoint: forward %.2f ms, forward+backward %.2f ms (stage store %s), with "
        "checkpoints %.2f ms" % (res["forward_ms"], res["forward_backward_ms"],
                                 res["stage_store"], res["forward_backward_checkpoints_ms"]))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-problem batched leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint leg")
    ap.add_argument("--no-adaptive", action="store_true", help="skip the error-control leg")
    ap.add_argument("--no-bruss", action="store_true", help="skip the Brusselator leg")
    ap.add_argument("--only", choices=("bruss-throughput", "batched", "adjoint", "porous2d", "heat1d",
                                       "fourth-order"),
                    help="run only this measurement and print its JSON (for profiling)")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 1D heat and 2D porous-medium legs")
    ap.add_argument("--tblock", type=int, default=0, choices=(0, 1, 2, 3),
                    help="stages fused per HBM pass in the timed run (0: autotune)")
    ap.add_argument("--tile", type=int, default=0, help="tile shape with --tblock (0: automatic)")
    ap.add_argument("--zchunk", type=int, default=0, help="z planes per workgroup with --tblock")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="write the kernel-trace summary under profiles/ from a rocprofv3 "
                         "--kernel-trace run of this script (no GPU needed)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the HBM traffic summary under profiles/ from rocprofv3 --pmc "
                         "FETCH_SIZE and WRITE_SIZE runs of this script (no GPU needed)")
    ap.add_argument("--summarize-sq", nargs="+", metavar=("OUT_MD", "DIR"),
                    help="write the SQ-counter summary of one kernel (--sq-kernel, --sq-title) "
                         "from rocprofv3 --pmc directories (one per pass) and exit")
    ap.add_argument("--trace-kernel", default=None, help="with --summarize-trace: kernel name part")
    ap.add_argument("--trace-title", default=None)
    ap.add_argument("--trace-note", default=None)
    ap.add_argument("--trace-out", default=None, help="with --summarize-trace: output file")
    ap.add_argument("--trace-by-kernel", action="store_true",
                    help="with --summarize-trace: one row per kernel over all grid sizes")
    ap.add_argument("--sq-kernel", default="tb3d_stage<1, 1, 3, false, false, false, false, 64, ")
    ap.add_argument("--sq-title", default="3D variable-D interior pass, 256^3, s = 100, k = 3")
    ap.add_argument("--command", action="append", default=[],
                    help="with --summarize-*: the command line(s) that produced the data")
    args = ap.parse_args()
    if args.summarize_sq:
        summarize_sq(args.summarize_sq[1:], args.sq_kernel, args.command, args.sq_title,
                     args.summarize_sq[0])
        return
    if args.summarize_trace or args.summarize_counters:
        k = args.tblock or 2
        tile = args.tile or (4 if k >= 2 else 1)
        if args.summarize_trace:
            out_md = os.path.join(ROOT, "profiles", "kernel_trace_stage3d_256.md")
            if args.trace_out:
                out_md = args.trace_out
            avg = summarize_trace(args.summarize_trace, args.command[0], k, tile, out_md,
                                  args.trace_kernel, args.trace_title, args.trace_note,
                                  args.trace_by_kernel)
            print("dominant kernel average %.2f us" % avg)
        else:
            t = summarize_counters(args.summarize_counters[0], args.summarize_counters[1],
                                   args.command[0], args.command[1], k, tile, args.zchunk,
                                   os.path.join(ROOT, "profiles", "counters_stage3d_256.md"))
            print(json.dumps(t))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the FRKC2 superstep here is a single-GPU build "
              "(multi-GPU sharding is designed but not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1702_03818_amd import frkc2 as F
    from paper_1702_03818_amd import workloads as wl

    torch.cuda.set_device(0)
    if args.only:
        legs = {"bruss-throughput": brusselator_throughput, "batched": batched_leg,
                "adjoint": adjoint_leg, "porous2d": porous2d_leg, "heat1d": heat1d_leg,
                "fourth-order": fourth_order_leg}
        print(json.dumps({args.only: legs[args.only](F, wl, torch)}), flush=True)
        return
    log("generating the 3D workload (n=%d)" % args.n)
    prob = wl.diffusion3d(n=args.n)
    N = prob.npoints
    w0 = torch.tensor(prob.w0.reshape(-1), dtype=torch.float64, device="cuda")
    D = torch.tensor(prob.D.reshape(-1), dtype=torch.float64, device="cuda")
    w = w0.clone()
    a_re, a_im, info, _ = F.frkc2_coeffs(S_STAGES, NU)
    rho = F.frkc2_rho_bound(prob, None, D)
    T = CFL * info["beta_bar"] / rho
    log("rho=%.6e T=%.6e beta_bar=%.3f" % (rho, T, info["beta_bar"]))

    # Launch configuration: measured by the library's autotuner on this grid
    # (outside the timed region), or fixed from the command line.
    if args.tblock == 0:
        tune = F.frkc2_autotune(prob, w, D, s=S_STAGES, nu=NU, reps=2)
        kdepth, tile, zchunk = tune["tblock"], tune["tile"], tune["zchunk"]
        log("autotune: k=%d tile=%d zchunk=%d (%.3f ms per superstep; default %.3f ms; "
            "%d candidates)" % (kdepth, tile, zchunk, tune["ms_best"], tune["ms_default"],
                                tune["candidates"]))
    else:
        tune = None
        kdepth, tile, zchunk = args.tblock, args.tile, args.zchunk
        F.frkc2_set_option(F.OPT_TBLOCK, kdepth)
        F.frkc2_set_option(F.OPT_TILE, tile)
        F.frkc2_set_option(F.OPT_ZCHUNK, zchunk)
        if tile == 0:
            tile = 4 if kdepth >= 2 else 1

    def restore_config():
        F.frkc2_set_option(F.OPT_TBLOCK, 0 if tune is not None else kdepth)

    def step():
        st = F.frkc2_step(prob, w, D, T=T, s=S_STAGES, nsteps=SUPERSTEPS, stats=True)
        nrm = F.frkc2_reduce(F.RED_SUMSQ, w)
        return st, nrm

    # A plain device-to-device copy of known size: the achievable streaming
    # bandwidth of this GPU, and the reference dispatch for scaling the
    # FETCH_SIZE / WRITE_SIZE counters.
    copy_bytes = 1 << 30
    src = torch.empty(copy_bytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    dst.copy_(src)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * copy_bytes / (e0.elapsed_time(e1) * 1e-3) / 1e9
    log("copy bandwidth %.1f GB/s" % copy_gbs)
    # The library's hand-written streaming copy (16 B per lane, four accesses in
    # flight, plain or nontemporal, 1..16 workgroups per CU): the best of these is
    # the measured HBM ceiling the stage kernels are compared with.
    stream = {}
    for bpc in (1, 2, 4, 8, 16):
        for nt in (False, True):
            F.frkc2_stream_copy(src, dst, bpc, nt)
            e0.record()
            for _ in range(5):
                F.frkc2_stream_copy(src, dst, bpc, nt)
            e1.record()
            torch.cuda.synchronize()
            stream[(bpc, nt)] = 5 * 2 * copy_bytes / (e0.elapsed_time(e1) * 1e-3) / 1e9
    best_stream = max(stream, key=stream.get)
    stream_gbs = stream[best_stream]
    assert torch.equal(dst, src)
    del src, dst
    log("streaming copy ceiling %.1f GB/s (%d workgroups per CU, %s)"
        % (stream_gbs, best_stream[0], "nontemporal" if best_stream[1] else "plain"))

    for i in range(args.warmup):
        step()
        log("warmup %d done" % i)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    last = None
    for i in range(args.steps):
        last = step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    log("timed %d steps: %.3f ms (events), %.3f s wall" % (args.steps, gpu_ms, wall))
    ms_per_step = gpu_ms / args.steps
    updates = N * S_STAGES * SUPERSTEPS * args.steps
    value = updates / (gpu_ms * 1e-3)

    # Roofline of the stage passes. Algorithmic (minimal) HBM bytes per point
    # and pass: input 8 (real w, first pass) or 16 (complex), D 8, output 16
    # (complex) or 8 (real w, last pass; the step's last superstep keeps W^L
    # complex for the Im diagnostic). The average launch time is the
    # event-timed region divided by the stage launches in it (every other
    # kernel in the region counts against it).
    sched = pass_schedule(S_STAGES, kdepth)
    passes = len(sched) * SUPERSTEPS * args.steps
    per_superstep = []
    for last_complex in (False, True):
        b = 0
        for i, _ in enumerate(sched):
            b += (8 if i == 0 else 16) + 8
            b += 8 if (i == len(sched) - 1 and not last_complex) else 16
        per_superstep.append(b)
    alg_bytes = N * args.steps * ((SUPERSTEPS - 1) * per_superstep[0] + per_superstep[1])
    avg_launch_ms = gpu_ms / passes
    achieved = alg_bytes / (gpu_ms * 1e-3) / 1e9
    traffic, traffic_note = measured_traffic(kdepth, tile, zchunk)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "traffic_note": traffic_note,
            "kernel": kernel_name(kdepth, tile),
            "stages_per_pass": kdepth, "tile": tile, "zchunk": zchunk,
            "autotuned": tune is not None, "bytes_per_point_per_pass": 40,
            "algorithmic_bytes_per_launch": 40 * N, "avg_launch_ms": avg_launch_ms,
            "measured_ceiling": stream_gbs, "frac_of_measured_ceiling": achieved / stream_gbs,
            "measured_ceiling_note": "best of the library's streaming copy (frkc2_stream_copy) "
                                     "over workgroups per CU and nontemporal accesses, 1 GiB"}
    # Update-rate caps: HBM at the pass schedule's minimal bytes per point-stage, and FP64
    # at the stage's flops per point (variable D, fused order: per face 2 subtractions,
    # 1 add and 2 fma; then 2 multiplies and 4 fma; an fma counts 2 flops: 52 flops).
    sched = pass_schedule(S_STAGES, kdepth)
    bytes_per_update = 40.0 * len(sched) / S_STAGES
    roof["update_caps"] = {
        "hbm": HBM_PEAK_GBS * 1e9 / bytes_per_update, "fp64": FP64_PEAK_TFLOPS * 1e12 / 52.0,
        "bytes_per_update": bytes_per_update, "flops_per_update": 52,
        "value_over_min_cap": value / min(HBM_PEAK_GBS * 1e9 / bytes_per_update,
                                          FP64_PEAK_TFLOPS * 1e12 / 52.0)}
    # one-stage-per-pass reference on the same state (diagnostic)
    F.frkc2_set_option(F.OPT_TBLOCK, 1)
    F.frkc2_step(prob, w, D, T=T, s=S_STAGES, nsteps=1)
    e0.record()
    for _ in range(3):
        F.frkc2_step(prob, w, D, T=T, s=S_STAGES, nsteps=1)
    e1.record()
    torch.cuda.synchronize()
    k1_ms = e0.elapsed_time(e1) / 3
    restore_config()
    k1_ach = N * (32 + (S_STAGES - 2) * 40 + 32) / (k1_ms * 1e-3) / 1e9
    k1_ref = {"ms_per_superstep": k1_ms, "value": N * S_STAGES / (k1_ms * 1e-3),
              "achieved_gbs": k1_ach, "frac": k1_ach / HBM_PEAK_GBS}
    log("one stage per pass: %.3f ms per superstep, %.1f GB/s" % (k1_ms, k1_ach))
    out = {
        "metric": "grid-point-stage updates/s (FRKC2 superstep) + % HBM roofline",
        "value": value, "unit": "grid-point-stage updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded lognormal D, Gaussian blobs)",
        "config": {"workload": "3D u_t=div(D grad u), %d^3 FP64, 7-point, lognormal D (sigma=1), "
                               "Dirichlet zero, FRKC2 s=%d, %d supersteps per step"
                               % (args.n, S_STAGES, SUPERSTEPS),
                   "grid": [args.n] * 3, "s": S_STAGES, "supersteps": SUPERSTEPS, "nu": NU,
                   "T": T, "parallelism": "single GPU"},
        "roofline": roof,
        "one_stage_per_pass": k1_ref,
        "diagnostics": {"copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                        "stream_ceiling_gbs": stream_gbs,
                        "stream_config": {"workgroups_per_cu": best_stream[0],
                                          "nontemporal": best_stream[1]},
                        "frac_of_stream_ceiling": achieved / stream_gbs,
                        "im_ratio": last[0]["im_ratio"], "l2_norm": float(np.sqrt(last[1])),
                        "q_realised": info["q_realised"], "n_shrink": info["n_shrink"]},
    }
    out["adaptive"] = None if args.no_adaptive else adaptive_leg(F, wl, torch, prob, D, rho, info)
    del w0, w, D
    torch.cuda.empty_cache()
    out["batched"] = None if args.no_batched else batched_leg(F, wl, torch)
    torch.cuda.empty_cache()
    F.release_workspaces()
    out["adjoint"] = None if args.no_adjoint else adjoint_leg(F, wl, torch)
    torch.cuda.empty_cache()
    out["brusselator"] = None if args.no_bruss else brusselator_leg(F, wl, torch)
    torch.cuda.empty_cache()
    out["fourth_order"] = None if args.no_bruss else fourth_order_leg(F, wl, torch)
    torch.cuda.empty_cache()
    out["heat1d"] = None if args.no_small else heat1d_leg(F, wl, torch)
    out["porous2d"] = None if args.no_small else porous2d_leg(F, wl, torch)
    if not args.no_cpu:
        log("timing the CPU oracle on one superstep")
        out["cpu_baseline"] = cpu_baseline(prob, T, info)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
