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
S_STAGES = 100
SUPERSTEPS = 10
NU = 0.01
CFL = 0.9


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("stage.hip", "tblock.hip", "device_common.h", "api.cpp")


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1702_03818_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_stage3d_256.json")
    if not os.path.exists(path):
        return None, "no counter summary"
    with open(path) as f:
        t = json.load(f)
    if t.get("sources_sha256") != kernel_sources_sha256():
        return None, "counters were taken on different kernel sources"
    return t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"], t.get("note", "")


def pass_schedule(s, k, supported=(2, 3)):
    """Stages per HBM pass for one superstep, as the library schedules them (3D)."""
    out, l = [], 0
    while l < s:
        kk = k if (k >= 2 and s - l >= k) else 1
        if l == 0 and kk == s:
            kk = s - 1
            while kk >= 2 and kk not in supported:
                kk -= 1
        out.append(kk)
        l += kk
    return out


def cpu_baseline(prob, T, c_lib):
    """Oracle superstep (s = 100) on the full 256^3 grid, timed on the host cores."""
    from oracle import frkc2_coeffs as ocoeffs
    from oracle import stage as ostage
    c = ocoeffs(S_STAGES, NU)
    t0 = time.perf_counter()
    ostage.superstep(prob, prob.w0, T * c.a_re, T * c.a_im)
    dt = time.perf_counter() - t0
    ups = prob.npoints * S_STAGES / dt
    return {"value": ups, "unit": "grid-point-stage updates/s", "cores": ostage.threads(),
            "kind": "oracle",
            "sample": "one superstep (s=100) of the same 256^3 variable-D problem, %.1f s" % dt}


def batched_leg(F, wl, torch, reps=3):
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
    args = F.BatchedArgs(grids, ws_list, D_list, T_list, s_list)
    F.frkc2_step_batched(args)          # builds and captures the graph
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
            "speedup_vs_plain": t_p / t_b}


def adjoint_leg(F, wl, torch, reps=3):
    """3D 128^3 variable D, s = 64, 8 supersteps, J = sum (w - target)^2: forward alone
    and forward + adjoint through the autograd function."""
    from paper_1702_03818_amd.autograd import superstep_fn
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

    def fwd_bwd():
        u = u0.clone().requires_grad_(True)
        ld = logD.clone().requires_grad_(True)
        J = ((superstep_fn(u, ld, p, T, s, nsteps) - tgt) ** 2).sum()
        J.backward()
        return J

    res = {}
    for name, fn in (("forward", fwd), ("forward_backward", fwd_bwd)):
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
    log("adjoint: forward %.2f ms, forward+backward %.2f ms"
        % (res["forward_ms"], res["forward_backward_ms"]))
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
    ap.add_argument("--tblock", type=int, default=2, choices=(1, 2, 3),
                    help="stages fused per HBM pass in the timed run")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the FRKC2 superstep here is a single-GPU build "
              "(multi-GPU sharding is designed but not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1702_03818_amd import frkc2 as F
    from paper_1702_03818_amd import workloads as wl

    torch.cuda.set_device(0)
    F.frkc2_set_option(F.OPT_TBLOCK, args.tblock)
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
    del src, dst
    log("copy bandwidth %.1f GB/s" % copy_gbs)

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
    sched = pass_schedule(S_STAGES, args.tblock)
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
    traffic, traffic_note = measured_traffic()
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "traffic_note": traffic_note,
            "kernel": ("tb_stage<VARCOEF, Dirichlet, 3D, K=%d>" % args.tblock if args.tblock >= 2
                       else "plane_stage<VARCOEF, Dirichlet, 3D>"),
            "stages_per_pass": args.tblock, "bytes_per_point_per_pass": 40,
            "algorithmic_bytes_per_launch": 40 * N, "avg_launch_ms": avg_launch_ms}
    # one-stage-per-pass reference on the same state (diagnostic)
    F.frkc2_set_option(F.OPT_TBLOCK, 1)
    F.frkc2_step(prob, w, D, T=T, s=S_STAGES, nsteps=1)
    e0.record()
    for _ in range(3):
        F.frkc2_step(prob, w, D, T=T, s=S_STAGES, nsteps=1)
    e1.record()
    torch.cuda.synchronize()
    k1_ms = e0.elapsed_time(e1) / 3
    F.frkc2_set_option(F.OPT_TBLOCK, args.tblock)
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
                        "im_ratio": last[0]["im_ratio"], "l2_norm": float(np.sqrt(last[1])),
                        "q_realised": info["q_realised"], "n_shrink": info["n_shrink"]},
    }
    del w0, w, D
    torch.cuda.empty_cache()
    out["batched"] = None if args.no_batched else batched_leg(F, wl, torch)
    torch.cuda.empty_cache()
    F.release_workspaces()
    out["adjoint"] = None if args.no_adjoint else adjoint_leg(F, wl, torch)
    if not args.no_cpu:
        log("timing the CPU oracle on one superstep")
        out["cpu_baseline"] = cpu_baseline(prob, T, info)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
