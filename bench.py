"""Benchmark: pixel-inner-iterations per second of Algorithm 1 on MI355X.

A step is one full solve (n_outer outer steps x n_inner local steps over all
subdomains) of the workload, with the input already resident in HBM.  The
default workload is ROF (L2) denoising of a 2048 x 2048 image with 16 x 16
subdomains of 128 x 128, alpha 8, 500 outer x 5 FISTA steps.

Prints one JSON line with the throughput, the roofline of the dominant kernel
(its algorithmic bytes per launch over its average launch time, measured with
HIP events on the solve stream) and the FP64 CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pixel-iterations/s + % HBM peak, 2048^2 ROF 16x16 subdomains; batched vs plain"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3  # MI355X vector FP32 (256 CUs x 128 lanes x 2 flops x 2.4 GHz)


# source files of each timed kernel (the counters in profiles/traffic.txt are keyed by their hash)
KERNEL_SOURCES = {
    "k_persist_fista": ["persist.hip", "exchange.h", "fused_common.h", "fista_ops.h", "dtvdd_internal.h"],
    "k_fused_fista": ["fused.hip", "fused_common.h", "fista_ops.h", "dtvdd_internal.h"],
    "k_fused_fista_staggered": ["fused.hip", "fused_common.h", "fista_ops.h", "dtvdd_internal.h"],
    "k_fista_step": ["kernels.hip", "fista_ops.h", "dtvdd_internal.h"],
    # (a one-step launch that ends an outer step is timed with the multi-step ones)
    "k_fista_multi": ["fista_multi.hip", "fista_multi.h", "cp2_multi.h", "kernels.hip", "fista_ops.h",
                      "dtvdd_internal.h"],
    "k_cp2_step": ["kernels.hip", "cp2_ops.h", "fista_ops.h", "dtvdd_internal.h"],
    # (a one-step launch that ends an outer step is timed with the multi-step ones)
    "k_cp2_multi": ["cp2_multi.hip", "cp2_multi.h", "kernels.hip", "cp2_ops.h", "fista_ops.h", "dtvdd_internal.h"],
    "k_fused_cp2": ["fused_cp2.hip", "cp2_tile.h", "cp2_ops.h", "fused_common.h", "fista_ops.h", "dtvdd_internal.h"],
    "k_persist_cp2": ["persist_cp2.hip", "cp2_tile.h", "cp2_ops.h", "exchange.h", "fused_common.h", "fista_ops.h",
                      "dtvdd_internal.h"],
    "k_fused_bwd": ["fused_bwd.hip", "bwd.h", "exchange.h", "fused_common.h", "fista_ops.h", "dtvdd_internal.h"],
    "k_persist_bwd": ["fused_bwd.hip", "bwd.h", "exchange.h", "fused_common.h", "fista_ops.h", "dtvdd_internal.h"],
    "k_fused_fista_rec": ["fused.hip", "fused_common.h", "fista_ops.h", "dtvdd_internal.h"],
}


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per dispatch from the committed counter passes, or None when
    there are none for this kernel and workload or the kernel changed since."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if kernel not in KERNEL_SOURCES or not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1901_00682_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    digest = h.hexdigest()[:16]
    with open(path) as fh:
        for line in fh:
            w = line.split()
            if len(w) == 7 and not line.startswith("#") and w[0] == kernel and w[1] == workload and w[2] == digest:
                return (float(w[3]) * float(w[5]) + float(w[4]) * float(w[6])) * 1024.0
    return None


def fista_flops_per_pixel(K: int) -> float:
    """Algorithmic FP32 operations per pixel of one outer step with K FISTA
    steps (an FMA counts 2): per edge, the extrapolation y = x + beta (x - x_prev)
    (3, steps k >= 3), the gradient step a y + c' - kL (d_b - d_a) (5) and the
    projection (1); per pixel, the divergence (3) over its two owned edges; per
    edge and outer step, c' = (phat / tau - (f_b - f_a)) / L (4)."""
    plain, mom = 2 * (5 + 1) + 3, 2 * (3 + 5 + 1) + 3
    return 2 * 4 + plain * min(K, 2) + mom * max(K - 2, 0)


CP2_PROX_FLOPS = {"L2": 4, "L1": 5, "CV": 8}


def cp2_flops_per_pixel(K: int, fidelity: str) -> float:
    """Algorithmic FP32 operations per pixel of one outer step with K local
    primal-dual steps (an FMA counts 2): per edge and step, the dual update
    x_k = clamp(c_keep (x - tau_k (u_b - u_a)) + c_anchor phat) (7); per edge
    and step but the last, xbar = x + theta (x - x_prev) (3); per pixel and
    step, the divergence of xbar (3) and the primal update prox(u + sigma_k d)
    (2 + the prox: L2 4, L1 5, Chan-Vese 8)."""
    return 2 * 7 * K + 2 * 3 * (K - 1) + K * (3 + 2 + CP2_PROX_FLOPS[fidelity])


def workload(name: str):
    from paper_1901_00682_amd import synth

    if name == "rof2048":
        return synth.config2()
    if name == "rof8192":
        return synth.config2(size=8192)
    if name == "rof2000":  # 16 x 16 equal subdomains of 125 x 125: every one framed, interfaces on all sides
        return synth.rof_case("rof2000_16x16", 2000, 2000, 16, 16, 8.0, 0.1, 500, 5, workload=2)
    if name == "tvl1":
        return synth.config3()
    if name == "cv2048":
        return synth.cv_case()
    if name == "cv2000":  # cut at multiples of 128: the last subdomain row and column (80 wide) are framed
        c = synth.cv_case(size=2000)
        c.name = "cv2000_128cuts"
        c.row_cuts = synth.tile_cuts(2000, 128)
        c.col_cuts = synth.tile_cuts(2000, 128)
        return c
    raise SystemExit(f"unknown workload {name}")


def batched_measure(steps: int, warmup: int, schedule: str = "auto") -> dict:
    """64 mixed-size ROF images in one plan (the persistent schedule runs them
    in groups of cooperative launches) against the same images solved one by
    one, back to back; both timed with the host clock around whole solves."""
    import torch

    from paper_1901_00682_amd import dtvdd, synth

    cases = synth.config4()
    dev = torch.device("cuda:0")
    imgs = [dtvdd.Image(c.f.shape[0], c.f.shape[1], c.row_cuts, c.col_cuts, c.alpha) for c in cases]
    n_outer, K = cases[0].n_outer, cases[0].n_inner
    px = sum(c.f.size for c in cases)
    tiles = sum((len(c.row_cuts) - 1) * (len(c.col_cuts) - 1) for c in cases)
    f = torch.from_numpy(np.concatenate([c.f.ravel() for c in cases])).to(dev)
    plan = dtvdd.Plan(imgs, n_outer=n_outer, n_inner=K, schedule=schedule, device=dev)
    st = plan.new_state()
    for _ in range(max(warmup, 1)):
        plan.solve(f, state=st, want_stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.solve(f, state=st, want_stats=False, check=False)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    plan.status()
    # the same images one plan each, solved back to back
    plans = [dtvdd.Plan([im], n_outer=n_outer, n_inner=K, schedule=schedule, device=dev) for im in imgs]
    fs = [torch.from_numpy(c.f.ravel()).to(dev) for c in cases]
    sts = [p.new_state() for p in plans]
    for p, fi, si in zip(plans, fs, sts):
        p.solve(fi, state=si, want_stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, fi, si in zip(plans, fs, sts):
        p.solve(fi, state=si, want_stats=False, check=False)
    torch.cuda.synchronize()
    dt_seq = time.perf_counter() - t0
    for p in plans:
        p.status()
        p.close()
    out = {"workload": f"{len(cases)} ROF images, {px} pixels, {tiles} subdomains (cut at multiples of 128, "
                       f"ragged edge tiles), {n_outer} outer x {K} inner",
           "value": px * n_outer * K / dt, "unit": "pixel-inner-iterations/s", "ms_per_solve": dt * 1e3,
           "steps": steps, "schedule": plan.schedule(),
           "sequential_plain": {"value": px * n_outer * K / dt_seq, "ms": dt_seq * 1e3},
           "over_sequential": dt_seq / dt}
    plan.close()
    return out


def run_batched(args):
    """The batched workload alone, with the timing of its dominant kernel."""
    import torch

    from paper_1901_00682_amd import dtvdd, synth

    b = batched_measure(args.steps, args.warmup, args.schedule)
    cases = synth.config4()
    dev = torch.device("cuda:0")
    imgs = [dtvdd.Image(c.f.shape[0], c.f.shape[1], c.row_cuts, c.col_cuts, c.alpha) for c in cases]
    n_outer, K = cases[0].n_outer, cases[0].n_inner
    px = sum(c.f.size for c in cases)
    f = torch.from_numpy(np.concatenate([c.f.ravel() for c in cases])).to(dev)
    plan = dtvdd.Plan(imgs, n_outer=n_outer, n_inner=K, schedule=args.schedule, device=dev, time_kernels=True)
    st = plan.new_state()
    plan.solve(f, state=st, want_stats=False)
    plan.solve(f, state=st, want_stats=False)
    torch.cuda.synchronize()
    dt = b["ms_per_solve"] * 1e-3
    dt_seq = b["sequential_plain"]["ms"] * 1e-3
    kt = plan.kernel_time()
    tiles = sum((len(c.row_cuts) - 1) * (len(c.col_cuts) - 1) for c in cases)
    return {
        "metric": METRIC, "value": px * n_outer * K / dt, "unit": "pixel-inner-iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched: {len(cases)} ROF images, {px} pixels, {tiles} subdomains (128-cuts, ragged), "
                               f"{n_outer} outer x {K} inner", "schedule": plan.schedule()},
        "sequential_plain": {"value": px * n_outer * K / dt_seq, "ms": dt_seq * 1e3},
        "batched_over_sequential": dt_seq / dt,
        "kernel": {"name": kt["name"], "avg_launch_us": kt["avg_ms"] * 1e3, "bytes_per_launch": kt["bytes_per_launch"],
                   "achieved_GBs": kt["bytes_per_launch"] / (kt["avg_ms"] * 1e-3) / 1e9},
    }


def backward_measure(steps: int, warmup: int, schedule: str = "auto") -> dict:
    """Forward and reverse mode of 16 unrolled 512 x 512 ROF solves (loss
    |u - g|^2): the plain forward, the forward that keeps checkpoints, and the
    backward, each timed with the host clock around the call; then one more
    backward with HIP events around every launch of the reverse kernel and of
    the recording forward (their rooflines: algorithmic bytes over the average
    launch).  Then the same with keep_records (the forward keeps every outer
    step's records, the backward recomputes nothing)."""
    import torch

    from paper_1901_00682_amd import dtvdd, synth

    cases = synth.config5()
    dev = torch.device("cuda:0")
    B = len(cases)
    H, W = cases[0].f.shape
    f = torch.from_numpy(np.stack([c.f for c in cases])).to(dev)
    g = torch.from_numpy(np.stack([c.clean for c in cases])).to(dev)
    imgs = [dtvdd.Image(H, W, c.row_cuts, c.col_cuts, c.alpha) for c in cases]
    n_outer, K = cases[0].n_outer, cases[0].n_inner
    plan = dtvdd.Plan(imgs, n_outer=n_outer, n_inner=K, save_for_backward=True, ckpt_every=20,
                      schedule=schedule, device=dev)
    plain = dtvdd.Plan(imgs, n_outer=n_outer, n_inner=K, schedule=schedule, device=dev)
    fl = f.reshape(-1)
    st, sp = plan.new_state(), plain.new_state()
    tf, tb, tp = [], [], []
    for it in range(warmup + steps):
        torch.cuda.synchronize(); t0 = time.perf_counter()
        plain.solve(fl, state=sp, want_stats=False)
        torch.cuda.synchronize(); t1 = time.perf_counter()
        plan.solve(fl, state=st, want_stats=False)
        torch.cuda.synchronize(); t2 = time.perf_counter()
        u = st["u"][: B * H * W]
        gu = 2.0 * (u - g.reshape(-1))
        plan.backward(fl, gu)
        torch.cuda.synchronize(); t3 = time.perf_counter()
        if it >= warmup:
            tp.append(t1 - t0); tf.append(t2 - t1); tb.append(t3 - t2)
    # the kernels of one more backward, timed launch by launch
    tplan = dtvdd.Plan(imgs, n_outer=n_outer, n_inner=K, save_for_backward=True, ckpt_every=20,
                       schedule=schedule, device=dev, time_kernels=True)
    ts = tplan.new_state()
    tplan.solve(fl, state=ts, want_stats=False)
    tplan.backward(fl, 2.0 * (ts["u"][: B * H * W] - g.reshape(-1)))
    torch.cuda.synchronize()
    sched = plan.schedule()
    kern = {}
    for which in (0, 1):
        kt = tplan.backward_kernel_time(which)
        if kt["launches"] > 0:
            gbs = kt["bytes_per_launch"] / (kt["avg_ms"] * 1e-3) / 1e9
            kern["reverse" if which == 0 else "recording_forward"] = {
                "bound": "hbm", "kernel": kt["name"], "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS, "traffic": measured_traffic(kt["name"].split()[0] + (
                    "_rec" if which == 1 else ""), "diff"),
                "avg_launch_us": kt["avg_ms"] * 1e3, "launches": kt["launches"],
                "bytes_per_launch": kt["bytes_per_launch"]}
    for p in (plan, tplan):
        p.close()
    del plan, tplan, st, ts
    # keep_records: the forward keeps the state before every outer step and that step's records
    # (the recording kernel runs in the forward), so the backward only reverses
    kr = {}
    if schedule in ("auto", "fused"):
        trf, trb = [], []
        rplan = dtvdd.Plan(imgs, n_outer=n_outer, n_inner=K, save_for_backward=True, keep_records=True, device=dev)
        sr = rplan.new_state()
        for it in range(warmup + steps):
            torch.cuda.synchronize(); t0 = time.perf_counter()
            rplan.solve(fl, state=sr, want_stats=False)
            torch.cuda.synchronize(); t1 = time.perf_counter()
            rplan.backward(fl, 2.0 * (sr["u"][: B * H * W] - g.reshape(-1)))
            torch.cuda.synchronize(); t2 = time.perf_counter()
            if it >= warmup:
                trf.append(t1 - t0); trb.append(t2 - t1)
        ws_gb = rplan.ws.numel() / 1e9
        rplan.close()
        del rplan, sr
        rplan = dtvdd.Plan(imgs, n_outer=n_outer, n_inner=K, save_for_backward=True, keep_records=True, device=dev,
                           time_kernels=True)
        sr = rplan.new_state()
        rplan.solve(fl, state=sr, want_stats=False)
        rplan.backward(fl, 2.0 * (sr["u"][: B * H * W] - g.reshape(-1)))
        torch.cuda.synchronize()
        rk = {}
        for key, kt in (("recording_forward", rplan.kernel_time()), ("reverse", rplan.backward_kernel_time(0))):
            gbs = kt["bytes_per_launch"] / (kt["avg_ms"] * 1e-3) / 1e9
            rk[key] = {"bound": "hbm", "kernel": kt["name"], "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": gbs / HBM_PEAK_GBS,
                       "traffic": measured_traffic(kt["name"].split()[0] + ("_rec" if key == "recording_forward"
                                                                            else ""), "diff_kr"),
                       "avg_launch_us": kt["avg_ms"] * 1e3, "launches": kt["launches"],
                       "bytes_per_launch": kt["bytes_per_launch"]}
            if key == "reverse":  # one launch reverses every outer step of the solve
                rk[key]["per_outer_step_us"] = kt["avg_ms"] * 1e3 * kt["launches"] / n_outer
        rplan.close()
        del rplan, sr
        fr, br = float(np.median(trf)) * 1e3, float(np.median(trb)) * 1e3
        kr = {"forward_ms": fr, "backward_ms": br, "forward_plus_backward_ms": fr + br,
              "backward_over_forward": br / (float(np.median(tp)) * 1e3), "workspace_GB": ws_gb, "kernels": rk}
    px = B * H * W
    out = {"workload": f"differentiation: {B} x {H}x{W} ROF, 4x4 subdomains, {n_outer} outer x {K} inner, "
                       "loss |u - g|^2, gradient in f and alpha, checkpoint every 20 outer steps",
           "plain_forward_ms": float(np.median(tp)) * 1e3,
           "forward_with_checkpoints_ms": float(np.median(tf)) * 1e3,
           "backward_ms": float(np.median(tb)) * 1e3,
           "backward_over_forward": float(np.median(tb)) / float(np.median(tp)),
           "forward_value": px * n_outer * K / float(np.median(tp)), "unit": "pixel-inner-iterations/s",
           "forward_plus_backward_ms": (float(np.median(tf)) + float(np.median(tb))) * 1e3,
           "steps": steps, "schedule": sched, "kernels": kern, "keep_records": kr}
    plain.close()
    return out


def copy_calibration(dev):
    """A plain 256 MiB device copy, four times: what the HBM byte counters read
    for it scales them (run with --calibrate-copy under the counter passes)."""
    import torch

    nbytes = 256 << 20
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).uniform_()
    dst = torch.empty_like(src)
    for _ in range(4):
        dst.copy_(src)
    torch.cuda.synchronize()


def run_diff(args):
    """Forward and reverse mode of 16 unrolled 512 x 512 ROF solves."""
    import torch

    b = backward_measure(args.steps, args.warmup, args.schedule)
    if args.calibrate_copy:
        copy_calibration(torch.device("cuda:0"))
    return {
        "metric": METRIC, "value": b["forward_value"], "unit": "pixel-inner-iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": b["forward_with_checkpoints_ms"] + b["backward_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": b["workload"], "schedule": b["schedule"]},
        "roofline": b["kernels"].get("reverse"), "backward": b,
    }


def run_dd_vs_full(args):
    """Decomposed against undecomposed on one GPU (Sec. 5 compares the method
    with the primal-dual method on the full-dimension problem): wall-clock time
    of a plain solve until the relative primal energy error (J(u) - J*)/J*
    falls below 1e-5 (the outer stopping rule of Sec. 5.1), on the 2048 x 2048
    ROF image.  J* comes from a long undecomposed FISTA run whose FP64
    primal-dual gap bounds its own error.  Each iteration count of a doubling
    sequence is a separate timed solve (no diagnostics inside the timed
    region); J(u) is evaluated after it with the FP64 diagnostics."""
    import torch

    from paper_1901_00682_amd import dtvdd, synth

    c = synth.config2()
    H, W = c.f.shape
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    f = torch.from_numpy(np.ascontiguousarray(c.f).ravel()).to(dev)
    full_img = dtvdd.Image(H, W, np.array([0, H]), np.array([0, W]), c.alpha)
    dd_img = dtvdd.Image(H, W, c.row_cuts, c.col_cuts, c.alpha)
    tol = 1e-5

    def timed(plan):
        st = plan.new_state()
        plan.solve(f, state=st, want_stats=False)  # warm-up (and the autotuner's first look)
        torch.cuda.synchronize()
        ts = []
        for _ in range(max(1, args.steps // 5)):
            t0 = time.perf_counter()
            plan.solve(f, state=st, want_stats=False)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        J, D, gap, _ = plan.diagnostics(f, st)[0]
        return float(np.median(ts)), float(J), float(D)

    ref = dtvdd.Plan([full_img], full_problem=True, n_outer=1, n_inner=args.ref_iters, device=dev)
    st = ref.new_state()
    ref.solve(f, state=st, want_stats=False)
    Jr, Dr, gr, _ = (float(x) for x in ref.diagnostics(f, st)[0])
    Jstar = Jr
    methods = {
        "dd_16x16_fista5": (lambda n: dtvdd.Plan([dd_img], n_outer=n, n_inner=c.n_inner, device=dev),
                            [25 * 2 ** k for k in range(11)], c.n_inner),
        "dd_16x16_fista10": (lambda n: dtvdd.Plan([dd_img], n_outer=n, n_inner=10, device=dev),
                             [25 * 2 ** k for k in range(10)], 10),
        "dd_16x16_adaptive": (lambda n: dtvdd.Plan([dd_img], n_outer=n, n_inner=args.adaptive_cap,
                                                   inner_tol=args.adaptive_tol, device=dev),
                              [25 * 2 ** k for k in range(9)], None),
        "full_fista": (lambda n: dtvdd.Plan([full_img], full_problem=True, n_outer=1, n_inner=n, device=dev),
                       [100 * 2 ** k for k in range(9)], 1),
        "full_cp": (lambda n: dtvdd.Plan([full_img], full_problem=True, inner="CP2", n_outer=1, n_inner=n,
                                         tau0=10.0, sigma0=1.0 / 80.0, gamma=1.0 / 400.0, device=dev),
                    [100 * 2 ** k for k in range(9)], 1),
    }
    res = {}
    for name, (mk, counts, per) in methods.items():
        rows, hit = [], None
        for n in counts:
            plan = mk(n)
            dt, J, D = timed(plan)
            err = (J - Jstar) / Jstar
            rows.append({"count": n, "ms": dt * 1e3, "rel_energy_error": err, "schedule": plan.schedule()})
            if per is None:  # adaptive: local steps actually taken (mean over subdomains)
                rows[-1]["inner_steps"] = float(plan.inner_counts()[:, 0].mean())
            print(f"[dd_vs_full] {name} count {n}: {dt * 1e3:.2f} ms, rel err {err:.3e}", file=sys.stderr, flush=True)
            del plan
            if err < tol:
                hit = rows[-1]
                break
        res[name] = {"runs": rows, "reached": hit is not None,
                     "ms_to_tol": hit["ms"] if hit else None,
                     "iterations_to_tol": (hit.get("inner_steps", hit["count"] * (per or 0))) if hit else None}
    dd = min([v["ms_to_tol"] for k, v in res.items() if k.startswith("dd_") and v["ms_to_tol"]], default=None)
    best_full = min([v["ms_to_tol"] for k, v in res.items() if k.startswith("full_") and v["ms_to_tol"]],
                    default=None)
    return {
        "metric": "ms to (J - J*)/J* < 1e-5, 2048^2 ROF: 16x16 decomposition (fastest variant) vs undecomposed",
        "value": dd, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": dd, "higher_is_better": False, "scaling": "strong", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{c.name}: {H}x{W}, alpha {c.alpha}; counts double until the tolerance is met",
                   "tolerance": tol},
        "reference": {"iterations": args.ref_iters, "J": Jr, "D": Dr, "gap_over_J": gr / Jr},
        "methods": res,
        "full_over_dd": (best_full / dd) if (dd and best_full) else None,
    }


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(c, outer_sample: int, outer_single: int) -> dict:
    """The FP64 oracle on the host cores: the first outer_sample outer steps
    with every thread of its parallel loop over subdomains, and the first
    outer_single steps on one thread."""
    import oracle

    def timed(n_outer):
        o = oracle.Oracle(oracle.Problem(c.f.astype(np.float64), c.alpha, c.row_cuts, c.col_cuts,
                                         fidelity=c.fidelity, inner=c.inner, mask=c.mask, tau=c.tau, sigma=c.sigma,
                                         tau0=c.tau0, sigma0=c.sigma0, gamma=c.gamma, n_inner=c.n_inner, **c.extra))
        t0 = time.perf_counter()
        o.run(n_outer)
        return time.perf_counter() - t0

    H, W = c.f.shape
    threads = oracle.threads()
    dt = timed(outer_sample)
    out = {"value": H * W * outer_sample * c.n_inner / dt, "unit": "pixel-inner-iterations/s",
           "cores": threads, "kind": "oracle", "cpu_model": cpu_model(), "logical_cpus": os.cpu_count(),
           "sample": f"first {outer_sample} of {c.n_outer} outer steps of the same workload, FP64, {threads} "
                     f"threads, {dt:.1f} s"}
    if outer_single > 0:
        oracle.set_threads(1)
        try:
            d1 = timed(outer_single)
        finally:
            oracle.set_threads(threads)
        out["single_thread"] = {"value": H * W * outer_single * c.n_inner / d1, "cores": 1,
                                "sample": f"first {outer_single} outer steps, FP64, 1 thread, {d1:.1f} s"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rof2048")
    ap.add_argument("--schedule", default="auto")
    ap.add_argument("--rows", type=int, default=0, help="streaming strip height (0: the plan picks)")
    ap.add_argument("--steps-per-launch", type=int, default=0,
                    help="streaming schedule: the most local steps per launch (1 .. 5; 0: the plan's default)")
    ap.add_argument("--cpu-outer", type=int, default=500, help="outer steps of the oracle sample (0: skip)")
    ap.add_argument("--cpu-outer-single", type=int, default=20, help="outer steps of the one-thread oracle sample")
    ap.add_argument("--no-extra", action="store_true", help="default workload: skip the batched and backward blocks")
    ap.add_argument("--ref-iters", type=int, default=20000, help="dd_vs_full: FISTA iterations of the J* run")
    ap.add_argument("--adaptive-tol", type=float, default=1e-3, help="dd_vs_full: inner_tol of the adaptive run")
    ap.add_argument("--adaptive-cap", type=int, default=100, help="dd_vs_full: local step cap of the adaptive run")
    ap.add_argument("--calibrate-copy", action="store_true", help="also run a 256 MiB device copy (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (the subdomain grid would be "
              "block-partitioned across GPUs with one interface exchange per outer step; see DESIGN.md)",
              file=sys.stderr)
        raise SystemExit(2)

    import torch

    from paper_1901_00682_amd import dtvdd

    if args.workload == "batched":
        print(json.dumps(run_batched(args)), flush=True)
        return
    if args.workload == "diff":
        print(json.dumps(run_diff(args)), flush=True)
        return
    if args.workload == "dd_vs_full":
        print(json.dumps(run_dd_vs_full(args)), flush=True)
        return
    c = workload(args.workload)
    H, W = c.f.shape
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    f = torch.from_numpy(np.ascontiguousarray(c.f).ravel()).to(dev)
    m = None if c.mask is None else torch.from_numpy(c.mask.ravel()).to(dev)
    stream = torch.cuda.current_stream(dev)
    img = dtvdd.Image(H, W, c.row_cuts, c.col_cuts, c.alpha)
    kw = dict(fidelity=c.fidelity, inner=c.inner, has_mask=c.mask is not None, tau=c.tau, sigma=c.sigma,
              tau0=c.tau0, sigma0=c.sigma0, gamma=c.gamma, n_outer=c.n_outer, n_inner=c.n_inner,
              schedule=args.schedule, rows=args.rows, steps_per_launch=args.steps_per_launch, device=dev, **c.extra)
    plan = dtvdd.Plan([img], **kw)
    state = plan.new_state()
    for _ in range(args.warmup):
        plan.solve(f, m, state=state, stream=stream, want_stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.solve(f, m, state=state, stream=stream, want_stats=False, check=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.status(stream)
    px_it = H * W * c.n_outer * c.n_inner * args.steps / dt
    # kernel timing: the same solves with HIP events around every launch of the
    # dominant kernel on the solve stream
    tplan = dtvdd.Plan([img], time_kernels=True, **kw)
    tstate = tplan.new_state()
    tplan.solve(f, m, state=tstate, stream=stream, want_stats=False)
    launch_ms = []
    for _ in range(max(1, args.steps // 2)):
        tplan.solve(f, m, state=tstate, stream=stream, want_stats=False)
        launch_ms.append(tplan.kernel_time()["avg_ms"])
    torch.cuda.synchronize()
    kt = tplan.kernel_time()
    avg_ms = float(np.mean(launch_ms))
    achieved = kt["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9
    if kt["name"] in ("k_persist_fista", "k_persist_cp2"):
        # one launch per solve, iterates on chip across outer steps: bound by the vector ALUs
        per_px = (fista_flops_per_pixel(c.n_inner) if kt["name"] == "k_persist_fista"
                  else cp2_flops_per_pixel(c.n_inner, c.fidelity))
        flops = per_px * H * W * c.n_outer
        tflops = flops / (avg_ms * 1e-3) / 1e12
        roofline = {"bound": "alu", "kernel": kt["name"], "achieved": tflops, "peak": FP32_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": tflops / FP32_PEAK_TFLOPS,
                    "traffic": measured_traffic(kt["name"], args.workload),
                    "avg_launch_us": avg_ms * 1e3, "flops_per_launch": flops,
                    "bytes_per_launch": kt["bytes_per_launch"], "hbm_GBs": achieved,
                    "launches_per_step": kt["launches"]}
    else:
        roofline = {"bound": "hbm", "kernel": kt["name"], "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                    "traffic": measured_traffic(kt["name"], args.workload),
                    "avg_launch_us": avg_ms * 1e3, "bytes_per_launch": kt["bytes_per_launch"],
                    "launches_per_step": kt["launches"]}
        if kt["name"] in ("k_cp2_multi", "k_fista_multi"):
            # several local steps per launch: the launch moves a fraction of the one-step bytes and
            # is limited by instruction issue and latency, not by HBM (the VALU counter passes of
            # profiles/k_cp2_multi_tvl1.md and profiles/k_fista_multi_rof2048.md: 86 % and 67 % busy)
            roofline["limiter"] = "vector ALU issue and latency (HBM figure: algorithmic bytes / launch time)"
    if args.calibrate_copy:
        copy_calibration(dev)
    out = {
        "metric": METRIC,
        "value": px_it,
        "unit": "pixel-inner-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{c.name}: {H}x{W}, {len(c.row_cuts) - 1}x{len(c.col_cuts) - 1} subdomains, "
                               f"{c.fidelity}/{c.inner}, alpha {c.alpha}, {c.n_outer} outer x {c.n_inner} inner",
                   "H": H, "W": W, "subdomains": [len(c.row_cuts) - 1, len(c.col_cuts) - 1],
                   "n_outer": c.n_outer, "n_inner": c.n_inner, "schedule": plan.schedule()},
        "roofline": roofline,
    }
    # the whole hot path against the streaming byte model (every inner step
    # reading x_k, x_{k-1}, the anchor and f and writing x_{k+1}; u written once
    # per outer step): an effective bandwidth, above HBM peak when the fused
    # schedule keeps the inner iterates on chip
    E = (H + out["config"]["subdomains"][0]) * W + H * (W + out["config"]["subdomains"][1])
    N = H * W
    K = c.n_inner
    per_outer = 4.0 * (2 * E + N) + (K - 1) * 4.0 * (4 * E + N) + 4.0 * N
    eff = per_outer * c.n_outer / (dt / args.steps) / 1e9
    out["hot_path_streaming_model"] = {"bytes_per_outer_step": per_outer, "effective_GBs": eff,
                                       "frac_of_hbm_peak": eff / HBM_PEAK_GBS}
    plan.close()
    tplan.close()
    if args.workload == "rof2048" and not args.no_extra:
        # the rest of the metric (batched vs plain, and the reverse mode), measured in the same run
        b = batched_measure(min(args.steps, 5), 1)
        b["over_plain"] = b["value"] / px_it
        out["batched"] = b
        out["backward"] = backward_measure(min(args.steps, 5), 1)
    if args.cpu_outer > 0:
        out["cpu_baseline"] = cpu_baseline(c, min(args.cpu_outer, c.n_outer), min(args.cpu_outer_single, c.n_outer))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
