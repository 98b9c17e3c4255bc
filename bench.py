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


def workload(name: str):
    from paper_1901_00682_amd import synth

    if name == "rof2048":
        return synth.config2()
    if name == "rof8192":
        return synth.config2(size=8192)
    if name == "tvl1":
        return synth.config3()
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(c, outer_sample: int) -> dict:
    import oracle

    o = oracle.Oracle(oracle.Problem(c.f.astype(np.float64), c.alpha, c.row_cuts, c.col_cuts, fidelity=c.fidelity,
                                     inner=c.inner, mask=c.mask, tau=c.tau, sigma=c.sigma, tau0=c.tau0,
                                     sigma0=c.sigma0, gamma=c.gamma, n_inner=c.n_inner))
    t0 = time.perf_counter()
    o.run(outer_sample)
    dt = time.perf_counter() - t0
    H, W = c.f.shape
    return {"value": H * W * outer_sample * c.n_inner / dt, "unit": "pixel-inner-iterations/s",
            "cores": oracle.threads(), "kind": "oracle",
            "sample": f"first {outer_sample} of {c.n_outer} outer steps of the same workload, FP64, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rof2048")
    ap.add_argument("--schedule", default="auto")
    ap.add_argument("--cpu-outer", type=int, default=100, help="outer steps of the oracle sample (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (the subdomain grid would be "
              "block-partitioned across GPUs with one interface exchange per outer step; see DESIGN.md)",
              file=sys.stderr)
        raise SystemExit(2)

    import torch

    from paper_1901_00682_amd import dtvdd

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
              schedule=args.schedule, device=dev)
    plan = dtvdd.Plan([img], time_kernels=True, **kw)
    state = plan.new_state()
    for _ in range(args.warmup):
        plan.solve(f, m, state=state, stream=stream, want_stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    launch_ms = []
    for _ in range(args.steps):
        plan.solve(f, m, state=state, stream=stream, want_stats=False)
        launch_ms.append(plan.kernel_time()["avg_ms"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = plan.kernel_time()
    px_it = H * W * c.n_outer * c.n_inner * args.steps / dt
    avg_ms = float(np.mean(launch_ms))
    achieved = kt["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9
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
        "roofline": {"bound": "hbm", "kernel": kt["name"], "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "avg_launch_us": avg_ms * 1e3, "bytes_per_launch": kt["bytes_per_launch"],
                     "launches_per_step": kt["launches"]},
    }
    if args.cpu_outer > 0:
        out["cpu_baseline"] = cpu_baseline(c, args.cpu_outer)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
