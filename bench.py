#!/usr/bin/env python3
"""Throughput of the batched TaylorF2 likelihood on one MI355X.

Workload (default): three detectors, 128 s segments at 4096 Hz sampling,
bins 20-2048 Hz at delta_f = 1/128 Hz (259,585 bins per detector), a batch of
4096 parameter samples (9 parameters each) drawn from the box prior, data =
seeded Gaussian noise plus an injected TaylorF2 signal.  One step is one
gw_lnl_batch call: event preparation, per-sample preparation, the tile kernel
and the final reduction, i.e. the whole likelihood path for one batch, with
every input already resident in device memory.

Prints one JSON line.  `value` is lnL evaluations per second.  `roofline`
prices the hot tile kernel's algorithmic FP64 flops (the per-(sample, bin)
tally below) per launch against the MI355X FP64 vector peak; its duration is
the mean of HIP events the library records around that kernel on the stream
it runs on.  `cpu_baseline` times the CPU oracle (OpenMP over samples, all
host cores it is given) on a bounded number of the same samples.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 vector peak
HBM_PEAK_GBS = 8000.0


def flops_per_pair(n_det: int) -> int:
    """Algorithmic FP64 flops of the tile kernel per (sample, bin) pair
    (FMA = 2, multiply = 1): half-phase polynomial 19, phasor from the half
    phase 43, detector-0 accumulation 8, and for every further detector
    rotate (6) + accumulate (8) + advance the delay rotation (6)."""
    return 19 + 43 + 8 + 20 * (n_det - 1)


def build_inputs(name: str, n_samples: int | None):
    import numpy as np
    import torch

    import paper_1904_02863_amd as gw
    import synth

    if name == "bbh-3det-128s":
        w = synth.bbh_3det_128s(n_samples or 4096)
    elif name == "bbh-1det-4s":
        w = synth.bbh_1det_4s(n_samples or 1000)
    else:
        raise SystemExit(f"unknown workload {name}")
    dev = torch.device("cuda", 0)
    theta = torch.from_numpy(np.ascontiguousarray(w.theta)).to(dev)
    inj = torch.from_numpy(np.ascontiguousarray(w.theta_inj[None, :])).to(dev)
    # the injection is made with the library's own waveform generator
    h = gw.waveform_batch(w.grid, w.tensors if w.n_param == 9 else w.tensors, w.vertices, inj)[0]
    data = (torch.from_numpy(w.noise).to(dev) + h).contiguous()
    psd = torch.from_numpy(w.psd).to(dev)
    torch.cuda.synchronize()
    return w, data, psd, theta


def cpu_baseline(w, data, budget_s: float):
    """Oracle evals/s on a bounded number of the workload's samples."""
    import numpy as np

    import oracle

    g = w.grid
    d = data.cpu().numpy()
    threads = oracle.max_threads()
    n = max(threads, 8)
    done, spent = 0, 0.0
    while spent < budget_s and done < w.n_samples:
        take = min(n, w.n_samples - done)
        t0 = time.perf_counter()
        vals = oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, d, w.psd,
                          w.theta[done:done + take])
        spent += time.perf_counter() - t0
        assert np.isfinite(vals).all()
        done += take
        # grow the chunk so that the next one lands near the remaining budget
        per = spent / done
        n = int(max(threads, min(4 * n, (budget_s - spent) / per)))
    return {"value": done / spent, "unit": "lnL evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} of the {w.n_samples} samples (rows 0..{done - 1}), all {g.n_bins} bins x "
                      f"{w.n_det} detectors, {spent:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="bbh-3det-128s", choices=["bbh-3det-128s", "bbh-1det-4s"])
    ap.add_argument("--samples", type=int, default=None)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="CPU-baseline budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(samples shard trivially across GPUs; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1904_02863_amd as gw

    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible: the benchmark runs the HIP library only")
    w, data, psd, theta = build_inputs(args.workload, args.samples)
    g = w.grid
    ws = gw.Workspace(0)
    ws.reserve(g.n_bins, w.n_det, w.n_samples)
    out = torch.empty(w.n_samples, dtype=torch.float64, device=theta.device)

    def step():
        gw.lnl_batch(g, w.tensors, w.vertices, data, psd, theta, out=out, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ws.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms, launches = ws.kernel_time()
    ws.set_timing(False)
    if not torch.isfinite(out).all():
        raise SystemExit("non-finite lnL in the benchmark batch")

    evals = w.n_samples * args.steps
    kernel_avg_s = kernel_ms / 1e3 / max(launches, 1)
    flops_launch = flops_per_pair(w.n_det) * w.n_samples * g.n_bins
    achieved = flops_launch / kernel_avg_s / 1e12
    result = {
        "metric": "lnL evals/s (3-det,128 s TaylorF2)" if args.workload == "bbh-3det-128s" else "lnL evals/s",
        "value": evals / elapsed,
        "unit": "lnL evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_samples": w.n_samples, "n_det": w.n_det, "n_bins": g.n_bins,
                   "delta_f": g.delta_f, "f_low": g.f_low, "f_high": g.f_high, "n_param": w.n_param,
                   "precision": "fp64"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "kernel": f"lnl_tile_kernel<{w.n_det}>", "kernel_ms": kernel_avg_s * 1e3,
                     "flops_per_launch": flops_launch, "flops_per_pair": flops_per_pair(w.n_det)},
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, data, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
