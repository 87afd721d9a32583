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
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 vector peak
HBM_PEAK_GBS = 8000.0
PROFILE_SUMMARY = "profiles/lnl_tile_kernel_bbh-3det-128s.md"
WAVEFORM_PROFILE = "profiles/waveform_kernel_bbh-3det-128s.md"
RELBIN_PROFILE = "profiles/relbin_lnl_kernel_bns-15hz-512s.md"
# Sources whose content fixes each profiled kernel's machine code and launch;
# a profile summary records their SHA-256 next to the figures it measured.
_CSRC = "paper_1904_02863_amd/csrc/"
_COMMON = tuple(_CSRC + f for f in ("gw_device_math.h", "gw_internal.h", "gw_template.h", "gw_phasor_table.h")) + (
    "paper_1904_02863_amd/build.py",)
PROFILE_SOURCES = {
    PROFILE_SUMMARY: (_CSRC + "gw_kernels.hip", _CSRC + "gw_plan.h") + _COMMON,
    WAVEFORM_PROFILE: (_CSRC + "gw_waveform.hip",) + _COMMON,
    RELBIN_PROFILE: (_CSRC + "gw_relbin.hip",) + _COMMON,
}


def flops_per_pair(n_det: int, mixed: bool = False, direct: bool = False) -> int:
    """Algorithmic FP64 flops of the tile kernel per (sample, bin) pair
    (FMA = 2, multiply or add = 1, rounding to an integer not counted):
    phase polynomial in u = f^(1/3) 19 (9 FMA + 1 multiply), phasor
    e^{-2 pi i x} from the phase in turns at a fixed tally of 34 (the count of
    the polynomial phasor gw_phasor_turns, 15 FMA + 3 multiplies + 1 add,
    whichever implementation runs: the FP64 tile loop takes it from an LDS
    table and two short polynomials, about 17 flops in 14 operations),
    detector-0 complex accumulation 8 (4 FMA), and for every further detector
    one Horner step S <- S conj(rho) + D e^{-i Phi} 14 (6 FMA + 2 multiplies).
    The mixed path replaces the phasor by the reduction to a fractional turn
    (1 add) and two FP32 hardware transcendentals, which are not counted.
    Direct form (GW_FLAG_DIRECT): per detector the residual d/a - T e^{-i Phi}
    and a^2/S |.|^2 accumulated, 13 (6 FMA + 1 multiply), plus for every
    further detector the rotation T <- T rho, 6 (2 FMA + 2 multiplies)."""
    per_det = (13, 19) if direct else (8, 14)
    return 19 + (1 if mixed else 34) + per_det[0] + per_det[1] * (n_det - 1)


def kernel_fingerprint(summary: str = PROFILE_SUMMARY) -> str:
    """SHA-256 over the sources of the kernel a profile summary covers."""
    h = hashlib.sha256()
    for rel in PROFILE_SOURCES[summary]:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _profile_value(name: str, summary: str, sources: str | None = None):
    """A named figure of a committed counter summary, or None when the
    sources of its kernel (those of `sources`, a key of PROFILE_SOURCES,
    by default the summary itself) changed since it was taken."""
    path = os.path.join(ROOT, summary)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    sha = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    val = re.search(rf"{re.escape(name)}:\s*([0-9.eE+]+)", text)
    if not sha or not val or sha.group(1) != kernel_fingerprint(sources or summary):
        return None
    return float(val.group(1))


def measured_traffic(key: str, summary: str = PROFILE_SUMMARY, sources: str | None = None):
    """HBM bytes per launch of a kernel from a committed counter summary, or
    None when the kernel sources changed since it was taken."""
    return _profile_value(f"traffic_bytes_per_launch_{key}", summary, sources)


def measured_executed_flops(key: str, summary: str = PROFILE_SUMMARY, sources: str | None = None):
    """FP64 flops per launch the hardware counters saw the kernel execute
    (FMA = 2), or None as for measured_traffic."""
    return _profile_value(f"executed_fp64_flops_per_launch_{key}", summary, sources)


# (sample, bin) pairs of one launch of the batch the tile kernel's counter
# summary was taken on: 4096 samples x 259,585 bins
PROFILED_PAIRS = 4096 * 259585


def executed_flops_per_pair(precision: str, summary: str = PROFILE_SUMMARY, sources: str | None = None):
    """FP64 flops the counters saw the split-form tile loop execute per
    (sample, bin) pair at this precision: the mean over the plans of a
    matching summary, or None when there is none."""
    plans = profiled_plans(precision, summary, sources)
    if not plans:
        return None
    total = sum(measured_executed_flops(f"{precision}@{p}", summary, sources) for p in plans)
    return total / len(plans) / PROFILED_PAIRS


def plan_key(precision: str, plan: dict) -> str:
    """Key of a likelihood plan's figures in the tile kernel's counter
    summary: precision@TILExROUNDS."""
    return f"{precision}@{plan['tile_bins']}x{plan['rounds']}"


def profiled_plans(precision: str, summary: str = PROFILE_SUMMARY, sources: str | None = None) -> list[str]:
    """The plans (TILExROUNDS) a counter summary holds executed-flop figures
    for at this precision, while its kernel sources still match."""
    path = os.path.join(ROOT, summary)
    if not os.path.exists(path):
        return []
    found = re.findall(rf"executed_fp64_flops_per_launch_{re.escape(precision)}@(\d+x\d+):", open(path).read())
    return [p for p in found if _profile_value(f"executed_fp64_flops_per_launch_{precision}@{p}", summary, sources)
            is not None]


def calibration_copy(mib: int, device):
    """One plain device-to-device copy of `mib` MiB (the reference dispatch
    for scaling hardware traffic counters)."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device=device)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def build_inputs(name: str, n_samples: int | None, spins: bool = False):
    import dataclasses

    import numpy as np
    import torch

    import paper_1904_02863_amd as gw
    import synth

    if name == "bbh-3det-128s":
        w = synth.bbh_3det_128s(n_samples or 4096)
    elif name == "bbh-1det-4s":
        w = synth.bbh_1det_4s(n_samples or 1000)
    elif name == "bns-15hz-512s":
        w = synth.long_bns(15.0, 512.0, 3, n_samples or 4096)
    else:
        raise SystemExit(f"unknown workload {name}")
    if spins:       # aligned spins chi1, chi2 ~ U[-1, 1] appended to every row and the injection
        rng = np.random.default_rng(11)
        w = dataclasses.replace(w, theta_inj=synth.add_spins(w.theta_inj, rng)[0],
                                theta=synth.add_spins(w.theta, rng), n_param=w.n_param + 2)
    dev = torch.device("cuda", 0)
    theta = torch.from_numpy(np.ascontiguousarray(w.theta)).to(dev)
    inj = torch.from_numpy(np.ascontiguousarray(w.theta_inj[None, :])).to(dev)
    # the injection is made with the library's own waveform generator
    h = gw.waveform_batch(w.grid, w.tensors, w.vertices, inj)[0]
    data = (torch.from_numpy(w.noise).to(dev) + h).contiguous()
    psd = torch.from_numpy(w.psd).to(dev)
    torch.cuda.synchronize()
    return w, data, psd, theta


def cpu_model() -> str:
    """The host CPU's model name (first processor in /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, data, budget_s: float, flags: int = 0):
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
                          w.theta[done:done + take], isco=bool(flags & 2), add_norm=bool(flags & 4))
        spent += time.perf_counter() - t0
        assert np.isfinite(vals).all()
        done += take
        # grow the chunk so that the next one lands near the remaining budget
        per = spent / done
        n = int(max(threads, min(4 * n, (budget_s - spent) / per)))
    # one thread, for comparison with single-core CPU codes
    one, spent1 = 0, 0.0
    while spent1 < budget_s / 3 and one < w.n_samples:
        t0 = time.perf_counter()
        vals = oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, d, w.psd,
                          w.theta[one:one + 1], n_threads=1, isco=bool(flags & 2), add_norm=bool(flags & 4))
        spent1 += time.perf_counter() - t0
        assert np.isfinite(vals).all()
        one += 1
    return {"value": done / spent, "unit": "lnL evals/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{done} of the {w.n_samples} samples (rows 0..{done - 1}), all {g.n_bins} bins x "
                      f"{w.n_det} detectors, {spent:.1f} s",
            "single_thread": {"value": one / spent1, "cores": 1,
                              "sample": f"rows 0..{one - 1} one at a time, {spent1:.1f} s"}}


def bench_ragged(args):
    """256 neutron-star events of 8..256 s (16,225..519,169 bins), 3 detectors,
    512 proposals each: one gw_lnl_ragged pass (persistent launch replayed from
    a HIP graph) per step, against 256 separate gw_lnl_batch calls."""
    import numpy as np
    import torch

    import paper_1904_02863_amd as gw
    import synth

    evs = synth.bns_ragged(n_events=256, n_samples=512)
    dev = torch.device("cuda", 0)
    ws = gw.Workspace(0)
    datas, psds, thetas = [], [], []
    for e in evs:
        inj = torch.from_numpy(np.ascontiguousarray(e.theta_inj[None])).to(dev)
        h = gw.waveform_batch(e.grid, e.tensors, e.vertices, inj, workspace=ws)[0]
        datas.append((torch.from_numpy(e.noise).to(dev) + h).reshape(-1))
        psds.append(torch.from_numpy(e.psd.ravel()).to(dev))
        thetas.append(e.theta)
    counts = [e.theta.shape[0] for e in evs]
    events, total, rows = gw.make_events([e.grid for e in evs], [e.tensors for e in evs],
                                         [e.vertices for e in evs], counts)
    data = torch.cat(datas).contiguous()
    psd = torch.cat(psds).contiguous()
    del datas, psds
    theta = torch.from_numpy(np.ascontiguousarray(np.concatenate(thetas))).to(dev)
    out = torch.empty(rows, dtype=torch.float64, device=dev)
    prec = args.precision

    def ragged_step():
        gw.lnl_ragged(events, len(evs), data, psd, theta, out=out, workspace=ws, precision=prec)

    views = []
    for i, e in enumerate(evs):
        m, off = e.grid.n_bins, events[i].data_offset
        views.append((e, data[off:off + 3 * m].view(3, m), psd[off:off + 3 * m].view(3, m),
                      theta[events[i].theta_offset:events[i].theta_offset + counts[i]],
                      out[events[i].theta_offset:events[i].theta_offset + counts[i]]))

    def separate_step():
        for e, d, s, th, o in views:
            gw.lnl_batch(e.grid, e.tensors, e.vertices, d, s, th, out=o, workspace=ws, precision=prec)

    def timed(fn, warmup, steps):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    steps = max(1, args.steps // 10)
    sep_s = timed(separate_step, 1, steps)
    ragged_step()                      # first call: autotune and capture (untimed)
    torch.cuda.synchronize()
    tuning = ws.ragged_tuning()
    rag_s = timed(ragged_step, 2, steps)
    if not torch.isfinite(out).all():
        raise SystemExit("non-finite lnL in the ragged batch")
    pairs = sum(c * e.grid.n_bins for c, e in zip(counts, evs))
    flops = flops_per_pair(3, prec == "mixed") * pairs
    # the ragged kernel runs the tile kernel's per-tile loop, so the flops the
    # counters saw that loop execute per pair price this pass too
    per_pair = executed_flops_per_pair(prec)
    executed = per_pair * pairs if per_pair is not None else None
    result = {
        "metric": "lnL evals/s (256 ragged BNS events, 3 det, 512 proposals each)",
        "value": rows / rag_s, "unit": "lnL evals/s", "n_gpus": 1, "steps": steps, "warmup": 2,
        "ms_per_step": rag_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32" if prec == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": "bns-ragged-256", "n_events": len(evs), "rows": rows, "bins_total": total // 3,
                   "sample_bin_pairs": pairs, "precision": prec, "tile_bins": tuning[0], "chunk_bins": tuning[1]},
        "separate_launches": {"value": rows / sep_s, "ms_per_step": sep_s * 1e3},
        "speedup_vs_separate": sep_s / rag_s,
        "roofline": {"bound": "alu", "achieved": executed / rag_s / 1e12 if executed else None,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": executed / rag_s / 1e12 / FP64_PEAK_TFLOPS if executed else None, "traffic": None,
                     "kernel": "whole ragged pass (graph)",
                     "flops_source": ("executed FP64 flops per (sample, bin) of the same tile loop, from the counters "
                                      "in " + PROFILE_SUMMARY if executed
                                      else "no counter summary of these kernel sources"),
                     "executed_flops_per_pair": per_pair,
                     "frac_tally": flops / rag_s / 1e12 / FP64_PEAK_TFLOPS,
                     "flops_per_pair_tally": flops_per_pair(3, prec == "mixed")},
    }
    if not args.no_cpu_baseline:
        import oracle
        rng = np.random.default_rng(7)
        order = rng.permutation(len(evs))
        threads = oracle.max_threads()
        spent, done_pairs = 0.0, 0
        used = []
        for i in order:
            if spent >= args.cpu_seconds:
                break
            e = evs[i]
            g = e.grid
            d = data[events[i].data_offset:events[i].data_offset + 3 * g.n_bins].view(3, g.n_bins).cpu().numpy()
            n = threads
            t0 = time.perf_counter()
            oracle.lnl(g.f_low, g.delta_f, g.n_bins, e.tensors, e.vertices, d, e.psd, e.theta[:n])
            spent += time.perf_counter() - t0
            done_pairs += n * g.n_bins
            used.append(int(i))
        pair_rate = done_pairs / spent
        result["cpu_baseline"] = {
            "value": pair_rate * rows / pairs, "unit": "lnL evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{threads} rows of each of {len(used)} seeded random events ({done_pairs} sample-bin pairs, "
                      f"{spent:.1f} s), extrapolated to the batch by sample-bin pairs"}
    print(json.dumps(result), flush=True)


def flow_problem(spins: bool, precision: str = "fp64"):
    """The learned-proposal workload: the 3-detector 128 s data (seeded noise)
    with one injection at network optimal SNR 25, built with the library's
    waveform; the prior box of sampler.injection_box."""
    import math

    import numpy as np
    import torch

    import paper_1904_02863_amd as gw
    import synth
    from paper_1904_02863_amd import sampler

    w = synth.bbh_3det_128s(1)
    g = w.grid
    dev = torch.device("cuda", 0)
    ws = gw.Workspace(0)
    # the default likelihood plan: a plan tuned on the box would change the
    # sums' rounding, and through the accept decisions the chains, from box to box
    ws.set_tuning(False)
    psd = torch.from_numpy(w.psd).to(dev)
    inj = w.theta_inj.copy()
    zero = torch.zeros((3, g.n_bins), dtype=torch.complex128, device=dev)
    hh = -2.0 * gw.lnl_batch(g, w.tensors, w.vertices, zero, psd, torch.from_numpy(inj[None]).to(dev),
                             workspace=ws).item()
    inj[2] *= math.sqrt(hh) / 25.0                      # network optimal SNR 25
    h = gw.waveform_batch(g, w.tensors, w.vertices, torch.from_numpy(inj[None]).to(dev), workspace=ws)[0]
    data = torch.from_numpy(np.ascontiguousarray(w.noise + h.cpu().numpy())).to(dev)
    lo, hi, p_inj = sampler.injection_box(inj)
    prob = sampler.Problem(g, w.tensors, w.vertices, data, psd, lo, hi, precision, spins=spins)
    return prob, p_inj, ws


def flow_comparison(args, spins: bool):
    """Random-walk and flow-proposal MH on flow_problem (see
    sampler.compare_samplers): 4096 chains, 2.1e5 training samples, 8
    couplings of 11 -> 256 -> 256 -> 22."""
    from paper_1904_02863_amd import sampler
    prob, p_inj, ws = flow_problem(spins, args.precision)
    burn = args.mcmc_burn if args.mcmc_burn is not None else (120000 if spins else 4000)
    t0 = time.perf_counter()
    res = sampler.compare_samplers(prob, p_inj, ws, n_chains=4096, burn=burn, steps=args.mcmc_steps,
                                   log=lambda m: print(m, file=sys.stderr, flush=True),
                                   flow_steps=args.flow_steps, lr=args.flow_lr,
                                   lr_final=args.flow_lr_final if args.flow_lr_final > 0 else None)
    res["wall_seconds"] = time.perf_counter() - t0
    res["burn_in_steps"] = burn
    res["spins"] = spins
    res.pop("states")
    return res


def bench_flow(args):
    """Learned proposal on the 3-detector 128 s data with one injection at
    network SNR 25, 11 sampler coordinates (9 physical + two aligned spins,
    prior-only unless --spins passes them to the likelihood), 4096 chains:
    random-walk MH (burn-in with covariance adaptation, then production), a
    flow trained on 2.1e5 of its samples, then flow-proposal MH (every 8th
    step a random-walk step) from the same states.  Reports ESS/s of both
    (bulk ESS, minimum over coordinates, from 256 chains recorded at every
    step and scaled to all chains), the standardised difference of every
    coordinate's mean (by the two ESS), and two-sample KS p-values between
    the final states of the 4096 random-walk chains and the 4096 flow chains."""
    res = flow_comparison(args, args.spins)
    result = {
        "metric": "ESS/s flow vs plain MCMC (3-det 128 s, SNR 25, 11 coordinates, 4096 chains)",
        "value": res["flow"]["ess_per_s"], "unit": "ESS/s", "n_gpus": 1, "steps": args.mcmc_steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+bf16", "data": "synthetic",
        "config": {"workload": "flow-mcmc", "chains": 4096, "ess_chains": 256, "snr": 25.0,
                   "burn_in_steps": res["burn_in_steps"], "flow_train_steps": args.flow_steps,
                   "flow_lr": args.flow_lr, "flow_lr_final": args.flow_lr_final,
                   "train_samples": res["train_samples"], "precision": args.precision, "spins": args.spins},
    }
    result.update(res)
    print(json.dumps(result), flush=True)


def bench_flow_train(args):
    """Training of the learned proposal alone: the flow of the flow-mcmc
    workload (8 couplings 11 -> 256 -> 256 -> 22) fitted to 208,896 synthetic
    11-parameter rows (a seeded correlated Gaussian, the size of the
    random-walk training set), minibatches of 4096, --flow-steps Adam steps
    with the flow-mcmc schedule.  Reports Adam steps per second and the MFMA
    rate of the step's matrix products (three products of 2 n (D H + H^2 +
    2 D H) flops per layer: forward, input gradients, weight gradients)."""
    import numpy as np
    import torch

    from paper_1904_02863_amd import sampler
    rng = np.random.default_rng(20190408)
    d, n_rows = 11, 208896
    a = rng.standard_normal((d, d)) * 0.3 + np.eye(d)
    x = torch.from_numpy(rng.standard_normal((n_rows, d)) @ a.T + rng.uniform(-5, 5, d)).to("cuda")
    lr_final = args.flow_lr_final if args.flow_lr_final > 0 else None
    sampler.train_flow(x, steps=max(1, args.warmup), lr=args.flow_lr, lr_final=lr_final)       # warm-up
    flow, hist, secs = sampler.train_flow(x, steps=args.flow_steps, lr=args.flow_lr, lr_final=lr_final,
                                          log_every=max(1, args.flow_steps // 4))
    h, layers, batch = 256, 8, 4096
    flops = 3 * 2 * batch * (d * h + h * h + 2 * d * h) * layers
    per = secs / args.flow_steps
    result = {
        "metric": "flow training Adam steps/s (8 couplings 11-256-256-22, batch 4096)",
        "value": 1.0 / per, "unit": "steps/s", "n_gpus": 1, "steps": args.flow_steps,
        "warmup": max(1, args.warmup), "ms_per_step": per * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16+f32+f64", "data": "synthetic",
        "config": {"workload": "flow-train", "rows": n_rows, "dim": d, "hidden": h, "layers": layers,
                   "batch": batch, "lr": args.flow_lr, "lr_final": lr_final},
        "loss_history": hist,
        "roofline": {"bound": "mfma", "achieved": flops / per / 1e12, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": flops / per / 1e12 / 2500.0, "traffic": None,
                     "kernel": "whole training step (5 launches: the minibatch gather, one through all 8 couplings "
                               "in each direction, one of all couplings' weight-gradient GEMMs, one for the "
                               "gradient sums and Adam)",
                     "gemm_flops_per_step": flops},
    }
    print(json.dumps(result), flush=True)


MIXED_REPORT = "profiles/mixed_precision_bbh-3det-128s.md"


def mixed_comparison(args, step_args, fp64_out, fp64_s: float) -> dict:
    """The precision extension on the same batch, after the timed FP64 steps:
    the mixed path timed the same way (its own workspace, first call tuning
    its plan), its largest |lnL difference| from the FP64 values of the batch,
    and the per-injection figures of the committed 1024-injection report."""
    import torch

    import paper_1904_02863_amd as gw
    g, w, data, psd, theta = step_args
    ws = gw.Workspace(0)
    out = torch.empty_like(fp64_out)

    def step():
        gw.lnl_batch(g, w.tensors, w.vertices, data, psd, theta, out=out, workspace=ws, precision="mixed")

    step()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    res = {"value": w.n_samples / t, "unit": "lnL evals/s", "ms_per_step": t * 1e3, "speedup_vs_fp64": fp64_s / t,
           "plan": ws.lnl_plan(g.n_bins, w.n_det, w.n_samples, "mixed"),
           "max_abs_dlnl_vs_fp64_this_batch": float((out - fp64_out).abs().max().item()), "tolerance": 1e-3}
    path = os.path.join(ROOT, MIXED_REPORT)
    if os.path.exists(path):
        text = open(path).read()
        for key in ("max_abs_dlnl_vs_oracle", "max_rel_dh_vs_oracle", "injections"):
            m = re.search(rf"{key}:\s*([0-9.eE+-]+)", text)
            if m:
                res[f"report_{key}"] = float(m.group(1))
        res["report"] = MIXED_REPORT
    return res


def flow_summary(res: dict) -> dict:
    """The compact learned-proposal figures carried on the default line."""
    return {"workload": "flow-mcmc", "spins": res["spins"], "chains": 4096, "burn_in_steps": res["burn_in_steps"],
            "ess_per_s_flow": res["flow"]["ess_per_s"],
            "ess_per_s_flow_with_training": res["flow"]["ess_per_s_with_training"],
            "ess_per_s_random_walk": res["random_walk"]["ess_per_s"],
            "speedup": res["speedup_ess_per_s"], "speedup_with_training": res["speedup_with_training"],
            "ks_min_p": res["ks_min_p"], "acceptance_flow": res["flow"]["acceptance"],
            "acceptance_random_walk": res["random_walk"]["acceptance"],
            "train_seconds": res["flow"]["train_seconds"], "train_samples": res["train_samples"],
            "wall_seconds": res["wall_seconds"]}


def bench_population(args):
    """Population likelihood of Eq. (poplike): 200 events x 20,000 posterior
    samples (4e6 samples, where the paper's GPU saturates), synthetic
    stand-ins for the GWTC-1 releases, prepared once (gw_pop_prepare: the
    per-sample logarithms).  Two regimes: one hyper-parameter point per call
    (the paper's setting; each call streams the 256 MB of prepared samples)
    and 64 points per call (the samples stay in registers while the points
    loop; bounded by the FP64 VALU).  The same calls on the raw samples are
    reported beside."""
    import numpy as np
    import torch

    import paper_1904_02863_amd as gw
    import synth

    n_events, n_per = 200, 20000
    samples = synth.population_samples(n_events, n_per)
    rng = np.random.default_rng(7)
    k = 64
    hyper = np.empty((k, 12))
    hyper[:] = [2.3, 1.2, 6.0, 70.0, 0.15, 33.0, 4.0, 2.0, 5.0, 0.6, 0.5, 0.9]
    hyper *= rng.uniform(0.9, 1.1, hyper.shape)
    hyper[:, [4, 9]] = np.clip(hyper[:, [4, 9]], 0.0, 1.0)
    dev = torch.device("cuda", 0)
    s_t = torch.from_numpy(samples).to(dev)
    h_t = torch.from_numpy(hyper).to(dev)
    ws = gw.Workspace(0)
    out = torch.empty(k, dtype=torch.float64, device=dev)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p_t = gw.pop_prepare(s_t)          # once per sample set: the per-sample logarithms
    torch.cuda.synchronize()
    prep_s = time.perf_counter() - t0

    def timed(n_hyper, steps, warmup, src):
        """(wall seconds per call, mean seconds of the weights kernel from HIP events)"""
        h = h_t[:n_hyper].contiguous()
        o = out[:n_hyper]
        for _ in range(warmup):
            gw.pop_lnl(src, h, out=o, workspace=ws)
        torch.cuda.synchronize()
        ws.set_timing(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            gw.pop_lnl(src, h, out=o, workspace=ws)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        kernel_ms, launches = ws.kernel_time()
        ws.set_timing(False)
        return wall, kernel_ms / launches / 1e3

    t1r, k1r = timed(1, max(args.steps, 50), args.warmup, s_t)
    tkr, kkr = timed(k, args.steps, args.warmup, s_t)
    t1, k1 = timed(1, max(args.steps, 50), args.warmup, p_t)
    tk, kk = timed(k, args.steps, args.warmup, p_t)
    if not torch.isfinite(out).all():
        raise SystemExit("non-finite population lnL")
    n = n_events * n_per
    bytes_per_call = 8 * 8 * n        # the prepared samples: 8 doubles each
    result = {
        "metric": "population lnL evals/s (200 events x 20,000 samples)",
        "value": k / tk, "unit": "lnL evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": tk * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "population", "n_events": n_events, "n_per_event": n_per, "hyper_per_call": k},
        "weights_kernel_ms": kk * 1e3,
        "samples": "prepared once (gw_pop_prepare), then reused by every call",
        "preparation_ms": prep_s * 1e3,
        "raw_samples": {"value": k / tkr, "ms_per_call": tkr * 1e3, "one_point_per_second": 1.0 / t1r,
                        "one_point_kernel_ms": k1r * 1e3},
        "one_point_per_call": {"value": 1.0 / t1, "ms_per_call": t1 * 1e3,
                               "roofline": {"bound": "hbm", "achieved": bytes_per_call / k1 / 1e9,
                                            "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                            "frac": bytes_per_call / k1 / 1e9 / HBM_PEAK_GBS,
                                            "kernel": "weights_kernel", "kernel_ms": k1 * 1e3,
                                            "algorithmic_bytes": bytes_per_call}},
    }
    if not args.no_cpu_baseline:
        from oracle import population as pop
        done, spent = 0, 0.0
        while spent < args.cpu_seconds / 2 and done < k:
            t0 = time.perf_counter()
            pop.lnl(samples, hyper[done:done + 1])
            spent += time.perf_counter() - t0
            done += 1
        result["cpu_baseline"] = {"value": done / spent, "unit": "lnL evals/s", "cores": 1, "kind": "oracle",
                                  "sample": f"{done} hyper-parameter points over all 4e6 samples, {spent:.1f} s"}
    ws.close()
    print(json.dumps(result), flush=True)


def bench_waveform(args):
    """gw_waveform_batch (the template of Sec. II, Fig. 1): detector responses
    of 256 samples on the 3-detector 128 s grid, 3.19 GB of complex128 written
    per call, so the call is bounded by HBM write bandwidth."""
    import torch

    import paper_1904_02863_amd as gw
    import synth

    n = args.samples or 256
    w = synth.bbh_3det_128s(n)
    g = w.grid
    dev = torch.device("cuda", 0)
    theta = torch.from_numpy(w.theta).to(dev)
    out = torch.empty((n, w.n_det, g.n_bins), dtype=torch.complex128, device=dev)
    ws = gw.Workspace(0)
    for _ in range(args.warmup):
        gw.waveform_batch(g, w.tensors, w.vertices, theta, out=out, workspace=ws)
    torch.cuda.synchronize()
    ws.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gw.waveform_batch(g, w.tensors, w.vertices, theta, out=out, workspace=ws)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    kernel_ms, launches = ws.kernel_time()
    ws.set_timing(False)
    kernel_s = kernel_ms / launches / 1e3
    if args.calibrate_copy > 0:
        calibration_copy(args.calibrate_copy, dev)
    if not torch.isfinite(torch.view_as_real(out)).all():
        raise SystemExit("non-finite waveform")
    written = out.numel() * 16
    read = g.n_bins * (32 + 16)
    # the write ceiling: the library's plain store kernel over the same buffer
    for _ in range(3):
        gw.fill_c128(out, 0.0)
    t_fill = []
    for _ in range(max(args.steps // 5, 5)):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        gw.fill_c128(out, 0.0)
        b.record()
        t_fill.append((a, b))
    torch.cuda.synchronize()
    fill_s = sum(a.elapsed_time(b) for a, b in t_fill) / len(t_fill) / 1e3
    store_gbs = written / fill_s / 1e9
    achieved = (written + read) / kernel_s / 1e9
    result = {
        "metric": "waveforms/s (3-det,128 s TaylorF2 responses)", "value": n / t, "unit": "waveforms/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "waveform", "n_samples": n, "n_det": w.n_det, "n_bins": g.n_bins},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("waveform", WAVEFORM_PROFILE) if n == 256 else None,
                     "kernel": "waveform_kernel", "kernel_ms": kernel_s * 1e3,
                     "algorithmic_bytes": written + read,
                     "store_ceiling": {"kernel": "fill_c128_kernel", "bytes_written": written,
                                       "kernel_ms": fill_s * 1e3, "achieved": store_gbs},
                     "frac_of_store_ceiling": achieved / store_gbs},
    }
    if not args.no_cpu_baseline:
        import oracle
        done, spent = 0, 0.0
        while spent < args.cpu_seconds / 3 and done < n:
            t0 = time.perf_counter()
            oracle.waveform(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, w.theta[done:done + 16])
            spent += time.perf_counter() - t0
            done += 16
        result["cpu_baseline"] = {"value": done / spent, "unit": "waveforms/s", "cores": oracle.max_threads(),
                                  "kind": "oracle", "sample": f"{done} of the {n} samples, {spent:.1f} s"}
    ws.close()
    print(json.dumps(result), flush=True)


def rb_flops_per_pair(n_det: int, mixed: bool = False) -> int:
    """Algorithmic FP64 flops of the relative-binning kernel per (sample, bin),
    i.e. per edge (FMA = 2, multiply or add = 1): the phase-difference
    polynomial 19 (9 FMA + 1 multiply); per detector the phasor 34, the ratio
    (P/P0) e^{-i dPhi} 6, the linear term 4, the squared term 5 and the cross
    term with the previous edge 5, plus 2 for the delay term on every
    detector but the first.  The mixed path replaces the phasor by the
    reduction to a fractional turn (1 add) and two FP32 hardware
    transcendentals, which are not counted."""
    return 19 + (54 - (33 if mixed else 0)) * n_det + 2 * (n_det - 1)


def bench_relbin(args):
    """Relative binning (named in Secs. I and V): the 15 Hz / 512 s neutron-star
    event (3 detectors, 1,040,897 bins, network SNR 30; or with --rb-band
    5hz-8192s one detector, 16,736,257 bins) cut into ~10^3 bins by the
    phase-bound rule (chi 1, eps 0.03); one step = one gw_rb_lnl call over
    65,536 rows near the fiducial (the injection)."""
    import torch

    import paper_1904_02863_amd as gw
    import synth

    n = args.samples or 65536
    dev = torch.device("cuda", 0)
    ws = gw.Workspace(0)
    f_low, duration, n_det = {"15hz-512s": (15.0, 512.0, 3), "5hz-8192s": (5.0, 8192.0, 1)}[args.rb_band]
    w = synth.relbin_bns(f_low, duration, n_det, n, index=6)
    g = w.grid
    psd = torch.from_numpy(w.psd).to(dev)
    h = gw.waveform_batch(g, w.tensors, w.vertices, torch.from_numpy(w.theta_inj[None]).to(dev), workspace=ws)[0]
    rho = math.sqrt(float((4.0 * g.delta_f * (h.real ** 2 + h.imag ** 2) / psd).sum()))
    w = synth.scale_distance(w, rho / 30.0)
    data = torch.from_numpy(w.noise).to(dev) + h * (30.0 / rho)
    del h
    edges = gw.rb_edges(g, 1.0, 0.03)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rbh = gw.RelativeBinning(g, w.tensors, w.vertices, data, psd, w.theta_inj, edges, workspace=ws)
    prep_s = time.perf_counter() - t0
    n_rb, n_det = rbh.shape
    theta = torch.from_numpy(w.theta).to(dev)
    out = torch.empty(n, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        rbh.lnl(theta, out=out, workspace=ws, precision=args.precision)
    torch.cuda.synchronize()
    ws.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rbh.lnl(theta, out=out, workspace=ws, precision=args.precision)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    kernel_ms, launches = ws.kernel_time()
    ws.set_timing(False)
    kernel_s = kernel_ms / launches / 1e3
    if args.calibrate_copy > 0:
        calibration_copy(args.calibrate_copy, dev)
    if not torch.isfinite(out).all():
        raise SystemExit("non-finite relative-binning lnL")
    # the full likelihood of the same event, for its rate and the estimate's error
    m = min(n, 4096)
    full = gw.lnl_batch(g, w.tensors, w.vertices, data, psd, theta[:m].contiguous(), workspace=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(3):
        gw.lnl_batch(g, w.tensors, w.vertices, data, psd, theta[:m].contiguous(), out=full, workspace=ws)
    torch.cuda.synchronize()
    full_s = (time.perf_counter() - t1) / 3
    rbh.lnl(theta, out=out, workspace=ws, precision=args.precision)
    err = (out[:m] - full).abs().max().item()
    mixed = args.precision == "mixed"
    flops = rb_flops_per_pair(n_det, mixed) * n * n_rb
    profiled = n == 65536 and args.rb_band == "15hz-512s" and not mixed
    executed = measured_executed_flops("relbin", RELBIN_PROFILE) if profiled else None
    result = {
        "metric": f"lnL evals/s (relative binning, BNS {f_low:g} Hz {duration:g} s, {n_det} det)", "value": n / t,
        "unit": "lnL evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32" if mixed else "f64", "data": "synthetic",
        "config": {"workload": f"bns-relbin-{args.rb_band}", "precision": args.precision, "n_samples": n, "n_det": n_det, "n_bins": g.n_bins,
                   "rb_bins": n_rb, "chi": 1.0, "eps": 0.03},
        "roofline": {"bound": "alu", "achieved": executed / kernel_s / 1e12 if executed else None,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": executed / kernel_s / 1e12 / FP64_PEAK_TFLOPS if executed else None,
                     "flops_source": ("executed FP64 flops from the counters in " + RELBIN_PROFILE if executed
                                      else "no counter summary of these kernel sources and this shape"),
                     "executed_flops_per_launch": executed,
                     "traffic": measured_traffic("relbin", RELBIN_PROFILE) if profiled else None,
                     "kernel": f"relative-binning lnl_kernel<{n_det}>", "kernel_ms": kernel_s * 1e3,
                     "frac_tally": flops / kernel_s / 1e12 / FP64_PEAK_TFLOPS,
                     "flops_per_pair_tally": rb_flops_per_pair(n_det, mixed)},
        "preparation_ms": prep_s * 1e3,
        "full_likelihood": {"value": m / full_s, "ms_per_call": full_s * 1e3, "rows": m},
        "max_abs_error_vs_full": err,
    }
    if not args.no_cpu_baseline:
        import oracle
        from oracle import relbin as rb
        d_np = data.cpu().numpy()
        t0 = time.perf_counter()
        summ = rb.summary(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, d_np, w.psd, w.theta_inj, edges)
        prep_cpu = time.perf_counter() - t0
        done, spent = 0, 0.0
        while spent < args.cpu_seconds / 2 and done < n:
            t0 = time.perf_counter()
            rb.lnl(summ, w.tensors, w.vertices, w.theta[done:done + 256])
            spent += time.perf_counter() - t0
            done += 256
        result["cpu_baseline"] = {"value": done / spent, "unit": "lnL evals/s", "cores": oracle.max_threads(),
                                  "kind": "oracle", "sample": f"{done} of the {n} rows, {spent:.1f} s "
                                  f"(summary data {prep_cpu:.1f} s, not counted)"}
    rbh.close()
    ws.close()
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--workload", default="bbh-3det-128s",
                    choices=["bbh-3det-128s", "bbh-1det-4s", "bns-15hz-512s", "bns-ragged", "flow-mcmc",
                             "flow-train", "population", "waveform", "bns-relbin"])
    ap.add_argument("--mcmc-burn", type=int, default=None,
                    help="flow-mcmc: random-walk burn-in steps (default 120000 with aligned spins, 4000 without)")
    ap.add_argument("--mcmc-steps", type=int, default=1024, help="flow-mcmc: production steps of each sampler")
    ap.add_argument("--flow-steps", type=int, default=1500, help="flow-mcmc: Adam steps")
    ap.add_argument("--flow-lr", type=float, default=2e-3, help="flow-mcmc: Adam step size")
    ap.add_argument("--flow-lr-final", type=float, default=2e-5,
                    help="flow-mcmc: the step size falls to this on a half cosine (<= 0: constant)")
    ap.add_argument("--samples", type=int, default=None)
    ap.add_argument("--plan", default=None, metavar="TILE,ROUNDS",
                    help="run this likelihood plan (LDS tile bins, work-queue rounds) instead of the autotuned one")
    ap.add_argument("--flags", type=int, default=0,
                    help="likelihood options: 1 direct form, 2 ISCO template end, 4 log prefactor (or-ed)")
    ap.add_argument("--rb-band", default="15hz-512s", choices=["15hz-512s", "5hz-8192s"],
                    help="bns-relbin: the neutron-star band (3 detectors from 15 Hz, or 1 detector from 5 Hz)")
    ap.add_argument("--spins", action="store_true",
                    help="single-event workloads: aligned spins chi1, chi2 ~ U[-1, 1] on every row; "
                         "flow-mcmc: the two spin coordinates enter the likelihood")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="CPU-baseline budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-flow", action="store_true",
                    help="default workload: skip the learned-proposal comparison appended to the line")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the timed steps, run one plain device-to-device copy of MIB MiB "
                         "(reference dispatch for scaling hardware traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(samples shard trivially across GPUs; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1904_02863_amd as gw

    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible: the benchmark runs the HIP library only")
    if args.workload == "bns-ragged":
        bench_ragged(args)
        return
    if args.workload == "flow-mcmc":
        bench_flow(args)
        return
    if args.workload == "flow-train":
        bench_flow_train(args)
        return
    if args.workload == "population":
        bench_population(args)
        return
    if args.workload == "waveform":
        bench_waveform(args)
        return
    if args.workload == "bns-relbin":
        bench_relbin(args)
        return
    w, data, psd, theta = build_inputs(args.workload, args.samples, args.spins)
    g = w.grid
    ws = gw.Workspace(0)
    ws.reserve(g.n_bins, w.n_det, w.n_samples)
    out = torch.empty(w.n_samples, dtype=torch.float64, device=theta.device)

    def step():
        gw.lnl_batch(g, w.tensors, w.vertices, data, psd, theta, out=out, workspace=ws, precision=args.precision,
                     flags=args.flags)

    if args.plan:
        tile, rounds = (int(v) for v in args.plan.split(","))
        ws.set_tuning(False)
        ws.set_plan(g.n_bins, w.n_det, w.n_samples, tile, rounds, args.precision, args.flags)
    step()                             # first call: times the candidate plans, keeps the fastest (untimed)
    plan = ws.lnl_plan(g.n_bins, w.n_det, w.n_samples, args.precision, args.flags)
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
    if args.calibrate_copy > 0:
        calibration_copy(args.calibrate_copy, theta.device)
    if not torch.isfinite(out).all():
        raise SystemExit("non-finite lnL in the benchmark batch")

    evals = w.n_samples * args.steps
    kernel_avg_s = kernel_ms / 1e3 / max(launches, 1)
    mixed = args.precision == "mixed"
    direct = bool(args.flags & 1)
    flops_launch = flops_per_pair(w.n_det, mixed, direct) * w.n_samples * g.n_bins
    tally_rate = flops_launch / kernel_avg_s / 1e12
    headline = args.workload == "bbh-3det-128s" and args.flags == 0 and not args.spins
    # the counters hold for the plan they were taken under
    key = plan_key(args.precision, plan)
    # FP64 flops the hardware counters saw one launch execute (FMA = 2), from
    # the committed summary of the same kernel sources; None when they changed
    executed = measured_executed_flops(key) if headline else None
    source = f"executed FP64 flops from the counters in {PROFILE_SUMMARY}" if executed is not None else None
    if executed is None and w.n_det == 3 and args.flags == 0:
        # another batch on the same 3-detector split-form loop (other bins,
        # samples or aligned spins, which change only the per-sample
        # coefficients): the counted flops per (sample, bin) of that loop
        per_pair = executed_flops_per_pair(args.precision)
        if per_pair is not None:
            executed = per_pair * w.n_samples * g.n_bins
            source = ("executed FP64 flops per (sample, bin) of the same tile loop, from the counters in "
                      + PROFILE_SUMMARY)
    achieved = executed / kernel_avg_s / 1e12 if executed is not None else None
    # VALU issue cycles per SIMD per launch (every instruction at its measured
    # issue cost: the mixed path's FP32 transcendentals take two slots)
    issue = _profile_value(f"valu_issue_cycles_per_simd_{key}", PROFILE_SUMMARY) if headline else None
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
        "dtype": "f64+f32" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_samples": w.n_samples, "n_det": w.n_det, "n_bins": g.n_bins,
                   "delta_f": g.delta_f, "f_low": g.f_low, "f_high": g.f_high, "n_param": w.n_param,
                   "precision": args.precision, "flags": args.flags, "spins": args.spins, "plan": plan},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS if achieved is not None else None,
                     "flops_source": (source if executed is not None else
                                      f"no counter summary of these kernel sources under plan {key} "
                                      f"(profiled: {profiled_plans(args.precision)})"),
                     "executed_flops_per_launch": executed,
                     "issue_frac": (issue / (kernel_avg_s * 2.4e9) if issue is not None else None),
                     "traffic": measured_traffic(key) if headline else None,
                     "kernel": f"lnl_tile_kernel<{w.n_det},{'mixed' if mixed else 'fp64'}>",
                     "kernel_ms": kernel_avg_s * 1e3,
                     # the algorithmic tally below prices the phasor at its
                     # polynomial cost; the table phasor the kernel runs costs less
                     "frac_tally": tally_rate / FP64_PEAK_TFLOPS, "flops_per_launch_tally": flops_launch,
                     "flops_per_pair_tally": flops_per_pair(w.n_det, mixed, direct)},
    }
    if args.flags & 2:
        # the kernel skips the bins above the batch's largest cut-off, so a
        # tally over every bin would overstate the rate
        result["roofline"] = None
    if headline and args.precision == "fp64":
        result["mixed_precision"] = mixed_comparison(args, step_args=(g, w, data, psd, theta), fp64_out=out,
                                                     fp64_s=elapsed / args.steps)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, data, args.cpu_seconds, args.flags)
    if args.workload == "bbh-3det-128s" and not args.no_flow:
        # the second half of the metric: the learned proposal against plain
        # random-walk MCMC on the same GPU (outside the timed region above)
        del data, psd, theta, out, ws
        result["flow_mcmc"] = flow_summary(flow_comparison(args, True))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
