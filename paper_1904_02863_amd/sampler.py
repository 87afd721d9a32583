"""Many-chain Metropolis-Hastings with the exact GPU likelihood and a learned
proposal.

The likelihood is gw_lnl_batch, Eq. (cbclike) of arXiv:1904.02863 (Sec. III).
The paper notes (Sec. I) that the sampling algorithm is hard to parallelise
while the likelihood is embarrassingly parallel; here thousands of chains step
together, every step is one batched likelihood call, and every proposal,
random number, acceptance decision and adaptation runs in the library's
kernels:

* random-walk MH: x' = x + L z (Philox normals), L the Cholesky factor of
  (2.38^2/d) s^2 Cov, Cov the chains' sample covariance and s a global scale
  tuned toward 23.4% acceptance, both adapted during burn-in
  (gw_mcmc_adapt_chol);
* learned proposal: an affine-coupling flow (gw_flow) trained by maximum
  likelihood on random-walk samples (minibatches drawn on the GPU,
  gw_gather_rows), used as an independence proposal x' = F(z).  The exact
  likelihood stays the judge.  Every rw_every-th step is a random-walk step
  for all chains (a fixed cycle of two kernels that both leave the posterior
  invariant, so the cycle does), and when the flow's acceptance over the
  first window of a run is below a threshold the run falls back to
  random-walk steps only.

Sampler coordinates are x_i = logit(u_i), u_i the position of parameter i in
a uniform prior box (see gw_mcmc_to_theta).  Host code here only orchestrates
calls, moves a few scalars and keeps statistics.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np

from . import (Flow, Workspace, chain_normals, gather_rows, lnl_batch, mcmc_accept, mcmc_adapt_chol, mcmc_count,
               mcmc_moments, mcmc_rw_propose, mcmc_to_theta)

# Philox streams used by the sampler (the kernels use 1 for random-walk
# normals and 2 for acceptance uniforms).
STREAM_FLOW = 3
STREAM_MINIBATCH = 4

PARAM_NAMES = ("mc", "q", "dl", "phic", "tc", "ra", "sindec", "psi", "cosiota", "chi1", "chi2")


@dataclasses.dataclass
class Problem:
    """One event's likelihood and the prior box of the sampler coordinates."""
    grid: object
    tensors: np.ndarray
    vertices: np.ndarray
    data: object            # torch complex128 [n_det, M] on the GPU
    psd: object             # torch float64 [n_det, M] on the GPU
    box_lo: np.ndarray      # [dim]
    box_hi: np.ndarray      # [dim]
    precision: str = "fp64"
    spins: bool = False     # dim 11: the last two coordinates enter lnL as aligned spins chi1, chi2

    @property
    def dim(self) -> int:
        return int(self.box_lo.shape[0])

    @property
    def theta_cols(self) -> int:
        return 11 if self.spins else 9


def to_sampler_coords(problem: Problem, params: np.ndarray) -> np.ndarray:
    """Box parameters (Mc, q, d_L, phi_c, t_c, RA, sin Dec, psi, cos iota[, chi1, chi2]) -> x."""
    u = (np.asarray(params, dtype=np.float64) - problem.box_lo) / (problem.box_hi - problem.box_lo)
    return np.log(u) - np.log1p(-u)


def from_sampler_coords(problem: Problem, x: np.ndarray) -> np.ndarray:
    u = 1.0 / (1.0 + np.exp(-np.asarray(x, dtype=np.float64)))
    return problem.box_lo + (problem.box_hi - problem.box_lo) * u


def injection_box(theta_inj, spins: bool = False):
    """The 11-coordinate prior box around an injection theta_inj (9 columns of
    gw_lnl_batch): Mc [25, 35], q [0.5, 1], d_L [0.2, 3] x its value,
    t_c [-0.1, 0.1], RA [0, 2 pi), sin Dec and cos iota [-1, 1], chi1, chi2
    [-1, 1], and phi_c and psi on one period of their symmetries centred on
    the injection: phi_c within pi of it (the phase is 2 pi periodic) and psi
    within pi/4 of it (psi -> psi + pi/2 with phi_c -> phi_c + pi gives the
    same signal, so a wider psi box would hold two copies of every mode).
    Returns (box_lo, box_hi, the injection in box coordinates with zero
    spins)."""
    inj = np.asarray(theta_inj, dtype=np.float64)
    lo = np.array([25.0, 0.5, 0.2 * inj[2], inj[3] - math.pi, -0.1, 0.0, -1.0, inj[7] - math.pi / 4, -1.0, -1.0,
                   -1.0])
    hi = np.array([35.0, 1.0, 3.0 * inj[2], inj[3] + math.pi, 0.1, 2 * math.pi, 1.0, inj[7] + math.pi / 4, 1.0,
                   1.0, 1.0])
    p_inj = np.array([inj[0], inj[1], inj[2], inj[3], inj[4], inj[5], math.sin(inj[6]), inj[7], math.cos(inj[8]),
                      0.0, 0.0])
    return lo, hi, p_inj


class _Buffers:
    def __init__(self, torch, n, dim, device, theta_cols=9):
        f64 = dict(dtype=torch.float64, device=device)
        self.x_prop = torch.empty((n, dim), **f64)
        self.theta = torch.empty((n, theta_cols), **f64)
        self.lp = torch.empty(n, **f64)
        self.lnl = torch.empty(n, **f64)
        self.z = torch.empty((n, dim), **f64)
        self.logq_prop = torch.empty(n, **f64)
        self.window = torch.zeros(n, dtype=torch.int32, device=device)
        self.total = torch.zeros(n, dtype=torch.int32, device=device)
        self.count = torch.zeros(1, dtype=torch.int64, device=device)

    def accepted(self, counters) -> int:
        """Sum of an acceptance counter array, summed on the GPU."""
        mcmc_count(counters, out=self.count)
        return int(self.count.item())


def _evaluate(problem: Problem, x, buf: _Buffers, ws: Workspace):
    """lnL and log prior of rows x into buf.lnl, buf.lp."""
    mcmc_to_theta(problem.box_lo, problem.box_hi, x, theta_out=buf.theta, logprior_out=buf.lp)
    lnl_batch(problem.grid, problem.tensors, problem.vertices, problem.data, problem.psd, buf.theta, out=buf.lnl,
              workspace=ws, precision=problem.precision)


def _records(torch, n_steps: int, record_every: int, track, x):
    """Device array for the records of the first `track` chains every
    record_every steps, or None when nothing is recorded."""
    n_records = n_steps // record_every if record_every else 0
    if n_records == 0:
        return None
    rows = x[:track].shape[0]
    return torch.empty((n_records, rows, x.shape[1]), dtype=x.dtype, device=x.device)


def _host(records):
    return None if records is None else records.cpu().numpy()


def _device_chol(chol, device):
    import torch
    if isinstance(chol, torch.Tensor):
        return chol.to(device=device, dtype=torch.float64).contiguous()
    return torch.from_numpy(np.ascontiguousarray(chol, dtype=np.float64)).to(device)


@dataclasses.dataclass
class ChainState:
    x: object        # torch [n, dim]
    lnp: object      # torch [n]: lnL + log prior at x
    logq: object     # torch [n]: flow log density at x (flow runs)
    step: int = 0


def init_chains(problem: Problem, x0: np.ndarray, ws: Workspace) -> ChainState:
    """Chains at the rows of x0 with lnp = lnL + log prior there: every chain
    starts at lnp = -inf and accepts x0 as its first proposal (a row whose
    lnL is not finite keeps lnp = -inf)."""
    import torch
    dev = problem.data.device
    n = x0.shape[0]
    x_start = torch.from_numpy(np.ascontiguousarray(x0, dtype=np.float64)).to(dev)
    x = torch.empty_like(x_start)
    lnp = torch.full((n,), -math.inf, dtype=torch.float64, device=dev)
    buf = _Buffers(torch, n, problem.dim, dev, problem.theta_cols)
    _evaluate(problem, x_start, buf, ws)
    mcmc_accept(0, 0, x, lnp, x_start, buf.lnl, buf.lp)
    return ChainState(x, lnp, torch.zeros_like(lnp), 0)


def run_random_walk(problem: Problem, state: ChainState, n_steps: int, seed: int, chol, ws: Workspace,
                    adapt_every: int = 0, record_every: int = 0, record_track: int | None = None,
                    collect_every: int = 0, target_accept: float = 0.234, progress=None):
    """n_steps random-walk MH steps on every chain.  With adapt_every > 0 the
    proposal is re-fitted that often on the GPU: the Cholesky factor of
    (2.38^2/d) s^2 times the chains' sample covariance, s a global scale that
    a Robbins-Monro step moves toward the acceptance rate target_accept over
    the last window (0.234, the optimum of Roberts, Gelman & Gilks 1997, by
    default).  Records the first record_track chains every record_every
    steps and collects all chains every collect_every steps, both into device
    arrays (the records are copied to the host once, after the last step, so
    that recording never makes the host wait for the GPU).  Returns (records [n_records, track, dim] or None,
    acceptance rate, seconds, final Cholesky factor (device), collected
    [n_collect * n_chains, dim] on the device or None).  progress, if given,
    is called with the number of steps done every 10,000 steps."""
    import torch
    n, dim = state.x.shape
    dev = state.x.device
    buf = _Buffers(torch, n, dim, dev, problem.theta_cols)
    chol_t = _device_chol(chol, dev)
    records = _records(torch, n_steps, record_every, record_track, state.x)
    n_collect = n_steps // collect_every if collect_every else 0
    collected = torch.empty((n_collect * n, dim), dtype=torch.float64, device=dev) if n_collect else None
    log_scale, window_start = 0.0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n_steps):
        step = state.step
        mcmc_rw_propose(state.x, chol_t, seed, step, buf.x_prop)
        _evaluate(problem, buf.x_prop, buf, ws)
        mcmc_accept(seed, step, state.x, state.lnp, buf.x_prop, buf.lnl, buf.lp, total_accepts=buf.total)
        state.step += 1
        if adapt_every and (i + 1) % adapt_every == 0:
            accepted = buf.accepted(buf.total)
            rate = (accepted - window_start) / (n * adapt_every)
            window_start = accepted
            log_scale = float(np.clip(log_scale + 2.0 * (rate - target_accept), -8.0, 2.0))
            mcmc_adapt_chol(state.x, scale=math.exp(log_scale), out=chol_t)
        if records is not None and (i + 1) % record_every == 0:
            records[(i + 1) // record_every - 1].copy_(state.x[:record_track])
        if collect_every and (i + 1) % collect_every == 0:
            k = (i + 1) // collect_every - 1
            collected[k * n:(k + 1) * n].copy_(state.x)
        if progress is not None and (i + 1) % 10000 == 0:
            progress(i + 1)
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    rate = buf.accepted(buf.total) / (n * max(n_steps, 1))
    return _host(records), rate, seconds, chol_t, collected


# ---------------------------------------------------------------- flow
def default_masks(dim: int, n_layers: int, seed: int = 0) -> np.ndarray:
    """Conditioning sets: alternating halves of a seeded permutation per pair of layers."""
    rng = np.random.default_rng(seed)
    masks = []
    for l in range(n_layers):
        if l % 2 == 0:
            perm = rng.permutation(dim)
            first = perm[: dim // 2]
        bits = 0
        chosen = first if l % 2 == 0 else np.setdiff1d(np.arange(dim), first)
        for i in chosen:
            bits |= 1 << int(i)
        masks.append(bits)
    return np.array(masks, dtype=np.uint32)


def init_flow_params(dim: int, hidden: int, n_layers: int, seed: int, scale_last: float = 0.0) -> np.ndarray:
    """Seeded uniform(+-1/sqrt(fan_in)) weights and biases; the output layer
    scaled by scale_last (0 starts from the identity map)."""
    rng = np.random.default_rng(seed)
    parts = []
    shapes = [("w1", (hidden, dim), dim), ("b1", (hidden,), dim), ("w2", (hidden, hidden), hidden),
              ("b2", (hidden,), hidden), ("w3", (2 * dim, hidden), hidden), ("b3", (2 * dim,), hidden)]
    for _ in range(n_layers):
        for name, shape, fan_in in shapes:
            v = rng.uniform(-1, 1, shape) / math.sqrt(fan_in)
            if name in ("w3", "b3"):
                v = v * scale_last
            parts.append(v.ravel())
    return np.concatenate(parts).astype(np.float32)


def train_flow(samples, n_layers: int = 8, hidden: int = 256, steps: int = 2000, batch: int = 4096,
               lr: float = 1e-3, seed: int = 0, device: int = 0, log_every: int = 0, lr_final: float | None = None):
    """Fit a flow to samples [n, dim] (device tensor or host array) by maximum
    likelihood: Adam on minibatches drawn with replacement on the GPU
    (gw_gather_rows), after an affine standardisation by the samples' mean and
    standard deviation (gw_mcmc_moments).  The step size is lr throughout, or
    with lr_final given falls from lr to lr_final on a half cosine over the
    steps.  Returns (flow, loss history, seconds)."""
    import torch
    dev = torch.device("cuda", device)
    if isinstance(samples, torch.Tensor):
        data = samples.to(device=dev, dtype=torch.float64).contiguous()
    else:
        data = torch.from_numpy(np.ascontiguousarray(samples, dtype=np.float64)).to(dev)
    n, dim = data.shape
    flow = Flow(dim, default_masks(dim, n_layers, seed), hidden=hidden, device=device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()                # the standardisation counts as training time
    mean, cov = mcmc_moments(data)
    mu = mean.cpu().numpy()
    sd = np.sqrt(np.diag(cov.cpu().numpy())) + 1e-12
    flow.set_params(init_flow_params(dim, hidden, n_layers, seed), mu, np.log(sd))
    batch = min(batch, n)
    mb = torch.empty((batch, dim), dtype=torch.float64, device=dev)
    loss_t = torch.empty(1, dtype=torch.float64, device=dev)
    history = []
    for s in range(steps):
        rate = lr
        if lr_final is not None and steps > 1:
            rate = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * s / (steps - 1)))
        gather_rows(data, batch, seed, STREAM_MINIBATCH, s, out=mb)
        flow.train_step(mb, rate, loss_out=loss_t)
        if log_every and (s % log_every == 0 or s == steps - 1):
            history.append((s, float(loss_t.item())))
    torch.cuda.synchronize()
    return flow, history, time.perf_counter() - t0


def run_flow_mh(problem: Problem, state: ChainState, flow: Flow, n_steps: int, seed: int, chol, ws: Workspace,
                rw_every: int = 8, window: int = 64, threshold: float = 0.05, record_every: int = 0,
                record_track: int | None = None):
    """Independence MH with flow proposals x' = F(z), alpha = min(1,
    pi(x') q(x) / (pi(x) q(x'))), and every rw_every-th step (by the global
    step count) a random-walk step for all chains, after which q is
    recomputed at the chains' states.  Both kernels leave the posterior
    invariant, so their fixed cycle does; the choice never depends on a
    chain's own history.  If the flow's acceptance over the first `window`
    flow steps of the run is below `threshold`, the rest of the run takes
    random-walk steps only (random-walk fallback).  Returns (records or None,
    acceptance rate, seconds, fraction of random-walk steps)."""
    import torch
    n, dim = state.x.shape
    dev = state.x.device
    buf = _Buffers(torch, n, dim, dev, problem.theta_cols)
    chol_t = _device_chol(chol, dev)
    flow_mode = torch.zeros(n, dtype=torch.int32, device=dev)
    flow.inverse(state.x, z_out=buf.z, logq_out=state.logq)
    records = _records(torch, n_steps, record_every, record_track, state.x)
    rw_steps, flow_steps, use_flow = 0, 0, True
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n_steps):
        step = state.step
        if not use_flow or (rw_every and step % rw_every == rw_every - 1):
            mcmc_rw_propose(state.x, chol_t, seed, step, buf.x_prop)
            _evaluate(problem, buf.x_prop, buf, ws)
            mcmc_accept(seed, step, state.x, state.lnp, buf.x_prop, buf.lnl, buf.lp, total_accepts=buf.total)
            if use_flow:
                flow.inverse(state.x, z_out=buf.z, logq_out=state.logq)     # q at the moved states
            rw_steps += 1
        else:
            chain_normals(dim, n, seed, STREAM_FLOW, step, out=buf.z)
            flow.forward(buf.z, x_out=buf.x_prop, logq_out=buf.logq_prop)
            _evaluate(problem, buf.x_prop, buf, ws)
            mcmc_accept(seed, step, state.x, state.lnp, buf.x_prop, buf.lnl, buf.lp, logq=state.logq,
                        logq_prop=buf.logq_prop, mode=flow_mode, window_accepts=buf.window, total_accepts=buf.total)
            flow_steps += 1
            if flow_steps == window and buf.accepted(buf.window) < threshold * n * window:
                use_flow = False
        state.step += 1
        if records is not None and (i + 1) % record_every == 0:
            records[(i + 1) // record_every - 1].copy_(state.x[:record_track])
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    rate = buf.accepted(buf.total) / (n * max(n_steps, 1))
    return _host(records), rate, seconds, rw_steps / max(n_steps, 1)


def compare_samplers(problem: Problem, p_inj: np.ndarray, ws: Workspace, n_chains: int = 4096, burn: int = 4000,
                     steps: int = 1024, flow_steps: int = 1500, hidden: int = 256, n_layers: int = 8,
                     seed: int = 20190408, track: int = 256, collect_every: int = 20, rw_every: int = 8,
                     lr: float = 2e-3, lr_final: float | None = 2e-5, log=None):
    """The learned proposal against the plain method on one event: n_chains
    random-walk chains start in a tight ball around the injection (spin
    coordinates that the likelihood ignores start from their prior), burn in
    with adaptation, then run `steps` production steps, recording `track`
    chains every step and collecting all chains every collect_every steps
    (the training set: steps / collect_every x n_chains samples, 2.1e5 by
    default); a flow is trained on them; flow-proposal MH continues from the
    random-walk states for one window, then for `steps` recorded steps.  ESS
    is the rank-normalised bulk ESS (minimum over coordinates) of the tracked
    chains scaled to all chains.  log, if given, receives a progress line
    every 10,000 burn-in steps.  Returns a dict of the figures and the two
    populations' final states (host arrays)."""
    import torch

    from . import diagnostics
    dim = problem.dim
    rng = np.random.default_rng(seed)
    x0 = to_sampler_coords(problem, p_inj)[None] + rng.normal(scale=1e-3, size=(n_chains, dim))
    if dim == 11 and not problem.spins:
        x0[:, 9:] = rng.normal(scale=1.0, size=(n_chains, 2))
    state = init_chains(problem, x0, ws)
    chol = np.diag(np.full(dim, 1e-3))
    def burn_progress(done):
        if log is not None:
            log(f"random-walk burn-in: {done} of {burn} steps")
    _, acc_burn, t_burn, chol, _ = run_random_walk(problem, state, burn, seed, chol, ws, adapt_every=100,
                                                   progress=burn_progress)
    rec_rw, acc_rw, t_rw, chol, collected = run_random_walk(problem, state, steps, seed, chol, ws, record_every=1,
                                                            record_track=track, collect_every=collect_every)
    n_train = int(collected.shape[0])
    flow, hist, t_train = train_flow(collected, n_layers=n_layers, hidden=hidden, steps=flow_steps, batch=4096,
                                     lr=lr, seed=seed + 2, log_every=max(1, flow_steps // 10), lr_final=lr_final)
    fstate = ChainState(state.x.clone(), state.lnp.clone(), torch.zeros_like(state.lnp), state.step)
    run_flow_mh(problem, fstate, flow, 64, seed + 3, chol, ws, rw_every=rw_every)
    rec_fl, acc_fl, t_fl, rw_frac = run_flow_mh(problem, fstate, flow, steps, seed + 3, chol, ws, rw_every=rw_every,
                                                record_every=1, record_track=track)
    rw_draws, fl_draws = rec_rw.transpose(1, 0, 2), rec_fl.transpose(1, 0, 2)
    ess_rw, per_rw = diagnostics.min_ess(rw_draws)
    ess_fl, per_fl = diagnostics.min_ess(fl_draws)
    scale = n_chains / track
    rw_final, fl_final = state.x.cpu().numpy(), fstate.x.cpu().numpy()
    ksp = diagnostics.ks_pvalues(rw_final, fl_final)
    a, b = rw_draws.reshape(-1, dim), fl_draws.reshape(-1, dim)
    zmean = (b.mean(axis=0) - a.mean(axis=0)) / (a.std(axis=0) * np.sqrt(1.0 / per_rw + 1.0 / per_fl))
    return {
        "random_walk": {"ess_per_s": ess_rw * scale / t_rw, "min_ess": ess_rw * scale, "seconds": t_rw,
                        "acceptance": acc_rw, "acceptance_burn_in": acc_burn, "burn_in_seconds": t_burn,
                        "ess_per_coordinate": (per_rw * scale).tolist()},
        "flow": {"ess_per_s": ess_fl * scale / t_fl, "ess_per_s_with_training": ess_fl * scale / (t_fl + t_train),
                 "min_ess": ess_fl * scale, "seconds": t_fl, "train_seconds": t_train, "acceptance": acc_fl,
                 "random_walk_step_fraction": rw_frac, "loss_history": hist,
                 "ess_per_coordinate": (per_fl * scale).tolist()},
        "speedup_ess_per_s": (ess_fl / t_fl) / (ess_rw / t_rw),
        "speedup_with_training": (ess_fl / (t_fl + t_train)) / (ess_rw / t_rw),
        "ks_pvalues_final_states": ksp.tolist(), "ks_min_p": float(ksp.min()),
        "mean_difference_z": zmean.tolist(), "train_samples": int(n_train),
        "states": {"random_walk": rw_final, "flow": fl_final, "flow_lnp": fstate.lnp.cpu().numpy()},
    }
