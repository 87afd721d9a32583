"""Many-chain Metropolis-Hastings with the exact GPU likelihood and a learned
proposal.

The likelihood is gw_lnl_batch, Eq. (cbclike) of arXiv:1904.02863 (Sec. III).
The paper notes (Sec. I) that the sampling algorithm is hard to parallelise
while the likelihood is embarrassingly parallel; here thousands of chains step
together, every step is one batched likelihood call, and every proposal,
random number and acceptance decision is computed by the library's kernels:

* random-walk MH: x' = x + L z (Philox normals), L the Cholesky factor of
  (2.38^2/d) times the chains' sample covariance and a global scale tuned
  toward 23.4% acceptance, both adapted during burn-in;
* learned proposal: an affine-coupling flow (gw_flow) trained by maximum
  likelihood on random-walk samples, used as an independence proposal
  x' = F(z); the exact likelihood stays the judge, and a chain whose flow
  acceptance over the last window falls below a threshold falls back to
  random-walk proposals until its rate recovers.

Sampler coordinates are x_i = logit(u_i), u_i the position of parameter i in
a uniform prior box (see gw_mcmc_to_theta).  Host code here only orchestrates
calls and keeps statistics; the arithmetic runs on the GPU.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np

from . import (Flow, Workspace, chain_normals, lnl_batch, mcmc_accept, mcmc_rw_propose, mcmc_to_theta,
               mcmc_update_mode)

# Philox streams used by the sampler (the kernels use 1 for random-walk
# normals and 2 for acceptance uniforms).
STREAM_FLOW = 3

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


def _evaluate(problem: Problem, x, buf: _Buffers, ws: Workspace):
    """lnL and log prior of rows x into buf.lnl, buf.lp."""
    mcmc_to_theta(problem.box_lo, problem.box_hi, x, theta_out=buf.theta, logprior_out=buf.lp)
    lnl_batch(problem.grid, problem.tensors, problem.vertices, problem.data, problem.psd, buf.theta, out=buf.lnl,
              workspace=ws, precision=problem.precision)


def adapted_cholesky(x: np.ndarray, floor: float = 1e-12) -> np.ndarray:
    """Cholesky factor of (2.38^2 / d) Cov(x) over the chains (Haario et al. 2001
    scaling), with a small diagonal floor."""
    d = x.shape[1]
    cov = np.cov(x, rowvar=False) * (2.38 ** 2 / d)
    cov += np.eye(d) * floor * max(1.0, float(np.trace(cov)) / d)
    return np.linalg.cholesky(cov)


@dataclasses.dataclass
class ChainState:
    x: object        # torch [n, dim]
    lnp: object      # torch [n]: lnL + log prior at x
    logq: object     # torch [n]: flow log density at x (flow runs)
    step: int = 0


def init_chains(problem: Problem, x0: np.ndarray, ws: Workspace) -> ChainState:
    import torch
    dev = problem.data.device
    x = torch.from_numpy(np.ascontiguousarray(x0, dtype=np.float64)).to(dev)
    buf = _Buffers(torch, x.shape[0], problem.dim, dev, problem.theta_cols)
    _evaluate(problem, x, buf, ws)
    lnp = (buf.lnl + buf.lp).contiguous()
    return ChainState(x, lnp, torch.zeros_like(lnp), 0)


def run_random_walk(problem: Problem, state: ChainState, n_steps: int, seed: int, chol: np.ndarray, ws: Workspace,
                    adapt_every: int = 0, record_every: int = 0, record_track: int | None = None,
                    collect_every: int = 0, target_accept: float = 0.234):
    """n_steps random-walk MH steps on every chain.  With adapt_every > 0 the
    proposal is re-fitted that often: the Cholesky factor of (2.38^2/d) times
    the chains' sample covariance, times a global scale that a Robbins-Monro
    step moves toward the acceptance rate target_accept over the last window
    (0.234, the optimum of Roberts, Gelman & Gilks 1997, by default).
    Records the first record_track chains every record_every steps and
    collects all chains every collect_every steps.  Returns (records
    [n_records, track, dim] or None, acceptance rate, seconds, final Cholesky
    factor, collected [n_collect * n_chains, dim] or None)."""
    import torch
    n, dim = state.x.shape
    dev = state.x.device
    buf = _Buffers(torch, n, dim, dev, problem.theta_cols)
    chol_t = torch.from_numpy(np.ascontiguousarray(chol)).to(dev)
    records, collected = [], []
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
            accepted = int(buf.total.sum().item())
            rate = (accepted - window_start) / (n * adapt_every)
            window_start = accepted
            log_scale = float(np.clip(log_scale + 2.0 * (rate - target_accept), -8.0, 2.0))
            chol = adapted_cholesky(state.x.cpu().numpy()) * math.exp(log_scale)
            chol_t = torch.from_numpy(np.ascontiguousarray(chol)).to(dev)
        if record_every and (i + 1) % record_every == 0:
            records.append(state.x[:record_track].cpu().numpy())
        if collect_every and (i + 1) % collect_every == 0:
            collected.append(state.x.cpu().numpy())
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    rate = float(buf.total.sum().item()) / (n * max(n_steps, 1))
    return ((np.stack(records) if records else None), rate, seconds, chol,
            (np.concatenate(collected) if collected else None))


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


def train_flow(samples: np.ndarray, n_layers: int = 8, hidden: int = 256, steps: int = 2000, batch: int = 4096,
               lr: float = 1e-3, seed: int = 0, device: int = 0, log_every: int = 0):
    """Fit a flow to samples [n, dim] by maximum likelihood (Adam on minibatches
    of a seeded shuffle).  Returns (flow, loss history, seconds)."""
    import torch
    dim = samples.shape[1]
    flow = Flow(dim, default_masks(dim, n_layers, seed), hidden=hidden, device=device)
    mu = samples.mean(axis=0)
    sd = samples.std(axis=0) + 1e-12
    flow.set_params(init_flow_params(dim, hidden, n_layers, seed), mu, np.log(sd))
    rng = np.random.default_rng(seed + 1)
    dev = torch.device("cuda", device)
    data = torch.from_numpy(np.ascontiguousarray(samples[rng.permutation(len(samples))])).to(dev)
    n = data.shape[0]
    batch = min(batch, n)
    per_epoch = max(1, n // batch)
    loss_t = torch.empty(1, dtype=torch.float64, device=dev)
    history = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        j = s % per_epoch
        if j == 0 and s > 0:
            data = data[torch.from_numpy(rng.permutation(n)).to(dev)].contiguous()
        flow.train_step(data[j * batch:(j + 1) * batch], lr, loss_out=loss_t)
        if log_every and (s % log_every == 0 or s == steps - 1):
            history.append((s, float(loss_t.item())))
    torch.cuda.synchronize()
    return flow, history, time.perf_counter() - t0


def run_flow_mh(problem: Problem, state: ChainState, flow: Flow, n_steps: int, seed: int, chol: np.ndarray,
                ws: Workspace, window: int = 64, threshold: float = 0.05, record_every: int = 0,
                record_track: int | None = None):
    """Independence MH with flow proposals (random-walk fallback per chain).
    Returns (records or None, acceptance rate, seconds, fraction of chain-steps
    in fallback mode)."""
    import torch
    n, dim = state.x.shape
    dev = state.x.device
    buf = _Buffers(torch, n, dim, dev, problem.theta_cols)
    chol_t = torch.from_numpy(np.ascontiguousarray(chol)).to(dev)
    mode = torch.zeros(n, dtype=torch.int32, device=dev)
    flow.inverse(state.x, z_out=buf.z, logq_out=state.logq)
    records, fallback = [], 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n_steps):
        step = state.step
        chain_normals(dim, n, seed, STREAM_FLOW, step, out=buf.z)
        flow.forward(buf.z, x_out=buf.x_prop, logq_out=buf.logq_prop)
        mcmc_rw_propose(state.x, chol_t, seed, step, buf.x_prop, mode=mode)
        _evaluate(problem, buf.x_prop, buf, ws)
        mcmc_accept(seed, step, state.x, state.lnp, buf.x_prop, buf.lnl, buf.lp, logq=state.logq,
                    logq_prop=buf.logq_prop, mode=mode, window_accepts=buf.window, total_accepts=buf.total)
        state.step += 1
        if (i + 1) % window == 0:
            mcmc_update_mode(buf.window, window, threshold, mode)
            flow.inverse(state.x, z_out=buf.z, logq_out=state.logq)     # refresh after random-walk moves
            fallback += int(mode.sum().item()) * window
        if record_every and (i + 1) % record_every == 0:
            records.append(state.x[:record_track].cpu().numpy())
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    rate = float(buf.total.sum().item()) / (n * max(n_steps, 1))
    return (np.stack(records) if records else None), rate, seconds, fallback / max(n * n_steps, 1)
