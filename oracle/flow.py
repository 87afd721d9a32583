"""FP64 reference of the affine-coupling flow -- TEST INFRASTRUCTURE (oracle side).

Plain PyTorch CPU operations in float64 (autograd supplies the gradients).
The model is the RealNVP affine coupling of Dinh, Sohl-Dickstein & Bengio
(ICLR 2017): x = mu + sigma * f_{L-1}(... f_0(z)), z ~ N(0, I); layer l keeps
the dimensions in its conditioning set and maps the others as
a -> a exp(s) + t, s = 3 tanh(r/3), (r, t) = MLP_l(m_l * a) with
MLP = Linear(D, H) ReLU Linear(H, H) ReLU Linear(H, 2D).  Parameters come
flat, per layer in the order W1 [H][D], b1 [H], W2 [H][H], b2 [H],
W3 [2D][H], b3 [2D].  log q(x) = log N(z) - sum over layers of sum s -
sum log sigma; the training loss is the mean of |z|^2/2 + sum s + sum log sigma.

Rounding models (``rounding=``).  The method fixes the MLPs at BF16 operands
with FP32 accumulation; everything else is FP64.  A matrix product in that
precision rounds each of its operands to BF16 once: the layer input, the
weights and the hidden activations on the way forward, and the gradient that
enters a product on the way back (the one of which the weight gradient and the
input gradient are both products).  Biases, bias gradients and the coupling
stay wider.  The gradient of a parameter is the one of the unrounded FP32
master value (the rounding passes gradients straight through), so only the
backward signals entering a product carry their own rounding.  A rounding
model is a callable v -> rounded v applied at exactly those points:

* ``rne_bf16`` rounds to the nearest bfloat16, ties to even;
* ``MonteCarloRounding(rng)`` multiplies by 1 + delta, delta uniform in
  [-u, u], u = 2^-8 the unit roundoff of bfloat16's 8-bit significand: the
  random-rounding model of Monte Carlo arithmetic (Parker, Pierce & Eggert,
  Comput. Sci. Eng. 2(4), 2000) under which the spread of repeated runs
  estimates the error that BF16 operands leave in each output element.
"""
from __future__ import annotations

import math

import numpy as np
import torch


def layer_sizes(dim: int, hidden: int):
    return [("w1", (hidden, dim)), ("b1", (hidden,)), ("w2", (hidden, hidden)), ("b2", (hidden,)),
            ("w3", (2 * dim, hidden)), ("b3", (2 * dim,))]


def round_bf16(t: torch.Tensor) -> torch.Tensor:
    """Round float64 values to the nearest bfloat16 (ties to even), as float64."""
    a = t.detach().numpy().astype(np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return torch.tensor(u.astype(np.uint32).view(np.float32).astype(np.float64))


BF16_UNIT_ROUNDOFF = 2.0 ** -8


def rne_bf16(t: torch.Tensor) -> torch.Tensor:
    """Rounding model: nearest bfloat16, ties to even."""
    return round_bf16(t).reshape(t.shape)


class MonteCarloRounding:
    """Rounding model: v (1 + delta), delta ~ U[-u, u] independently per
    element and per call, u = 2^-8 (bfloat16)."""

    def __init__(self, rng: np.random.Generator, u: float = BF16_UNIT_ROUNDOFF):
        self.rng, self.u = rng, u

    def __call__(self, t: torch.Tensor) -> torch.Tensor:
        d = self.rng.uniform(-self.u, self.u, tuple(t.shape))
        return t.detach() * (1.0 + torch.from_numpy(d))


class _RoundValue(torch.autograd.Function):
    """Rounds the value; the gradient passes through unchanged."""

    @staticmethod
    def forward(ctx, v, rounder):
        return rounder(v)

    @staticmethod
    def backward(ctx, g):
        return g, None


class _RoundGradient(torch.autograd.Function):
    """Leaves the value; rounds the gradient flowing back through it."""

    @staticmethod
    def forward(ctx, v, rounder):
        ctx.rounder = rounder
        return v.view_as(v)

    @staticmethod
    def backward(ctx, g):
        return ctx.rounder(g), None


class OracleFlow:
    """rounding=None computes in float64 throughout.  rounding=<model>
    applies the model at the BF16 operand points listed in the module
    docstring, forward and backward.  bf16=True is rounding=rne_bf16."""

    def __init__(self, dim, cond_masks, hidden, params, mu, log_sigma, bf16=False, rounding=None):
        self.rounding = rne_bf16 if bf16 and rounding is None else rounding
        self.dim, self.hidden = dim, hidden
        self.masks = [torch.tensor([(int(m) >> i) & 1 for i in range(dim)], dtype=torch.float64)
                      for m in cond_masks]
        flat = torch.tensor(np.asarray(params, dtype=np.float64))
        self.params = []
        off = 0
        for _ in cond_masks:
            layer = {}
            for name, shape in layer_sizes(dim, hidden):
                n = int(np.prod(shape))
                layer[name] = flat[off:off + n].reshape(shape).clone().requires_grad_(True)
                off += n
            self.params.append(layer)
        assert off == flat.numel()
        self.mu = torch.tensor(np.asarray(mu, dtype=np.float64))
        self.log_sigma = torch.tensor(np.asarray(log_sigma, dtype=np.float64))

    def _product(self, x, w):
        """x w^T with both operands and the gradient entering it rounded."""
        r = self.rounding
        prod = _RoundValue.apply(x, r) @ _RoundValue.apply(w, r).T
        return _RoundGradient.apply(prod, r)

    def _mlp(self, l, a):
        p = self.params[l]
        if self.rounding is not None:
            h1 = torch.relu(self._product(a * self.masks[l], p["w1"]) + p["b1"])
            h2 = torch.relu(self._product(h1, p["w2"]) + p["b2"])
            out = self._product(h2, p["w3"]) + p["b3"]
            return out[:, :self.dim], out[:, self.dim:]
        h1 = torch.relu((a * self.masks[l]) @ p["w1"].T + p["b1"])
        h2 = torch.relu(h1 @ p["w2"].T + p["b2"])
        out = h2 @ p["w3"].T + p["b3"]
        return out[:, :self.dim], out[:, self.dim:]

    def forward(self, z):
        """z [n, D] -> (x, log q(x))."""
        z = torch.as_tensor(z, dtype=torch.float64)
        a, sum_s = z, torch.zeros(z.shape[0], dtype=torch.float64)
        for l in range(len(self.params)):
            r, t = self._mlp(l, a)
            keep = self.masks[l]
            s = 3.0 * torch.tanh(r / 3.0) * (1 - keep)
            a = keep * a + (1 - keep) * (a * torch.exp(s) + t)
            sum_s = sum_s + s.sum(1)
        x = self.mu + torch.exp(self.log_sigma) * a
        sum_s = sum_s + self.log_sigma.sum()
        return x, self._logq(z, sum_s)

    def inverse(self, x):
        """x [n, D] -> (z, log q(x))."""
        x = torch.as_tensor(x, dtype=torch.float64)
        a = (x - self.mu) * torch.exp(-self.log_sigma)
        sum_s = self.log_sigma.sum() * torch.ones(x.shape[0], dtype=torch.float64)
        for l in reversed(range(len(self.params))):
            r, t = self._mlp(l, a)
            keep = self.masks[l]
            s = 3.0 * torch.tanh(r / 3.0) * (1 - keep)
            a = keep * a + (1 - keep) * ((a - t) * torch.exp(-s))
            sum_s = sum_s + s.sum(1)
        return a, self._logq(a, sum_s)

    def _logq(self, z, sum_s):
        return -0.5 * (z * z).sum(1) - 0.5 * self.dim * math.log(2 * math.pi) - sum_s

    def loss(self, x):
        """mean over rows of |z|^2/2 + sum s + sum log sigma."""
        z, logq = self.inverse(x)
        return (-logq).mean() - 0.5 * self.dim * math.log(2 * math.pi)

    def gradients(self, x):
        """(flat gradient in the parameter layout, loss)."""
        for layer in self.params:
            for t in layer.values():
                t.grad = None
        loss = self.loss(x)
        loss.backward()
        flat = torch.cat([layer[name].grad.reshape(-1) for layer in self.params
                          for name, _ in layer_sizes(self.dim, self.hidden)])
        return flat.detach().numpy(), float(loss.detach())


def init_params(dim: int, hidden: int, n_layers: int, seed: int, scale_last: float = 0.0) -> np.ndarray:
    """Seeded initial parameters: uniform(+-1/sqrt(fan_in)) weights and
    biases, the last layer scaled by scale_last (0 = identity flow)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_layers):
        for name, shape in layer_sizes(dim, hidden):
            fan_in = shape[1] if len(shape) == 2 else (dim if name == "b1" else hidden)
            v = rng.uniform(-1, 1, shape) / math.sqrt(fan_in)
            if name in ("w3", "b3"):
                v = v * scale_last
            out.append(v.ravel())
    return np.concatenate(out).astype(np.float32)


def parameter_groups(dim: int, hidden: int, n_layers: int):
    """[(name, slice)] over the flat parameter layout: every weight matrix
    and every bias vector of every layer, e.g. ("l3.w2", slice(...))."""
    out, off = [], 0
    for l in range(n_layers):
        for name, shape in layer_sizes(dim, hidden):
            n = int(np.prod(shape))
            out.append((f"l{l}.{name}", slice(off, off + n)))
            off += n
    return out


def rounding_spread(make_flow, evaluate, runs: int, seed: int):
    """(exact, sigma): evaluate(make_flow(None)), a float64 array, and element
    by element the root-mean-square deviation from it of `runs` evaluations
    of evaluate(make_flow(MonteCarloRounding(rng))) -- the error that BF16
    operands leave in each element under the random-rounding model."""
    exact = np.asarray(evaluate(make_flow(None)), dtype=np.float64)
    rng = np.random.default_rng(seed)
    acc = np.zeros_like(exact)
    for _ in range(runs):
        d = np.asarray(evaluate(make_flow(MonteCarloRounding(rng))), dtype=np.float64) - exact
        acc += d * d
    return exact, np.sqrt(acc / runs)


def rounding_tolerance(sigma: np.ndarray, groups, k: float = 6.0, rho: float = 0.5) -> np.ndarray:
    """Per-element bound k (sigma_i + rho sigma_G) on |result - exact|, where
    sigma_G is the root mean square of sigma over element i's group (the
    slices in `groups`; elements in none form one group).  The sigma_i term
    is the element's own rounding spread; the group term admits the rare
    large errors of a ReLU whose pre-activation sits within rounding of zero
    (an activation that turns on or off changes a whole row's contribution),
    which a finite number of random runs samples poorly."""
    sigma = np.asarray(sigma, dtype=np.float64)
    floor = np.empty_like(sigma)
    covered = np.zeros(sigma.shape, dtype=bool)
    flat_s, flat_f, flat_c = sigma.reshape(-1), floor.reshape(-1), covered.reshape(-1)
    for _, sl in groups:
        flat_f[sl] = math.sqrt(float(np.mean(flat_s[sl] ** 2))) if flat_s[sl].size else 0.0
        flat_c[sl] = True
    if not flat_c.all():
        rest = ~flat_c
        flat_f[rest] = math.sqrt(float(np.mean(flat_s[rest] ** 2)))
    return k * (sigma + rho * floor)
