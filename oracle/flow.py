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


class OracleFlow:
    """bf16=True rounds the MLP inputs, weights and hidden activations to
    bfloat16 (the precision the GPU kernels declare for their matrix-core
    MLPs) and otherwise computes in float64; it is for forward comparisons
    only (no gradients through the rounding)."""

    def __init__(self, dim, cond_masks, hidden, params, mu, log_sigma, bf16=False):
        self.bf16 = bf16
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

    def _mlp(self, l, a):
        p = self.params[l]
        if self.bf16:
            q = round_bf16
            h1 = q(torch.relu(q(a * self.masks[l]) @ q(p["w1"]).T + p["b1"].detach()))
            h2 = q(torch.relu(h1 @ q(p["w2"]).T + p["b2"].detach()))
            out = h2 @ q(p["w3"]).T + p["b3"].detach()
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
