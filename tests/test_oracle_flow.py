"""Pins of the FP64 flow oracle: inverse(forward(z)) = z, the same log q from
both directions, log |det dx/dz| from a brute-force finite-difference
Jacobian, and autograd gradients against central finite differences."""
import math

import numpy as np
import pytest
import torch

from oracle.flow import OracleFlow, init_params

DIM, HID = 11, 32
MASKS = [0b00000111111, 0b11111000000, 0b10101010101, 0b01010101010]


@pytest.fixture(scope="module")
def flow():
    p = init_params(DIM, HID, len(MASKS), seed=3, scale_last=0.3)
    rng = np.random.default_rng(0)
    return OracleFlow(DIM, MASKS, HID, p, rng.normal(size=DIM), rng.normal(size=DIM) * 0.3)


def test_inverse_of_forward(flow):
    z = torch.tensor(np.random.default_rng(1).standard_normal((64, DIM)))
    x, lq_f = flow.forward(z)
    z2, lq_i = flow.inverse(x)
    np.testing.assert_allclose(z2.detach().numpy(), z.numpy(), atol=1e-12)
    np.testing.assert_allclose(lq_i.detach().numpy(), lq_f.detach().numpy(), rtol=1e-12)


def test_logdet_matches_finite_difference_jacobian(flow):
    rng = np.random.default_rng(2)
    for _ in range(3):
        z0 = rng.standard_normal(DIM)
        h = 1e-6
        jac = np.empty((DIM, DIM))
        for j in range(DIM):
            zp, zm = z0.copy(), z0.copy()
            zp[j] += h
            zm[j] -= h
            xp = flow.forward(torch.tensor(zp[None]))[0].detach().numpy()[0]
            xm = flow.forward(torch.tensor(zm[None]))[0].detach().numpy()[0]
            jac[:, j] = (xp - xm) / (2 * h)
        logdet = np.linalg.slogdet(jac)[1]
        x, lq = flow.forward(torch.tensor(z0[None]))
        lognz = -0.5 * float(z0 @ z0) - 0.5 * DIM * math.log(2 * math.pi)
        # log q(x) = log N(z) - log |det dx/dz|
        assert float(lq[0]) == pytest.approx(lognz - logdet, abs=1e-6)


def test_gradients_match_central_differences():
    p = init_params(DIM, HID, 2, seed=5, scale_last=0.5)
    masks = MASKS[:2]
    rng = np.random.default_rng(3)
    mu, ls = rng.normal(size=DIM) * 0.1, rng.normal(size=DIM) * 0.1
    x = rng.standard_normal((16, DIM))
    g, loss = OracleFlow(DIM, masks, HID, p, mu, ls).gradients(x)
    for idx in rng.choice(p.size, 12, replace=False):
        h = 1e-5
        pp, pm = p.astype(np.float64).copy(), p.astype(np.float64).copy()
        pp[idx] += h
        pm[idx] -= h
        lp = float(OracleFlow(DIM, masks, HID, pp, mu, ls).loss(x))
        lm = float(OracleFlow(DIM, masks, HID, pm, mu, ls).loss(x))
        assert g[idx] == pytest.approx((lp - lm) / (2 * h), rel=1e-5, abs=1e-8)


def test_identity_initialisation_is_standard_normal():
    p = init_params(DIM, HID, 3, seed=1, scale_last=0.0)
    f = OracleFlow(DIM, MASKS[:3], HID, p, np.zeros(DIM), np.zeros(DIM))
    z = torch.tensor(np.random.default_rng(4).standard_normal((10, DIM)))
    x, lq = f.forward(z)
    np.testing.assert_allclose(x.detach().numpy(), z.numpy(), atol=0)
    ref = -0.5 * (z * z).sum(1) - 0.5 * DIM * math.log(2 * math.pi)
    np.testing.assert_allclose(lq.detach().numpy(), ref.numpy(), rtol=1e-15)


# ---------------------------------------------------------------- BF16 error model
# The GPU flow runs its matrix products on BF16 operands.  Its results are
# compared with the float64 oracle element by element within
# rounding_tolerance(sigma), sigma the spread of the oracle under random
# rounding at the BF16 operand points.  These tests show that the bound admits
# a real BF16 computation and rejects plausible mistakes.

def _tolerance_case(n=512, hid=64, layers=4, runs=24):
    from oracle.flow import parameter_groups, rounding_spread, rounding_tolerance
    p = init_params(DIM, hid, layers, seed=7, scale_last=0.5)
    rng = np.random.default_rng(8)
    mu, ls = rng.normal(size=DIM), rng.normal(size=DIM) * 0.3
    x = rng.standard_normal((n, DIM)) * 1.3 + 0.2
    masks = MASKS[:layers]

    def make(rounding, cls=OracleFlow):
        return cls(DIM, masks, hid, p, mu, ls, rounding=rounding)

    exact, sigma = rounding_spread(make, lambda f: f.gradients(x)[0], runs=runs, seed=1)
    tol = rounding_tolerance(sigma, parameter_groups(DIM, hid, layers))
    return make, x, exact, sigma, tol, parameter_groups(DIM, hid, layers)


@pytest.fixture(scope="module")
def tolerance_case():
    return _tolerance_case()


def test_rounding_spread_is_at_the_bf16_scale(tolerance_case):
    _, _, exact, sigma, _, groups = tolerance_case
    nz = exact != 0
    rel = sigma[nz] / np.abs(exact[nz])
    # u = 2^-8; averaged over rows and amplified through the layers, the
    # typical relative spread sits within a couple of decades of u/sqrt(3)
    assert 1e-4 < np.median(rel) < 3e-2
    # inputs outside a layer's conditioning set never reach its MLP: their
    # first-layer weight gradients are exactly zero, with zero spread
    where = dict(groups)
    for l, m in enumerate(MASKS[:4]):
        off = np.array([(m >> i) & 1 == 0 for i in range(DIM)])
        w1 = where[f"l{l}.w1"]
        assert (exact[w1].reshape(64, DIM)[:, off] == 0).all()
        assert (sigma[w1].reshape(64, DIM)[:, off] == 0).all()


def test_round_to_nearest_bf16_is_within_tolerance(tolerance_case):
    from oracle.flow import rne_bf16
    make, x, exact, _, tol, _ = tolerance_case
    got = make(rne_bf16).gradients(x)[0]
    worst = np.max(np.abs(got - exact) / np.maximum(tol, 1e-300))
    assert worst <= 1.0, worst


class _NoLogDet(OracleFlow):
    """Planted mistake: the loss forgets the log-determinant terms."""

    def loss(self, x):
        z, _ = self.inverse(x)
        return 0.5 * (z * z).sum(1).mean()


class _ShiftSign(OracleFlow):
    """Planted mistake: the inverse coupling adds the shift t."""

    def inverse(self, x):
        x = torch.as_tensor(x, dtype=torch.float64)
        a = (x - self.mu) * torch.exp(-self.log_sigma)
        sum_s = self.log_sigma.sum() * torch.ones(x.shape[0], dtype=torch.float64)
        for l in reversed(range(len(self.params))):
            r, t = self._mlp(l, a)
            keep = self.masks[l]
            s = 3.0 * torch.tanh(r / 3.0) * (1 - keep)
            a = keep * a + (1 - keep) * ((a + t) * torch.exp(-s))
            sum_s = sum_s + s.sum(1)
        return a, self._logq(a, sum_s)


class _ScaleSign(OracleFlow):
    """Planted mistake: the inverse coupling multiplies by exp(+s)."""

    def inverse(self, x):
        x = torch.as_tensor(x, dtype=torch.float64)
        a = (x - self.mu) * torch.exp(-self.log_sigma)
        sum_s = self.log_sigma.sum() * torch.ones(x.shape[0], dtype=torch.float64)
        for l in reversed(range(len(self.params))):
            r, t = self._mlp(l, a)
            keep = self.masks[l]
            s = 3.0 * torch.tanh(r / 3.0) * (1 - keep)
            a = keep * a + (1 - keep) * ((a - t) * torch.exp(s))
            sum_s = sum_s + s.sum(1)
        return a, self._logq(a, sum_s)


def test_tolerance_rejects_planted_mistakes(tolerance_case):
    make, x, exact, _, tol, groups = tolerance_case
    bad = lambda g: bool((np.abs(g - exact) > tol).any())
    where = dict(groups)
    # a bias gradient 25% off in one layer (BF16 operands alone move these
    # elements by about 1.5%), a weight gradient transposed
    g = exact.copy()
    g[where["l1.b1"]] *= 1.25
    assert bad(g)
    g = exact.copy()
    w2 = g[where["l2.w2"]].reshape(64, 64)
    g[where["l2.w2"]] = w2.T.ravel()
    assert bad(g)
    # a layer's output-bias gradient lost
    g = exact.copy()
    g[where["l3.b3"]] = 0.0
    assert bad(g)
    # mistakes in the model itself, each run through the same rounding
    for cls in (_NoLogDet, _ShiftSign, _ScaleSign):
        assert bad(make(None, cls).gradients(x)[0]), cls.__name__
