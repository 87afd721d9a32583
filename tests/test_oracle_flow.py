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
