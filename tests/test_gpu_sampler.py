"""GPU parity of the sampler pieces: Philox random numbers (bit-exact), the
coordinate map, random-walk proposals and Metropolis-Hastings decisions
(against numpy recomputations with the oracle's numbers), the BF16
matrix-core flow (against the FP64 flow oracle), its gradients, and MH with
flow proposals on an analytic target."""
import math

import numpy as np
import pytest
import torch
from scipy import stats

from oracle import philox
from oracle.flow import OracleFlow

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module")
def gw():
    import paper_1904_02863_amd as gw
    assert torch.cuda.is_available(), "these tests need the GPU"
    gw.load_library()
    return gw


def test_philox_known_answers_through_gpu_counter_layout(gw):
    # counter (index lo, index hi, step, stream), key (seed lo, seed hi)
    a = gw.philox_raw(0, 0, 0, 1)[0]
    assert tuple(int(v) for v in a) == (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)
    ones = gw.philox_raw(2 ** 64 - 1, 0xffffffff, 0xffffffff, 1, first=2 ** 64 - 1)[0]
    assert tuple(int(v) for v in ones) == (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)
    seed = 0x299f31d0 << 32 | 0xa4093822
    first = 0x85a308d3 << 32 | 0x243f6a88
    out = gw.philox_raw(seed, 0x03707344, 0x13198a2e, 3, first=first - 1)
    assert tuple(int(v) for v in out[1]) == (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)


@pytest.mark.parametrize("seed,stream,step", [(1, 1, 0), (2 ** 40 + 7, 3, 12345), (99, 2, 2 ** 31 + 5)])
def test_philox_blocks_bit_exact(gw, seed, stream, step):
    got = gw.philox_raw(seed, stream, step, 1000)
    for i in (0, 1, 17, 999):
        assert tuple(int(v) for v in got[i]) == philox.block(seed, stream, step, i)
    u = gw.philox_fill(seed, stream, step, 2001, normal=False).cpu().numpy()
    np.testing.assert_array_equal(u, philox.fill(seed, stream, step, 2001, normal=False))
    z = gw.philox_fill(seed, stream, step, 2001, normal=True).cpu().numpy()
    np.testing.assert_allclose(z, philox.fill(seed, stream, step, 2001, normal=True), rtol=1e-13, atol=1e-13)
    zc = gw.chain_normals(11, 37, seed, stream, step).cpu().numpy()
    np.testing.assert_allclose(zc, philox.chain_normals(11, 37, seed, stream, step), rtol=1e-13, atol=1e-13)


BOX_LO = np.array([25.0, 0.5, 100.0, 0.0, -0.1, 0.0, -1.0, 0.0, -1.0, -1.0, -1.0])
BOX_HI = np.array([35.0, 1.0, 2000.0, 2 * math.pi, 0.1, 2 * math.pi, 1.0, math.pi, 1.0, 1.0, 1.0])


def test_coordinates_to_theta(gw):
    rng = np.random.default_rng(0)
    x = rng.normal(scale=3.0, size=(300, 11))
    x[0] = 40.0
    x[1] = -40.0
    th, lp = gw.mcmc_to_theta(BOX_LO, BOX_HI, torch.from_numpy(x).to(DEV))
    u = 1 / (1 + np.exp(-x))
    p = BOX_LO + (BOX_HI - BOX_LO) * u
    ref = np.stack([p[:, 0], p[:, 1], p[:, 2], p[:, 3], p[:, 4], p[:, 5], np.arcsin(p[:, 6]), p[:, 7],
                    np.arccos(p[:, 8])], 1)
    np.testing.assert_allclose(th.cpu().numpy(), ref, rtol=1e-13, atol=1e-12)
    lp_ref = np.sum(-np.abs(x) - 2 * np.log1p(np.exp(-np.abs(x))), 1)
    np.testing.assert_allclose(lp.cpu().numpy(), lp_ref, rtol=1e-13)


def test_coordinates_to_theta_with_spins(gw):
    rng = np.random.default_rng(5)
    x = rng.normal(scale=3.0, size=(200, 11))
    lo, hi = BOX_LO.copy(), BOX_HI.copy()
    lo[9:], hi[9:] = [-0.9, -0.5], [0.8, 1.0]
    th9, _ = gw.mcmc_to_theta(lo, hi, torch.from_numpy(x).to(DEV))
    th11, lp = gw.mcmc_to_theta(lo, hi, torch.from_numpy(x).to(DEV), theta_cols=11)
    u = 1 / (1 + np.exp(-x))
    p = lo + (hi - lo) * u
    assert th11.shape == (200, 11)
    assert torch.equal(th11[:, :9], th9)
    np.testing.assert_allclose(th11[:, 9:].cpu().numpy(), p[:, 9:], rtol=1e-13, atol=1e-13)
    bad = hi.copy()
    bad[10] = 1.5
    with pytest.raises(gw.GwError):
        gw.mcmc_to_theta(lo, bad, torch.from_numpy(x).to(DEV), theta_cols=11)
    with pytest.raises(gw.GwError):
        gw.mcmc_to_theta(lo[:9], hi[:9], torch.from_numpy(x[:, :9].copy()).to(DEV), theta_cols=11)


def test_random_walk_proposal_and_acceptance(gw):
    rng = np.random.default_rng(1)
    n, d = 513, 11
    x = rng.normal(size=(n, d))
    a = rng.normal(size=(d, d)) * 0.1
    chol = np.linalg.cholesky(a @ a.T + np.eye(d) * 0.01)
    seed, step = 777, 41
    xt = torch.from_numpy(x.copy()).to(DEV)
    xp = torch.empty_like(xt)
    gw.mcmc_rw_propose(xt, torch.from_numpy(chol).to(DEV), seed, step, xp)
    z = philox.chain_normals(d, n, seed, 1, step)
    np.testing.assert_allclose(xp.cpu().numpy(), x + z @ chol.T, rtol=1e-13, atol=1e-13)
    # acceptance with given targets, in both modes
    lnp = rng.normal(size=n)
    lnl = lnp + rng.normal(size=n)
    lp = rng.normal(scale=0.1, size=n)
    logq = rng.normal(size=n)
    logq_p = rng.normal(size=n)
    mode = (rng.uniform(size=n) < 0.5).astype(np.int32)
    t = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to(DEV)
    lnp_t, logq_t, mode_t = t(lnp.copy()), t(logq.copy()), t(mode)
    total = torch.zeros(n, dtype=torch.int32, device=DEV)
    gw.mcmc_accept(seed, step, xt, lnp_t, xp, t(lnl), t(lp), logq=logq_t, logq_prop=t(logq_p), mode=mode_t,
                   total_accepts=total)
    u = np.array([philox.uniform_pair(philox.block(seed, 2, step, c))[0] for c in range(n)])
    log_alpha = (lnl + lp) - lnp + np.where(mode == 0, logq - logq_p, 0.0)
    ok = np.log(u) < log_alpha
    np.testing.assert_array_equal(total.cpu().numpy(), ok.astype(np.int32))
    np.testing.assert_array_equal(xt.cpu().numpy(), np.where(ok[:, None], xp.cpu().numpy(), x))
    np.testing.assert_allclose(lnp_t.cpu().numpy(), np.where(ok, lnl + lp, lnp))
    np.testing.assert_allclose(logq_t.cpu().numpy(), np.where(ok & (mode == 0), logq_p, logq))


def test_moments_and_adapted_cholesky(gw):
    rng = np.random.default_rng(21)
    n, d = 4097, 11
    a = rng.normal(size=(d, d))
    x = rng.normal(size=(n, d)) @ a.T + rng.normal(size=d) * 3
    xt = torch.from_numpy(x).to(DEV)
    mean, cov = gw.mcmc_moments(xt)
    np.testing.assert_allclose(mean.cpu().numpy(), x.mean(0), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(cov.cpu().numpy(), np.cov(x, rowvar=False), rtol=1e-11, atol=1e-12)
    chol = gw.mcmc_adapt_chol(xt, scale=0.7, floor=1e-9).cpu().numpy()
    c = np.cov(x, rowvar=False) * (2.38 ** 2 / d) * 0.49
    c += np.eye(d) * 1e-9 * max(1.0, np.trace(c) / d)
    np.testing.assert_allclose(chol, np.linalg.cholesky(c), rtol=1e-10, atol=1e-13)
    assert (np.triu(chol, 1) == 0).all()
    # identical rows: zero covariance, so the factor is sqrt(eps) I with eps = floor
    flat = gw.mcmc_adapt_chol(torch.ones((10, d), dtype=torch.float64, device=DEV), floor=1e-6).cpu().numpy()
    np.testing.assert_allclose(flat, np.eye(d) * 1e-3, rtol=1e-15)
    with pytest.raises(gw.GwError):
        gw.mcmc_adapt_chol(xt[:1].contiguous())


def test_count_and_gather_rows(gw):
    rng = np.random.default_rng(22)
    counts = rng.integers(0, 1000, size=10001).astype(np.int32)
    assert gw.mcmc_count(torch.from_numpy(counts).to(DEV)).item() == int(counts.sum())
    src = rng.normal(size=(777, 11))
    seed, stream, step = 2 ** 40 + 3, 4, 12
    got = gw.gather_rows(torch.from_numpy(src).to(DEV), 1001, seed, stream, step).cpu().numpy()
    u = philox.fill(seed, stream, step, 1001, normal=False)
    idx = np.minimum((u * 777).astype(np.int64), 776)
    np.testing.assert_array_equal(got, src[idx])
    # every source row is reachable and none outside: draws cover the set
    many = gw.gather_rows(torch.from_numpy(src).to(DEV), 200000, seed, stream, step + 1).cpu().numpy()
    assert len(np.unique(many[:, 0])) == 777


def _flow_pair(gw, dim=11, hidden=256, layers=8, scale_last=0.3, seed=3):
    from paper_1904_02863_amd import sampler
    masks = sampler.default_masks(dim, layers, seed)
    p = sampler.init_flow_params(dim, hidden, layers, seed, scale_last)
    rng = np.random.default_rng(seed)
    mu, ls = rng.normal(size=dim), rng.normal(size=dim) * 0.3
    f = gw.Flow(dim, masks, hidden=hidden)
    f.set_params(p, mu, ls)
    return f, (dim, masks, hidden, p, mu, ls)


def _check_within_rounding(name, got, exact, tol):
    """Element by element: |got - exact| <= tol (+ the FP32 rounding of
    results that come back in single precision)."""
    err = np.abs(got - exact)
    bound = tol + 2.0 ** -22 * np.abs(exact)
    ratio = err / np.maximum(bound, 1e-300)
    worst = int(np.argmax(ratio))
    print(f"{name}: worst |err|/bound {ratio[worst]:.3f} at {worst} (err {err[worst]:.3e}, "
          f"exact {exact[worst]:.3e}), median {np.median(ratio):.3f}")
    assert (err <= bound).all(), f"{name}: {(err > bound).sum()} elements outside the BF16 rounding bound"


def test_flow_matches_oracle(gw):
    """Forward pass against the float64 oracle, element by element, within the
    spread that BF16 operands produce under the oracle's random-rounding model."""
    from oracle.flow import rounding_spread, rounding_tolerance
    f, args = _flow_pair(gw)
    n = 1000
    z = np.random.default_rng(5).standard_normal((n, 11))
    x, lq = f.forward(torch.from_numpy(z).to(DEV))
    x, lq = x.cpu().numpy(), lq.cpu().numpy()
    # in place (x_out = z): the same values
    zz = torch.from_numpy(z).to(DEV)
    xi, lqi = f.forward(zz, x_out=zz)
    np.testing.assert_array_equal(xi.cpu().numpy(), x)
    np.testing.assert_array_equal(lqi.cpu().numpy(), lq)

    def evaluate(flow):
        ex, elq = flow.forward(torch.tensor(z))
        return np.concatenate([ex.detach().numpy().ravel(), elq.detach().numpy()])

    exact, sigma = rounding_spread(lambda r: OracleFlow(*args, rounding=r), evaluate, runs=24, seed=11)
    tol = rounding_tolerance(sigma, [("x", slice(0, 11 * n)), ("logq", slice(11 * n, 12 * n))])
    _check_within_rounding("x", x.ravel(), exact[:11 * n], tol[:11 * n])
    _check_within_rounding("log q", lq, exact[11 * n:], tol[11 * n:])
    # inverse of forward on the GPU: the same BF16 inputs in both directions
    z2, lq2 = f.inverse(torch.from_numpy(x).to(DEV))
    np.testing.assert_allclose(z2.cpu().numpy(), z, atol=1e-9)
    np.testing.assert_allclose(lq2.cpu().numpy(), lq, atol=1e-9)


@pytest.mark.parametrize("n", [4096, 1000])
def test_flow_gradients_match_oracle(gw, n):
    """Every weight and bias gradient of the 8-layer 11 -> 256 -> 256 -> 22
    flow against the float64 oracle's autograd gradient, element by element,
    within the BF16 rounding bound (grouped per layer and per matrix or bias
    vector); the loss likewise.  Batches of 4096 rows (16 split-K slices of
    256) and 1000 (3 slices of 352, two K chunks each, ragged row blocks).
    Smaller batches are left to the next test: there one row's share of a
    gradient (1/n) reaches the bound, and a ReLU whose pre-activation sits at
    zero can fall on either side under different roundings."""
    from oracle.flow import parameter_groups, rounding_spread, rounding_tolerance
    f, args = _flow_pair(gw, scale_last=0.5)
    x = np.random.default_rng(6).standard_normal((n, 11)) * 1.3 + 0.2
    g, loss = f.gradients(torch.from_numpy(x).to(DEV))
    g = g.cpu().numpy().astype(np.float64)

    def evaluate(flow):
        grad, l = flow.gradients(x)
        return np.concatenate([grad, [l]])

    exact, sigma = rounding_spread(lambda r: OracleFlow(*args, rounding=r), evaluate, runs=24, seed=12)
    groups = parameter_groups(11, 256, 8)
    npar = g.size
    tol = rounding_tolerance(sigma, groups + [("loss", slice(npar, npar + 1))])
    for name, sl in groups:
        _check_within_rounding(name, g[sl], exact[sl], tol[sl])
    _check_within_rounding("loss", np.array([float(loss.item())]), exact[npar:], tol[npar:])
    # first-layer weights of inputs outside a layer's conditioning set get no gradient
    where = dict(groups)
    for l, m in enumerate(args[1]):
        off = np.array([(int(m) >> i) & 1 == 0 for i in range(11)])
        assert (g[where[f"l{l}.w1"]].reshape(256, 11)[:, off] == 0).all()


def test_flow_rows_do_not_depend_on_the_batch(gw):
    """A row's way through the couplings never involves another row: the
    forward and inverse passes of the first k rows of a batch equal, bit for
    bit, those rows of the whole batch's passes, for batches that fill part
    of one 16-row block (k = 1, 5), spill into a second (17) or end one row
    short of the whole batch (999)."""
    f, _ = _flow_pair(gw)
    z = torch.from_numpy(np.random.default_rng(9).standard_normal((1000, 11))).to(DEV)
    x, lq = f.forward(z)
    zb, lqb = f.inverse(x)
    for k in (1, 5, 17, 999):
        xk, lqk = f.forward(z[:k].contiguous())
        assert torch.equal(xk, x[:k]) and torch.equal(lqk, lq[:k]), k
        zk, lqik = f.inverse(x[:k].contiguous())
        assert torch.equal(zk, zb[:k]) and torch.equal(lqik, lqb[:k]), k


def test_flow_longer_than_one_launch(gw):
    """20 couplings of hidden width 128: a launch carries the rows through at
    most 16 couplings of a pass, so the rows cross from one launch to the
    next in both directions.  The forward pass equals bit for bit two
    10-coupling flows in a row (the first with the identity normalisation),
    whose passes each fit one launch; the forward pass and every gradient
    agree with the float64 oracle within the BF16 rounding bound, as in the
    tests above (4096 rows, as there: one row's share of a gradient, which a
    ReLU decided on the other side of zero moves, stays below the bound), and
    the inverse undoes the forward."""
    from oracle.flow import parameter_groups, rounding_spread, rounding_tolerance
    layers, hidden = 20, 128
    f, args = _flow_pair(gw, hidden=hidden, layers=layers, seed=4)
    n = 600
    z = np.random.default_rng(7).standard_normal((n, 11))
    zt = torch.from_numpy(z).to(DEV)
    x, lq = f.forward(zt)
    _, masks, _, p, mu, ls = args
    per = p.size // layers
    first = gw.Flow(11, masks[:10], hidden=hidden)
    first.set_params(p[:10 * per], np.zeros(11), np.zeros(11))
    second = gw.Flow(11, masks[10:], hidden=hidden)
    second.set_params(p[10 * per:], mu, ls)
    u, _ = first.forward(zt)
    x2, _ = second.forward(u)
    assert torch.equal(x2, x)
    x, lq = x.cpu().numpy(), lq.cpu().numpy()

    def forward(flow):
        ex, elq = flow.forward(torch.tensor(z))
        return np.concatenate([ex.detach().numpy().ravel(), elq.detach().numpy()])

    exact, sigma = rounding_spread(lambda r: OracleFlow(*args, rounding=r), forward, runs=24, seed=13)
    tol = rounding_tolerance(sigma, [("x", slice(0, 11 * n)), ("logq", slice(11 * n, 12 * n))])
    _check_within_rounding("x", x.ravel(), exact[:11 * n], tol[:11 * n])
    _check_within_rounding("log q", lq, exact[11 * n:], tol[11 * n:])
    z2, lq2 = f.inverse(torch.from_numpy(x).to(DEV))
    np.testing.assert_allclose(z2.cpu().numpy(), z, atol=1e-9)
    np.testing.assert_allclose(lq2.cpu().numpy(), lq, atol=1e-9)

    xs = np.random.default_rng(8).standard_normal((4096, 11)) * 1.3 + 0.2
    g, loss = f.gradients(torch.from_numpy(xs).to(DEV))
    g = g.cpu().numpy().astype(np.float64)

    def gradients(flow):
        grad, l = flow.gradients(xs)
        return np.concatenate([grad, [l]])

    exact, sigma = rounding_spread(lambda r: OracleFlow(*args, rounding=r), gradients, runs=24, seed=14)
    groups = parameter_groups(11, hidden, layers)
    npar = g.size
    tol = rounding_tolerance(sigma, groups + [("loss", slice(npar, npar + 1))])
    for name, sl in groups:
        _check_within_rounding(name, g[sl], exact[sl], tol[sl])
    _check_within_rounding("loss", np.array([float(loss.item())]), exact[npar:], tol[npar:])


def test_flow_gradients_of_repeated_rows(gw):
    """The loss is a mean over rows, so a batch and the same batch twice have
    the same gradient.  300 rows (one K slice, ragged row blocks of 64 and
    256) against 600 (two slices): every element within FP32 rounding of
    sums of that length."""
    from oracle.flow import parameter_groups
    f, _ = _flow_pair(gw, scale_last=0.5)
    x = np.random.default_rng(8).standard_normal((300, 11)) * 1.3 + 0.2
    g1, l1 = f.gradients(torch.from_numpy(x).to(DEV))
    g2, l2 = f.gradients(torch.from_numpy(np.vstack([x, x])).to(DEV))
    g1, g2 = g1.cpu().numpy().astype(np.float64), g2.cpu().numpy().astype(np.float64)
    assert float(l1.item()) == pytest.approx(float(l2.item()), rel=1e-12)
    for name, sl in parameter_groups(11, 256, 8):
        a, b = g1[sl], g2[sl]
        bound = 1e-5 * np.abs(a).max() + 1e-6 * np.abs(a)
        err = np.abs(a - b)
        assert (err <= bound).all(), f"{name}: worst {err.max():.3e} (scale {np.abs(a).max():.3e})"
    assert np.abs(g1).max() > 0


def test_flow_learns_a_gaussian(gw):
    from paper_1904_02863_amd import sampler
    rng = np.random.default_rng(7)
    d = 11
    a = rng.normal(size=(d, d))
    cov = a @ a.T / d + np.eye(d) * 0.1
    mean = rng.normal(size=d) * 3
    data = rng.multivariate_normal(mean, cov, size=40000)
    flow, hist, secs = sampler.train_flow(data, n_layers=8, hidden=128, steps=600, batch=4096, lr=2e-3, seed=1,
                                          log_every=100)
    print("loss history", hist, f"{secs:.1f} s")
    entropy = 0.5 * np.linalg.slogdet(2 * math.pi * math.e * cov)[1]
    assert hist[-1][1] < hist[0][1]
    # at the optimum the loss (mean |z|^2/2 + log-det terms) is the entropy minus (d/2) log(2 pi)
    assert hist[-1][1] == pytest.approx(entropy - 0.5 * d * math.log(2 * math.pi), abs=0.3)
    z = torch.from_numpy(rng.standard_normal((40000, d))).to(DEV)
    xs, _ = flow.forward(z)
    xs = xs.cpu().numpy()
    np.testing.assert_allclose(xs.mean(0), mean, atol=0.08)
    np.testing.assert_allclose(np.cov(xs, rowvar=False), cov, atol=0.12)


def test_flow_mh_reaches_the_exact_target(gw):
    """Independence MH with a deliberately imperfect flow on a Gaussian target
    (log target computed by the test): the chains' marginals match the exact
    ones, which needs the log q terms with the right signs."""
    from paper_1904_02863_amd import sampler
    rng = np.random.default_rng(8)
    d, n = 5, 4096
    mean = np.array([1.0, -2.0, 0.5, 0.0, 3.0])
    sd = np.array([0.5, 1.0, 2.0, 0.3, 1.5])
    # flow trained on a wrong (shifted, wider) version of the target
    data = rng.normal(mean + 0.3, sd * 1.4, size=(20000, d))
    flow, _, _ = sampler.train_flow(data, n_layers=4, hidden=64, steps=300, batch=2048, lr=2e-3, seed=2)
    t = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to(DEV)
    mean_t, sd_t = t(mean), t(sd)
    x = t(rng.normal(mean, sd, size=(n, d)))
    logtarget = lambda v: (-0.5 * (((v - mean_t) / sd_t) ** 2).sum(1)).contiguous()
    lnp = logtarget(x)
    logq = torch.empty(n, dtype=torch.float64, device=DEV)
    zbuf = torch.empty_like(x)
    flow.inverse(x, z_out=zbuf, logq_out=logq)
    mode = torch.zeros(n, dtype=torch.int32, device=DEV)
    zero = torch.zeros(n, dtype=torch.float64, device=DEV)
    total = torch.zeros(n, dtype=torch.int32, device=DEV)
    xp = torch.empty_like(x)
    lqp = torch.empty(n, dtype=torch.float64, device=DEV)
    for step in range(200):
        gw.chain_normals(d, n, 11, 3, step, out=zbuf)
        flow.forward(zbuf, x_out=xp, logq_out=lqp)
        gw.mcmc_accept(11, step, x, lnp, xp, logtarget(xp), zero, logq=logq, logq_prop=lqp, mode=mode,
                       total_accepts=total)
    rate = total.sum().item() / (n * 200)
    xs = x.cpu().numpy()
    print(f"acceptance {rate:.3f}")
    assert rate > 0.2
    for j in range(d):
        p = stats.kstest(xs[:, j], stats.norm(mean[j], sd[j]).cdf).pvalue
        print(f"dim {j}: KS p = {p:.3f}")
        assert p > 1e-3
