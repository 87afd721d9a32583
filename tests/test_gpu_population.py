"""GPU parity of gw_pop_lnl (Eq. (poplike), Sec. IV) against the population
oracle.  Bar: |dlnL| <= 1e-10 max(1, |lnL|) for every hyper-parameter point
(FP64 throughout; the per-event sums of up to 1e4 weights and their logs are
the only differences in rounding).  Domain rules are compared exactly."""
import numpy as np
import pytest

import synth
from oracle import population as pop

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def gw():
    import torch
    import paper_1904_02863_amd as gw
    assert torch.cuda.is_available(), "these tests need the GPU"
    gw.load_library()
    return gw


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(torch.device("cuda", 0))


def _hyper(rng, k):
    """k hyper-parameter points spread over the ranges population studies use."""
    h = np.empty((k, 12))
    h[:, 0] = rng.uniform(-2.0, 4.0, k)       # alpha
    h[:, 1] = rng.uniform(-2.0, 4.0, k)       # beta
    h[:, 2] = rng.uniform(2.0, 10.0, k)       # m_min
    h[:, 3] = rng.uniform(40.0, 100.0, k)     # m_max
    h[:, 4] = rng.uniform(0.0, 1.0, k)        # lam
    h[:, 5] = rng.uniform(20.0, 50.0, k)      # mu_m
    h[:, 6] = rng.uniform(1.0, 10.0, k)       # sigma_m
    h[:, 7] = rng.uniform(0.5, 5.0, k)        # alpha_chi
    h[:, 8] = rng.uniform(0.5, 5.0, k)        # beta_chi
    h[:, 9] = rng.uniform(0.0, 1.0, k)        # xi
    h[:, 10] = rng.uniform(0.1, 4.0, k)       # sigma_1
    h[:, 11] = rng.uniform(0.1, 4.0, k)       # sigma_2
    return h


def _check(got, ref, label):
    both_inf = np.isneginf(got) & np.isneginf(ref)
    both_nan = np.isnan(got) & np.isnan(ref)
    fin = ~(both_inf | both_nan)
    assert np.isfinite(got[fin]).all() and np.isfinite(ref[fin]).all(), f"{label}: special values differ"
    err = np.abs(got[fin] - ref[fin])
    bound = TOL * np.maximum(1.0, np.abs(ref[fin]))
    print(f"{label}: max |dlnL| {err.max() if err.size else 0:.3e}", flush=True)
    assert (err <= bound).all(), f"{label}: {got[fin][err > bound]} vs {ref[fin][err > bound]}"


@pytest.mark.parametrize("n_events,n_per", [(1, 1), (3, 1000), (2, 1500), (5, 1024), (7, 3001)])
def test_small_batches_match_oracle(gw, n_events, n_per):
    import torch
    s = synth.population_samples(n_events, n_per, index=60 + n_events)
    h = _hyper(np.random.default_rng(n_per), 24)
    got = gw.pop_lnl(_dev(s), _dev(h))
    torch.cuda.synchronize()
    _check(got.cpu().numpy(), pop.lnl(s, h), f"{n_events} x {n_per}")


def test_special_points_and_domain(gw):
    import torch
    s = synth.population_samples(4, 700, index=70)
    base = np.array([2.3, 1.2, 4.0, 90.0, 0.15, 33.0, 4.0, 2.0, 5.0, 0.6, 0.5, 0.9])
    rows = []
    for idx, val in [(0, 1.0), (1, -1.0), (4, 0.0), (4, 1.0), (9, 0.0), (9, 1.0), (7, 1.0), (8, 1.0)]:
        r = base.copy()
        r[idx] = val
        rows.append(r)
    bad = [(2, 200.0), (6, 0.0), (4, -0.1), (9, 1.5), (7, 0.0), (10, -1.0), (2, -1.0)]
    for idx, val in bad:
        r = base.copy()
        r[idx] = val
        rows.append(r)
    r = base.copy()
    r[5] = np.nan
    rows.append(r)
    r = base.copy()
    r[3] = np.inf
    rows.append(r)
    h = np.array(rows)
    got = gw.pop_lnl(_dev(s), _dev(h))
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    ref = pop.lnl(s, h)
    assert np.isfinite(ref[:8]).all() and np.isneginf(ref[8:15]).all() and np.isnan(ref[15:]).all()
    _check(got, ref, "special points")


def test_event_with_no_support(gw):
    import torch
    s = synth.population_samples(3, 500, index=71)
    s[0, 1] = 150.0                 # every m1 of event 1 above any m_max used here
    h = _hyper(np.random.default_rng(4), 5)
    got = gw.pop_lnl(_dev(s), _dev(h)).cpu().numpy()
    torch.cuda.synchronize()
    assert np.isneginf(got).all() and np.isneginf(pop.lnl(s, h)).all()


def test_deterministic(gw):
    import torch
    s = _dev(synth.population_samples(6, 5000, index=72))
    h = _dev(_hyper(np.random.default_rng(5), 16))
    a = gw.pop_lnl(s, h).cpu().numpy()
    b = gw.pop_lnl(s, h).cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(a, b)


def test_benchmark_size_sampled(gw):
    """The benchmark's batch: 200 events x 20,000 samples (4e6 samples, where
    the paper's GPU saturates), 64 hyper-parameter points per call; three
    points against the oracle."""
    import torch
    s = synth.population_samples(200, 20000)
    h = np.empty((64, 12))
    h[:] = [2.3, 1.2, 6.0, 70.0, 0.15, 33.0, 4.0, 2.0, 5.0, 0.6, 0.5, 0.9]
    h *= np.random.default_rng(7).uniform(0.9, 1.1, h.shape)
    h[:, [4, 9]] = np.clip(h[:, [4, 9]], 0.0, 1.0)
    got = gw.pop_lnl(_dev(s), _dev(h))
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert np.isfinite(got).all()
    pick = [0, 31, 63]
    _check(got[pick], pop.lnl(s, h[pick]), "4e6 samples")


@pytest.mark.parametrize("n_events,n_per", [(1, 1), (3, 1000), (7, 3001), (200, 20000)])
def test_prepared_samples_give_identical_results(gw, n_events, n_per):
    """gw_pop_prepare + gw_pop_lnl_prepared equal gw_pop_lnl bit for bit (the
    prepared fields are the very values the raw path computes), including
    samples outside the supports and events without support."""
    import torch
    s = synth.population_samples(n_events, n_per, index=80 + n_events)
    if n_per > 1:
        s[1, 0, 0] = 1.5            # q > 1: outside the support
        s[2, 0, 1] = -0.2           # a1 < 0
        s[6, 0, 2] = np.inf         # non-finite prior density
    if n_events > 2:
        s[0, 2] = 150.0             # event 2: no support at all
    h = _hyper(np.random.default_rng(n_per + 1), 32)
    st = _dev(s)
    prep = gw.pop_prepare(st)
    assert tuple(prep.shape) == (8, n_events, n_per)
    a = gw.pop_lnl(st, _dev(h))
    b = gw.pop_lnl(prep, _dev(h))
    torch.cuda.synchronize()
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert np.array_equal(a, b, equal_nan=True)
    if n_events * n_per <= 30000:
        _check(b, pop.lnl(s, h), f"prepared {n_events} x {n_per}")
