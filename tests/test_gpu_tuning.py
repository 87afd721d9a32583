"""Plan autotuning of the single-event likelihood (gw_lnl_batch).

A plan splits the pass over the bins into LDS tiles and work items; the
autotuner times the candidates of a size class (the largest LDS tile and half
of it; 0, 4, 6 or 8 work-queue rounds, 0 only with the ISCO end) on the first
call of the class and keeps the fastest.  Plans differ only in where the bin
sums are cut into partial sums, so:

- FP64: every candidate plan, set explicitly with gw_workspace_set_plan, gives
  every row within 1e-12 relative of the default plan (the partial sums of
  2.6e5 bins each carry rounding near 1e-16 relative of the row's largest
  term; 1e-12 leaves room for the sums' cancellation between <d,h> and
  <h,h>), and a few rows of the tuned plan within 1e-10 of the oracle, the
  single-event parity bar.
- Mixed precision: within the mixed path's bar of 1e-3 in lnL of the default
  plan, since a tile boundary restarts the FP32 phasor rotation.
- The tuned plan is the one gw_lnl_plan reports, repeats bit for bit on its
  workspace and, set on a fresh workspace, on that one too; the tuning calls
  are not counted by the kernel timer; a captured call is never tuned.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

RTOL_PLAN = 1e-12
RTOL_ORACLE = 1e-10
TOL_MIXED = 1e-3

# (name, event factory): both above the tuner's threshold of 2^24 (sample, bin) pairs
CASES = [
    ("3 detectors x 259,585 bins x 1024 samples", lambda: synth.bbh_3det_128s(1024)),
    ("2 detectors x 100,003 bins x 700 samples", lambda: synth.small_event(41, 2, 100_003, 700, 9,
                                                                            delta_f=1.0 / 64.0)),
]


@pytest.fixture(scope="module")
def gw():
    import torch
    import paper_1904_02863_amd as gw
    assert torch.cuda.is_available(), "these tests need the GPU"
    gw.load_library()
    return gw


def _inputs(w):
    import torch
    dev = torch.device("cuda", 0)
    data = oracle.workload_data(w)
    return (torch.from_numpy(np.ascontiguousarray(data)).to(dev), torch.from_numpy(w.psd).to(dev),
            torch.from_numpy(np.ascontiguousarray(w.theta)).to(dev), data)


def _call(gw, w, inp, ws, precision, flags, out=None):
    import torch
    d, s, th, _ = inp
    r = gw.lnl_batch(w.grid, w.tensors, w.vertices, d, s, th, precision=precision, flags=flags, workspace=ws,
                     out=out)
    torch.cuda.synchronize()
    return r.cpu().numpy()


def _fixed(gw):
    ws = gw.Workspace(0)
    ws.set_tuning(False)
    return ws


def _modes(gw):
    return (("fp64", 0), ("mixed", 0), ("fp64", gw.FLAG_TERM_ISCO))


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_every_candidate_plan_agrees_with_the_default(gw, name, make):
    w = make()
    inp = _inputs(w)
    n_bins, n_det, n_samples = w.grid.n_bins, w.n_det, w.theta.shape[0]
    for precision, flags in _modes(gw):
        base_ws = _fixed(gw)
        default = base_ws.lnl_plan(n_bins, n_det, n_samples, precision, flags)
        ref = _call(gw, w, inp, base_ws, precision, flags)
        assert np.isfinite(ref).all()
        rounds = (0,) if flags & gw.FLAG_TERM_ISCO else (0, 4, 6, 8)
        for tile in (default["tile_bins"], default["tile_bins"] // 2):
            for r in rounds:
                ws = _fixed(gw)
                ws.set_plan(n_bins, n_det, n_samples, tile, r, precision, flags)
                plan = ws.lnl_plan(n_bins, n_det, n_samples, precision, flags)
                assert plan["tile_bins"] == tile and plan["rounds"] in (0, r), plan
                got = _call(gw, w, inp, ws, precision, flags)
                err = np.abs(got - ref)
                print(f"{name} {precision} flags {flags} tile {tile} rounds {r} -> {plan}: "
                      f"max |plan - default| {err.max():.3e}", flush=True)
                if precision == "mixed":
                    assert (err <= TOL_MIXED).all(), f"row {int(np.argmax(err))}"
                else:
                    worst = int(np.argmax(err / np.abs(ref)))
                    assert (err <= RTOL_PLAN * np.abs(ref)).all(), f"row {worst}: {got[worst]!r} vs {ref[worst]!r}"


def test_tuned_plan_is_reported_repeatable_and_reproducible(gw):
    w = synth.bbh_3det_128s(1024)
    inp = _inputs(w)
    g = w.grid
    n_bins, n_det, n_samples = g.n_bins, w.n_det, w.theta.shape[0]
    rows = np.array([0, 1, n_samples // 2, n_samples - 1])
    want = oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, inp[3], w.psd, w.theta[rows])
    for precision, flags in _modes(gw):
        ws = gw.Workspace(0)
        ws.set_timing(True)
        default = ws.lnl_plan(n_bins, n_det, n_samples, precision, flags)
        ref = _call(gw, w, inp, _fixed(gw), precision, flags)
        a = _call(gw, w, inp, ws, precision, flags)          # times the candidates, then runs the fastest
        tuned = ws.lnl_plan(n_bins, n_det, n_samples, precision, flags)
        print(f"{precision} flags {flags}: default {default}, tuned {tuned}", flush=True)
        _, launches = ws.kernel_time()
        assert launches == 1, "the tuning calls are not measurements of the caller's"
        b = _call(gw, w, inp, ws, precision, flags)
        np.testing.assert_array_equal(a, b)
        assert ws.lnl_plan(n_bins, n_det, n_samples, precision, flags) == tuned
        # the same plan on a fresh workspace gives the same values
        other = _fixed(gw)
        other.set_plan(n_bins, n_det, n_samples, tuned["tile_bins"], tuned["rounds"], precision, flags)
        assert other.lnl_plan(n_bins, n_det, n_samples, precision, flags) == tuned
        np.testing.assert_array_equal(_call(gw, w, inp, other, precision, flags), a)
        if precision == "mixed":
            assert np.all(np.abs(a - ref) <= TOL_MIXED)
        else:
            assert np.all(np.abs(a - ref) <= RTOL_PLAN * np.abs(ref))
            if flags == 0:
                assert np.all(np.abs(a[rows] - want) <= RTOL_ORACLE * np.abs(want))
        # forgetting the tuned plans restores the default one, and the call
        # after it is not tuned again
        ws.set_tuning(False, forget=True)
        assert ws.lnl_plan(n_bins, n_det, n_samples, precision, flags) == default
        np.testing.assert_array_equal(_call(gw, w, inp, ws, precision, flags), ref)
        assert ws.lnl_plan(n_bins, n_det, n_samples, precision, flags) == default
    with pytest.raises(gw.GwError):
        _fixed(gw).set_plan(n_bins, n_det, n_samples, 100, 0)        # not a multiple of 64
    with pytest.raises(gw.GwError):
        _fixed(gw).set_plan(n_bins, n_det, n_samples, 1 << 20, 0)    # beyond the LDS budget
    with pytest.raises(gw.GwError):
        _fixed(gw).set_plan(n_bins, n_det, n_samples, 256, 17)


def test_captured_call_is_not_tuned(gw):
    """A call first seen under stream capture runs the default plan (timing
    needs host waits, which capture forbids), and the workspace, pinned by the
    capture, is not tuned afterwards either.  Three replays, with eager calls
    on another workspace between them, equal the default plan's values."""
    import torch
    w = synth.small_event(43, 3, 60_000, 2000, 9, delta_f=1.0 / 64.0)
    d, s, th, data = _inputs(w)
    n_bins, n_det, n_samples = w.grid.n_bins, w.n_det, w.theta.shape[0]
    ref = _call(gw, w, (d, s, th, data), _fixed(gw), "fp64", 0)
    ws = gw.Workspace(0)
    ws.reserve(n_bins, n_det, n_samples)
    default = ws.lnl_plan(n_bins, n_det, n_samples)
    out = torch.empty(n_samples, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gw.lnl_batch(w.grid, w.tensors, w.vertices, d, s, th, workspace=ws, out=out)
    torch.cuda.synchronize()
    assert ws.lnl_plan(n_bins, n_det, n_samples) == default
    other = gw.Workspace(0)
    for rep in range(3):
        out.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), ref, err_msg=f"replay {rep}")
        gw.lnl_batch(w.grid, w.tensors, w.vertices, d, s, th.flip(0).contiguous(), workspace=other)
        torch.cuda.synchronize()
    # an eager call on the pinned workspace keeps the default plan too
    np.testing.assert_array_equal(_call(gw, w, (d, s, th, data), ws, "fp64", 0), ref)
    assert ws.lnl_plan(n_bins, n_det, n_samples) == default


def test_reserved_workspace_does_not_grow_while_tuning(gw):
    w = synth.small_event(44, 3, 60_000, 2000, 9, delta_f=1.0 / 64.0)
    inp = _inputs(w)
    ws = gw.Workspace(0)
    ws.reserve(w.grid.n_bins, w.n_det, w.theta.shape[0])
    before = ws.nbytes
    for precision, flags in _modes(gw):
        _call(gw, w, inp, ws, precision, flags)
    assert ws.nbytes == before
