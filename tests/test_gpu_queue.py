"""The single-event tile kernel's work-queue launch (a persistent grid over
one queue per XCD, chunks in rounds of halving size) against the CPU oracle.

The small parity cases of test_gpu_lnl.py run one block per (sample group,
chunk) item; these shapes are large enough for the queue (checked with
gw_lnl_plan before each call) and ragged in both sample count and bin count.
Bar: every row within 1e-10 relative of the oracle.  The queue hands items to
blocks in an order that changes from call to call, but each item's partial
sums are formed over fixed bins in a fixed order and added in chunk order,
so repeated calls, also on another stream, agree bit for bit.  The tests
run the default plan (plan autotuning off), whose shape they check.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-10

# (seed, n_det, n_bins, n_samples, spins)
QUEUE_CASES = [
    (31, 3, 40_001, 4000, False),
    (32, 2, 100_003, 700, False),
    (33, 1, 60_000, 2000, False),
    (34, 5, 30_011, 5000, True),
]


@pytest.fixture(scope="module")
def gw():
    import torch
    import paper_1904_02863_amd as gw
    assert torch.cuda.is_available(), "these tests need the GPU"
    gw.load_library()
    return gw


def _ws(gw):
    ws = gw.Workspace(0)
    ws.set_tuning(False)
    return ws


def _event(seed, n_det, n_bins, n_samples, spins):
    w = synth.small_event(seed, n_det, n_bins, n_samples, 9, delta_f=1.0 / 64.0)
    theta = synth.add_spins(w.theta, np.random.default_rng(seed), 0.8) if spins else w.theta
    return w, theta, oracle.workload_data(w)


def _run(gw, w, theta, data, ws, stream=None):
    import torch
    dev = torch.device("cuda", 0)
    d = torch.from_numpy(np.ascontiguousarray(data)).to(dev)
    s = torch.from_numpy(w.psd).to(dev)
    th = torch.from_numpy(np.ascontiguousarray(theta)).to(dev)
    torch.cuda.synchronize()
    if stream is None:
        out = gw.lnl_batch(w.grid, w.tensors, w.vertices, d, s, th, workspace=ws)
    else:
        with torch.cuda.stream(stream):
            out = gw.lnl_batch(w.grid, w.tensors, w.vertices, d, s, th, workspace=ws)
        stream.synchronize()
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("seed,n_det,n_bins,n_samples,spins", QUEUE_CASES)
def test_queue_launch_matches_oracle(gw, seed, n_det, n_bins, n_samples, spins):
    w, theta, data = _event(seed, n_det, n_bins, n_samples, spins)
    ws = _ws(gw)
    plan = ws.lnl_plan(n_bins, n_det, n_samples)
    print(f"seed {seed} det {n_det} bins {n_bins} S {n_samples} spins {spins}: plan {plan}", flush=True)
    assert plan["rounds"] > 0 and plan["n_chunks"] % plan["rounds"] == 0
    got = _run(gw, w, theta, data, ws)
    g = w.grid
    ref = oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data, w.psd, theta)
    err = np.abs(got - ref)
    assert np.isfinite(got).all()
    worst = int(np.argmax(err / np.abs(ref)))
    assert (err <= RTOL * np.abs(ref)).all(), f"row {worst}: {got[worst]!r} oracle {ref[worst]!r}"


def test_queue_launch_is_bitwise_repeatable(gw):
    import torch
    w, theta, data = _event(31, 3, 40_001, 4000, False)
    ws = _ws(gw)
    assert ws.lnl_plan(40_001, 3, 4000)["rounds"] > 0
    a = _run(gw, w, theta, data, ws)
    b = _run(gw, w, theta, data, ws)
    c = _run(gw, w, theta, data, _ws(gw), stream=torch.cuda.Stream())
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(a, c)


def test_plan_rules(gw):
    ws = _ws(gw)
    # small events: one block per item
    assert ws.lnl_plan(3001, 3, 300)["rounds"] == 0
    # the template end keeps one block per item (its band is known only on the device)
    assert ws.lnl_plan(259_585, 3, 4096, flags=gw.FLAG_TERM_ISCO)["rounds"] == 0
    big = ws.lnl_plan(259_585, 3, 4096)
    assert big["rounds"] > 0 and big["tile_bins"] >= 256
    mixed = ws.lnl_plan(259_585, 3, 4096, precision="mixed")
    assert mixed["rounds"] > 0
    with pytest.raises(gw.GwError):
        ws.lnl_plan(0, 3, 4096)
    with pytest.raises(gw.GwError):
        ws.lnl_plan(1000, 3, 10, flags=1 << 20)


def test_queue_launch_replays_from_a_graph(gw):
    """gw_lnl_batch captured in a graph: the queue counters are zeroed by a
    kernel of the call itself, so every replay starts from empty queues.
    Three replays, with eager calls on another workspace and host
    synchronisations between them, each equal the eager result bit for bit."""
    import torch
    w, theta, data = _event(31, 3, 40_001, 4000, False)
    dev = torch.device("cuda", 0)
    d = torch.from_numpy(np.ascontiguousarray(data)).to(dev)
    s = torch.from_numpy(w.psd).to(dev)
    th = torch.from_numpy(np.ascontiguousarray(theta)).to(dev)
    ws = _ws(gw)
    assert ws.lnl_plan(40_001, 3, 4000)["rounds"] > 0
    eager = gw.lnl_batch(w.grid, w.tensors, w.vertices, d, s, th, workspace=ws).clone()
    out = torch.empty_like(eager)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        gw.lnl_batch(w.grid, w.tensors, w.vertices, d, s, th, workspace=ws, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gw.lnl_batch(w.grid, w.tensors, w.vertices, d, s, th, workspace=ws, out=out)
    torch.cuda.synchronize()
    other = _ws(gw)
    th2 = th.flip(0).contiguous()
    for rep in range(3):
        out.zero_()
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), eager.cpu().numpy(), err_msg=f"replay {rep}")
        gw.lnl_batch(w.grid, w.tensors, w.vertices, d, s, th2, workspace=other)
        torch.cuda.synchronize()


def test_captured_call_keeps_its_tables_and_pins_the_workspace(gw):
    """A graph captured from gw_lnl_batch records the bin-table kernel too:
    eager calls on the same workspace with another grid of the same size
    (which rewrite the tables in the arena) between the replays leave every
    replay equal to the eager result, and those eager calls, made after a
    replay has rewritten the arena, equal a fresh workspace's.  The captured
    workspace then refuses to grow."""
    import torch
    w, theta, data = _event(35, 3, 40_001, 4000, False)
    dev = torch.device("cuda", 0)
    d = torch.from_numpy(np.ascontiguousarray(data)).to(dev)
    s = torch.from_numpy(w.psd).to(dev)
    th = torch.from_numpy(np.ascontiguousarray(theta)).to(dev)
    other_grid = (w.grid.f_low + 7.0, w.grid.delta_f, w.grid.n_bins)
    ws = _ws(gw)
    eager = gw.lnl_batch(w.grid, w.tensors, w.vertices, d, s, th, workspace=ws).clone()
    want_b = gw.lnl_batch(other_grid, w.tensors, w.vertices, d, s, th, workspace=_ws(gw)).clone()
    out = torch.empty_like(eager)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gw.lnl_batch(w.grid, w.tensors, w.vertices, d, s, th, workspace=ws, out=out)
    torch.cuda.synchronize()
    for rep in range(3):
        got_b = gw.lnl_batch(other_grid, w.tensors, w.vertices, d, s, th, workspace=ws)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got_b.cpu().numpy(), want_b.cpu().numpy(), err_msg=f"eager {rep}")
        out.zero_()
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), eager.cpu().numpy(), err_msg=f"replay {rep}")
    big = torch.zeros((3, 2 * w.grid.n_bins), dtype=torch.complex128, device=dev)
    big_s = torch.ones((3, 2 * w.grid.n_bins), dtype=torch.float64, device=dev)
    with pytest.raises(gw.GwError, match="cannot grow"):
        gw.lnl_batch((w.grid.f_low, w.grid.delta_f, 2 * w.grid.n_bins), w.tensors, w.vertices, big, big_s, th,
                     workspace=ws)
