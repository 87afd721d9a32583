"""The allocation-free likelihood entry point, gw_lnl_batch_static, against
gw_lnl_batch on a workspace: the same values bit for bit (and so within the
1e-10 relative FP64 bar of Eq. (cbclike) against the oracle, which the
workspace call's own tests establish), on two calls in a row, the second
smaller than the first, so that whatever the first left in the shared
static array must not leak into the second; the mixed path and the
template-end form, whose work-queue counters and cut-off live in the array;
and a call larger than the array, refused before anything is enqueued."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def _inputs(w):
    data = torch.from_numpy(oracle.workload_data(w)).to(DEV)
    psd = torch.from_numpy(np.ascontiguousarray(w.psd)).to(DEV)
    theta = torch.from_numpy(np.ascontiguousarray(w.theta)).to(DEV)
    return data, psd, theta


def test_static_entry_matches_workspace_call_on_two_calls():
    import paper_1904_02863_amd as gw
    gw.load_library()
    ws = gw.Workspace(0)
    ws.set_tuning(False)                 # the default plan, which the static entry point uses
    cap = gw.lnl_batch_static_capacity()
    assert cap == 64 << 20
    big = synth.bbh_3det_128s(4096)
    small = synth.small_event(3, 2, 5003, 300)
    for name, w in (("3 detectors x 259,585 bins x 4096 samples", big), ("2 x 5,003 x 300", small)):
        print(f"case {name}", flush=True)
        need = gw.lnl_batch_static_bytes(w.grid, w.n_det, w.theta.shape[0])
        assert 0 < need <= cap
        data, psd, theta = _inputs(w)
        for precision, flags in (("fp64", 0), ("mixed", 0), ("fp64", gw.FLAG_TERM_ISCO)):
            ref = gw.lnl_batch(w.grid, w.tensors, w.vertices, data, psd, theta, precision=precision, flags=flags,
                               workspace=ws)
            out = torch.full_like(ref, float("nan"))
            got = gw.lnl_batch_static(w.grid, w.tensors, w.vertices, data, psd, theta, precision=precision,
                                      flags=flags, out=out)
            torch.cuda.synchronize()
            assert got.data_ptr() == out.data_ptr()
            a, b = got.cpu().numpy(), ref.cpu().numpy()
            print(f"  {precision} flags {flags}: max |static - workspace| {np.max(np.abs(a - b)):.3e}", flush=True)
            np.testing.assert_array_equal(a, b)
            assert np.isfinite(a).all()
        # a few rows of the FP64 result against the oracle directly
        rows = np.array([0, w.theta.shape[0] // 2, w.theta.shape[0] - 1])
        got = gw.lnl_batch_static(w.grid, w.tensors, w.vertices, data, psd, theta).cpu().numpy()[rows]
        g = w.grid
        want = oracle.lnl(g.f_low, g.delta_f, g.n_bins, w.tensors, w.vertices, data.cpu().numpy(), w.psd,
                          w.theta[rows])
        assert np.all(np.abs(got - want) <= 1e-10 * np.abs(want))


def test_static_entry_refuses_calls_beyond_its_array():
    import paper_1904_02863_amd as gw
    w = synth.small_event(4, 3, 800_000, 4096)
    need = gw.lnl_batch_static_bytes(w.grid, 3, 4096)
    assert need > gw.lnl_batch_static_capacity()
    data = torch.zeros((3, w.grid.n_bins), dtype=torch.complex128, device=DEV)
    psd = torch.ones((3, w.grid.n_bins), dtype=torch.float64, device=DEV)
    theta = torch.from_numpy(np.ascontiguousarray(w.theta)).to(DEV)
    out = torch.full((4096,), 7.0, dtype=torch.float64, device=DEV)
    with pytest.raises(gw.GwError, match="static"):
        gw.lnl_batch_static(w.grid, w.tensors, w.vertices, data, psd, theta, out=out)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
