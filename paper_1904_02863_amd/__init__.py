"""Python binding of libgwlnl.so, the MI355X (gfx950) batched TaylorF2
likelihood library declared in include/gwlnl.h.

This module only marshals arguments: PyTorch tensors supply device memory and
the current HIP stream, ctypes passes their pointers to the C ABI, and every
step of the computation runs in the library's HIP kernels.  There is no CPU
fallback: if the library is not built, or no GPU is present, the calls raise.

The likelihood is the exponent of Eq. (cbclike) of arXiv:1904.02863 (Sec. III),
lnL = -(2/T) sum_det sum_bins |d - h|^2 / S, for the TaylorF2 template of Sec. II
projected onto each detector and shifted by exp(-2 pi i f dt_det).
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgwlnl.so")

GW_OK, GW_EINVAL, GW_ENOMEM, GW_EDEVICE, GW_EUNSUPPORTED, GW_EABI = 0, -1, -2, -3, -4, -5
# The library version this binding's argument types describe (gw_version).
ABI_VERSION = 301
PRECISIONS = {"fp64": 0, "mixed": 1}
MAX_DET = 8
# Options of the likelihood and waveform calls (GW_FLAG_* of include/gwlnl.h).
FLAG_DIRECT = 1
FLAG_TERM_ISCO = 2
FLAG_ADD_NORM = 4

# Every symbol include/gwlnl.h declares.
EXPORTED = ("gw_workspace_create", "gw_workspace_destroy", "gw_workspace_reserve", "gw_workspace_bytes",
            "gw_workspace_set_timing", "gw_workspace_set_tuning", "gw_workspace_kernel_time", "gw_waveform_batch", "gw_fill_c128", "gw_lnl_batch",
            "gw_lnl_batch_static", "gw_lnl_batch_static_bytes", "gw_lnl_batch_static_capacity",
            "gw_lnl_ragged", "gw_lnl_plan", "gw_workspace_set_plan", "gw_ragged_tuning", "gw_pop_lnl", "gw_pop_prepare", "gw_pop_lnl_prepared",
            "gw_rb_edges", "gw_rb_create", "gw_rb_destroy", "gw_rb_lnl", "gw_rb_shape", "gw_rb_summary", "gw_last_error",
            "gw_version", "gw_abi_layout", "gw_source_hash",
            "gw_philox_raw", "gw_philox_fill", "gw_philox_chain_normals", "gw_mcmc_to_theta", "gw_mcmc_rw_propose",
            "gw_mcmc_accept", "gw_mcmc_update_mode", "gw_mcmc_adapt_chol", "gw_mcmc_moments", "gw_mcmc_count", "gw_gather_rows",
            "gw_flow_create", "gw_flow_destroy", "gw_flow_num_params",
            "gw_flow_set_params", "gw_flow_get_params", "gw_flow_forward", "gw_flow_inverse", "gw_flow_gradients",
            "gw_flow_train_step")


class GwError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"gwlnl error {code}: {message}")
        self.code = code


class GwGrid(ctypes.Structure):
    _fields_ = [("f_low", ctypes.c_double), ("delta_f", ctypes.c_double), ("n_bins", ctypes.c_int64)]


class GwDetector(ctypes.Structure):
    _fields_ = [("tensor", ctypes.c_double * 9), ("vertex", ctypes.c_double * 3)]


class GwEvent(ctypes.Structure):
    _fields_ = [("grid", GwGrid), ("n_det", ctypes.c_int), ("dets", GwDetector * MAX_DET),
                ("data_offset", ctypes.c_int64), ("theta_offset", ctypes.c_int64), ("n_samples", ctypes.c_int64)]


_lib = None


def _layout() -> list[int]:
    """What gw_abi_layout must report for the structures declared above:
    sizeof gw_c128, gw_grid, gw_detector, gw_event, offsetof(gw_event, dets), GW_MAX_DET."""
    return [16, ctypes.sizeof(GwGrid), ctypes.sizeof(GwDetector), ctypes.sizeof(GwEvent), GwEvent.dets.offset,
            MAX_DET]


def check_library(path: str, sources: bool = True) -> ctypes.CDLL:
    """Open the shared library at `path` and check, before any argument types
    are installed or any call with arguments is made, that it is the library
    this binding describes: the same gw_version, the same structure layouts
    (gw_abi_layout, which also fails when the library was linked from objects
    of different builds) and, when `sources` is set and the source tree is
    present, the same source hash as that tree (a library left over from
    older sources is refused).  Raises RuntimeError otherwise."""
    lib = ctypes.CDLL(path)
    for name in ("gw_version", "gw_abi_layout", "gw_source_hash", "gw_last_error"):
        if not hasattr(lib, name):
            raise RuntimeError(f"{path} does not export {name}: not a library this binding can use")
    lib.gw_version.argtypes = []
    lib.gw_version.restype = ctypes.c_int
    version = lib.gw_version()
    if version != ABI_VERSION:
        raise RuntimeError(f"{path} reports version {version}; this binding is for version {ABI_VERSION}")
    lib.gw_last_error.argtypes = []
    lib.gw_last_error.restype = ctypes.c_char_p
    lib.gw_abi_layout.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.gw_abi_layout.restype = ctypes.c_int
    want = _layout()
    got = (ctypes.c_int64 * 16)()
    n = lib.gw_abi_layout(got, 16)
    if n < 0:
        raise RuntimeError(f"{path}: {lib.gw_last_error().decode()}")
    if n != len(want) or list(got[:n]) != want:
        raise RuntimeError(f"{path} lays out its structures as {list(got[:max(n, 0)])}; this binding expects {want}")
    lib.gw_source_hash.argtypes = []
    lib.gw_source_hash.restype = ctypes.c_char_p
    if sources:
        from . import build as _build
        if all(os.path.exists(f) for f in _build.source_files()):
            have, tree = lib.gw_source_hash().decode(), _build.source_hash()
            if have != tree:
                raise RuntimeError(f"{path} was built from other sources than this tree ({have[:12]} against "
                                   f"{tree[:12]}); rebuild it with `python -m paper_1904_02863_amd.build`")
    return lib


def load_library() -> ctypes.CDLL:
    """Load libgwlnl.so, checked by check_library (raises if it has not been
    built, or is not the library this binding describes)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1904_02863_amd.build`")
        lib = check_library(LIB_PATH)
        vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint
        lib.gw_workspace_create.argtypes = [ctypes.POINTER(vp), i32]
        lib.gw_workspace_destroy.argtypes = [vp]
        lib.gw_workspace_reserve.argtypes = [vp, i64, i32, i64]
        lib.gw_workspace_bytes.argtypes = [vp]
        lib.gw_workspace_bytes.restype = i64
        lib.gw_workspace_set_timing.argtypes = [vp, i32]
        lib.gw_workspace_set_tuning.argtypes = [vp, i32]
        lib.gw_workspace_set_plan.argtypes = [vp, i64, i32, i64, i32, u32, i32, i32]
        lib.gw_workspace_kernel_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
        lib.gw_waveform_batch.argtypes = [vp, ctypes.POINTER(GwGrid), i32, ctypes.POINTER(GwDetector), vp, i32, i64,
                                          vp, u32, vp]
        lib.gw_lnl_batch.argtypes = [vp, ctypes.POINTER(GwGrid), i32, ctypes.POINTER(GwDetector), vp, vp, vp, i32,
                                     i64, vp, i32, u32, vp]
        lib.gw_fill_c128.argtypes = [vp, i64, ctypes.c_double, ctypes.c_double, vp]
        lib.gw_lnl_batch_static.argtypes = [ctypes.POINTER(GwGrid), i32, ctypes.POINTER(GwDetector), vp, vp, vp,
                                            i32, i64, vp, i32, u32, vp]
        lib.gw_lnl_batch_static_bytes.argtypes = [ctypes.POINTER(GwGrid), i32, i64, i32, u32]
        lib.gw_lnl_batch_static_bytes.restype = i64
        lib.gw_lnl_batch_static_capacity.argtypes = []
        lib.gw_lnl_batch_static_capacity.restype = i64
        lib.gw_lnl_ragged.argtypes = [vp, i32, ctypes.POINTER(GwEvent), vp, vp, vp, i32, vp, i32, u32, vp]
        lib.gw_ragged_tuning.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64)]
        lib.gw_lnl_plan.argtypes = [vp, i64, i32, i64, i32, u32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                    ctypes.POINTER(i32)]
        lib.gw_pop_lnl.argtypes = [vp, i64, i64, vp, i64, vp, vp, vp]
        lib.gw_pop_prepare.argtypes = [i64, i64, vp, vp, vp]
        lib.gw_pop_lnl_prepared.argtypes = [vp, i64, i64, vp, i64, vp, vp, vp]
        lib.gw_rb_edges.argtypes = [ctypes.POINTER(GwGrid), ctypes.c_double, ctypes.c_double, vp, i64,
                                    ctypes.POINTER(i64)]
        lib.gw_rb_create.argtypes = [vp, ctypes.POINTER(GwGrid), i32, ctypes.POINTER(GwDetector), vp, vp, vp, i32,
                                     vp, i64, u32, ctypes.POINTER(vp), vp]
        lib.gw_rb_destroy.argtypes = [vp]
        lib.gw_rb_lnl.argtypes = [vp, vp, vp, i64, vp, i32, vp]
        lib.gw_rb_shape.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i32)]
        lib.gw_rb_summary.argtypes = [vp, vp, vp]
        u64, u32p = ctypes.c_uint64, ctypes.c_uint32
        lib.gw_philox_raw.argtypes = [u64, u32p, u32p, u64, i64, vp, vp]
        lib.gw_philox_fill.argtypes = [u64, u32p, u32p, i32, i64, vp, vp]
        lib.gw_philox_chain_normals.argtypes = [i32, i64, u64, u32p, u32p, vp, vp]
        lib.gw_mcmc_to_theta.argtypes = [i32, i64, vp, vp, vp, i32, vp, vp, vp]
        lib.gw_mcmc_rw_propose.argtypes = [i32, i64, vp, vp, u64, u32p, vp, vp, vp]
        lib.gw_mcmc_accept.argtypes = [i32, i64, u64, u32p, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.gw_mcmc_update_mode.argtypes = [i64, vp, i32, ctypes.c_double, vp, vp]
        lib.gw_mcmc_adapt_chol.argtypes = [i32, i64, vp, ctypes.c_double, ctypes.c_double, vp, vp]
        lib.gw_mcmc_moments.argtypes = [i32, i64, vp, vp, vp, vp]
        lib.gw_mcmc_count.argtypes = [i64, vp, vp, vp]
        lib.gw_gather_rows.argtypes = [i32, i64, vp, i64, u64, u32p, u32p, vp, vp]
        lib.gw_flow_create.argtypes = [ctypes.POINTER(vp), i32, i32, i32, i32, vp]
        lib.gw_flow_destroy.argtypes = [vp]
        lib.gw_flow_num_params.argtypes = [vp]
        lib.gw_flow_num_params.restype = i64
        lib.gw_flow_set_params.argtypes = [vp, vp, vp, vp]
        lib.gw_flow_get_params.argtypes = [vp, vp, vp, vp]
        lib.gw_flow_forward.argtypes = [vp, vp, i64, vp, vp, vp]
        lib.gw_flow_inverse.argtypes = [vp, vp, i64, vp, vp, vp]
        lib.gw_flow_gradients.argtypes = [vp, vp, i64, vp, vp, vp]
        lib.gw_flow_train_step.argtypes = [vp, vp, i64, ctypes.c_float, vp, vp]
        for name in EXPORTED:
            getattr(lib, name).restype = getattr(lib, name).restype or i32
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != GW_OK:
        raise GwError(rc, load_library().gw_last_error().decode())


def _torch():
    import torch
    return torch


class Workspace:
    """Library-owned device buffers (gw_workspace) bound to one GPU."""

    def __init__(self, device: int | None = None):
        lib = load_library()
        self._h = ctypes.c_void_p()
        self.device = -1 if device is None else int(device)
        _check(lib.gw_workspace_create(ctypes.byref(self._h), self.device))

    def reserve(self, n_bins: int, n_det: int, n_samples: int):
        _check(load_library().gw_workspace_reserve(self._h, int(n_bins), int(n_det), int(n_samples)))

    @property
    def nbytes(self) -> int:
        return load_library().gw_workspace_bytes(self._h)

    def set_timing(self, enable: bool):
        """Record HIP events around the hot kernel of every likelihood call."""
        _check(load_library().gw_workspace_set_timing(self._h, 1 if enable else 0))

    def set_tuning(self, enable: bool, forget: bool = False):
        """Time candidate plans on the first likelihood call of each size class
        and use the fastest (on by default).  forget=True turns tuning off and
        drops the tuned plans, so that the default plans are used again."""
        _check(load_library().gw_workspace_set_tuning(self._h, -1 if forget else (1 if enable else 0)))

    def kernel_time(self) -> tuple[float, int]:
        """(total milliseconds, launches) of the hot kernel since timing was enabled."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(load_library().gw_workspace_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def lnl_plan(self, n_bins: int, n_det: int, n_samples: int, precision: str = "fp64", flags: int = 0) -> dict:
        """How gw_lnl_batch splits a call of this shape (the tuned plan of its
        size class once one is tuned): LDS tile bins, chunks per sample group
        and work-queue rounds (0: one block per item)."""
        t, c, r = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(load_library().gw_lnl_plan(self._h, n_bins, n_det, n_samples, PRECISIONS[precision], int(flags),
                                          ctypes.byref(t), ctypes.byref(c), ctypes.byref(r)))
        return {"tile_bins": t.value, "n_chunks": c.value, "rounds": r.value}

    def set_plan(self, n_bins: int, n_det: int, n_samples: int, tile_bins: int, rounds: int,
                 precision: str = "fp64", flags: int = 0):
        """Use this plan (LDS tile bins, work-queue rounds) for every
        gw_lnl_batch call of this size class on the workspace; tile_bins=0
        and rounds=0 drop the class's plan."""
        _check(load_library().gw_workspace_set_plan(self._h, n_bins, n_det, n_samples, PRECISIONS[precision],
                                                    int(flags), tile_bins, rounds))

    def ragged_tuning(self) -> tuple[int, int]:
        """(LDS tile bins, bins per work item) of the last ragged call."""
        t, c = ctypes.c_int(), ctypes.c_int64()
        _check(load_library().gw_ragged_tuning(self._h, ctypes.byref(t), ctypes.byref(c)))
        return t.value, c.value

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            load_library().gw_workspace_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ws: dict[int, Workspace] = {}


def default_workspace(device: int) -> Workspace:
    if device not in _default_ws:
        _default_ws[device] = Workspace(device)
    return _default_ws[device]


def make_grid(grid) -> GwGrid:
    """A gw_grid from any object with f_low, delta_f, n_bins (or a 3-tuple)."""
    if isinstance(grid, GwGrid):
        return grid
    if isinstance(grid, (tuple, list)):
        f_low, delta_f, n_bins = grid
    else:
        f_low, delta_f, n_bins = grid.f_low, grid.delta_f, grid.n_bins
    return GwGrid(float(f_low), float(delta_f), int(n_bins))


def make_detectors(tensors, vertices) -> ctypes.Array:
    t = np.ascontiguousarray(tensors, dtype=np.float64).reshape(-1, 9)
    v = np.ascontiguousarray(vertices, dtype=np.float64).reshape(-1, 3)
    if t.shape[0] != v.shape[0] or not 1 <= t.shape[0] <= MAX_DET:
        raise ValueError("tensors and vertices must describe 1..8 detectors")
    arr = (GwDetector * t.shape[0])()
    for i in range(t.shape[0]):
        arr[i].tensor[:] = t[i].tolist()
        arr[i].vertex[:] = v[i].tolist()
    return arr


def _cuda_tensor(x, dtype, name, shape=None):
    torch = _torch()
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch.Tensor")
    if x.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {x.dtype}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(x.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(x.shape)}")
    return x


def _stream_ptr(device: int, stream=None) -> ctypes.c_void_p:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def lnl_batch(grid, tensors, vertices, data, psd, theta, *, precision: str = "fp64", flags: int = 0, out=None,
              workspace: Workspace | None = None, stream=None):
    """lnL for every row of theta (Eq. (cbclike) without its constant factor).

    data: complex128 [n_det, M]; psd: float64 [n_det, M]; theta: float64 [S, 5, 7, 9 or 11],
    all on the same GPU.  flags: FLAG_DIRECT | FLAG_TERM_ISCO | FLAG_ADD_NORM.
    Returns (or fills `out`) float64 [S] on that GPU.
    """
    torch = _torch()
    g = make_grid(grid)
    theta = _cuda_tensor(theta, torch.float64, "theta")
    if theta.dim() != 2:
        raise ValueError("theta must be [n_samples, n_param]")
    n_samples, n_param = theta.shape
    n_det = data.shape[0] if data.dim() == 2 else -1
    data = _cuda_tensor(data, torch.complex128, "data", (n_det, g.n_bins))
    psd = _cuda_tensor(psd, torch.float64, "psd", (n_det, g.n_bins))
    dev = theta.device.index
    if data.device.index != dev or psd.device.index != dev:
        raise ValueError("data, psd and theta must be on the same device")
    if out is None:
        out = torch.empty(n_samples, dtype=torch.float64, device=theta.device)
    out = _cuda_tensor(out, torch.float64, "out", (n_samples,))
    dets = make_detectors(tensors, vertices) if n_param in (9, 11) or tensors is not None else (GwDetector * 1)()
    ws = workspace or default_workspace(dev)
    _check(load_library().gw_lnl_batch(ws.handle, ctypes.byref(g), n_det, dets, data.data_ptr(), psd.data_ptr(),
                                       theta.data_ptr(), n_param, n_samples, out.data_ptr(),
                                       PRECISIONS[precision], int(flags), _stream_ptr(dev, stream)))
    return out


def fill_c128(out, value: complex = 0.0, stream=None):
    """out[...] = value for a contiguous complex128 CUDA tensor (gw_fill_c128)."""
    torch = _torch()
    out = _cuda_tensor(out, torch.complex128, "out")
    dev = out.device.index
    with torch.cuda.device(dev):
        _check(load_library().gw_fill_c128(out.data_ptr(), out.numel(), float(complex(value).real),
                                           float(complex(value).imag), _stream_ptr(dev, stream)))
    return out


def lnl_batch_static(grid, tensors, vertices, data, psd, theta, *, precision: str = "fp64", flags: int = 0,
                     out=None, stream=None):
    """lnl_batch through gw_lnl_batch_static: no workspace, no device
    allocation by the library (its buffers are a static array per GPU).
    `out` must be given by callers that may not allocate either."""
    torch = _torch()
    g = make_grid(grid)
    theta = _cuda_tensor(theta, torch.float64, "theta")
    if theta.dim() != 2:
        raise ValueError("theta must be [n_samples, n_param]")
    n_samples, n_param = theta.shape
    n_det = data.shape[0] if data.dim() == 2 else -1
    data = _cuda_tensor(data, torch.complex128, "data", (n_det, g.n_bins))
    psd = _cuda_tensor(psd, torch.float64, "psd", (n_det, g.n_bins))
    dev = theta.device.index
    if data.device.index != dev or psd.device.index != dev:
        raise ValueError("data, psd and theta must be on the same device")
    if out is None:
        out = torch.empty(n_samples, dtype=torch.float64, device=theta.device)
    out = _cuda_tensor(out, torch.float64, "out", (n_samples,))
    dets = make_detectors(tensors, vertices) if n_param in (9, 11) or tensors is not None else (GwDetector * 1)()
    with torch.cuda.device(dev):
        _check(load_library().gw_lnl_batch_static(ctypes.byref(g), n_det, dets, data.data_ptr(), psd.data_ptr(),
                                                  theta.data_ptr(), n_param, n_samples, out.data_ptr(),
                                                  PRECISIONS[precision], int(flags), _stream_ptr(dev, stream)))
    return out


def lnl_batch_static_bytes(grid, n_det: int, n_samples: int, precision: str = "fp64", flags: int = 0,
                           device: int = 0) -> int:
    """Bytes of the static array a gw_lnl_batch_static call of this shape needs."""
    torch = _torch()
    g = make_grid(grid)
    with torch.cuda.device(device):
        n = load_library().gw_lnl_batch_static_bytes(ctypes.byref(g), int(n_det), int(n_samples),
                                                     PRECISIONS[precision], int(flags))
    if n < 0:
        _check(int(n))
    return int(n)


def lnl_batch_static_capacity() -> int:
    """GW_STATIC_SCRATCH_BYTES: the size of the static array per GPU."""
    return int(load_library().gw_lnl_batch_static_capacity())


def waveform_batch(grid, tensors, vertices, theta, *, flags: int = 0, out=None, workspace: Workspace | None = None,
                   stream=None):
    """Detector responses [S, n_det, M] (complex128); with tensors None the
    polarisations [S, 2, M] (h_plus, h_cross).  flags: 0 or FLAG_TERM_ISCO."""
    torch = _torch()
    g = make_grid(grid)
    theta = _cuda_tensor(theta, torch.float64, "theta")
    if theta.dim() != 2:
        raise ValueError("theta must be [n_samples, n_param]")
    n_samples, n_param = theta.shape
    if tensors is None:
        n_det, n_out, dets = 0, 2, None
    else:
        dets = make_detectors(tensors, vertices)
        n_det = n_out = len(dets)
    dev = theta.device.index
    if out is None:
        out = torch.empty((n_samples, n_out, g.n_bins), dtype=torch.complex128, device=theta.device)
    out = _cuda_tensor(out, torch.complex128, "out", (n_samples, n_out, g.n_bins))
    ws = workspace or default_workspace(dev)
    _check(load_library().gw_waveform_batch(ws.handle, ctypes.byref(g), n_det, dets, theta.data_ptr(), n_param,
                                            n_samples, out.data_ptr(), int(flags), _stream_ptr(dev, stream)))
    return out


def make_events(grids: Sequence, tensors: Sequence, vertices: Sequence, n_samples: Sequence[int]):
    """Host gw_event array with packed offsets; returns (events, total_data_elems, total_rows)."""
    n = len(grids)
    events = (GwEvent * max(n, 1))()
    doff, toff = 0, 0
    for i in range(n):
        g = make_grid(grids[i])
        dets = make_detectors(tensors[i], vertices[i])
        ev = events[i]
        ev.grid = g
        ev.n_det = len(dets)
        for d in range(len(dets)):
            ev.dets[d] = dets[d]
        ev.data_offset = doff
        ev.theta_offset = toff
        ev.n_samples = int(n_samples[i])
        doff += len(dets) * g.n_bins
        toff += int(n_samples[i])
    return events, doff, toff


def lnl_ragged(events, n_events: int, data_packed, psd_packed, theta_packed, *, precision: str = "fp64",
               flags: int = 0, out=None, workspace: Workspace | None = None, stream=None):
    """lnL of many events of different durations, each with its own rows of
    theta_packed (see gw_lnl_ragged); flags as for lnl_batch."""
    torch = _torch()
    theta_packed = _cuda_tensor(theta_packed, torch.float64, "theta_packed")
    data_packed = _cuda_tensor(data_packed, torch.complex128, "data_packed")
    psd_packed = _cuda_tensor(psd_packed, torch.float64, "psd_packed")
    n_rows, n_param = theta_packed.shape
    total = max((events[i].data_offset + events[i].n_det * events[i].grid.n_bins for i in range(n_events)), default=0)
    rows = max((events[i].theta_offset + events[i].n_samples for i in range(n_events)), default=0)
    if data_packed.numel() < total or psd_packed.numel() < total or n_rows < rows:
        raise ValueError("packed arrays are smaller than the events describe")
    dev = theta_packed.device.index
    if out is None:
        out = torch.empty(n_rows, dtype=torch.float64, device=theta_packed.device)
    out = _cuda_tensor(out, torch.float64, "out")
    if out.numel() < rows:
        raise ValueError("out is smaller than the events describe")
    ws = workspace or default_workspace(dev)
    _check(load_library().gw_lnl_ragged(ws.handle, int(n_events), events, data_packed.data_ptr(),
                                        psd_packed.data_ptr(), theta_packed.data_ptr(), n_param, out.data_ptr(),
                                        PRECISIONS[precision], int(flags), _stream_ptr(dev, stream)))
    return out


def pop_prepare(samples, *, out=None, stream=None):
    """Prepared samples [8, n_events, n] (gw_pop_prepare) from raw samples [7, n_events, n]."""
    torch = _torch()
    samples = _cuda_tensor(samples, torch.float64, "samples")
    if samples.dim() != 3 or samples.shape[0] != 7:
        raise ValueError("samples must be [7, n_events, n_per_event]")
    shape = (8, samples.shape[1], samples.shape[2])
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=samples.device)
    out = _cuda_tensor(out, torch.float64, "out", shape)
    _check(load_library().gw_pop_prepare(samples.shape[1], samples.shape[2], samples.data_ptr(), out.data_ptr(),
                                         _stream_ptr(samples.device.index, stream)))
    return out


def pop_lnl(samples, hyper, *, out=None, workspace: Workspace | None = None, stream=None):
    """Population ln L (Eq. (poplike)) for every row of hyper [K, 12] over
    samples [7, n_events, n] (m1, q, a1, a2, cos t1, cos t2, ln prior), or over
    prepared samples [8, n_events, n] from `pop_prepare`, both float64 on the
    same GPU; returns float64 [K] there."""
    torch = _torch()
    samples = _cuda_tensor(samples, torch.float64, "samples")
    if samples.dim() != 3 or samples.shape[0] not in (7, 8):
        raise ValueError("samples must be [7, n_events, n_per_event] (raw) or [8, ...] (prepared)")
    hyper = _cuda_tensor(hyper, torch.float64, "hyper")
    if hyper.dim() != 2 or hyper.shape[1] != 12:
        raise ValueError("hyper must be [n_hyper, 12]")
    dev = samples.device.index
    if hyper.device.index != dev:
        raise ValueError("samples and hyper must be on the same device")
    k = hyper.shape[0]
    if out is None:
        out = torch.empty(k, dtype=torch.float64, device=samples.device)
    out = _cuda_tensor(out, torch.float64, "out", (k,))
    ws = workspace or default_workspace(dev)
    fn = load_library().gw_pop_lnl_prepared if samples.shape[0] == 8 else load_library().gw_pop_lnl
    _check(fn(ws.handle, samples.shape[1], samples.shape[2], samples.data_ptr(), k, hyper.data_ptr(), out.data_ptr(),
              _stream_ptr(dev, stream)))
    return out


def rb_edges(grid, chi: float = 1.0, eps: float = 0.5) -> np.ndarray:
    """Relative-binning bin edges (grid indices) by the phase-bound rule of
    gw_rb_edges; a host computation."""
    g = make_grid(grid)
    lib = load_library()
    n = ctypes.c_int64()
    _check(lib.gw_rb_edges(ctypes.byref(g), float(chi), float(eps), None, 0, ctypes.byref(n)))
    out = np.empty(n.value, dtype=np.int64)
    _check(lib.gw_rb_edges(ctypes.byref(g), float(chi), float(eps), out.ctypes.data_as(ctypes.c_void_p), out.size,
                           ctypes.byref(n)))
    return out


class RelativeBinning:
    """One event prepared for the relative-binning likelihood (gw_relbin).

    data complex128 [n_det, M] and psd float64 [n_det, M] on one GPU; theta0
    the fiducial parameters (host, 5, 7, 9 or 11 values); edges the bin edges (host
    int64, from `rb_edges` or any strictly rising list from 0 to M - 1);
    flags 0 or FLAG_ADD_NORM.  The preparation is synchronous."""

    def __init__(self, grid, tensors, vertices, data, psd, theta0, edges, *, flags: int = 0,
                 workspace: Workspace | None = None, stream=None):
        torch = _torch()
        g = make_grid(grid)
        th0 = np.ascontiguousarray(theta0, dtype=np.float64).reshape(-1)
        n_param = th0.size
        n_det = data.shape[0] if data.dim() == 2 else -1
        data = _cuda_tensor(data, torch.complex128, "data", (n_det, g.n_bins))
        psd = _cuda_tensor(psd, torch.float64, "psd", (n_det, g.n_bins))
        dev = data.device.index
        if psd.device.index != dev:
            raise ValueError("data and psd must be on the same device")
        e = np.ascontiguousarray(edges, dtype=np.int64).reshape(-1)
        dets = make_detectors(tensors, vertices) if n_param in (9, 11) or tensors is not None else (GwDetector * 1)()
        self.device = dev
        self.n_param = n_param
        self._ws = workspace or default_workspace(dev)
        h = ctypes.c_void_p()
        _check(load_library().gw_rb_create(self._ws.handle, ctypes.byref(g), n_det, dets, data.data_ptr(),
                                           psd.data_ptr(), th0.ctypes.data_as(ctypes.c_void_p), n_param,
                                           e.ctypes.data_as(ctypes.c_void_p), e.size, int(flags), ctypes.byref(h),
                                           _stream_ptr(dev, stream)))
        self._h = h

    @property
    def shape(self) -> tuple[int, int]:
        """(bins B, detectors)."""
        nb, nd = ctypes.c_int64(), ctypes.c_int()
        _check(load_library().gw_rb_shape(self._h, ctypes.byref(nb), ctypes.byref(nd)))
        return nb.value, nd.value

    def lnl(self, theta, *, out=None, precision: str = "fp64", workspace: Workspace | None = None, stream=None):
        """Relative-binning lnL of every row of theta (float64 [S, n_param] on the handle's GPU);
        precision "fp64" or "mixed" (FP32 hardware phasor of the ratio)."""
        torch = _torch()
        theta = _cuda_tensor(theta, torch.float64, "theta")
        if theta.dim() != 2 or theta.shape[1] != self.n_param:
            raise ValueError(f"theta must be [n_samples, {self.n_param}]")
        if theta.device.index != self.device:
            raise ValueError("theta must be on the handle's device")
        n = theta.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=theta.device)
        out = _cuda_tensor(out, torch.float64, "out", (n,))
        ws = workspace or self._ws
        _check(load_library().gw_rb_lnl(ws.handle, self._h, theta.data_ptr(), n, out.data_ptr(),
                                        PRECISIONS[precision], _stream_ptr(self.device, stream)))
        return out

    def summary(self) -> tuple[np.ndarray, np.ndarray]:
        """(raw [B, n_det, 7]: A0 re, A0 im, A1 re, A1 im, B0, B1, B2; totals [<d,d>, sum ln 2 pi S])."""
        nb, nd = self.shape
        raw = np.empty((nb, nd, 7))
        tot = np.empty(2)
        _check(load_library().gw_rb_summary(self._h, raw.ctypes.data_as(ctypes.c_void_p),
                                            tot.ctypes.data_as(ctypes.c_void_p)))
        return raw, tot

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(load_library().gw_rb_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def version() -> int:
    return load_library().gw_version()


# ---------------------------------------------------------------- sampler calls
def _ptr_or_null(t):
    return None if t is None else t.data_ptr()


def philox_raw(seed: int, stream_id: int, step: int, n_blocks: int, first: int = 0, device=0, stream=None):
    """Philox4x32-10 blocks first .. first + n_blocks - 1 as a numpy uint32
    array [n_blocks, 4] (computed on the GPU)."""
    torch = _torch()
    out = torch.empty((int(n_blocks), 4), dtype=torch.int32, device=torch.device("cuda", device))
    _check(load_library().gw_philox_raw(int(seed), int(stream_id), int(step), int(first) % 2 ** 64, int(n_blocks),
                                        out.data_ptr(), _stream_ptr(device, stream)))
    return out.cpu().numpy().view(np.uint32)


def philox_fill(seed: int, stream_id: int, step: int, n: int, normal: bool, device=0, stream=None, out=None):
    """n uniforms (normal=False) or standard normals from (seed, stream_id, step) as float64 on the GPU."""
    torch = _torch()
    if out is None:
        out = torch.empty(int(n), dtype=torch.float64, device=torch.device("cuda", device))
    _check(load_library().gw_philox_fill(int(seed), int(stream_id), int(step), 1 if normal else 0, int(n),
                                         out.data_ptr(), _stream_ptr(device, stream)))
    return out


def chain_normals(dim: int, n_chains: int, seed: int, stream_id: int, step: int, out=None, device=0, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty((int(n_chains), int(dim)), dtype=torch.float64, device=torch.device("cuda", device))
    _check(load_library().gw_philox_chain_normals(int(dim), int(n_chains), int(seed), int(stream_id), int(step),
                                                  out.data_ptr(), _stream_ptr(device, stream)))
    return out


def mcmc_to_theta(box_lo, box_hi, x, theta_out=None, logprior_out=None, stream=None, theta_cols: int | None = None):
    """theta [n, theta_cols] and log prior [n] of sampler coordinates x [n, dim].
    theta_cols 9 (default), or 11 with dim 11 to pass the spin coordinates on
    as chi1, chi2; with theta_out given its width decides."""
    torch = _torch()
    x = _cuda_tensor(x, torch.float64, "x")
    n, dim = x.shape
    lo = np.ascontiguousarray(box_lo, dtype=np.float64)
    hi = np.ascontiguousarray(box_hi, dtype=np.float64)
    if lo.shape != (dim,) or hi.shape != (dim,):
        raise ValueError("box_lo and box_hi must have one entry per coordinate")
    if theta_cols is None:
        theta_cols = theta_out.shape[1] if theta_out is not None else 9
    if theta_out is None:
        theta_out = torch.empty((n, theta_cols), dtype=torch.float64, device=x.device)
    theta_out = _cuda_tensor(theta_out, torch.float64, "theta_out", (n, theta_cols))
    if logprior_out is None:
        logprior_out = torch.empty(n, dtype=torch.float64, device=x.device)
    _check(load_library().gw_mcmc_to_theta(dim, n, lo.ctypes.data, hi.ctypes.data, x.data_ptr(), theta_cols,
                                           theta_out.data_ptr(), logprior_out.data_ptr(),
                                           _stream_ptr(x.device.index, stream)))
    return theta_out, logprior_out


def mcmc_rw_propose(x, chol, seed: int, step: int, x_prop, mode=None, stream=None):
    torch = _torch()
    x = _cuda_tensor(x, torch.float64, "x")
    n, dim = x.shape
    chol = _cuda_tensor(chol, torch.float64, "chol", (dim, dim))
    x_prop = _cuda_tensor(x_prop, torch.float64, "x_prop", (n, dim))
    if mode is not None:
        mode = _cuda_tensor(mode, torch.int32, "mode", (n,))
    _check(load_library().gw_mcmc_rw_propose(dim, n, x.data_ptr(), chol.data_ptr(), int(seed), int(step),
                                             _ptr_or_null(mode), x_prop.data_ptr(), _stream_ptr(x.device.index, stream)))
    return x_prop


def mcmc_accept(seed: int, step: int, x, lnp, x_prop, lnl_prop, lp_prop, logq=None, logq_prop=None, mode=None,
                window_accepts=None, total_accepts=None, stream=None):
    """One Metropolis-Hastings decision per chain (see gw_mcmc_accept)."""
    torch = _torch()
    x = _cuda_tensor(x, torch.float64, "x")
    n, dim = x.shape
    for name, t in (("lnp", lnp), ("lnl_prop", lnl_prop), ("lp_prop", lp_prop)):
        _cuda_tensor(t, torch.float64, name, (n,))
    _cuda_tensor(x_prop, torch.float64, "x_prop", (n, dim))
    for name, t in (("window_accepts", window_accepts), ("total_accepts", total_accepts), ("mode", mode)):
        if t is not None:
            _cuda_tensor(t, torch.int32, name, (n,))
    _check(load_library().gw_mcmc_accept(dim, n, int(seed), int(step), x.data_ptr(), lnp.data_ptr(),
                                         _ptr_or_null(logq), x_prop.data_ptr(), lnl_prop.data_ptr(), lp_prop.data_ptr(),
                                         _ptr_or_null(logq_prop), _ptr_or_null(mode), _ptr_or_null(window_accepts),
                                         _ptr_or_null(total_accepts), _stream_ptr(x.device.index, stream)))


def mcmc_update_mode(window_accepts, window: int, threshold: float, mode, stream=None):
    n = mode.shape[0]
    _check(load_library().gw_mcmc_update_mode(n, window_accepts.data_ptr(), int(window), float(threshold),
                                              mode.data_ptr(), _stream_ptr(mode.device.index, stream)))
    return mode


def mcmc_adapt_chol(x, scale: float = 1.0, floor: float = 1e-12, out=None, stream=None):
    """Cholesky factor [dim, dim] of (2.38^2/dim) scale^2 Cov(x) + floor
    max(1, tr/dim) I over the rows of x [n, dim] (gw_mcmc_adapt_chol)."""
    torch = _torch()
    x = _cuda_tensor(x, torch.float64, "x")
    n, dim = x.shape
    if out is None:
        out = torch.empty((dim, dim), dtype=torch.float64, device=x.device)
    out = _cuda_tensor(out, torch.float64, "out", (dim, dim))
    _check(load_library().gw_mcmc_adapt_chol(dim, n, x.data_ptr(), float(scale), float(floor), out.data_ptr(),
                                             _stream_ptr(x.device.index, stream)))
    return out


def mcmc_moments(x, stream=None):
    """(mean [dim], covariance [dim, dim]) of the rows of x [n, dim] on the GPU (gw_mcmc_moments)."""
    torch = _torch()
    x = _cuda_tensor(x, torch.float64, "x")
    n, dim = x.shape
    mean = torch.empty(dim, dtype=torch.float64, device=x.device)
    cov = torch.empty((dim, dim), dtype=torch.float64, device=x.device)
    _check(load_library().gw_mcmc_moments(dim, n, x.data_ptr(), mean.data_ptr(), cov.data_ptr(),
                                          _stream_ptr(x.device.index, stream)))
    return mean, cov


def mcmc_count(counts, out=None, stream=None):
    """Sum of the int32 counters `counts` [n] as a device int64 [1] (gw_mcmc_count)."""
    torch = _torch()
    counts = _cuda_tensor(counts, torch.int32, "counts")
    if out is None:
        out = torch.empty(1, dtype=torch.int64, device=counts.device)
    out = _cuda_tensor(out, torch.int64, "out", (1,))
    _check(load_library().gw_mcmc_count(counts.shape[0], counts.data_ptr(), out.data_ptr(),
                                        _stream_ptr(counts.device.index, stream)))
    return out


def gather_rows(src, n_out: int, seed: int, stream_id: int, step: int, out=None, stream=None):
    """n_out rows of src [n_src, dim] drawn with replacement by Philox
    (seed, stream_id, step) (gw_gather_rows)."""
    torch = _torch()
    src = _cuda_tensor(src, torch.float64, "src")
    n_src, dim = src.shape
    if out is None:
        out = torch.empty((int(n_out), dim), dtype=torch.float64, device=src.device)
    out = _cuda_tensor(out, torch.float64, "out", (int(n_out), dim))
    _check(load_library().gw_gather_rows(dim, int(n_out), src.data_ptr(), n_src, int(seed), int(stream_id),
                                         int(step), out.data_ptr(), _stream_ptr(src.device.index, stream)))
    return out


class Flow:
    """Affine-coupling normalising flow on the GPU (gw_flow): BF16 matrix-core
    MLPs, FP64 coupling and densities, Adam training."""

    def __init__(self, dim: int, cond_masks, hidden: int = 256, device: int = 0):
        lib = load_library()
        masks = np.ascontiguousarray(cond_masks, dtype=np.uint32)
        self.dim, self.layers, self.hidden, self.device = int(dim), len(masks), int(hidden), int(device)
        self.cond_masks = masks.copy()
        self._h = ctypes.c_void_p()
        _check(lib.gw_flow_create(ctypes.byref(self._h), self.device, self.dim, self.layers, self.hidden,
                                  masks.ctypes.data))
        self.n_params = lib.gw_flow_num_params(self._h)

    def set_params(self, params, mu, log_sigma):
        p = np.ascontiguousarray(params, dtype=np.float32)
        m = np.ascontiguousarray(mu, dtype=np.float64)
        ls = np.ascontiguousarray(log_sigma, dtype=np.float64)
        if p.shape != (self.n_params,) or m.shape != (self.dim,) or ls.shape != (self.dim,):
            raise ValueError("parameter shapes do not match the flow")
        _check(load_library().gw_flow_set_params(self._h, p.ctypes.data, m.ctypes.data, ls.ctypes.data))

    def get_params(self):
        p = np.empty(self.n_params, dtype=np.float32)
        m = np.empty(self.dim)
        ls = np.empty(self.dim)
        _check(load_library().gw_flow_get_params(self._h, p.ctypes.data, m.ctypes.data, ls.ctypes.data))
        return p, m, ls

    def _rows(self, a, name):
        torch = _torch()
        a = _cuda_tensor(a, torch.float64, name)
        if a.dim() != 2 or a.shape[1] != self.dim:
            raise ValueError(f"{name} must be [n, {self.dim}]")
        return a

    def forward(self, z, x_out=None, logq_out=None, stream=None):
        torch = _torch()
        z = self._rows(z, "z")
        x_out = torch.empty_like(z) if x_out is None else x_out
        logq_out = torch.empty(z.shape[0], dtype=torch.float64, device=z.device) if logq_out is None else logq_out
        _check(load_library().gw_flow_forward(self._h, z.data_ptr(), z.shape[0], x_out.data_ptr(), logq_out.data_ptr(),
                                              _stream_ptr(self.device, stream)))
        return x_out, logq_out

    def inverse(self, x, z_out=None, logq_out=None, stream=None):
        torch = _torch()
        x = self._rows(x, "x")
        z_out = torch.empty_like(x) if z_out is None else z_out
        logq_out = torch.empty(x.shape[0], dtype=torch.float64, device=x.device) if logq_out is None else logq_out
        _check(load_library().gw_flow_inverse(self._h, x.data_ptr(), x.shape[0], z_out.data_ptr(), logq_out.data_ptr(),
                                              _stream_ptr(self.device, stream)))
        return z_out, logq_out

    def gradients(self, x, stream=None):
        torch = _torch()
        x = self._rows(x, "x")
        grad = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float64, device=x.device)
        _check(load_library().gw_flow_gradients(self._h, x.data_ptr(), x.shape[0], grad.data_ptr(), loss.data_ptr(),
                                                _stream_ptr(self.device, stream)))
        return grad, loss

    def train_step(self, x, lr: float, loss_out=None, stream=None):
        torch = _torch()
        x = self._rows(x, "x")
        loss_out = torch.empty(1, dtype=torch.float64, device=x.device) if loss_out is None else loss_out
        _check(load_library().gw_flow_train_step(self._h, x.data_ptr(), x.shape[0], float(lr), loss_out.data_ptr(),
                                                 _stream_ptr(self.device, stream)))
        return loss_out

    def close(self):
        if self._h:
            load_library().gw_flow_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
