"""FFT-based psi_r and SCV bandwidth-selector hot path on MI355X (HIP, gfx950).

Python face of libkdefft (include/kdefft.h): every step runs in the library's
HIP kernels; this module only allocates device memory through torch, passes
pointers and the current stream, and raises on error codes.  It refuses to
work without the built library.

    import paper_1511_07482_amd as kf
    g   = kf.grid_auto(X, G, M=256)                     # X: cuda float64 [n, d]
    psi = kf.psi(X, G, r=4, grid=g)                     # unique entries of psi_4
    ds  = kf.Dataset(X, G_pilot, M=256)                 # binned + transformed once
    obj, grad = kf.scv([ds], vechL)                     # many H in one launch
    obj = kf.SCV.apply(vechL, ds)                       # autograd: backward = adjoint
"""
from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import (FUN_ETA1, FUN_ETA2, FUN_PSI, FUN_SCV_GRAD, FUN_SCV_OBJ, FUN_SCV_OBJGRAD, Grid,  # noqa: F401
                   KdefftError)

__all__ = ["Grid", "Dataset", "KdefftError", "grid_plan", "grid_auto", "linbin", "psi", "psi_batch", "scv",
           "scv_adjoint", "scv_plain", "SCV", "unique_tuples", "autotune", "set_row_launch", "library_path",
           "timing_start", "timing_stop", "crit", "crit_adjoint", "pi", "expand_full", "Criterion", "PI",
           "CRIT_SCV", "CRIT_LSCV", "CRIT_LSCV_EXACT", "CRIT_QR", "fftl_plan", "psi_fftl",
           "get_row_launch", "row_launch", "lag_layout", "scv_batch_noalloc", "minimize", "CRIT_PI",
           "MIN_CONVERGED", "MIN_RUNNING", "MIN_STALLED", "MIN_BAD_START", "set_fft_schedule",
           "get_fft_schedule", "fft_schedule", "FFT_SCHEDULES", "scv_walk_runs"]


def library_path():
    return _lib.LIB_PATH


def _L():
    return _lib.load()


def _stream(device=None):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _as_X(X):
    if not isinstance(X, torch.Tensor) or not X.is_cuda:
        raise TypeError("X must be a CUDA (HIP) tensor")
    if X.dtype != torch.float64 or X.dim() != 2:
        raise TypeError("X must be float64 [n, d]")
    return X.contiguous()


def _mat(A, d, name):
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
    if A.shape != (d, d):
        raise ValueError(f"{name} must be {d}x{d}")
    return A


def _ws(grid: Grid, op, r, batch, device):
    n = C.c_size_t()
    _lib.check(_L().kdefft_ws_bytes(C.byref(grid), op, r, int(batch), C.byref(n)), "kdefft_ws_bytes")
    return torch.empty(max(int(n.value), 256), dtype=torch.uint8, device=device)


def unique_tuples(d: int, r: int):
    cnt = _L().kdefft_unique_count(d, r)
    if cnt < 0:
        _lib.check(cnt, "kdefft_unique_count")
    if r == 0:
        return [()]
    buf = (C.c_int32 * (cnt * r))()
    _lib.check(_L().kdefft_unique_index(d, r, buf), "kdefft_unique_index")
    return [tuple(buf[k * r:(k + 1) * r]) for k in range(cnt)]


def grid_plan(M, lo, hi, P=None) -> Grid:
    lo = np.asarray(lo, dtype=np.float64)
    d = len(lo)
    M = np.broadcast_to(np.asarray(M, dtype=np.int32), (d,)).copy()
    hi = np.asarray(hi, dtype=np.float64)
    Pa = None if P is None else np.broadcast_to(np.asarray(P, dtype=np.int32), (d,)).copy()
    g = Grid()
    _lib.check(_L().kdefft_grid_plan(d, M.ctypes.data, None if Pa is None else Pa.ctypes.data,
                                     lo.ctypes.data, hi.ctypes.data, C.byref(g)), "kdefft_grid_plan")
    return g


def grid_auto(X: torch.Tensor, G, M, pad_sd: float = 4.0) -> Grid:
    X = _as_X(X)
    n, d = X.shape
    Gm = _mat(G, d, "G")
    Ma = np.broadcast_to(np.asarray(M, dtype=np.int32), (d,)).copy()
    probe = Grid()
    probe.d = d
    for k in range(d):
        probe.M[k], probe.P[k], probe.delta[k] = 2, 4, 1.0
    ws = _ws(probe, _lib.OP_GRID_AUTO, 0, n, X.device)
    g = Grid()
    _lib.check(_L().kdefft_grid_auto(_ptr(X), n, d, Gm.ctypes.data, Ma.ctypes.data, float(pad_sd), C.byref(g),
                                     _ptr(ws), ws.numel(), _stream(X.device)), "kdefft_grid_auto")
    return g


def linbin(X: torch.Tensor, grid: Grid):
    """Int64 fixed-point counts [M_0, ..., M_{d-1}] (2^-40 quanta) and the out-of-grid count."""
    X = _as_X(X)
    n, d = X.shape
    shape = tuple(grid.M[:grid.d])
    counts = torch.empty(shape, dtype=torch.int64, device=X.device)
    nout = torch.zeros(2, dtype=torch.int32, device=X.device)
    _lib.check(_L().kdefft_linbin(_ptr(X), n, C.byref(grid), _ptr(counts), _ptr(nout), _stream(X.device)),
               "kdefft_linbin")
    return counts, nout[:1]


def psi(X: torch.Tensor, G, r: int, M=None, grid: Optional[Grid] = None, mode: str = "plain",
        pad_sd: float = 4.0) -> torch.Tensor:
    """Unique entries of psi_r(G) of the sample X by the binned FFT route.
    With an explicit grid, points outside it are dropped (see linbin)."""
    X = _as_X(X)
    n, d = X.shape
    Gm = _mat(G, d, "G")
    if grid is None:
        if M is None:
            raise ValueError("give M or grid")
        grid = grid_auto(X, Gm, M, pad_sd)
    m = {"plain": _lib.PSI_PLAIN, "fused": _lib.PSI_FUSED}[mode]
    ws = _ws(grid, _lib.OP_PSI_PLAIN if m == _lib.PSI_PLAIN else _lib.OP_PSI_FUSED, r, 1, X.device)
    cnt = _L().kdefft_unique_count(d, r)
    out = torch.empty(max(cnt, 1), dtype=torch.float64, device=X.device)
    _lib.check(_L().kdefft_psi(_ptr(X), n, C.byref(grid), Gm.ctypes.data, r, _ptr(out), m, _ptr(ws), ws.numel(),
                               _stream(X.device)), "kdefft_psi")
    return out


def fftl_plan(grid: Grid, S, tau: float = 3.7):
    """(L, P) of the fft-L variant (Eq. (26)-(27)) for bandwidth S on grid."""
    d = grid.d
    Sm = _mat(S, d, "S")
    L = np.zeros(d, dtype=np.int32)
    P = np.zeros(d, dtype=np.int32)
    _lib.check(_L().kdefft_fftl_plan(C.byref(grid), Sm.ctypes.data, float(tau), L.ctypes.data, P.ctypes.data),
               "kdefft_fftl_plan")
    return L.tolist(), P.tolist()


def psi_fftl(X: torch.Tensor, G, r: int, M=None, grid: Optional[Grid] = None, tau: float = 3.7,
             pad_sd: float = 4.0):
    """psi_r(G) by the fft-L variant (kernel support cut to |l_k| <= L_k,
    transforms of the Eq. (27) lengths); returns (psi, L, P)."""
    X = _as_X(X)
    n, d = X.shape
    Gm = _mat(G, d, "G")
    if grid is None:
        if M is None:
            raise ValueError("give M or grid")
        grid = grid_auto(X, Gm, M, pad_sd)
    ws = _ws(grid, _lib.OP_PSI_FFTL, r, 1, X.device)
    cnt = _L().kdefft_unique_count(d, r)
    out = torch.empty(max(cnt, 1), dtype=torch.float64, device=X.device)
    L = np.zeros(d, dtype=np.int32)
    P = np.zeros(d, dtype=np.int32)
    _lib.check(_L().kdefft_psi_fftl(_ptr(X), n, C.byref(grid), Gm.ctypes.data, r, float(tau), _ptr(out),
                                    L.ctypes.data, P.ctypes.data, _ptr(ws), ws.numel(), _stream(X.device)),
               "kdefft_psi_fftl")
    return out, L.tolist(), P.tolist()


class Dataset:
    """A sample binned on a grid and transformed once (counts, spectra,
    autocorrelation, constant SCV term).  Without an explicit grid the grid is
    planned on the device (no host round trip); ``grid`` reads it back on first
    use."""

    def __init__(self, X: torch.Tensor, G_pilot, M=None, grid: Optional[Grid] = None, pad_sd: float = 4.0):
        X = _as_X(X)
        n, d = X.shape
        self.G_pilot = _mat(G_pilot, d, "G_pilot")
        self.device = X.device
        self.n = n
        self.d = d
        self.desc = _lib.Dataset()
        if grid is None:
            if M is None:
                raise ValueError("give M or grid")
            Ms = np.broadcast_to(np.asarray(M, dtype=np.int32), (d,)).copy()
            shape = grid_plan(Ms, [0.0] * d, [1.0] * d)
            nb = C.c_size_t()
            _lib.check(_L().kdefft_dataset_bytes(C.byref(shape), C.byref(nb)), "kdefft_dataset_bytes")
            self.mem = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=X.device)
            base = self.mem.data_ptr()
            off = (-base) % 256
            ws = _ws(shape, _lib.OP_PREPARE_AUTO, 0, n, X.device)
            _lib.check(_L().kdefft_dataset_prepare_auto(_ptr(X), n, d, Ms.ctypes.data, float(pad_sd),
                                                        self.G_pilot.ctypes.data, C.c_void_p(base + off),
                                                        int(nb.value), C.byref(self.desc), _ptr(ws), ws.numel(),
                                                        _stream(X.device)), "kdefft_dataset_prepare_auto")
            self.shape_grid = shape
            self._grid = None
        else:
            nb = C.c_size_t()
            _lib.check(_L().kdefft_dataset_bytes(C.byref(grid), C.byref(nb)), "kdefft_dataset_bytes")
            self.mem = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=X.device)
            base = self.mem.data_ptr()
            off = (-base) % 256
            ws = _ws(grid, _lib.OP_PREPARE, 0, 1, X.device)
            _lib.check(_L().kdefft_dataset_prepare(_ptr(X), n, C.byref(grid), self.G_pilot.ctypes.data,
                                                   C.c_void_p(base + off), int(nb.value), C.byref(self.desc),
                                                   _ptr(ws), ws.numel(), _stream(X.device)), "kdefft_dataset_prepare")
            self.shape_grid = grid
            self._grid = grid

    @property
    def grid(self) -> Grid:
        """The grid with its origin and spacing; a device-planned grid is read
        back once (one stream synchronisation) and kept in the descriptor, so
        later calls that need it on the host (the plain path) do not wait."""
        if self._grid is None:
            g = Grid()
            _lib.check(_L().kdefft_dataset_grid(C.byref(self.desc), C.byref(g), _stream(self.device)),
                       "kdefft_dataset_grid")
            self._grid = g
            self.desc.grid = g
        return self._grid

    @property
    def q(self):
        return self.d * (self.d + 1) // 2

    def out_of_grid(self) -> int:
        v = C.c_int32()
        rc = _L().kdefft_check_binning(C.c_void_p(self.desc.n_out), C.byref(v), _stream(self.device))
        if rc not in (_lib.OK, _lib.E_OUT_OF_GRID):
            _lib.check(rc, "kdefft_check_binning")
        return int(v.value)

    def lag_array(self) -> torch.Tensor:
        """Copy of the prepared lag array: prod P times the count
        autocorrelation, lag l at index l mod P (float64 [P_0, ..., P_{d-1}];
        exact zeros where the last-axis lag exceeds M - 1)."""
        shape = tuple(self.shape_grid.P[:self.d])
        numel = int(np.prod(shape))
        start = self.desc.alag - self.mem.data_ptr()
        return self.mem[start:start + 8 * numel].view(torch.float64).view(shape).clone()

    def transform(self):
        """Recompute the count transform (spectrum, mixed spectrum, lag array)
        from the counts with the current FFT schedule (kdefft_dataset_transform)."""
        _lib.check(_L().kdefft_dataset_transform(C.byref(self.desc), _stream(self.device)),
                   "kdefft_dataset_transform")

    def counts(self) -> torch.Tensor:
        """Copy of the int64 grid counts."""
        shape = tuple(self.shape_grid.M[:self.d])
        numel = int(np.prod(shape))
        base = self.mem.data_ptr()
        start = self.desc.counts - base
        return self.mem[start:start + 8 * numel].view(torch.int64).view(shape).clone()


def _ds_array(datasets: Sequence[Dataset]):
    arr = (_lib.Dataset * len(datasets))()
    for j, ds in enumerate(datasets):
        arr[j] = ds.desc
    return arr


def psi_batch(datasets: Sequence[Dataset], Gs, r: int) -> torch.Tensor:
    """psi_r at Gs[j] for each prepared dataset j, one launch (up to 32 datasets per call)."""
    datasets = list(datasets)
    d = datasets[0].d
    dev = datasets[0].device
    cnt = _L().kdefft_unique_count(d, r)
    out = torch.empty((len(datasets), max(cnt, 1)), dtype=torch.float64, device=dev)
    for s in range(0, len(datasets), _lib.MAX_PSI_DS):
        part = datasets[s:s + _lib.MAX_PSI_DS]
        Gh = np.zeros((len(part), 16))
        for j in range(len(part)):
            Gh[j, :d * d] = _mat(Gs[s + j], d, "G").ravel()
        ws = _ws(part[0].shape_grid, _lib.OP_PSI_BATCH, r, len(part), dev)
        arr = _ds_array(part)
        _lib.check(_L().kdefft_psi_batch(arr, len(part), Gh.ctypes.data, r, _ptr(out[s:s + len(part)]), _ptr(ws),
                                         ws.numel(), _stream(dev)), "kdefft_psi_batch")
    return out


def _offsets(datasets, counts):
    off = np.zeros(len(datasets) + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    return off


def _split_counts(datasets, vechL, per_ds):
    if per_ds is None:
        if len(datasets) != 1:
            raise ValueError("give per_ds (candidates per dataset) for several datasets")
        per_ds = [vechL.shape[0]]
    per_ds = [int(c) for c in per_ds]
    if sum(per_ds) != vechL.shape[0]:
        raise ValueError("per_ds must add up to the number of candidates")
    return per_ds


CRIT_SCV, CRIT_LSCV, CRIT_LSCV_EXACT, CRIT_QR, CRIT_PI = 0, 1, 2, 3, 4
_CRIT_NAMES = {"scv": CRIT_SCV, "lscv": CRIT_LSCV, "lscv_exact": CRIT_LSCV_EXACT, "qr": CRIT_QR, "pi": CRIT_PI}
# outcomes of minimize (include/kdefft.h KDEFFT_MIN_*)
MIN_CONVERGED, MIN_RUNNING, MIN_STALLED, MIN_BAD_START = 0, 1, 2, 3


def _crit_code(crit):
    if isinstance(crit, str):
        return _CRIT_NAMES[crit]
    return int(crit)


def crit(datasets: Sequence[Dataset], vechL: torch.Tensor, crit="scv", r: int = 0, per_ds=None,
         grad: bool = True, status: bool = False):
    """Batched criterion ("scv", "lscv", "lscv_exact" or "qr", include/kdefft.h)
    for candidates vechL [B, q] (H = L L^T; for "qr" the matrix S itself);
    candidates are grouped by dataset in order, per_ds[j] of them for dataset j.
    Gradients (d/d vechL) exist for r = 0 and the SCV / LSCV criteria."""
    code = _crit_code(crit)
    datasets = list(datasets)
    dev = datasets[0].device
    vechL = vechL.to(device=dev, dtype=torch.float64).contiguous()
    B, q = vechL.shape
    per_ds = _split_counts(datasets, vechL, per_ds)
    obj = torch.empty(B, dtype=torch.float64, device=dev)
    g = torch.empty((B, q), dtype=torch.float64, device=dev) if grad else None
    st = torch.empty(B, dtype=torch.int32, device=dev)
    start = 0
    for s in range(0, len(datasets), _lib.MAX_BATCH_DS):
        part = datasets[s:s + _lib.MAX_BATCH_DS]
        cnts = per_ds[s:s + _lib.MAX_BATCH_DS]
        nb = sum(cnts)
        if nb == 0:
            continue
        off = _offsets(part, cnts)
        ws = _ws(part[0].shape_grid, _lib.OP_SCV_BATCH, 2, nb, dev)
        arr = _ds_array(part)
        sl = slice(start, start + nb)
        _lib.check(_L().kdefft_crit_batch(arr, len(part), off.ctypes.data, _ptr(vechL[sl]), code, int(r),
                                          _ptr(obj[sl]), _ptr(g[sl]) if grad else None, _ptr(st[sl]), _ptr(ws),
                                          ws.numel(), _stream(dev)), "kdefft_crit_batch")
        start += nb
    if status:
        return obj, g, st
    return (obj, g) if grad else obj


def crit_adjoint(datasets: Sequence[Dataset], vechL: torch.Tensor, grad_out: torch.Tensor, crit="scv",
                 per_ds=None):
    """grad_out[b] * d crit(H_b) / d vechL_b (r = 0, SCV / LSCV criteria)."""
    code = _crit_code(crit)
    datasets = list(datasets)
    dev = datasets[0].device
    vechL = vechL.to(device=dev, dtype=torch.float64).contiguous()
    grad_out = grad_out.to(device=dev, dtype=torch.float64).contiguous()
    B, q = vechL.shape
    per_ds = _split_counts(datasets, vechL, per_ds)
    out = torch.empty((B, q), dtype=torch.float64, device=dev)
    start = 0
    for s in range(0, len(datasets), _lib.MAX_BATCH_DS):
        part = datasets[s:s + _lib.MAX_BATCH_DS]
        cnts = per_ds[s:s + _lib.MAX_BATCH_DS]
        nb = sum(cnts)
        if nb == 0:
            continue
        off = _offsets(part, cnts)
        ws = _ws(part[0].shape_grid, _lib.OP_SCV_BATCH, 2, nb, dev)
        arr = _ds_array(part)
        sl = slice(start, start + nb)
        if code == CRIT_SCV:
            rc = _L().kdefft_scv_adjoint(arr, len(part), off.ctypes.data, _ptr(vechL[sl]), _ptr(grad_out[sl]),
                                         _ptr(out[sl]), _ptr(ws), ws.numel(), _stream(dev))
            _lib.check(rc, "kdefft_scv_adjoint")
        else:
            rc = _L().kdefft_crit_adjoint(arr, len(part), off.ctypes.data, _ptr(vechL[sl]), code,
                                          _ptr(grad_out[sl]), _ptr(out[sl]), _ptr(ws), ws.numel(), _stream(dev))
            _lib.check(rc, "kdefft_crit_adjoint")
        start += nb
    return out


def scv(datasets: Sequence[Dataset], vechL: torch.Tensor, per_ds=None, grad: bool = True, status: bool = False):
    """SCV objective (and d/d vechL) for candidates vechL [B, q]; candidates are
    grouped by dataset in order, per_ds[j] of them for dataset j."""
    datasets = list(datasets)
    dev = datasets[0].device
    vechL = vechL.to(device=dev, dtype=torch.float64).contiguous()
    B, q = vechL.shape
    per_ds = _split_counts(datasets, vechL, per_ds)
    obj = torch.empty(B, dtype=torch.float64, device=dev)
    g = torch.empty((B, q), dtype=torch.float64, device=dev) if grad else None
    st = torch.empty(B, dtype=torch.int32, device=dev)
    start = 0
    for s in range(0, len(datasets), _lib.MAX_BATCH_DS):
        part = datasets[s:s + _lib.MAX_BATCH_DS]
        cnts = per_ds[s:s + _lib.MAX_BATCH_DS]
        nb = sum(cnts)
        if nb == 0:
            continue
        off = _offsets(part, cnts)
        ws = _ws(part[0].shape_grid, _lib.OP_SCV_BATCH, 2, nb, dev)
        arr = _ds_array(part)
        sl = slice(start, start + nb)
        _lib.check(_L().kdefft_scv_batch(arr, len(part), off.ctypes.data, _ptr(vechL[sl]), _ptr(obj[sl]),
                                         _ptr(g[sl]) if grad else None, _ptr(st[sl]), _ptr(ws), ws.numel(),
                                         _stream(dev)), "kdefft_scv_batch")
        start += nb
    if status:
        return obj, g, st
    return (obj, g) if grad else obj


def scv_walk_runs(datasets: Sequence[Dataset], vechL: torch.Tensor, per_ds=None) -> int:
    """Runs the compacted lag walk visits for the SCV objective + gradient of
    these candidates (kdefft_scv_walk_runs; synchronizes)."""
    datasets = list(datasets)
    if len(datasets) > _lib.MAX_BATCH_DS:
        raise ValueError(f"at most {_lib.MAX_BATCH_DS} datasets per call")
    dev = datasets[0].device
    vechL = vechL.to(device=dev, dtype=torch.float64).contiguous()
    per_ds = _split_counts(datasets, vechL, per_ds)
    off = _offsets(datasets, per_ds)
    ws = _ws(datasets[0].shape_grid, _lib.OP_SCV_BATCH, 2, vechL.shape[0], dev)
    out = C.c_int64()
    _lib.check(_L().kdefft_scv_walk_runs(_ds_array(datasets), len(datasets), off.ctypes.data, _ptr(vechL),
                                         C.byref(out), _ptr(ws), ws.numel(), _stream(dev)), "kdefft_scv_walk_runs")
    return int(out.value)


def scv_batch_noalloc(datasets: Sequence[Dataset], vechL: torch.Tensor, obj: torch.Tensor,
                      grad: Optional[torch.Tensor] = None, status: Optional[torch.Tensor] = None, per_ds=None):
    """kdefft_scv_batch_noalloc: the batched SCV objective (and gradient) into the
    caller's obj [B] (and grad [B, q], status [B]) with the library's fixed
    device scratch as workspace; allocates nothing (up to 64 datasets)."""
    datasets = list(datasets)
    if len(datasets) > _lib.MAX_BATCH_DS:
        raise ValueError(f"at most {_lib.MAX_BATCH_DS} datasets per call")
    dev = datasets[0].device
    per_ds = _split_counts(datasets, vechL, per_ds)
    off = _offsets(datasets, per_ds)
    arr = _ds_array(datasets)
    _lib.check(_L().kdefft_scv_batch_noalloc(arr, len(datasets), off.ctypes.data, _ptr(vechL), _ptr(obj),
                                             _ptr(grad), _ptr(status), _stream(dev)), "kdefft_scv_batch_noalloc")


def scv_adjoint(datasets: Sequence[Dataset], vechL: torch.Tensor, grad_out: torch.Tensor, per_ds=None):
    return crit_adjoint(datasets, vechL, grad_out, "scv", per_ds)


def minimize(vechL0: torch.Tensor, crit="scv", datasets: Optional[Sequence[Dataset]] = None, per_ds=None,
             psi4: Optional[torch.Tensor] = None, ns: Optional[Sequence[int]] = None, evals: int = 80,
             tol: float = 1e-9):
    """kdefft_minimize: quasi-Newton minimisation of the criterion ("scv",
    "lscv", "lscv_exact" on prepared datasets, or "pi" from psi4 [n_ds, C(d+3,4)]
    and sample sizes ns) from each starting point vechL0 [B, q] independently,
    `evals` batched evaluations enqueued without host synchronisation.
    Returns (vechL [B, q], crit values [B], info [B, 2] = (outcome, accepted
    steps)); outcomes MIN_CONVERGED / MIN_RUNNING / MIN_STALLED / MIN_BAD_START."""
    import ctypes as C
    code = _crit_code(crit)
    if code == CRIT_PI:
        if psi4 is None or ns is None:
            raise ValueError("the PI criterion needs psi4 and ns")
        dev = psi4.device
        psi4 = psi4.to(dtype=torch.float64).contiguous()
        nn = np.array([int(v) for v in ns], dtype=np.int64)
        nds = len(nn)
        arr, grid_p = None, None
    else:
        datasets = list(datasets)
        if len(datasets) > _lib.MAX_BATCH_DS:
            raise ValueError(f"at most {_lib.MAX_BATCH_DS} datasets per call")
        dev = datasets[0].device
        nds = len(datasets)
        arr = _ds_array(datasets)
        grid_p = C.byref(datasets[0].shape_grid)
        nn = None
    x0 = vechL0.to(device=dev, dtype=torch.float64).contiguous()
    B, q = x0.shape
    d = int(round((np.sqrt(8 * q + 1) - 1) / 2))
    if per_ds is None:
        if nds != 1:
            raise ValueError("give per_ds (candidates per dataset) for several datasets")
        per_ds = [B]
    per_ds = [int(c) for c in per_ds]
    if sum(per_ds) != B or len(per_ds) != nds:
        raise ValueError("per_ds must have one count per dataset and add up to B")
    off = np.zeros(nds + 1, dtype=np.int64)
    off[1:] = np.cumsum(per_ds)
    need = C.c_size_t()
    _lib.check(_L().kdefft_minimize_ws_bytes(grid_p, d, B, C.byref(need)), "kdefft_minimize_ws_bytes")
    ws = torch.empty(max(int(need.value), 256), dtype=torch.uint8, device=dev)
    x = torch.empty((B, q), dtype=torch.float64, device=dev)
    f = torch.empty(B, dtype=torch.float64, device=dev)
    info = torch.empty((B, 2), dtype=torch.int32, device=dev)
    _lib.check(_L().kdefft_minimize(arr, nds, off.ctypes.data, code, d,
                                    nn.ctypes.data if nn is not None else None,
                                    _ptr(psi4) if code == CRIT_PI else None, _ptr(x0), int(evals), float(tol),
                                    _ptr(x), _ptr(f), _ptr(info), _ptr(ws), ws.numel(), _stream(dev)),
               "kdefft_minimize")
    return x, f, info


def pi(psi4: torch.Tensor, ns: Sequence[int], vechL: torch.Tensor, per_ds=None, grad: bool = True,
       status: bool = False):
    """Plug-in criterion for candidates vechL [B, q] from psi_4 [n_ds, C(d+3,4)]
    of each dataset (sample sizes ns), candidates grouped by dataset in order."""
    dev = psi4.device
    psi4 = psi4.to(dtype=torch.float64).contiguous()
    vechL = vechL.to(device=dev, dtype=torch.float64).contiguous()
    B, q = vechL.shape
    d = int(round((np.sqrt(8 * q + 1) - 1) / 2))
    ns = [int(v) for v in ns]
    if per_ds is None:
        if len(ns) != 1:
            raise ValueError("give per_ds (candidates per dataset) for several datasets")
        per_ds = [B]
    per_ds = [int(c) for c in per_ds]
    if sum(per_ds) != B or len(per_ds) != len(ns) or psi4.shape[0] != len(ns):
        raise ValueError("per_ds, ns and psi4 must describe the same datasets and add up to B")
    obj = torch.empty(B, dtype=torch.float64, device=dev)
    g = torch.empty((B, q), dtype=torch.float64, device=dev) if grad else None
    st = torch.empty(B, dtype=torch.int32, device=dev)
    start = 0
    for s in range(0, len(ns), _lib.MAX_BATCH_DS):
        cnts = per_ds[s:s + _lib.MAX_BATCH_DS]
        nb = sum(cnts)
        if nb == 0:
            continue
        nn = np.array(ns[s:s + _lib.MAX_BATCH_DS], dtype=np.int64)
        off = np.zeros(len(cnts) + 1, dtype=np.int64)
        off[1:] = np.cumsum(cnts)
        sl = slice(start, start + nb)
        _lib.check(_L().kdefft_pi_batch(d, len(cnts), nn.ctypes.data, _ptr(psi4[s:s + len(cnts)]),
                                        off.ctypes.data, _ptr(vechL[sl]), _ptr(obj[sl]),
                                        _ptr(g[sl]) if grad else None, _ptr(st[sl]), _stream(dev)),
                   "kdefft_pi_batch")
        start += nb
    if status:
        return obj, g, st
    return (obj, g) if grad else obj


def expand_full(vals, d: int, r: int) -> np.ndarray:
    """Unique entries -> the d^r Kronecker-ordered vector (host)."""
    u = np.ascontiguousarray(np.asarray(vals, dtype=np.float64))
    out = np.empty(d ** r, dtype=np.float64)
    _lib.check(_L().kdefft_expand_full(d, r, u.ctypes.data, out.ctypes.data), "kdefft_expand_full")
    return out


def scv_plain(dataset: Dataset, H) -> torch.Tensor:
    """[SCV(H), d SCV / d vechL] for one H by the paper's literal steps."""
    Hm = _mat(H, dataset.d, "H")
    ws = _ws(dataset.shape_grid, _lib.OP_SCV_PLAIN, 2, 1, dataset.device)
    out = torch.empty(1 + dataset.q, dtype=torch.float64, device=dataset.device)
    arr = _ds_array([dataset])
    _lib.check(_L().kdefft_scv_plain(arr, Hm.ctypes.data, _ptr(out), _ptr(ws), ws.numel(), _stream(dataset.device)),
               "kdefft_scv_plain")
    return out


class Criterion(torch.autograd.Function):
    """obj[b] = crit(H_b) (SCV or LSCV at r = 0); backward runs the adjoint
    kernel (Hessian grids recomputed, never stored)."""

    @staticmethod
    def forward(ctx, vechL, dataset, crit_name="lscv", per_ds=None):
        datasets = dataset if isinstance(dataset, (list, tuple)) else [dataset]
        obj = crit(datasets, vechL.detach(), crit_name, 0, per_ds=per_ds, grad=False)
        ctx.datasets = datasets
        ctx.per_ds = per_ds
        ctx.crit = crit_name
        ctx.save_for_backward(vechL.detach())
        return obj

    @staticmethod
    def backward(ctx, grad_out):
        (vechL,) = ctx.saved_tensors
        g = crit_adjoint(ctx.datasets, vechL, grad_out.detach(), ctx.crit, per_ds=ctx.per_ds)
        return g, None, None, None


class PI(torch.autograd.Function):
    """obj[b] = PI(H_b) from psi_4; the exact gradient comes from the same
    launch and is kept for backward."""

    @staticmethod
    def forward(ctx, vechL, psi4, ns, per_ds=None):
        obj, g = pi(psi4, ns, vechL.detach(), per_ds=per_ds, grad=True)
        ctx.save_for_backward(g)
        return obj

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out[:, None] * g, None, None, None


class SCV(torch.autograd.Function):
    """obj[b] = SCV(H_b), H_b = L_b L_b^T from vechL [B, q]; backward runs the
    adjoint kernel (Hessian grids recomputed, never stored)."""

    @staticmethod
    def forward(ctx, vechL, dataset, per_ds=None):
        datasets = dataset if isinstance(dataset, (list, tuple)) else [dataset]
        obj = scv(datasets, vechL.detach(), per_ds=per_ds, grad=False)
        ctx.datasets = datasets
        ctx.per_ds = per_ds
        ctx.save_for_backward(vechL.detach())
        return obj

    @staticmethod
    def backward(ctx, grad_out):
        (vechL,) = ctx.saved_tensors
        g = scv_adjoint(ctx.datasets, vechL, grad_out.detach(), per_ds=ctx.per_ds)
        return g, None, None


def lag_layout(N: int, moments: bool = True):
    """(lags per run, runs per segment, rows per block pass) of the compiled
    lag-domain kernels for last-axis length N."""
    run, seg, rows = C.c_int(), C.c_int(), C.c_int()
    _lib.check(_L().kdefft_lag_layout(int(N), int(bool(moments)), C.byref(run), C.byref(seg), C.byref(rows)),
               "kdefft_lag_layout")
    return run.value, seg.value, rows.value


def set_row_launch(kind: int, d: int, r: int, N: int, variant: int, grid_blocks: int = 0):
    """Pin the batched launch of one kernel family and shape (variant -1 drops the pin)."""
    _lib.check(_L().kdefft_set_row_launch(kind, d, r, N, variant, grid_blocks), "kdefft_set_row_launch")


def get_row_launch(kind: int, d: int, r: int, N: int):
    """(variant, grid_blocks) the batched calls of this family and shape use now."""
    v, gb = C.c_int(), C.c_int()
    _lib.check(_L().kdefft_get_row_launch(kind, d, r, N, C.byref(v), C.byref(gb)), "kdefft_get_row_launch")
    return v.value, gb.value


FFT_SCHEDULES = _lib.FFT_SCHEDULES


def set_fft_schedule(P, sched: int):
    """Pin the count transform's FFT schedule for grids with last-axis lengths
    P (one entry per axis); sched -1 drops the pin (include/kdefft.h)."""
    Pa = np.asarray(P, dtype=np.int32)
    _lib.check(_L().kdefft_set_fft_schedule(len(Pa), Pa.ctypes.data, int(sched)), "kdefft_set_fft_schedule")


def get_fft_schedule(P) -> int:
    """The FFT schedule the count transform uses now for grids of lengths P."""
    Pa = np.asarray(P, dtype=np.int32)
    out = C.c_int()
    _lib.check(_L().kdefft_get_fft_schedule(len(Pa), Pa.ctypes.data, C.byref(out)), "kdefft_get_fft_schedule")
    return out.value


class fft_schedule:
    """Context manager: pin an FFT schedule for one grid shape, restore on exit."""

    def __init__(self, P, sched: int):
        self.P = list(P)
        self.sched = sched
        self.saved = None

    def __enter__(self):
        self.saved = get_fft_schedule(self.P)
        set_fft_schedule(self.P, self.sched)
        return self

    def __exit__(self, *exc):
        set_fft_schedule(self.P, self.saved)
        return False


class row_launch:
    """Context manager: pin (variant, grid_blocks) for the given families of
    one shape, and restore the previous choices on exit."""

    def __init__(self, kinds, d: int, r: int, N: int, variant: int, grid_blocks: int = 0):
        self.kinds = [kinds] if isinstance(kinds, int) else list(kinds)
        self.key = (d, r, N)
        self.launch = (variant, grid_blocks)
        self.saved = []

    def __enter__(self):
        d, r, N = self.key
        self.saved = [(k, get_row_launch(k, d, r, N)) for k in self.kinds]
        for k in self.kinds:
            set_row_launch(k, d, r, N, *self.launch)
        return self

    def __exit__(self, *exc):
        d, r, N = self.key
        for k, (v, gb) in self.saved:
            set_row_launch(k, d, r, N, v, gb)
        return False


def autotune(dataset: Dataset, cache_path: Optional[str] = None) -> str:
    ws = _ws(dataset.shape_grid, _lib.OP_AUTOTUNE, 2, 256, dataset.device)
    arr = _ds_array([dataset])
    _lib.check(_L().kdefft_autotune(arr, _ptr(ws), ws.numel(), cache_path.encode() if cache_path else None,
                                    _stream(dataset.device)), "kdefft_autotune")
    return _L().kdefft_last_error_detail().decode()


def timing_start(max_launches: int = 1024):
    """Arm the row-kernel timer for the next `max_launches` batched row launches."""
    _lib.check(_L().kdefft_timing_start(int(max_launches)), "kdefft_timing_start")


def timing_stop(cap: int = _lib.MAX_TIMED):
    """Disarm the timer; returns [(ms, family, r), ...] in launch order."""
    import ctypes as C
    ms = (C.c_float * cap)()
    tag = (C.c_int32 * cap)()
    cnt = C.c_int(0)
    _lib.check(_L().kdefft_timing_stop(ms, tag, cap, C.byref(cnt)), "kdefft_timing_stop")
    return [(float(ms[k]), int(tag[k]) // 16, int(tag[k]) % 16) for k in range(cnt.value)]
