"""Host-side checks of the C-ABI library (no GPU needed, nothing launched).

* the library loads and exports every function include/kdefft.h declares;
* the unique-index order, grid planning and padded sizes agree with the
  CPU reference bit for bit;
* invalid arguments return the documented error codes before any launch.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import grid as ogrid
from oracle import multiindex


def _declared(repo_root):
    txt = open(os.path.join(repo_root, "include", "kdefft.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(kdefft_[a-z_0-9]+)\s*\(", txt)))


def test_exports_every_declared_symbol(kf, repo_root):
    lib = kf._lib.load()
    names = _declared(repo_root)
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(kf._lib.EXPORTS)
    assert lib.kdefft_version() >= 10000


def test_strerror(kf):
    lib = kf._lib.load()
    for code in range(0, -9, -1):
        s = lib.kdefft_strerror(code).decode()
        assert s and s != "unknown error"


@pytest.mark.parametrize("d,r", [(1, 0), (1, 8), (2, 4), (2, 8), (3, 2), (3, 6), (4, 4)])
def test_unique_order(kf, d, r):
    got = kf.unique_tuples(d, r)
    want = multiindex.unique_tuples(d, r) if r else [()]
    assert got == want


def test_grid_plan_matches_oracle(kf):
    rng = np.random.default_rng(1)
    for d in (1, 2, 3, 4):
        for _ in range(20):
            lo = rng.standard_normal(d) * 10
            hi = lo + rng.random(d) * 7 + 1e-3
            M = rng.integers(2, {1: 2000, 2: 300, 3: 100, 4: 30}[d], size=d)
            g = kf.grid_plan(M, lo, hi).to_dict()
            o = ogrid.plan(lo, hi, M)
            assert np.array_equal(g["lo"], o["lo"])
            assert np.array_equal(g["delta"], o["delta"])     # bitwise
            assert np.array_equal(g["P"], o["P"])


def _grid(kf, d=2, M=16):
    return kf.grid_plan([M] * d, [0.0] * d, [1.0] * d)


def test_ws_bytes(kf):
    lib = kf._lib.load()
    g = _grid(kf, 2, 256)
    n = C.c_size_t()
    sizes = {}
    for op in range(1, 9):
        assert lib.kdefft_ws_bytes(C.byref(g), op, 4, 256, C.byref(n)) == 0
        sizes[op] = n.value
        assert n.value > 0
    assert sizes[kf._lib.OP_PSI_PLAIN] >= 2 * 512 * 512 * 8
    small, big = C.c_size_t(), C.c_size_t()
    lib.kdefft_ws_bytes(C.byref(g), kf._lib.OP_SCV_BATCH, 2, 16, C.byref(small))
    lib.kdefft_ws_bytes(C.byref(g), kf._lib.OP_SCV_BATCH, 2, 4096, C.byref(big))
    assert big.value > small.value
    assert lib.kdefft_ws_bytes(C.byref(g), 99, 0, 1, C.byref(n)) == kf._lib.E_ARG


def test_dataset_bytes(kf):
    lib = kf._lib.load()
    g = _grid(kf, 4, 32)
    n = C.c_size_t()
    assert lib.kdefft_dataset_bytes(C.byref(g), C.byref(n)) == 0
    assert n.value >= 32 ** 4 * 8 + 2 * 64 ** 3 * 33 * 16


def test_grid_validation(kf):
    lib = kf._lib.load()
    g = kf._lib.Grid()
    M = np.array([8, 8], dtype=np.int32)
    lo = np.zeros(2)
    hi = np.ones(2)
    assert lib.kdefft_grid_plan(5, M.ctypes.data, None, lo.ctypes.data, hi.ctypes.data, C.byref(g)) == kf._lib.E_ARG
    M1 = np.array([1, 8], dtype=np.int32)
    assert lib.kdefft_grid_plan(2, M1.ctypes.data, None, lo.ctypes.data, hi.ctypes.data, C.byref(g)) == kf._lib.E_ARG
    P = np.array([12, 16], dtype=np.int32)     # not a power of two
    assert lib.kdefft_grid_plan(2, M.ctypes.data, P.ctypes.data, lo.ctypes.data, hi.ctypes.data, C.byref(g)) == kf._lib.E_ARG
    P = np.array([8, 16], dtype=np.int32)      # 8 < 2*8-1
    assert lib.kdefft_grid_plan(2, M.ctypes.data, P.ctypes.data, lo.ctypes.data, hi.ctypes.data, C.byref(g)) == kf._lib.E_ARG
    bad = np.array([0.0, 2.0])
    assert lib.kdefft_grid_plan(2, M.ctypes.data, None, lo.ctypes.data, bad.ctypes.data, C.byref(g)) == kf._lib.E_ARG


def test_compute_entry_validation(kf):
    """Errors raised on the host before any launch (pointers are never touched)."""
    lib = kf._lib.load()
    L = kf._lib
    g = _grid(kf, 2, 16)
    fake = C.c_void_p(0x1000)
    G = np.array([[0.1, 0.02], [0.02, 0.2]])
    ws = C.c_void_p(0x100000)
    psi = lib.kdefft_psi
    assert psi(fake, 10, C.byref(g), G.ctypes.data, 3, fake, 0, ws, 1 << 30, None) == L.E_ODD_R
    assert psi(fake, 10, C.byref(g), G.ctypes.data, 10, fake, 0, ws, 1 << 30, None) == L.E_UNSUPPORTED
    assert psi(fake, 1 << 23, C.byref(g), G.ctypes.data, 2, fake, 0, ws, 1 << 30, None) == L.E_OVERFLOW
    assert psi(fake, 0, C.byref(g), G.ctypes.data, 2, fake, 0, ws, 1 << 30, None) == L.E_ARG
    assert psi(None, 10, C.byref(g), G.ctypes.data, 2, fake, 0, ws, 1 << 30, None) == L.E_ARG
    assert psi(fake, 10, C.byref(g), G.ctypes.data, 2, fake, 7, ws, 1 << 30, None) == L.E_ARG
    notspd = np.array([[0.1, 0.3], [0.3, 0.2]])
    assert psi(fake, 10, C.byref(g), notspd.ctypes.data, 2, fake, 0, ws, 1 << 30, None) == L.E_NOT_SPD
    asym = np.array([[0.1, 0.02], [0.03, 0.2]])
    assert psi(fake, 10, C.byref(g), asym.ctypes.data, 2, fake, 0, ws, 1 << 30, None) == L.E_NOT_SPD
    assert psi(fake, 10, C.byref(g), G.ctypes.data, 2, fake, 0, ws, 64, None) == L.E_WORKSPACE
    assert "workspace" in lib.kdefft_last_error_detail().decode()
    g3 = _grid(kf, 3, 8)
    G3 = np.eye(3)
    assert psi(fake, 10, C.byref(g3), G3.ctypes.data, 8, fake, 0, ws, 1 << 30, None) == L.E_UNSUPPORTED
    assert lib.kdefft_linbin(fake, 1 << 23, C.byref(g), fake, None, None) == L.E_OVERFLOW
    assert lib.kdefft_unique_count(5, 2) == L.E_ARG


def test_dataset_entry_validation(kf):
    lib = kf._lib.load()
    L = kf._lib
    g = _grid(kf, 2, 16)
    fake = C.c_void_p(0x1000)
    G = np.eye(2) * 0.1
    out = kf._lib.Dataset()
    # misaligned dataset buffer
    assert lib.kdefft_dataset_prepare(fake, 10, C.byref(g), G.ctypes.data, C.c_void_p(0x1008), 1 << 30,
                                      C.byref(out), fake, 1 << 30, None) == L.E_WORKSPACE
    # too small dataset buffer
    assert lib.kdefft_dataset_prepare(fake, 10, C.byref(g), G.ctypes.data, C.c_void_p(0x1000), 64,
                                      C.byref(out), fake, 1 << 30, None) == L.E_WORKSPACE
    # unprepared dataset in a batch
    ds = (kf._lib.Dataset * 1)()
    ds[0].grid = g
    ds[0].n = 10
    off = np.array([0, 4], dtype=np.int64)
    assert lib.kdefft_scv_batch(ds, 1, off.ctypes.data, fake, fake, None, None, fake, 1 << 30, None) == L.E_ARG
    assert lib.kdefft_set_row_launch(2, 2, 2, 512, 7, 0) == L.E_ARG
    assert lib.kdefft_set_row_launch(2, 2, 2, 512, -2, 0) == L.E_ARG
    assert lib.kdefft_set_row_launch(2, 2, 2, 3, 0, 0) == L.E_UNSUPPORTED


def test_timing_hook_validation(kf):
    """Out-of-range arming and bad output arrays fail before any HIP call;
    stopping an unarmed timer reports no launches."""
    lib = kf._lib.load()
    L = kf._lib
    assert lib.kdefft_timing_start(0) == L.E_ARG
    assert lib.kdefft_timing_start(L.MAX_TIMED + 1) == L.E_ARG
    cnt = C.c_int(-1)
    assert lib.kdefft_timing_stop(None, None, 4, C.byref(cnt)) == L.E_ARG
    assert lib.kdefft_timing_stop(None, None, 0, None) == L.E_ARG
    assert lib.kdefft_timing_stop(None, None, 0, C.byref(cnt)) == L.OK and cnt.value == 0
    assert kf.timing_stop() == []


def _fake_prepared(kf, d=2, M=16, n=100):
    """A dataset descriptor that passes the host checks (pointers never touched)."""
    ds = (kf._lib.Dataset * 1)()
    ds[0].grid = _grid(kf, d, M)
    ds[0].n = n
    for f in ("counts", "spec", "wmix", "alag", "scal", "n_out", "rec"):
        setattr(ds[0], f, 0x100000)
    return ds


def test_criterion_entry_validation(kf):
    lib = kf._lib.load()
    L = kf._lib
    ds = _fake_prepared(kf)
    fake = C.c_void_p(0x1000)
    off = np.array([0, 4], dtype=np.int64)
    cb = lib.kdefft_crit_batch
    # gradient only for r = 0 and the SCV / LSCV criteria
    assert cb(ds, 1, off.ctypes.data, fake, kf.CRIT_LSCV, 2, fake, fake, None, fake, 1 << 30, None) == L.E_UNSUPPORTED
    assert cb(ds, 1, off.ctypes.data, fake, kf.CRIT_QR, 0, fake, fake, None, fake, 1 << 30, None) == L.E_UNSUPPORTED
    assert cb(ds, 1, off.ctypes.data, fake, 7, 0, fake, None, None, fake, 1 << 30, None) == L.E_ARG
    assert cb(ds, 1, off.ctypes.data, fake, kf.CRIT_QR, 9, fake, None, None, fake, 1 << 30, None) == L.E_ARG
    assert cb(ds, 1, off.ctypes.data, fake, kf.CRIT_SCV, 2, fake, None, None, fake, 1 << 30, None) == L.E_UNSUPPORTED
    assert cb(ds, 1, off.ctypes.data, fake, kf.CRIT_LSCV, 0, None, None, None, fake, 1 << 30, None) == L.E_ARG
    assert cb(ds, 1, off.ctypes.data, fake, kf.CRIT_LSCV, 0, fake, None, None, fake, 64, None) == L.E_WORKSPACE
    ds1 = _fake_prepared(kf, n=1)
    assert cb(ds1, 1, off.ctypes.data, fake, kf.CRIT_LSCV_EXACT, 0, fake, None, None, fake, 1 << 30,
              None) == L.E_ARG
    ca = lib.kdefft_crit_adjoint
    assert ca(ds, 1, off.ctypes.data, fake, kf.CRIT_QR, fake, fake, fake, 1 << 30, None) == L.E_UNSUPPORTED
    assert ca(ds, 1, off.ctypes.data, fake, kf.CRIT_LSCV, None, fake, fake, 1 << 30, None) == L.E_ARG
    pb = lib.kdefft_pi_batch
    nn = np.array([100], dtype=np.int64)
    assert pb(5, 1, nn.ctypes.data, fake, off.ctypes.data, fake, fake, None, None, None) == L.E_ARG
    assert pb(2, 0, nn.ctypes.data, fake, off.ctypes.data, fake, fake, None, None, None) == L.E_ARG
    assert pb(2, 1, nn.ctypes.data, fake, off.ctypes.data, fake, None, None, None, None) == L.E_ARG
    bad = np.array([1, 4], dtype=np.int64)
    assert pb(2, 1, nn.ctypes.data, fake, bad.ctypes.data, fake, fake, None, None, None) == L.E_ARG
    n0 = np.array([0], dtype=np.int64)
    assert pb(2, 1, n0.ctypes.data, fake, off.ctypes.data, fake, fake, None, None, None) == L.E_ARG


def test_fft_schedule_table(kf):
    lib = kf._lib.load()
    L = kf._lib
    P = np.array([64, 128], dtype=np.int32)
    out = C.c_int(-5)
    assert lib.kdefft_get_fft_schedule(2, P.ctypes.data, C.byref(out)) == L.OK and out.value == 0
    for sched in range(kf.FFT_SCHEDULES):
        assert lib.kdefft_set_fft_schedule(2, P.ctypes.data, sched) == L.OK
        assert lib.kdefft_get_fft_schedule(2, P.ctypes.data, C.byref(out)) == L.OK and out.value == sched
    assert lib.kdefft_set_fft_schedule(2, P.ctypes.data, -1) == L.OK
    assert lib.kdefft_get_fft_schedule(2, P.ctypes.data, C.byref(out)) == L.OK and out.value == 0
    assert lib.kdefft_set_fft_schedule(2, P.ctypes.data, kf.FFT_SCHEDULES) == L.E_ARG
    assert lib.kdefft_set_fft_schedule(2, P.ctypes.data, -2) == L.E_ARG
    assert lib.kdefft_set_fft_schedule(5, P.ctypes.data, 0) == L.E_ARG
    bad = np.array([64, 96], dtype=np.int32)
    assert lib.kdefft_set_fft_schedule(2, bad.ctypes.data, 0) == L.E_ARG
    assert lib.kdefft_set_fft_schedule(2, None, 0) == L.E_ARG
    assert lib.kdefft_get_fft_schedule(2, P.ctypes.data, None) == L.E_ARG
    with kf.fft_schedule([64, 128], 3):
        assert kf.get_fft_schedule([64, 128]) == 3
    assert kf.get_fft_schedule([64, 128]) == 0


def test_minimize_entry_validation(kf):
    lib = kf._lib.load()
    L = kf._lib
    ds = _fake_prepared(kf)
    fake = C.c_void_p(0x1000)
    off = np.array([0, 4], dtype=np.int64)
    nn = np.array([100], dtype=np.int64)
    mz = lib.kdefft_minimize
    big = 1 << 30

    def call(crit=kf.CRIT_SCV, d=2, evals=10, tol=1e-9, ws_bytes=big, psi4=fake, offs=off, x_out=fake, dsa=ds):
        return mz(dsa, 1, offs.ctypes.data, crit, d, nn.ctypes.data, psi4, fake, evals, tol, x_out, None, None,
                  fake, ws_bytes, None)

    assert call(evals=0) == L.E_ARG
    assert call(evals=100001) == L.E_ARG
    assert call(tol=0.0) == L.E_ARG
    assert call(tol=float("nan")) == L.E_ARG
    assert call(crit=kf.CRIT_QR) == L.E_ARG       # no gradient
    assert call(crit=9) == L.E_ARG
    assert call(x_out=None) == L.E_ARG
    assert call(offs=np.array([1, 4], dtype=np.int64)) == L.E_ARG
    assert call(offs=np.array([0, 0], dtype=np.int64)) == L.E_ARG
    assert call(ws_bytes=64) == L.E_WORKSPACE
    assert call(crit=kf.CRIT_PI, d=5, dsa=None) == L.E_ARG
    assert call(crit=kf.CRIT_PI, psi4=None, dsa=None) == L.E_ARG
    assert call(crit=kf.CRIT_PI, ws_bytes=64, dsa=None) == L.E_WORKSPACE
    n = C.c_size_t()
    assert lib.kdefft_minimize_ws_bytes(None, 2, 8, C.byref(n)) == L.OK and n.value > 8 * 8 * 8
    pi_only = n.value
    g = kf.grid_plan([32, 32], lo=[0.0, 0.0], hi=[1.0, 1.0])
    assert lib.kdefft_minimize_ws_bytes(C.byref(g), 0, 8, C.byref(n)) == L.OK and n.value > pi_only
    assert lib.kdefft_minimize_ws_bytes(None, 0, 8, C.byref(n)) == L.E_ARG
    assert lib.kdefft_minimize_ws_bytes(None, 2, 0, C.byref(n)) == L.E_ARG


@pytest.mark.parametrize("d,r", [(1, 0), (1, 4), (2, 0), (2, 4), (3, 2), (3, 4), (4, 4), (2, 8), (4, 3)])
def test_expand_full_matches_oracle(kf, d, r):
    u = np.arange(1, multiindex.n_unique(d, r) + 1, dtype=np.float64) * 1.5
    np.testing.assert_array_equal(kf.expand_full(u, d, r), multiindex.expand_full(u, d, r))


def test_fftl_plan_table2_from_table3(kf, repo_root):
    """The library's Eq. (27) turns Table 3's L values into Table 2's P values:
    pick S and delta so that Eq. (26) returns exactly the printed L."""
    from test_oracle_fftl import _tables
    L, P = _tables(repo_root)
    for (n, M) in sorted(set(L) & set(P)):
        # axis spacings chosen so that 3.7 * sqrt(1) / delta_k is just below L_k
        lo = np.zeros(2)
        hi = np.array([3.7 / (L[(n, M)][0] - 0.5) * (M - 1), 3.7 / (L[(n, M)][1] - 0.5) * (M - 1)])
        g = kf.grid_plan([M, M], lo, hi)
        Lg, Pg = kf.fftl_plan(g, np.eye(2))
        assert tuple(Lg) == L[(n, M)] and tuple(Pg) == P[(n, M)], (n, M, Lg, Pg)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_fftl_plan_matches_oracle(kf, d):
    from oracle import fftl
    rng = np.random.default_rng(60 + d)
    checked = 0
    for t in range(40):
        M = [int(m) for m in rng.integers(8, 200 if d <= 2 else 40, size=d)]
        lo = rng.normal(size=d)
        hi = lo + rng.uniform(1.0, 6.0, size=d)
        g = kf.grid_plan(M, lo, hi)
        Q, _ = np.linalg.qr(rng.normal(size=(d, d)))
        S = Q @ np.diag(10 ** rng.uniform(-3, 0, d)) @ Q.T
        S = 0.5 * (S + S.T)
        tau = float(rng.uniform(2.0, 5.0))
        gd = g.to_dict()
        lam = float(np.max(np.linalg.eigvalsh(S)))
        ratios = tau * np.sqrt(lam) / gd["delta"]
        if np.any(np.abs(ratios - np.round(ratios)) < 1e-9):
            continue   # a ceiling at an exact integer could round either way
        Lg, Pg = kf.fftl_plan(g, S, tau)
        Lo = fftl.plan_L(gd, S, tau)
        assert Lg == Lo and Pg == fftl.plan_P(M, Lo), (M, Lg, Lo)
        checked += 1
    assert checked >= 30


def test_prepare_auto_validation(kf):
    lib = kf._lib.load()
    L = kf._lib
    fake = C.c_void_p(0x1000)
    M = np.array([16, 16], dtype=np.int32)
    G = np.eye(2) * 0.1
    out = kf._lib.Dataset()
    pa = lib.kdefft_dataset_prepare_auto
    assert pa(None, 10, 2, M.ctypes.data, 4.0, G.ctypes.data, fake, 1 << 30, C.byref(out), fake, 1 << 30,
              None) == L.E_ARG
    assert pa(fake, 10, 5, M.ctypes.data, 4.0, G.ctypes.data, fake, 1 << 30, C.byref(out), fake, 1 << 30,
              None) == L.E_ARG
    assert pa(fake, 10, 2, M.ctypes.data, -1.0, G.ctypes.data, fake, 1 << 30, C.byref(out), fake, 1 << 30,
              None) == L.E_ARG
    bad = np.array([[0.1, 0.3], [0.3, 0.1]])
    assert pa(fake, 10, 2, M.ctypes.data, 4.0, bad.ctypes.data, fake, 1 << 30, C.byref(out), fake, 1 << 30,
              None) == L.E_NOT_SPD
    assert pa(fake, 10, 2, M.ctypes.data, 4.0, G.ctypes.data, C.c_void_p(0x1008), 1 << 30, C.byref(out), fake,
              1 << 30, None) == L.E_WORKSPACE
    assert pa(fake, 10, 2, M.ctypes.data, 4.0, G.ctypes.data, fake, 64, C.byref(out), fake, 1 << 30,
              None) == L.E_WORKSPACE
    assert pa(fake, 10, 2, M.ctypes.data, 4.0, G.ctypes.data, fake, 1 << 30, C.byref(out), fake, 64,
              None) == L.E_WORKSPACE
    assert lib.kdefft_dataset_grid(None, C.byref(kf._lib.Grid()), None) == L.E_ARG
