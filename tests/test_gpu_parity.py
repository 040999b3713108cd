"""Parity of the HIP path with the CPU oracle (GPU, through the C-ABI).

* binning: int64 counts bit-identical to oracle.linbin (every case shape,
  ragged grids, the hand-derived fixture, out-of-grid counting);
* grid planning: bitwise identical lo/delta;
* psi_r: FFT route (paper-literal plain path and the fused Parseval path) vs
  the oracle's direct lag-domain binned sum, <= 1e-11 relative per entry;
* full-size workloads (d=2 n=1e5 M=256 r=4; d=3 n=2e5 M=64 r=2) at the same
  launch configuration the benchmark uses.
"""
import os

import numpy as np
import pytest
import torch

import synth
from oracle import binned, grid, linbin, multiindex

from _gpu_util import assert_psi_close, log, mixture_sample, oracle_autocorr, spd

pytestmark = pytest.mark.gpu

_AC = {}


def _case(name, X, G, M):
    """Oracle side of a case: grid, counts, real counts, autocorrelation (cached)."""
    if name not in _AC:
        g = grid.plan_auto(X, G, [M] * X.shape[1])
        counts, skipped = linbin.linbin(X, g)
        c = linbin.counts_to_real(counts)
        _AC[name] = (g, counts, skipped, c, oracle_autocorr(c))
    return _AC[name]


def _to_dev(X, dev):
    return torch.from_numpy(np.ascontiguousarray(X)).to(dev)


CASES = {
    "d1": lambda: (mixture_sample(5000, 1, 1), spd(1, 1, 0.05), 100),
    "d2_case1": lambda: (synth.case1().X[0], synth.case1().G_psi[0], 64),
    "d2_ragged": lambda: (mixture_sample(2000, 2, 2), spd(2, 2), 37),
    "d3": lambda: (mixture_sample(3000, 3, 3), spd(3, 3), 20),
    "d4": lambda: (mixture_sample(2000, 4, 4), spd(4, 4, 0.2), 8),
    "d4_m12": lambda: (mixture_sample(4000, 4, 5), spd(4, 5, 0.2), 12),
}


@pytest.mark.parametrize("name", list(CASES))
def test_grid_and_linbin_bitexact(kf, gpu, name):
    X, G, M = CASES[name]()
    log(f"[linbin] case={name} n={X.shape[0]} d={X.shape[1]} M={M}")
    g_o, counts_o, skipped, _, _ = _case(name, X, G, M)
    Xd = _to_dev(X, gpu)
    g = kf.grid_auto(Xd, G, M)
    gd = g.to_dict()
    assert np.array_equal(gd["lo"], g_o["lo"]) and np.array_equal(gd["delta"], g_o["delta"])
    counts, nout = kf.linbin(Xd, g)
    torch.cuda.synchronize()
    assert skipped == 0 and int(nout.item()) == 0
    np.testing.assert_array_equal(counts.cpu().numpy(), counts_o)


@pytest.mark.parametrize("name", list(CASES))
def test_prepare_auto_bitexact(kf, gpu, name):
    """A dataset planned on the device (no host round trip) has the host
    planner's grid bit for bit and the oracle's counts."""
    X, G, M = CASES[name]()
    g_o, counts_o, skipped, _, _ = _case(name, X, G, M)
    ds = kf.Dataset(_to_dev(X, gpu), G, M=M)
    gd = ds.grid.to_dict()
    assert np.array_equal(gd["lo"], g_o["lo"]) and np.array_equal(gd["delta"], g_o["delta"])
    np.testing.assert_array_equal(ds.counts().cpu().numpy(), counts_o)
    assert ds.out_of_grid() == 0


def test_prepare_auto_nonfinite_data(kf, gpu):
    """A NaN coordinate is ignored by the bounds and its point is counted out
    of the grid (as on the host path); an infinite one leaves no valid grid:
    every point is counted out and reading the grid back reports the error."""
    X = np.random.default_rng(3).normal(size=(500, 2))
    X[7, 1] = np.nan
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), np.eye(2) * 0.1, M=16)
    assert ds.out_of_grid() == 1
    g_o = grid.plan_auto(np.delete(X, 7, axis=0), np.eye(2) * 0.1, [16, 16])
    assert np.array_equal(ds.grid.to_dict()["delta"], g_o["delta"])
    X[7, 1] = np.inf
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), np.eye(2) * 0.1, M=16)
    assert ds.out_of_grid() == 500
    with pytest.raises(kf.KdefftError):
        ds.grid


@pytest.mark.parametrize("name", list(CASES))
def test_lag_array_vs_oracle(kf, gpu, name):
    """The prepared lag array against the oracle's direct autocorrelation of
    the same counts (every lag with |l_k| <= M_k - 1), and exact zeros at the
    last-axis positions beyond M - 1."""
    X, G, M = CASES[name]()
    log(f"[lag array] case={name} n={X.shape[0]} d={X.shape[1]} M={M}")
    _, _, _, _, A = _case(name, X, G, M)
    Xd = _to_dev(X, gpu)
    g = kf.grid_auto(Xd, G, M)
    ds = kf.Dataset(Xd, G, grid=g)
    al = ds.lag_array().cpu().numpy()
    d = X.shape[1]
    P = [int(p) for p in g.P[:d]]
    Mv = [int(m) for m in g.M[:d]]
    idx = [np.arange(-(m - 1), m) % p for m, p in zip(Mv, P)]
    got = al[np.ix_(*idx)] / float(np.prod(P))
    np.testing.assert_allclose(got, A, rtol=0, atol=1e-12 * np.abs(A).max())
    zero = np.arange(P[-1])
    zero = zero[(zero > Mv[-1] - 1) & (zero < P[-1] - (Mv[-1] - 1))]
    assert zero.size > 0 and np.all(al[..., zero] == 0.0)


def test_linbin_fixture(kf, gpu, repo_root):
    from test_oracle_linbin import _read_fixture
    cases = _read_fixture(os.path.join(repo_root, "tests", "golden", "linbin_tiny.txt"))
    for name, c in cases.items():
        g0 = c["grid"]
        d = g0["d"]
        hi = g0["lo"] + (g0["M"] - 1) * g0["delta"]
        g = kf.grid_plan(g0["M"], g0["lo"], hi)
        assert np.array_equal(g.to_dict()["delta"], g0["delta"])
        counts, nout = kf.linbin(_to_dev(np.array(c["points"]).reshape(-1, d), gpu), g)
        want = np.zeros(tuple(g0["M"]), dtype=np.int64)
        for idx, v in c["counts"]:
            want[idx] += v
        np.testing.assert_array_equal(counts.cpu().numpy(), want, err_msg=name)
        assert int(nout.item()) == c["skipped"]


def test_linbin_out_of_grid_and_edges(kf, gpu):
    g = kf.grid_plan([5, 4], [0.0, -1.0], [1.0, 2.0])
    pts = np.array([[0.0, -1.0], [1.0, 2.0], [0.5, 0.5], [-1e-12, 0.0], [0.3, 2.0 + 1e-9], [0.25, 1.0]])
    counts, nout = kf.linbin(_to_dev(pts, gpu), g)
    co, sk = linbin.linbin(pts, {"d": 2, "M": np.array([5, 4]), "lo": np.array([0.0, -1.0]),
                                 "delta": g.to_dict()["delta"]})
    np.testing.assert_array_equal(counts.cpu().numpy(), co)
    assert int(nout.item()) == sk == 2


def test_linbin_full_sizes(kf, gpu):
    """Case-2 (d=2 n=1e5 M=256), case-3 (d=3 n=2e5 M=64) and one case-5 dataset
    (d=4 M=32) binned bit-identically."""
    w5 = synth.case5(n_datasets=1, B=1, n_lo=200_000, n_hi=200_000)
    for name, X, G, M in [("case2", synth.case2().X[0], synth.case2().G_psi[0], 256),
                          ("case3", synth.case3().X[0], synth.case3().G_psi[0], 64),
                          ("case5", w5.X[0], w5.G_pilot[0], 32)]:
        log(f"[linbin-full] {name} n={X.shape[0]}")
        g_o = grid.plan_auto(X, G, [M] * X.shape[1])
        co, sk = linbin.linbin(X, g_o)
        Xd = _to_dev(X, gpu)
        g = kf.grid_auto(Xd, G, M)
        counts, nout = kf.linbin(Xd, g)
        np.testing.assert_array_equal(counts.cpu().numpy(), co)
        assert int(counts.sum().item()) == X.shape[0] << 40


def test_linbin_max_n(kf, gpu):
    """The largest accepted n (2^23 - 1): random points bin bit-identically, and
    the same point repeated n times fills its largest corner to within 2^40 of
    2^63 without overflow (every bin equals n times the one-point quanta)."""
    n = (1 << 23) - 1
    rng = np.random.default_rng(151107482 + 23)
    X = rng.standard_normal((n, 2))
    G = np.array([[0.01, 0.002], [0.002, 0.02]])
    log(f"[linbin-max] random n={n}")
    g_o = grid.plan_auto(X, G, [256, 256])
    co, sk = linbin.linbin(X, g_o)
    Xd = _to_dev(X, gpu)
    g = kf.grid_auto(Xd, G, 256)
    counts, nout = kf.linbin(Xd, g)
    np.testing.assert_array_equal(counts.cpu().numpy(), co)
    assert int(nout.item()) == sk == 0
    del Xd, counts
    log(f"[linbin-max] repeated point n={n}")
    g1 = kf.grid_plan([5, 4], [0.0, -1.0], [1.0, 2.0])
    p1 = np.array([[0.5 + 1e-3, 0.25 - 2e-3]])
    g1o = {"d": 2, "M": np.array([5, 4]), "lo": np.array([0.0, -1.0]), "delta": g1.to_dict()["delta"]}
    one, _ = linbin.linbin(p1, g1o)
    Xr = _to_dev(np.repeat(p1, n, axis=0), gpu)
    counts, nout = kf.linbin(Xr, g1)
    got = counts.cpu().numpy()
    np.testing.assert_array_equal(got, one * n)
    assert int(got.max()) > (1 << 62) and int(got.sum()) == n << 40


PSI_CASES = [("d1", 0), ("d1", 4), ("d1", 8), ("d2_case1", 0), ("d2_ragged", 2), ("d2_ragged", 4),
             ("d2_ragged", 8), ("d3", 2), ("d3", 4), ("d3", 6), ("d4", 2), ("d4", 4), ("d4_m12", 2)]


@pytest.mark.parametrize("name,r", PSI_CASES)
@pytest.mark.parametrize("mode", ["plain", "fused"])
def test_psi_vs_oracle(kf, gpu, name, r, mode):
    X, G, M = CASES[name]()
    d = X.shape[1]
    log(f"[psi] case={name} r={r} mode={mode} M={M}")
    g_o, _, _, c, A = _case(name, X, G, M)
    n = X.shape[0]
    want = binned.psi(A, n, g_o, G, r)
    sabs = binned.abs_scale(A, n, g_o, G, multiindex.unique_alphas(d, r))
    Xd = _to_dev(X, gpu)
    got = kf.psi(Xd, G, r, M=M, mode=mode).cpu().numpy()
    assert_psi_close(got, want, sabs, what=f"{name} r={r} {mode}")


def test_psi_case2_full(kf, gpu):
    """d=2, n=1e5 four-component mixture, M=256 (P=512), psi_4: both paths."""
    w = synth.case2()
    X, G = w.X[0], w.G_psi[0]
    log("[psi-full] case2 psi_4")
    g_o, _, _, c, A = _case("case2", X, G, 256)
    want = binned.psi(A, X.shape[0], g_o, G, 4)
    sabs = binned.abs_scale(A, X.shape[0], g_o, G, multiindex.unique_alphas(2, 4))
    Xd = _to_dev(X, gpu)
    for mode in ("plain", "fused"):
        got = kf.psi(Xd, G, 4, M=256, mode=mode).cpu().numpy()
        assert_psi_close(got, want, sabs, what=f"case2 {mode}")


def test_psi_case3_full(kf, gpu):
    """d=3, n=2e5 three-component mixture, M=64 (P=128), psi_2: both paths."""
    w = synth.case3()
    X, G = w.X[0], w.G_psi[0]
    log("[psi-full] case3 psi_2")
    g_o, _, _, c, A = _case("case3", X, G, 64)
    want = binned.psi(A, X.shape[0], g_o, G, 2)
    sabs = binned.abs_scale(A, X.shape[0], g_o, G, multiindex.unique_alphas(3, 2))
    Xd = _to_dev(X, gpu)
    for mode in ("plain", "fused"):
        got = kf.psi(Xd, G, 2, M=64, mode=mode).cpu().numpy()
        assert_psi_close(got, want, sabs, what=f"case3 {mode}")


def test_psi_edge_cases(kf, gpu):
    """n = 1; all points identical; smallest grid M = 2; oversized padding P = 4M."""
    G = np.array([[0.2, 0.05], [0.05, 0.3]])
    # single point: counts spread over one cell
    for X in (np.array([[0.3, -0.7]]), np.tile(np.array([[1.0, 2.0]]), (50, 1))):
        g_o = grid.plan_auto(X, G, [16, 16])
        co, _ = linbin.linbin(X, g_o)
        c = linbin.counts_to_real(co)
        A = binned.autocorr_direct(c)
        want = binned.psi(A, X.shape[0], g_o, G, 2)
        sabs = binned.abs_scale(A, X.shape[0], g_o, G, multiindex.unique_alphas(2, 2))
        for mode in ("plain", "fused"):
            got = kf.psi(_to_dev(X, gpu), G, 2, M=16, mode=mode).cpu().numpy()
            assert_psi_close(got, want, sabs, what=f"identical points {mode}")
    X = mixture_sample(300, 2, 9)
    for M, P in ((2, None), (8, 64), (9, 32)):
        g_o = grid.plan_auto(X, G, [M, M])
        co, _ = linbin.linbin(X, g_o)
        A = binned.autocorr_direct(linbin.counts_to_real(co))
        want = binned.psi(A, 300, g_o, G, 4)
        sabs = binned.abs_scale(A, 300, g_o, G, multiindex.unique_alphas(2, 4))
        hi = g_o["lo"] + (g_o["M"] - 1) * g_o["delta"]
        g = kf.grid_plan([M, M], g_o["lo"], hi, P=P)
        for mode in ("plain", "fused"):
            got = kf.psi(_to_dev(X, gpu), G, 4, grid=g, mode=mode).cpu().numpy()
            assert_psi_close(got, want, sabs, what=f"M={M} P={P} {mode}")


def test_psi_deterministic(kf, gpu):
    X, G, M = CASES["d3"]()
    Xd = _to_dev(X, gpu)
    for mode in ("plain", "fused"):
        a = kf.psi(Xd, G, 4, M=M, mode=mode).cpu().numpy()
        b = kf.psi(Xd, G, 4, M=M, mode=mode).cpu().numpy()
        assert np.array_equal(a, b)
