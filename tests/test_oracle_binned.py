"""Pins of oracle.binned and oracle.layout (Sec. 4, Eq. (14), (17)-(24)).

* literal Eq. (14): the quadruple sum over node pairs at tiny grids equals the
  lag-domain form;
* autocorrelation by shifted slices and by slab products equals a
  brute-force double loop and the numpy.fft route;
* data on grid nodes: binned psi equals the unbinned psi of oracle.direct;
* the paper's zero-padded layout (P = 2^ceil(log2(3M-1))) and the circular
  P = 2M layout both equal the lag-domain form;
* negative control for the paper's central claim: a kernel grid mirrored
  from one quadrant (valid only for diagonal G) gives a different result for
  a correlated G, while reflecting one axis of both data and G flips exactly
  the entries with an odd power of that axis;
* binning error behaves as the first-order prediction
  d psi_a ~ 1/2 sum_k (delta_k^2/3) psi_{a+2e_k}.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import binned, direct, gauss, grid, layout, linbin, multiindex


def _binned_case(d, n, M, seed, G=None):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((d, d)) * 0.6 + np.eye(d)
    X = rng.standard_normal((n, d)) @ A.T
    if G is None:
        B = rng.standard_normal((d, d))
        G = 0.05 * (B @ B.T) + 0.08 * np.eye(d)
    g = grid.plan_auto(X, G, [M] * d)
    counts, skipped = linbin.linbin(X, g)
    assert skipped == 0
    return X, G, g, linbin.counts_to_real(counts)


@pytest.mark.parametrize("d,M,r", [(1, 9, 4), (2, 6, 0), (2, 5, 4), (3, 4, 2)])
def test_literal_eq14(d, M, r):
    X, G, g, c = _binned_case(d, 200, M, 1 + d)
    n = X.shape[0]
    nodes = [grid.nodes(g, k) for k in range(d)]
    pts = list(itertools.product(*[range(M)] * d))
    alphas = multiindex.unique_alphas(d, r)
    tot = np.zeros(len(alphas))
    for i in pts:
        for j in pts:
            diff = np.array([nodes[k][i[k]] - nodes[k][j[k]] for k in range(d)])
            tot += gauss.dphi_many(diff, G, alphas) * c[i] * c[j]
    want = tot / n ** 2
    A = binned.autocorr_direct(c)
    got = binned.psi(A, n, g, G, r)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-14 * np.abs(want).max())


@pytest.mark.parametrize("shape", [(7,), (5, 6), (3, 4, 5), (3, 2, 4, 3)])
def test_autocorr_routes(shape):
    rng = np.random.default_rng(2)
    c = rng.random(shape)
    A = binned.autocorr_direct(c)
    d = len(shape)
    brute = np.zeros(A.shape)
    for i in itertools.product(*[range(m) for m in shape]):
        for j in itertools.product(*[range(m) for m in shape]):
            lag = tuple(jj - ii for ii, jj in zip(i, j))
            brute[tuple(l + m - 1 for l, m in zip(lag, shape))] += c[i] * c[j]
    np.testing.assert_allclose(A, brute, rtol=1e-13)
    np.testing.assert_allclose(binned.autocorr_fft(c), brute, rtol=1e-12, atol=1e-12 * brute.max())
    np.testing.assert_allclose(binned.autocorr_gemm(c), brute, rtol=1e-13)
    assert d == A.ndim


@pytest.mark.parametrize("shape", [(9, 5), (6, 7, 5), (5, 4, 6, 3), (4, 4, 4, 4)])
def test_autocorr_gemm_matches_slices(shape):
    """The slab-product route (used for the large grids of the GPU parity
    tests) equals the shifted-slice definition on sparse ragged grids, and is
    exactly centrally symmetric (A_{-l} = A_l bit for bit)."""
    rng = np.random.default_rng(sum(shape))
    c = rng.random(shape) * (rng.random(shape) < 0.6)
    A = binned.autocorr_direct(c)
    B = binned.autocorr_gemm(c)
    np.testing.assert_allclose(B, A, rtol=1e-13, atol=1e-15 * A.max())
    assert np.array_equal(B, B[tuple(slice(None, None, -1) for _ in shape)])
    # zero lag: the sum of squares
    assert B[tuple(m - 1 for m in shape)] == pytest.approx(float(np.sum(c * c)), rel=1e-14)


@pytest.mark.parametrize("d,r", [(1, 6), (2, 0), (2, 4), (3, 2)])
def test_on_nodes_equals_unbinned(d, r):
    rng = np.random.default_rng(20 + d)
    M = 12
    lo = -np.ones(d) * 2.0
    hi = np.ones(d) * 3.5
    g = grid.plan(lo, hi, [M] * d)
    idx = rng.integers(0, M, size=(300, d))
    X = lo + idx * g["delta"]
    G = np.diag(np.linspace(0.3, 0.6, d))
    if d > 1:
        G[0, 1] = G[1, 0] = 0.1
    counts, skipped = linbin.linbin(X, g)
    assert skipped == 0
    c = linbin.counts_to_real(counts)
    got = binned.psi(binned.autocorr_direct(c), X.shape[0], g, G, r)
    want = direct.psi(X, G, r)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-14 * np.abs(want).max())


@pytest.mark.parametrize("d,M,r", [(1, 40, 4), (2, 24, 4), (2, 17, 0), (3, 10, 2)])
def test_layouts_equal_lag_form(d, M, r):
    X, G, g, c = _binned_case(d, 1500, M, 30 + d)
    n = X.shape[0]
    ref = binned.psi(binned.autocorr_direct(c), n, g, G, r)
    scale = np.abs(ref).max()
    np.testing.assert_allclose(layout.psi_paper(c, n, g, G, r), ref, rtol=1e-12, atol=1e-13 * scale)
    np.testing.assert_allclose(layout.psi_wrap(c, n, g, G, r), ref, rtol=1e-12, atol=1e-13 * scale)


def test_paper_P_rule():
    assert layout.paper_P(64) == 256
    assert layout.paper_P(256) == 1024
    assert layout.paper_P(20) == 64


def test_quadrant_mirror_fails_for_full_G():
    G = np.array([[0.10, 0.06], [0.06, 0.20]])
    X, G, g, c = _binned_case(2, 2000, 32, 5, G=G)
    n = X.shape[0]
    ref = binned.psi(binned.autocorr_direct(c), n, g, G, 0)
    wand = layout.psi_wand_quadrant(c, n, g, G, 0)
    assert abs(wand[0] - ref[0]) > 1e-3 * abs(ref[0])
    # for a diagonal G the mirrored grid is exact
    Gd = np.diag(np.diag(G))
    refd = binned.psi(binned.autocorr_direct(c), n, g, Gd, 0)
    np.testing.assert_allclose(layout.psi_wand_quadrant(c, n, g, Gd, 0), refd, rtol=1e-12)


def test_sign_flip_of_off_diagonal():
    rng = np.random.default_rng(6)
    X = rng.standard_normal((400, 2)) @ np.array([[1.0, 0.0], [0.7, 0.7]])
    G = np.array([[0.10, 0.06], [0.06, 0.20]])
    Gf = G * np.array([[1, -1], [-1, 1]])
    r = 4
    a = direct.psi(X, G, r)
    b = direct.psi(X, Gf, r)
    assert abs(a[0] - b[0]) > 1e-3 * abs(a[0])
    c = direct.psi(X * np.array([1.0, -1.0]), Gf, r)
    signs = np.array([(-1) ** al[1] for al in multiindex.unique_alphas(2, r)])
    np.testing.assert_allclose(c, signs * a, rtol=1e-13)


def test_binning_error_first_order():
    rng = np.random.default_rng(7)
    n = 800
    X = rng.standard_normal((n, 2)) @ np.array([[1.0, 0.0], [0.7, 0.71]])
    G = np.array([[0.10, 0.06], [0.06, 0.20]])
    exact = direct.psi(X, G, 0)[0]
    second = direct.psi(X, G, 2)            # (0,0),(0,1),(1,1)
    errs, preds = [], []
    for M in (64, 128):
        g = grid.plan_auto(X, G, [M, M])
        counts, _ = linbin.linbin(X, g)
        c = linbin.counts_to_real(counts)
        val = binned.psi(binned.autocorr_direct(c), n, g, G, 0)[0]
        errs.append(val - exact)
        dl = g["delta"]
        preds.append(0.5 * (dl[0] ** 2 / 3 * second[0] + dl[1] ** 2 / 3 * second[2]))
    for e, p in zip(errs, preds):
        assert e == pytest.approx(p, rel=0.1)
    assert abs(errs[1]) < abs(errs[0]) / 3.0
    assert math.isfinite(exact)
