"""Pins of oracle.fftl (fft-L, Sec. 4 Eq. (25)-(27); Sec. 6.3 Tables 2 and 3).

* Eq. (27) applied to the L values the paper prints in Table 3 reproduces its
  Table 2 at every (n, M) cell the two tables share (tests/golden/fftl_tables.txt);
* Eq. (26) on hand-computed cases (largest eigenvalue of a rotated matrix,
  ceiling, clamp at M - 1);
* with L_k = M_k - 1 the truncated sum is the full binned sum;
* data on grid nodes: the truncated binned sum equals the unbinned pair sum
  restricted to pairs with |X_ik - X_jk| <= L_k delta_k (brute force).
"""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import binned, fftl, gauss, grid, linbin, multiindex


def _tables(repo_root):
    L, P = {}, {}
    for line in open(os.path.join(repo_root, "tests", "golden", "fftl_tables.txt")):
        if line.startswith("#") or not line.strip():
            continue
        kind, n, M, a, b = line.split()
        (L if kind == "L" else P)[(int(n), int(M))] = (int(a), int(b))
    return L, P


def test_table2_from_table3(repo_root):
    L, P = _tables(repo_root)
    shared = sorted(set(L) & set(P))
    assert len(shared) == 20
    for (n, M) in shared:
        assert tuple(fftl.plan_P([M, M], L[(n, M)])) == P[(n, M)], (n, M)


def test_plan_L_hand_cases():
    g = grid.plan(np.array([0.0, 0.0]), np.array([19.9, 59.7]), [200, 200])   # delta 0.1, 0.3
    assert np.allclose(g["delta"], [0.1, 0.3])
    c, s = math.cos(0.4), math.sin(0.4)
    R = np.array([[c, -s], [s, c]])
    S = R @ np.diag([4.0, 1.0]) @ R.T            # largest eigenvalue 4
    # 3.7 * 2 / 0.1 = 74 exactly in real arithmetic; 7.4 / 0.3 = 24.67 -> 25
    L = fftl.plan_L(g, S)
    assert L[1] == 25
    assert L[0] in (74, 75)                       # 74 up to the rounding of 7.4 / 0.1
    g2 = grid.plan(np.array([0.0, 0.0]), np.array([4.9, 0.49]), [50, 50])     # delta 0.1, 0.01
    assert fftl.plan_L(g2, np.diag([0.25, 0.01])) == [19, 49]   # ceil(18.5) = 19; 185 clamped to 49
    assert fftl.plan_P([50, 50], [19, 49]) == [128, 256]          # 87 -> 128, 147 -> 256


def _setup(seed, M=18):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(400, 2)) * 0.6
    G = np.array([[0.04, 0.01], [0.01, 0.03]])
    g = grid.plan_auto(X, G, [M, M])
    co, _ = linbin.linbin(X, g)
    A = binned.autocorr_direct(linbin.counts_to_real(co))
    return X, G, g, A


@pytest.mark.parametrize("r", [0, 2, 4])
def test_full_L_is_full_sum(r):
    X, G, g, A = _setup(3)
    n = X.shape[0]
    full = binned.psi(A, n, g, G, r)
    tr = fftl.psi_truncated(A, n, g, G, r, [int(m) - 1 for m in g["M"]])
    np.testing.assert_allclose(tr, full, rtol=1e-13, atol=1e-15 * np.abs(full).max())


@pytest.mark.parametrize("r", [0, 2])
def test_truncated_equals_restricted_pairs_on_nodes(r):
    M = 14
    g = grid.plan(np.array([-1.0, -1.5]), np.array([1.6, 1.1]), [M, M])
    rng = np.random.default_rng(4)
    idx = rng.integers(0, M, size=(70, 2))
    X = g["lo"] + idx * g["delta"]
    co, _ = linbin.linbin(X, g)
    A = binned.autocorr_direct(linbin.counts_to_real(co))
    n = X.shape[0]
    G = np.array([[0.08, 0.02], [0.02, 0.05]])
    L = [4, 6]
    tr = fftl.psi_truncated(A, n, g, G, r, L)
    alphas = multiindex.unique_alphas(2, r)
    acc = np.zeros(len(alphas))
    for i, j in itertools.product(range(n), repeat=2):
        dl = idx[i] - idx[j]
        if abs(dl[0]) <= L[0] and abs(dl[1]) <= L[1]:
            acc += gauss.dphi_many(X[i] - X[j], G, alphas)
    np.testing.assert_allclose(tr, acc / n ** 2, rtol=1e-12, atol=1e-14 * np.abs(acc / n ** 2).max())


def test_truncation_error_is_small_at_tau():
    X, G, g, A = _setup(5, M=40)
    n = X.shape[0]
    L = fftl.plan_L(g, G)
    assert all(l < int(m) - 1 for l, m in zip(L, g["M"]))
    full = binned.psi(A, n, g, G, 0)[0]
    tr = fftl.psi_truncated(A, n, g, G, 0, L)[0]
    assert tr <= full and abs(tr - full) <= 1e-3 * full
