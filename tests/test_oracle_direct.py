"""Pins of oracle.direct: the unbinned double sum psi_r (Eq. (13)).

* 50-digit brute force (mpmath) over all n^2 ordered pairs with derivatives
  from symbolic differentiation (sympy), n <= 40;
* n = 1 reduces to D^alpha phi_G(0);
* expectation over samples of a normal mixture, closed form
  E psi_alpha = (1-1/n) sum_lm w_l w_m D^alpha phi_{G+S_l+S_m}(mu_l-mu_m)
               + n^-1 D^alpha phi_G(0)   (z-test over seeds);
* invariances: X->2X, G->4G scales psi_r by 2^-(d+r); X->X R^T, G->R G R^T
  maps the full derivative vector by R^{(x)r}; coordinate permutation.
"""
import itertools

import mpmath
import numpy as np
import pytest
import sympy as sp

from oracle import direct, gauss, multiindex


def _mp_derivs(S, alphas):
    d = S.shape[0]
    xs = sp.symbols(f"x0:{d}")
    Ss = sp.Matrix(d, d, lambda i, j: sp.nsimplify(S[i, j]))
    P = Ss.inv()
    xv = sp.Matrix(xs)
    q = (xv.T * P * xv)[0, 0]
    f = (2 * sp.pi) ** sp.Rational(-d, 2) / sp.sqrt(Ss.det()) * sp.exp(-q / 2)
    fns = []
    for a in alphas:
        e = f
        for k in range(d):
            if a[k]:
                e = sp.diff(e, xs[k], a[k])
        fns.append(sp.lambdify(xs, e, modules="mpmath"))
    return fns


@pytest.mark.parametrize("d,r,n", [(2, 0, 40), (2, 4, 30), (3, 2, 25)])
def test_mpmath_brute_force(d, r, n):
    rng = np.random.default_rng(11 + d + r)
    X = rng.standard_normal((n, d))
    A = rng.standard_normal((d, d))
    G = 0.3 * (A @ A.T) / d + 0.1 * np.eye(d)
    G = np.round(G, 6)
    alphas = multiindex.unique_alphas(d, r)
    fns = _mp_derivs(G, alphas)
    mpmath.mp.dps = 50
    want = []
    for fn in fns:
        acc = mpmath.mpf(0)
        for i in range(n):
            for j in range(n):
                acc += fn(*[mpmath.mpf(float(X[i, k])) - mpmath.mpf(float(X[j, k])) for k in range(d)])
        want.append(acc / n ** 2)
    got = direct.psi(X, G, r)
    for g, w in zip(got, want):
        w = float(w)
        assert abs(g - w) <= 1e-14 * max(abs(w), 1e-3), (g, w)


def test_single_point():
    G = np.array([[0.2, 0.05], [0.05, 0.1]])
    X = np.array([[0.3, -1.2]])
    for r in (0, 2, 4):
        al = multiindex.unique_alphas(2, r)
        np.testing.assert_allclose(direct.psi(X, G, r), gauss.dphi_many(np.zeros(2), G, al), rtol=1e-15)


def test_mixture_expectation_z():
    """Closed-form mean of the V-statistic over random samples (pins the pair
    structure: the diagonal term, the factor 2 and n^-2)."""
    w = np.array([0.6, 0.4])
    mu = np.array([[0.0, 0.0], [1.0, -0.5]])
    S = np.array([[[0.5, 0.2], [0.2, 0.4]], [[0.3, -0.1], [-0.1, 0.6]]])
    G = np.array([[0.15, 0.04], [0.04, 0.1]])
    n, r, reps = 60, 2, 200
    alphas = multiindex.unique_alphas(2, r)
    expect = gauss.dphi_many(np.zeros(2), G, alphas) / n
    for l in range(2):
        for m in range(2):
            expect = expect + (1 - 1 / n) * w[l] * w[m] * gauss.dphi_many(mu[l] - mu[m], G + S[l] + S[m], alphas)
    rng = np.random.default_rng(123)
    vals = []
    for _ in range(reps):
        lab = rng.choice(2, size=n, p=w)
        X = np.empty((n, 2))
        for l in range(2):
            idx = lab == l
            X[idx] = mu[l] + rng.standard_normal((idx.sum(), 2)) @ np.linalg.cholesky(S[l]).T
        vals.append(direct.psi(X, G, r))
    vals = np.array(vals)
    z = (vals.mean(0) - expect) / (vals.std(0, ddof=1) / np.sqrt(reps))
    assert np.all(np.abs(z) < 4.0), z


def test_scaling_invariance():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((150, 2))
    G = np.array([[0.2, -0.07], [-0.07, 0.3]])
    for r in (0, 2, 4):
        a = direct.psi(X, G, r)
        b = direct.psi(2 * X, 4 * G, r)
        np.testing.assert_allclose(b, a * 2.0 ** (-(2 + r)), rtol=1e-13)


def test_rotation_covariance():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((120, 2)) @ np.array([[1.0, 0.0], [0.6, 0.8]])
    G = np.array([[0.2, 0.05], [0.05, 0.15]])
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    r = 4
    a = multiindex.expand_full(direct.psi(X, G, r), 2, r)
    b = multiindex.expand_full(direct.psi(X @ R.T, R @ G @ R.T, r), 2, r)
    Rk = R
    for _ in range(r - 1):
        Rk = np.kron(Rk, R)
    np.testing.assert_allclose(b, Rk @ a, rtol=1e-12, atol=1e-12 * np.abs(a).max())


def test_permutation():
    rng = np.random.default_rng(8)
    X = rng.standard_normal((100, 3))
    G = np.array([[0.3, 0.1, 0.0], [0.1, 0.2, -0.05], [0.0, -0.05, 0.4]])
    perm = [2, 0, 1]
    r = 2
    a = direct.psi(X, G, r)
    b = direct.psi(X[:, perm], G[np.ix_(perm, perm)], r)
    tup = multiindex.unique_tuples(3, r)
    pos = {t: i for i, t in enumerate(tup)}
    for i, t in enumerate(tup):
        # axis k of the permuted data is axis perm[k] of the original
        orig = tuple(sorted(perm[k] for k in t))
        assert b[i] == pytest.approx(a[pos[orig]], rel=1e-13)


def test_workers_match_serial():
    rng = np.random.default_rng(9)
    X = rng.standard_normal((2500, 2))
    G = np.eye(2) * 0.1
    a = direct.psi(X, G, 2, workers=1)
    b = direct.psi(X, G, 2, workers=2)
    np.testing.assert_array_equal(a, b)
