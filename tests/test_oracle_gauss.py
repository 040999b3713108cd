"""Pins of oracle.gauss: the Gaussian derivatives against independent routes.

* symbolic differentiation of the density (sympy), full covariance, d=2 r=4,
  d=3 r=2, d=2 r=6;
* d=1: (-1)^r s^-r He_r(x/s) phi, with He_r from numpy.polynomial.hermite_e;
* diagonal covariance: product of one-dimensional derivatives;
* x = 0: Isserlis' theorem (moments of N(0, Sigma^{-1}) via the Fourier
  transform of phi_Sigma).
"""
import itertools
import math

import numpy as np
import pytest
import sympy as sp
from numpy.polynomial import hermite_e

from oracle import gauss, multiindex


def _sym_density(S):
    d = S.shape[0]
    xs = sp.symbols(f"x0:{d}")
    Ss = sp.Matrix(d, d, lambda i, j: sp.nsimplify(S[i, j]))
    P = Ss.inv()
    xv = sp.Matrix(xs)
    q = (xv.T * P * xv)[0, 0]
    f = (2 * sp.pi) ** sp.Rational(-d, 2) / sp.sqrt(Ss.det()) * sp.exp(-q / 2)
    return xs, f


@pytest.mark.parametrize("S,r,x", [
    (np.array([[0.10, 0.06], [0.06, 0.20]]), 4, (0.13, -0.21)),
    (np.array([[0.7, -0.3], [-0.3, 0.5]]), 6, (0.4, 0.25)),
    (np.array([[1.0, 0.2, -0.1], [0.2, 0.8, 0.3], [-0.1, 0.3, 0.6]]), 2, (0.3, -0.2, 0.5)),
    (np.array([[1.0, 0.2, -0.1], [0.2, 0.8, 0.3], [-0.1, 0.3, 0.6]]), 4, (-0.1, 0.35, 0.2)),
])
def test_against_sympy(S, r, x):
    xs, f = _sym_density(S)
    d = S.shape[0]
    alphas = multiindex.unique_alphas(d, r)
    got = gauss.dphi_many(np.array(x), S, alphas)
    for a, g in zip(alphas, got):
        expr = f
        for k in range(d):
            if a[k]:
                expr = sp.diff(expr, xs[k], a[k])
        want = float(expr.subs(dict(zip(xs, [sp.nsimplify(v) for v in x]))).evalf(30))
        assert abs(g - want) <= 2e-14 * max(1.0, abs(want)), (a, g, want)


@pytest.mark.parametrize("r", [0, 1, 2, 3, 4, 6, 8])
def test_univariate_hermite_e(r):
    s2 = 0.37
    s = math.sqrt(s2)
    x = np.linspace(-2.0, 2.0, 41)[:, None]
    got = gauss.dphi(x, np.array([[s2]]), (r,))
    coef = np.zeros(r + 1)
    coef[r] = 1.0
    u = x[:, 0] / s
    phi1 = np.exp(-0.5 * u * u) / math.sqrt(2 * math.pi * s2)
    want = (-1) ** r * s ** (-r) * hermite_e.hermeval(u, coef) * phi1
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-14 * np.abs(want).max())


def test_diagonal_is_product():
    S = np.diag([0.3, 1.7, 0.8])
    x = np.array([[0.2, -0.5, 0.9], [1.0, 0.1, -0.3]])
    for a in multiindex.unique_alphas(3, 4):
        got = gauss.dphi(x, S, a)
        want = np.ones(len(x))
        for k in range(3):
            want = want * gauss.dphi(x[:, k:k + 1], np.array([[S[k, k]]]), (a[k],))
        np.testing.assert_allclose(got, want, rtol=1e-13)


def _pairings(idx):
    if not idx:
        yield []
        return
    a = idx[0]
    for t in range(1, len(idx)):
        rest = idx[1:t] + idx[t + 1:]
        for p in _pairings(rest):
            yield [(a, idx[t])] + p


@pytest.mark.parametrize("d,r", [(2, 2), (2, 4), (3, 4), (4, 2), (2, 6)])
def test_isserlis_at_zero(d, r):
    rng = np.random.default_rng(5)
    A = rng.standard_normal((d, d))
    S = A @ A.T + d * np.eye(d)
    P = np.linalg.inv(S)
    phi0 = gauss.phi(np.zeros(d), S)
    for t in multiindex.unique_tuples(d, r):
        a = multiindex.tuple_to_alpha(t, d)
        want = sum(np.prod([P[i, j] for i, j in pr]) for pr in _pairings(list(t)))
        want *= (-1) ** (r // 2) * phi0
        got = gauss.dphi(np.zeros(d), S, a)
        assert abs(got - want) <= 1e-13 * max(abs(want), phi0), (t, got, want)


def test_odd_order_is_odd_function():
    S = np.array([[0.5, 0.1], [0.1, 0.3]])
    x = np.array([0.3, -0.7])
    for a in multiindex.unique_alphas(2, 3):
        assert gauss.dphi(x, S, a) == pytest.approx(-gauss.dphi(-x, S, a), rel=1e-14)


def test_unique_order_and_expand():
    assert multiindex.unique_tuples(2, 4) == [(0, 0, 0, 0), (0, 0, 0, 1), (0, 0, 1, 1), (0, 1, 1, 1), (1, 1, 1, 1)]
    assert multiindex.n_unique(4, 4) == 35
    v = np.arange(5.0)
    full = multiindex.expand_full(v, 2, 4)
    for flat, idx in enumerate(itertools.product(range(2), repeat=4)):
        assert full[flat] == sum(idx)
