"""Pins of oracle.eta: eta_r, Q_r and LSCV_r.

* eta_r against an independent derivation: by the heat equation of the normal
  density, eta_r(x; S) = d^r/dt^r phi_{S + 2tI}(x) at t = 0, so eta_r / phi_S is
  the complete Bell polynomial of the t-cumulants
  kappa_m = (-1)^{m+1} (m-1)!/2 (m U_m - T_m),
  U_m = x^T S^-1 (2 S^-1)^m x, T_m = tr (2 S^-1)^m   (d = 1..4, r = 0..8);
* the same t-derivative by central finite differences (r = 1, 2);
* one dimension: sigma^{-2r} He_{2r}(x/sigma) phi (numpy.polynomial.hermite_e);
* x = 0, S = I: (-1)^r (2 pi)^{-d/2} 2^r Gamma(d/2 + r) / Gamma(d/2)
  (Fourier side: the r-th power of -|w|^2 against a standard normal);
* Q_0 = psi_0 and Q_1 = trace of psi_2 (binned and unbinned);
* LSCV (r = 0, Eq. (35)) against its definition Eq. (8)-(10): the integral of
  the squared estimate by quadrature and the leave-one-out sum, 1-D and 2-D;
* the sign (-1)^r: the integral of the squared r-th derivative of the 1-D
  estimate equals (-1)^r n^-2 sum sum eta_r(.; 2h^2);
* data on grid nodes: binned = unbinned; LSCV gradient by central differences.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import hermite_e

from oracle import binned, direct, eta, gauss, grid, linbin, multiindex

from test_oracle_scv import _fd_richardson, _vech_to_H


def _spd(d, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(d, d)))
    return scale * Q @ np.diag(10 ** rng.uniform(-0.5, 0.3, d)) @ Q.T


def _eta_bell(x, S, r):
    """eta_r via cumulants of log phi_{S+2tI}(x) in t and the Bell recursion."""
    P = np.linalg.inv(S)
    d = S.shape[0]
    B = 2.0 * P
    kap = [0.0] * (r + 1)
    Bm = np.eye(d)
    for m in range(1, r + 1):
        Bm = Bm @ B
        U = float(x @ P @ Bm @ x)
        T = float(np.trace(Bm))
        kap[m] = (-1) ** (m + 1) * math.factorial(m - 1) / 2.0 * (m * U - T)
    Y = [1.0]
    for m in range(r):
        Y.append(sum(math.comb(m, k) * kap[k + 1] * Y[m - k] for k in range(m + 1)))
    return Y[r] * float(gauss.phi(x, S))


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_eta_vs_cumulant_bell(d):
    rng = np.random.default_rng(11 + d)
    S = _spd(d, 5 + d)
    rmax = 8 if d <= 2 else (6 if d == 3 else 4)
    for r in range(rmax + 1):
        pts = rng.normal(size=(6, d)) * 0.8
        a = np.array([float(eta.eta(p, S, r)) for p in pts])
        b = np.array([_eta_bell(p, S, r) for p in pts])
        np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-12 * np.abs(b).max())


def test_eta_t_derivative_fd():
    S = _spd(2, 3)
    x = np.array([0.4, -0.3])
    h = 1e-4
    f = lambda t: float(gauss.phi(x, S + 2 * t * np.eye(2)))
    d1 = (f(h) - f(-h)) / (2 * h)
    d2 = (f(h) - 2 * f(0) + f(-h)) / h ** 2
    assert float(eta.eta(x, S, 1)) == pytest.approx(d1, rel=1e-7)
    assert float(eta.eta(x, S, 2)) == pytest.approx(d2, rel=1e-5)


@pytest.mark.parametrize("r", [0, 1, 2, 3, 5, 8])
def test_eta_one_dimension(r):
    s2 = 0.7
    s = math.sqrt(s2)
    for x in (-1.3, 0.0, 0.25, 2.1):
        c = np.zeros(2 * r + 1)
        c[-1] = 1.0
        want = s ** (-2 * r) * hermite_e.hermeval(x / s, c) * float(gauss.phi(np.array([x]), np.array([[s2]])))
        got = float(eta.eta(np.array([x]), np.array([[s2]]), r))
        assert got == pytest.approx(want, rel=1e-11, abs=1e-14 * abs(want) + 1e-300)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
@pytest.mark.parametrize("r", [0, 1, 2, 4])
def test_eta_at_zero_identity(d, r):
    want = (-1) ** r * (2 * math.pi) ** (-d / 2) * 2 ** r * math.gamma(d / 2 + r) / math.gamma(d / 2)
    assert float(eta.eta(np.zeros(d), np.eye(d), r)) == pytest.approx(want, rel=1e-13)


def _setup(n, d, M, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, d)) * 0.7
    G = _spd(d, seed + 1, 0.05)
    g = grid.plan_auto(X, G, [M] * d)
    co, _ = linbin.linbin(X, g)
    A = binned.autocorr_direct(linbin.counts_to_real(co))
    return X, G, g, A


def test_q0_q1_are_psi_contractions():
    X, G, g, A = _setup(300, 2, 20, 21)
    n = X.shape[0]
    S = _spd(2, 9, 0.1)
    assert eta.qr_binned(A, n, g, S, 0) == pytest.approx(binned.psi(A, n, g, S, 0)[0], rel=1e-13)
    p2 = binned.psi(A, n, g, S, 2)
    tr = sum(p2[k] for k, t in enumerate(multiindex.unique_tuples(2, 2)) if t[0] == t[1])
    assert eta.qr_binned(A, n, g, S, 1) == pytest.approx(tr, rel=1e-12)
    p2d = direct.psi(X[:120], S, 2)
    trd = sum(p2d[k] for k, t in enumerate(multiindex.unique_tuples(2, 2)) if t[0] == t[1])
    assert eta.qr_direct(X[:120], S, 1) == pytest.approx(trd, rel=1e-12)


def _fhat_1d(X, h2, xs, r=0):
    """r-th derivative of the 1-D normal-kernel estimate on the points xs."""
    s = math.sqrt(h2)
    c = np.zeros(r + 1)
    c[-1] = 1.0
    u = (xs[:, None] - X[None, :]) / s
    dens = np.exp(-0.5 * u * u) / (math.sqrt(2 * math.pi) * s)
    return ((-1) ** r * s ** (-r) * hermite_e.hermeval(u, c) * dens).mean(axis=1)


def test_lscv_definition_1d():
    rng = np.random.default_rng(4)
    X = rng.normal(size=(25, 1))
    n = 25
    h2 = 0.09
    xs = np.linspace(X.min() - 3, X.max() + 3, 200001)
    dx = xs[1] - xs[0]
    int_f2 = float(np.sum(_fhat_1d(X[:, 0], h2, xs) ** 2) * dx)
    s = math.sqrt(h2)
    D = X[:, 0][:, None] - X[:, 0][None, :]
    K = np.exp(-0.5 * D * D / h2) / (math.sqrt(2 * math.pi) * s)
    loo = (K.sum(axis=1) - K.diagonal()) / (n - 1)
    want = int_f2 - 2.0 / n * loo.sum()
    got = eta.lscv_r_direct(X, np.array([[h2]]), 0, exact=True)
    assert got == pytest.approx(want, rel=1e-9)


def test_lscv_definition_2d():
    rng = np.random.default_rng(5)
    n = 12
    X = rng.normal(size=(n, 2)) * 0.5
    H = np.array([[0.05, 0.02], [0.02, 0.08]])
    ax = [np.linspace(X[:, k].min() - 2, X[:, k].max() + 2, 801) for k in range(2)]
    mesh = np.stack(np.meshgrid(*ax, indexing="ij"), axis=-1)
    f = np.mean([gauss.phi(mesh - X[i], H) for i in range(n)], axis=0)
    int_f2 = float(np.sum(f * f) * (ax[0][1] - ax[0][0]) * (ax[1][1] - ax[1][0]))
    K = np.array([[float(gauss.phi(X[i] - X[j], H)) for j in range(n)] for i in range(n)])
    loo = (K.sum(axis=1) - K.diagonal()) / (n - 1)
    want = int_f2 - 2.0 / n * loo.sum()
    got = eta.lscv_r_direct(X, H, 0, exact=True)
    assert got == pytest.approx(want, rel=1e-7)
    # Eq. (36): n - 1 -> n
    approx = eta.lscv_r_direct(X, H, 0, exact=False)
    V2 = eta.vstat_direct(X, [(1.0, 2 * H)], 0)
    V1 = eta.vstat_direct(X, [(1.0, H)], 0)
    assert approx == pytest.approx(V2 - 2 * V1 + 2.0 / n * float(gauss.phi(np.zeros(2), H)), rel=1e-13)


@pytest.mark.parametrize("r", [1, 2])
def test_sign_of_lscv_r_first_term_1d(r):
    rng = np.random.default_rng(8 + r)
    X = rng.normal(size=(15, 1))
    h2 = 0.12
    xs = np.linspace(X.min() - 3, X.max() + 3, 400001)
    dx = xs[1] - xs[0]
    int_dr2 = float(np.sum(_fhat_1d(X[:, 0], h2, xs, r) ** 2) * dx)
    V = eta.vstat_direct(X, [(1.0, np.array([[2 * h2]]))], r)
    assert (-1) ** r * V == pytest.approx(int_dr2, rel=1e-8)


def test_binned_equals_direct_on_nodes():
    d, M = 2, 12
    g = grid.plan(np.array([-1.0, -2.0]), np.array([1.75, 1.3]), [M, M])
    rng = np.random.default_rng(2)
    idx = rng.integers(0, M, size=(60, d))
    X = g["lo"] + idx * g["delta"]
    co, _ = linbin.linbin(X, g)
    A = binned.autocorr_direct(linbin.counts_to_real(co))
    n = X.shape[0]
    H = _spd(2, 4, 0.2)
    for r in (0, 1, 3):
        a = eta.lscv_r_binned(A, n, g, H, r)
        b = eta.lscv_r_direct(X, H, r)
        assert a == pytest.approx(b, rel=1e-12, abs=1e-14 * eta.lscv_abs_scale(A, n, g, H, r))
        assert eta.qr_binned(A, n, g, H, r) == pytest.approx(eta.qr_direct(X, H, r), rel=1e-12)


@pytest.mark.parametrize("exact", [False, True])
def test_lscv_gradient_fd(exact):
    X, G, g, A = _setup(400, 2, 24, 31)
    n = X.shape[0]
    H = _spd(2, 12, 0.1)
    L = np.linalg.cholesky(H)
    v = np.concatenate([L[j:, j] for j in range(2)])
    _, gr = eta.lscv_binned(A, n, g, H, exact)
    fd = _fd_richardson(lambda w: eta.lscv_binned(A, n, g, _vech_to_H(w, 2), exact, with_grad=False)[0], v, 1e-4)
    np.testing.assert_allclose(gr, fd, rtol=1e-7, atol=1e-9 * np.abs(gr).max())
    _, grd = eta.lscv_direct(X[:150], H, exact)
    fdd = _fd_richardson(lambda w: eta.lscv_direct(X[:150], _vech_to_H(w, 2), exact, with_grad=False)[0], v, 1e-4)
    np.testing.assert_allclose(grd, fdd, rtol=1e-7, atol=1e-9 * np.abs(grd).max())


@pytest.mark.parametrize("exact", [False, True])
def test_lscv_scales_bound_values(exact):
    """lscv_binned_scales bounds |LSCV| and every |gradient entry|; the
    objective's scale stays within two orders of magnitude of it, and the
    gradient's (whose entries cancel strongly near the minimiser) within two
    orders of the objective's scale over the smallest diagonal entry of L."""
    X, G, g, A = _setup(400, 2, 24, 31)
    n = X.shape[0]
    for seed in range(4):
        H = _spd(2, 20 + seed, 0.1)
        o, gr = eta.lscv_binned(A, n, g, H, exact)
        so, sg = eta.lscv_binned_scales(A, n, g, H, exact)
        assert abs(o) <= so * (1 + 1e-13)
        assert np.all(np.abs(gr) <= sg * (1 + 1e-13))
        lmin = np.abs(np.diag(np.linalg.cholesky(H))).min()
        assert so <= 100 * abs(o) and np.all(sg <= 100 * so / lmin)
