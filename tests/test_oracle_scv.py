"""Pins of oracle.scv: the SCV objective and its gradient.

* the first term equals n^-1 phi_{2H}(0) (closed form of R(K)|H|^-1/2 for the
  normal kernel);
* heat identity of the normal density: d phi_S/d S_ij (symmetric
  perturbation) = D_ij phi_S off the diagonal and 1/2 D_ii phi_S on it, by
  central differences;
* gradient w.r.t. vech(chol H): central differences with Richardson
  extrapolation, for the unbinned and the binned objective (<= 1e-7 rel);
* the phi_{2G} term does not depend on H; direct and binned objectives agree
  exactly when the data sit on grid nodes.
"""
import numpy as np
import pytest

from oracle import binned, gauss, grid, linbin, scv


def _vech_to_H(v, d):
    L = np.zeros((d, d))
    k = 0
    for j in range(d):
        for i in range(j, d):
            L[i, j] = v[k]
            k += 1
    return L @ L.T


def _fd_richardson(f, v, h):
    g = np.empty_like(v)
    for k in range(len(v)):
        e = np.zeros_like(v)
        e[k] = 1.0
        d1 = (f(v + h * e) - f(v - h * e)) / (2 * h)
        d2 = (f(v + 0.5 * h * e) - f(v - 0.5 * h * e)) / h
        g[k] = (4 * d2 - d1) / 3
    return g


def test_first_term_closed_form():
    H = np.array([[0.3, 0.1], [0.1, 0.2]])
    n = 17
    assert scv.first_term(H, n) == pytest.approx(gauss.phi(np.zeros(2), 2 * H) / n, rel=1e-14)


def test_heat_identity():
    S = np.array([[0.6, 0.2], [0.2, 0.4]])
    x = np.array([0.3, -0.5])
    h = 1e-5
    E12 = np.array([[0.0, 1.0], [1.0, 0.0]])
    E11 = np.array([[1.0, 0.0], [0.0, 0.0]])
    d12 = (gauss.phi(x, S + h * E12) - gauss.phi(x, S - h * E12)) / (2 * h)
    d11 = (gauss.phi(x, S + h * E11) - gauss.phi(x, S - h * E11)) / (2 * h)
    # perturbing S_12 and S_21 together is twice the one-sided derivative
    assert d12 == pytest.approx(2 * 0.5 * gauss.dphi(x, S, (1, 1)), rel=1e-8)
    assert d11 == pytest.approx(0.5 * gauss.dphi(x, S, (2, 0)), rel=1e-8)


@pytest.mark.parametrize("d", [2, 3])
def test_gradient_direct_fd(d):
    rng = np.random.default_rng(40 + d)
    n = 120
    X = rng.standard_normal((n, d)) @ (np.eye(d) + 0.4 * rng.standard_normal((d, d)))
    G = 0.15 * np.eye(d)
    Hq = np.eye(d) * 0.3 + 0.05
    L = np.linalg.cholesky(Hq)
    v = np.concatenate([L[j:, j] for j in range(d)])
    obj, grad = scv.objective_direct(X, Hq, G)
    fd = _fd_richardson(lambda w: scv.objective_direct(X, _vech_to_H(w, d), G, with_grad=False)[0], v, 1e-3)
    np.testing.assert_allclose(grad, fd, rtol=1e-7, atol=1e-9 * np.abs(fd).max())


def test_gradient_binned_fd():
    rng = np.random.default_rng(50)
    n, d = 500, 2
    X = rng.standard_normal((n, d)) @ np.array([[1.0, 0.0], [-0.5, 0.8]])
    G = np.array([[0.08, -0.02], [-0.02, 0.06]])
    g = grid.plan_auto(X, G, [24, 24])
    counts, _ = linbin.linbin(X, g)
    A = binned.autocorr_direct(linbin.counts_to_real(counts))
    H = np.array([[0.2, -0.05], [-0.05, 0.15]])
    L = np.linalg.cholesky(H)
    v = np.array([L[0, 0], L[1, 0], L[1, 1]])
    obj, grad = scv.objective_binned(A, n, g, H, G)
    fd = _fd_richardson(lambda w: scv.objective_binned(A, n, g, _vech_to_H(w, d), G, with_grad=False)[0], v, 1e-3)
    np.testing.assert_allclose(grad, fd, rtol=1e-7)


def test_constant_term_and_on_nodes():
    rng = np.random.default_rng(51)
    d, M = 2, 10
    lo, hi = np.array([-2.0, -1.0]), np.array([2.5, 3.0])
    g = grid.plan(lo, hi, [M, M])
    X = lo + rng.integers(0, M, size=(150, d)) * g["delta"]
    G = np.array([[0.1, 0.03], [0.03, 0.2]])
    counts, _ = linbin.linbin(X, g)
    A = binned.autocorr_direct(linbin.counts_to_real(counts))
    H1 = np.array([[0.3, 0.1], [0.1, 0.25]])
    H2 = np.array([[0.5, -0.2], [-0.2, 0.4]])
    _, _, c1 = scv.objective_binned_parts(A, 150, g, H1, G)
    _, _, c2 = scv.objective_binned_parts(A, 150, g, H2, G)
    assert c1 == c2
    ob, gb = scv.objective_binned(A, 150, g, H1, G)
    od, gd = scv.objective_direct(X, H1, G)
    assert ob == pytest.approx(od, rel=1e-13)
    np.testing.assert_allclose(gb, gd, rtol=1e-12)


def test_abs_scales_bound_the_values():
    """The absolute-value scales that judge near-cancelling entries: for one
    positive kernel (psi_0) the scale equals the value; for the SCV objective
    and every gradient entry it bounds the value (triangle inequality) and is
    strictly larger where the Hessian kernels change sign."""
    rng = np.random.default_rng(31)
    d, n, M = 2, 300, 12
    X = rng.standard_normal((n, d)) @ np.array([[1.0, 0.0], [0.5, 0.8]])
    G = np.array([[0.06, 0.02], [0.02, 0.09]])
    g = grid.plan_auto(X, G, [M, M])
    counts, _ = linbin.linbin(X, g)
    A = binned.autocorr_direct(linbin.counts_to_real(counts))
    zero = [(0, 0)]
    v = binned.vstat(A, n, g, [(1.0, G)], zero)
    s = binned.vstat_abs(A, n, g, [(1.0, G)], zero)
    assert s[0] == pytest.approx(v[0], rel=1e-14)
    H = np.array([[0.2, -0.05], [-0.05, 0.1]])
    obj, gr = scv.objective_binned(A, n, g, H, G)
    s_obj, s_gr = scv.objective_binned_scales(A, n, g, H, G)
    assert s_obj >= abs(obj)
    assert np.all(s_gr >= np.abs(gr)) and np.all(s_gr > np.abs(gr) * (1 + 1e-6))
