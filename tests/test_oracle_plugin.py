"""Pins of oracle.plugin: the plug-in (AMISE) objective and its gradient.

* normal reference: with psi_4 of N(0, Sigma) integrated exactly, the AMISE
  is minimised by the normal-scale bandwidth
  H = (4/(d+2))^{2/(d+4)} n^{-2/(d+4)} Sigma (Wand & Jones, multivariate
  normal-scale rule), so the gradient vanishes there and the objective rises
  in every direction around it;
* diagonal Sigma and H: the quadratic term has the closed form
  phi_{2 Sigma}(0)/16 [(sum_i h_i/s_i)^2 + 2 sum_i (h_i/s_i)^2]
  (h_i = H_ii, s_i = Sigma_ii; fourth moments of a normal by Isserlis'
  theorem), independent of the Hermite recurrence and the Kronecker fill;
* one dimension: R(K)/(n h) + h^4 psi_4 / 4 with its minimiser
  h^5 = R(K) / (n psi_4);
* gradient w.r.t. vech(chol H) against central differences with Richardson
  extrapolation.
"""
import numpy as np
import pytest

from oracle import gauss, plugin

from test_oracle_scv import _fd_richardson, _vech_to_H


def _vech(H):
    L = np.linalg.cholesky(H)
    d = H.shape[0]
    return np.concatenate([L[j:, j] for j in range(d)])


def _spd(d, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(d, d)))
    return Q @ np.diag(10 ** rng.uniform(-0.7, 0.3, d)) @ Q.T


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_normal_scale_is_the_minimiser(d):
    n = 5000
    Sigma = _spd(d, 40 + d)
    p4 = plugin.normal_psi4(Sigma)
    Hns = (4.0 / (d + 2)) ** (2.0 / (d + 4)) * n ** (-2.0 / (d + 4)) * Sigma
    obj, g = plugin.objective(p4, n, Hns)
    # scale of the two terms' gradients separately
    from oracle import scv
    ref = np.abs(scv.vech_grad_from_matrix_grad(scv.first_term_grad(Hns, n), Hns)).max()
    assert np.abs(g).max() <= 1e-12 * ref
    rng = np.random.default_rng(7)
    v0 = _vech(Hns)
    for _ in range(8):
        dv = rng.normal(size=v0.shape) * 0.02 * np.abs(v0).max()
        assert plugin.objective(p4, n, _vech_to_H(v0 + dv, d), with_grad=False)[0] > obj


@pytest.mark.parametrize("d", [2, 3])
def test_diagonal_closed_form(d):
    rng = np.random.default_rng(3 + d)
    s = rng.uniform(0.3, 2.0, d)
    h = rng.uniform(0.05, 0.4, d)
    Sigma, H = np.diag(s), np.diag(h)
    n = 300
    obj, _ = plugin.objective(plugin.normal_psi4(Sigma), n, H, with_grad=False)
    c0 = gauss.phi(np.zeros(d), 2 * Sigma)
    t = h / s
    quad = c0 / 16.0 * (t.sum() ** 2 + 2.0 * (t ** 2).sum())
    first = (4 * np.pi) ** (-d / 2) / np.sqrt(np.prod(h)) / n
    assert obj == pytest.approx(first + quad, rel=1e-13)


def test_one_dimension():
    sigma2, n = 1.7, 400
    p4 = plugin.normal_psi4(np.array([[sigma2]]))
    # psi_4 of N(0, s^2) is 3 / (8 sqrt(pi) s^5)
    assert p4[0] == pytest.approx(3.0 / (8.0 * np.sqrt(np.pi) * sigma2 ** 2.5), rel=1e-14)
    R = 1.0 / (2.0 * np.sqrt(np.pi))
    h = 0.37
    obj, _ = plugin.objective(p4, n, np.array([[h * h]]), with_grad=False)
    assert obj == pytest.approx(R / (n * h) + 0.25 * h ** 4 * p4[0], rel=1e-14)
    hopt = (R / (n * p4[0])) ** 0.2
    _, g = plugin.objective(p4, n, np.array([[hopt * hopt]]))
    assert abs(g[0]) <= 1e-12 * R / (n * hopt * hopt)


@pytest.mark.parametrize("d", [2, 4])
def test_gradient_fd(d):
    n = 700
    p4 = plugin.normal_psi4(_spd(d, 90 + d)) * np.linspace(0.7, 1.3, len(plugin.normal_psi4(np.eye(d))))
    H = _spd(d, 70 + d) * 0.05
    v = _vech(H)
    _, g = plugin.objective(p4, n, H)
    fd = _fd_richardson(lambda w: plugin.objective(p4, n, _vech_to_H(w, d), with_grad=False)[0], v, 1e-4)
    np.testing.assert_allclose(g, fd, rtol=1e-7, atol=1e-9 * np.abs(g).max())


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_scales_bound_values(d):
    """objective_scales bounds |PI| and every |gradient entry|; with diagonal
    Sigma and H every term of the quadratic form is positive, so the objective's
    scale equals the objective itself."""
    n = 800
    Sigma = _spd(d, 70 + d)
    p4 = plugin.normal_psi4(Sigma)
    for seed in range(4):
        H = _spd(d, 80 + 7 * d + seed) * 0.1
        o, g = plugin.objective(p4, n, H)
        so, sg = plugin.objective_scales(p4, n, H)
        assert abs(o) <= so * (1 + 1e-14)
        assert np.all(np.abs(g) <= sg * (1 + 1e-14))
        assert np.all(sg <= 100 * np.abs(g).max())
    Sd = np.diag(np.linspace(0.5, 1.5, d))
    Hd = np.diag(np.linspace(0.05, 0.2, d))
    p4d = plugin.normal_psi4(Sd)
    o, _ = plugin.objective(p4d, n, Hd)
    so, _ = plugin.objective_scales(p4d, n, Hd)
    assert so == pytest.approx(o, rel=1e-13)
