"""Pins of the reference side of the minimiser tests (CPU): scipy's BFGS over
vech(chol H) on the oracle's PI objective with the exact psi_4 of a normal
density must land on the normal-scale bandwidth, the closed-form minimiser of
the normal-kernel AMISE for normal data; and on the oracle's SCV objective a
reference minimiser must be a stationary point that no nearby H improves."""
import numpy as np
import pytest

from oracle import binned, grid, linbin, plugin, scv

from _minref import H_of, argmin_vech, normal_scale_H


def _spd(d, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((d, d))
    return A @ A.T / d + 0.3 * np.eye(d)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_pi_reference_minimiser_is_normal_scale(d):
    Sigma = _spd(d, 7 + d)
    n = 1000
    psi4 = plugin.normal_psi4(Sigma)
    fun = lambda H: plugin.objective(psi4, n, H)
    L0 = np.linalg.cholesky(0.5 * np.eye(d))
    v0 = np.concatenate([L0[j:, j] for j in range(d)])
    v, _ = argmin_vech(fun, v0, d)
    H = H_of(v, d)
    Hns = normal_scale_H(Sigma, n)
    assert np.abs(H - Hns).max() <= 1e-7 * np.abs(Hns).max(), (H, Hns)


def test_scv_reference_minimiser_is_a_local_minimum():
    rng = np.random.default_rng(5)
    n, d, M = 800, 2, 24
    X = rng.standard_normal((n, d)) @ np.array([[1.0, 0.0], [0.5, 0.7]])
    G = 0.1 * np.cov(X.T)
    g = grid.plan_auto(X, G, [M, M])
    co, sk = linbin.linbin(X, g)
    assert sk == 0
    A = binned.autocorr_direct(linbin.counts_to_real(co))
    fun = lambda H: scv.objective_binned(A, n, g, H, G)
    H0 = 0.3 * np.cov(X.T)
    L0 = np.linalg.cholesky(H0)
    v, fmin = argmin_vech(fun, np.concatenate([L0[j:, j] for j in range(d)]), d)
    _, gr = fun(H_of(v, d))
    assert np.abs(gr).max() * np.abs(v).max() <= 1e-7 * abs(fmin)
    for k in range(v.size):
        for s in (1e-3, -1e-3):
            w = v.copy()
            w[k] *= 1 + s
            assert fun(H_of(w, d))[0] >= fmin
