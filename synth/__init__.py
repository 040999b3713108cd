"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws data and bandwidth matrices.  It holds none of the
method's arithmetic (no binning, no kernel derivatives, no sums): the CPU
reference in ``oracle/`` and the HIP library both receive what is drawn here
as plain arrays.

Workloads follow the shapes of the paper's own experiments (Sec. 6: bivariate
normal mixtures, N(0, I) speed runs) widened to the five benchmark cases of
this project.  Every draw comes from ``numpy.random.default_rng(151107482 + k)``
for case ``k``, so a case is reproducible bit for bit on any host.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

SEED_BASE = 151107482


def rng_for(case: int, salt: int = 0) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + case + 1000 * salt)


# ---------------------------------------------------------------- sampling


def sample_mixture(n, weights, means, covs, rng):
    """n draws from sum_l w_l N(mu_l, Sigma_l), shape [n, d], float64."""
    weights = np.asarray(weights, dtype=np.float64)
    means = np.asarray(means, dtype=np.float64)
    covs = np.asarray(covs, dtype=np.float64)
    d = means.shape[1]
    lab = rng.choice(len(weights), size=n, p=weights / weights.sum())
    z = rng.standard_normal((n, d))
    X = np.empty((n, d))
    for l in range(len(weights)):
        idx = lab == l
        Lc = np.linalg.cholesky(covs[l])
        X[idx] = means[l] + z[idx] @ Lc.T
    return X


def haar_orthogonal(d, rng):
    """Haar-distributed orthogonal matrix (QR of a Gaussian matrix, sign-fixed)."""
    A = rng.standard_normal((d, d))
    Q, R = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(R))[None, :]
    return Q


def unit_vector(d, rng):
    v = rng.standard_normal(d)
    return v / np.linalg.norm(v)


def rot2(theta):
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[c, -s], [s, c]])


def sample_cov(X):
    """Unbiased sample covariance."""
    return np.cov(X, rowvar=False, ddof=1).reshape(X.shape[1], X.shape[1])


def normal_scale_pilot(X, rate_den):
    """G = n^{-2/rate_den} * S_hat (documented stand-in for a pilot bandwidth)."""
    n = X.shape[0]
    return n ** (-2.0 / rate_den) * sample_cov(X)


def normal_scale_H(X):
    """Normal-scale bandwidth (4/(d+2))^{2/(d+4)} n^{-2/(d+4)} S_hat."""
    n, d = X.shape
    return (4.0 / (d + 2)) ** (2.0 / (d + 4)) * n ** (-2.0 / (d + 4)) * sample_cov(X)


def random_H_2d(B, rng):
    """B random SPD 2x2: R_theta diag(e^u1, e^u2) R_theta^T, u~U[-3,0], theta~U[0,pi)."""
    out = np.empty((B, 2, 2))
    for b in range(B):
        u = rng.uniform(-3.0, 0.0, size=2)
        th = rng.uniform(0.0, np.pi)
        R = rot2(th)
        out[b] = R @ np.diag(np.exp(u)) @ R.T
    return 0.5 * (out + out.transpose(0, 2, 1))


def random_H_haar(B, d, rng):
    """B random SPD dxd: Q diag(e^u) Q^T, u~U[-3,0]^d, Q Haar."""
    out = np.empty((B, d, d))
    for b in range(B):
        u = rng.uniform(-3.0, 0.0, size=d)
        Q = haar_orthogonal(d, rng)
        out[b] = Q @ np.diag(np.exp(u)) @ Q.T
    return 0.5 * (out + out.transpose(0, 2, 1))


def vech_chol(H):
    """vech of the lower Cholesky factor, columns of the lower triangle stacked:
    (L11, L21, ..., Ld1, L22, ..., Ldd).  H: [..., d, d] -> [..., d(d+1)/2]."""
    H = np.asarray(H, dtype=np.float64)
    L = np.linalg.cholesky(H)
    d = H.shape[-1]
    cols = [L[..., j:, j] for j in range(d)]
    return np.concatenate(cols, axis=-1)


# ---------------------------------------------------------------- workloads


@dataclasses.dataclass
class Workload:
    name: str
    d: int
    M: int
    r: int
    X: List[np.ndarray]                 # one [n_j, d] array per dataset
    G_psi: List[np.ndarray]             # bandwidth for psi_r per dataset
    G_pilot: List[Optional[np.ndarray]]  # SCV pilot per dataset (None: no SCV)
    H: List[Optional[np.ndarray]]       # SCV candidates per dataset [B_j, d, d]
    grid_G: List[np.ndarray]            # bandwidth whose sd pads the grid
    note: str = ""


def _mix2d_case2(n, rng):
    weights = np.full(4, 0.25)
    th = np.arange(4) * np.pi / 2
    means = 1.5 * np.stack([np.cos(th), np.sin(th)], axis=1)
    covs = []
    for _ in range(4):
        sd = rng.uniform(0.5, 1.0, size=2)
        rho = rng.uniform(-0.6, 0.6)
        covs.append(np.array([[sd[0] ** 2, rho * sd[0] * sd[1]],
                              [rho * sd[0] * sd[1], sd[1] ** 2]]))
    return sample_mixture(n, weights, means, np.array(covs), rng)


def _haar_cov(d, rng):
    lam = 10.0 ** rng.uniform(-1.0, 0.0, size=d)
    Q = haar_orthogonal(d, rng)
    S = Q @ np.diag(lam) @ Q.T
    return 0.5 * (S + S.T)


def case1(n=1000):
    """Plain psi_0, d=2: N(0, [[1,.7],[.7,1]]), G=[[.10,.06],[.06,.20]], M=64."""
    rng = rng_for(1)
    C = np.array([[1.0, 0.7], [0.7, 1.0]])
    X = rng.standard_normal((n, 2)) @ np.linalg.cholesky(C).T
    G = np.array([[0.10, 0.06], [0.06, 0.20]])
    return Workload("case1 psi_0 d=2 n=1e3 M=64", 2, 64, 0, [X], [G], [None], [None], [G])


def case2(n=100_000):
    """Plain psi_4, d=2: 4-component mixture, G = n^{-2/10} S_hat, M=256."""
    rng = rng_for(2)
    X = _mix2d_case2(n, rng)
    G = normal_scale_pilot(X, 10)
    return Workload("case2 psi_4 d=2 n=1e5 M=256", 2, 256, 4, [X], [G], [None], [None], [G])


def case3(n=200_000):
    """psi_2 + SCV, d=3: 3-component mixture (weights .5/.3/.2), M=64."""
    rng = rng_for(3)
    d = 3
    means = np.stack([1.5 * unit_vector(d, rng) for _ in range(3)])
    covs = np.stack([_haar_cov(d, rng) for _ in range(3)])
    X = sample_mixture(n, [0.5, 0.3, 0.2], means, covs, rng)
    G = normal_scale_pilot(X, 9)
    H = normal_scale_H(X)[None]
    return Workload("case3 psi_2+SCV d=3 n=2e5 M=64", 3, 64, 2, [X], [G], [G], [H], [G])


def case4(n=100_000, B=256):
    """Batched SCV + adjoint, d=2: case-2 mixture, pilot n^{-2/8} S_hat, 256 H, M=256."""
    rng = rng_for(2)            # same data as case 2
    X = _mix2d_case2(n, rng)
    Gpsi = normal_scale_pilot(X, 10)
    Gp = normal_scale_pilot(X, 8)
    H = random_H_2d(B, rng_for(4))
    return Workload("case4 SCV batch d=2 n=1e5 M=256 B=256", 2, 256, 4, [X], [Gpsi], [Gp], [H], [Gp])


def case5(n_datasets=32, B=64, n_lo=10_000, n_hi=1_000_000, M=32):
    """Uneven batched SCV + adjoint, d=4: 32 two-component mixtures, n~U[1e4,1e6]."""
    rng = rng_for(5)
    d = 4
    Xs, Gpsi, Gp, Hs = [], [], [], []
    ns = rng.integers(n_lo, n_hi + 1, size=n_datasets)
    for j in range(n_datasets):
        w = rng.uniform(0.3, 0.7)
        v = unit_vector(d, rng)
        covs = np.stack([_haar_cov(d, rng) for _ in range(2)])
        X = sample_mixture(int(ns[j]), [w, 1 - w], np.stack([v, -v]), covs, rng)
        Xs.append(X)
        Gpsi.append(normal_scale_pilot(X, 12))
        Gp.append(normal_scale_pilot(X, 10))
        Hs.append(random_H_haar(B, d, rng))
    return Workload(f"case5 uneven SCV batch d=4 {n_datasets} datasets M={M} B={B}/dataset",
                    d, M, 4, Xs, Gpsi, Gp, Hs, Gp)


CASES = {1: case1, 2: case2, 3: case3, 4: case4, 5: case5}
