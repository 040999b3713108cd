"""Gaussian density phi_Sigma and its partial derivatives D^alpha phi_Sigma.

The kernel of the paper is the normal density: K_H = phi_H with the squared
bandwidth H as covariance (Sec. 1, Eq. (1)-(2); Sec. 3 after Eq. (8)).  The
r-th derivative functional psi_r (Eq. (13)) needs every partial derivative
D^alpha phi_Sigma with |alpha| = r.

Derivatives use the multivariate Hermite polynomials of z = Sigma^{-1} x:

    D^alpha phi_Sigma(x) = (-1)^{|alpha|} He_alpha(x) phi_Sigma(x),
    He_0 = 1,
    He_{alpha+e_k} = z_k He_alpha - sum_j alpha_j P_kj He_{alpha-e_j},  P = Sigma^{-1}.

(Differentiate (-1)^{|a|} He_a phi once more along x_k: d phi/dx_k = -z_k phi and
d He_a/dx_k = sum_j a_j P_kj He_{a-e_j}.)  The paper defers this computation to
an external package; the recurrence here is derived from the density itself
and is pinned against symbolic differentiation in the tests.
"""
from __future__ import annotations

import numpy as np


def phi(x, S):
    """Normal density N(0, S) at points x [..., d]."""
    x = np.asarray(x, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    d = S.shape[0]
    P = np.linalg.inv(S)
    q = np.einsum("...i,ij,...j->...", x, P, x)
    return (2 * np.pi) ** (-d / 2) * np.linalg.det(S) ** -0.5 * np.exp(-0.5 * q)


def hermite_all(x, S, r):
    """He_alpha(x) for every multi-index with |alpha| <= r, as a dict."""
    x = np.asarray(x, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    d = S.shape[0]
    P = np.linalg.inv(S)
    z = np.einsum("ij,...j->...i", P, x)
    zero = (0,) * d
    He = {zero: np.ones(x.shape[:-1])}
    level = [zero]
    for _ in range(r):
        nxt = []
        for a in level:
            for k in range(d):
                b = list(a)
                b[k] += 1
                b = tuple(b)
                if b in He:
                    continue
                val = z[..., k] * He[a]
                for j in range(d):
                    if a[j] > 0:
                        am = list(a)
                        am[j] -= 1
                        val = val - a[j] * P[k, j] * He[tuple(am)]
                He[b] = val
                nxt.append(b)
        level = nxt
    return He


def dphi(x, S, alpha):
    """D^alpha phi_S(x) for one multi-index alpha."""
    r = int(sum(alpha))
    He = hermite_all(x, S, r)
    return (-1) ** r * He[tuple(alpha)] * phi(x, S)


def dphi_many(x, S, alphas):
    """[len(alphas), ...] array of D^alpha phi_S(x)."""
    r = max(int(sum(a)) for a in alphas)
    He = hermite_all(x, S, r)
    f = phi(x, S)
    return np.stack([(-1) ** int(sum(a)) * He[tuple(a)] * f for a in alphas])
