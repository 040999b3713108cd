"""fft-L: the truncated-support variant of the binned sum (Sec. 4, Eq. (25)-(27)).

Eq. (25) keeps only the lags |l_k| <= L_k of the binned double sum; Eq. (26)
chooses L_k = min(M_k - 1, ceil(tau sqrt(lambda) / delta_k)) with lambda the
largest eigenvalue of the bandwidth matrix and tau = 3.7 suggested for the
two-dimensional normal kernel; Eq. (27) pads each axis to
P_k = 2^ceil(log2(M_k + 2 L_k - 1)).  The truncated sum is an approximation
of Eq. (17) (exact when every L_k = M_k - 1).
"""
from __future__ import annotations

import math

import numpy as np

from . import binned, gauss, multiindex

TAU = 3.7


def plan_L(g, S, tau=TAU):
    """L_k of Eq. (26) for bandwidth matrix S on grid g."""
    lam = float(np.max(np.linalg.eigvalsh(np.asarray(S, dtype=np.float64))))
    out = []
    for k in range(g["d"]):
        m = int(g["M"][k])
        out.append(min(m - 1, math.ceil(tau * math.sqrt(abs(lam)) / float(g["delta"][k]))))
    return out


def plan_P(M, L):
    """P_k of Eq. (27): the smallest power of two >= M_k + 2 L_k - 1."""
    out = []
    for m, l in zip(M, L):
        x = int(m) + 2 * int(l) - 1
        p = 1
        while p < x:
            p *= 2
        out.append(p)
    return out


def psi_truncated(A, n, g, G, r, L, absval=False):
    """Binned psi_r(G) over the lags |l_k| <= L_k only (Eq. (25)); absval: the
    same sum of |kernel| (scale for near-zero entries)."""
    d = g["d"]
    M = [int(m) for m in g["M"]]
    alphas = multiindex.unique_alphas(d, r)
    # restrict the autocorrelation (index l + M - 1) to the box
    sl = tuple(slice(m - 1 - l, m + l) for m, l in zip(M, L))
    Ab = A[sl]
    axes = [np.arange(-l, l + 1) * g["delta"][k] for k, l in enumerate(L)]
    mesh = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1)
    vals = gauss.dphi_many(mesh, G, alphas)
    if absval:
        vals = np.abs(vals)
    return np.array([math.fsum((vals[t] * Ab).ravel()) for t in range(len(alphas))]) / float(n) ** 2
