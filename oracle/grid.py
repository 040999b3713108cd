"""Grid planning (Sec. 4, Eq. (15)-(16)).

The paper asks for an equally spaced grid g_{k1} < ... < g_{kM_k} per axis whose
span contains the data, with binwidth delta_k = (g_{kM_k} - g_{k1})/(M_k - 1)
(Eq. (16)).  It does not fix the span; this project pads the data range by
``pad_sd`` kernel standard deviations, sqrt(G_kk), on each side:

    lo_k = min_i X_ik - pad_sd*sqrt(G_kk),  hi_k = max_i X_ik + pad_sd*sqrt(G_kk),
    delta_k = (hi_k - lo_k) / (M_k - 1),

each step one IEEE float64 operation in that order, so that the HIP library
(which plans the grid on the host with the same operations) produces the
same bits.  The zero-padded transform length of the circular layout is the
smallest power of two P_k >= max(4, 2 M_k - 1) (any P_k >= 2M_k - 1 gives the
exact circular result; P_k = 2 M_k when M_k is a power of two).
"""
from __future__ import annotations

import math

import numpy as np


def plan(lo, hi, M):
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    M = np.asarray(M, dtype=np.int64)
    delta = (hi - lo) / (M - 1).astype(np.float64)
    P = np.array([max(4, 1 << int(2 * m - 2).bit_length()) for m in M], dtype=np.int64)
    return {"d": len(lo), "M": M, "P": P, "lo": lo.copy(), "delta": delta}


def plan_auto(X, G, M, pad_sd=4.0):
    X = np.asarray(X, dtype=np.float64)
    d = X.shape[1]
    if np.isscalar(M):
        M = [int(M)] * d
    sd = np.array([math.sqrt(float(G[k][k])) for k in range(d)])
    pad = np.array([pad_sd * sd[k] for k in range(d)])
    lo = np.array([float(X[:, k].min()) - pad[k] for k in range(d)])
    hi = np.array([float(X[:, k].max()) + pad[k] for k in range(d)])
    return plan(lo, hi, M)


def nodes(g, k):
    """Grid node coordinates along axis k: lo_k + j*delta_k, j = 0..M_k-1."""
    return g["lo"][k] + np.arange(g["M"][k]) * g["delta"][k]
