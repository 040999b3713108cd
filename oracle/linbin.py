"""Multivariate linear binning, bit-exact fixed-point contract (Sec. 4, first step).

The paper's first step replaces the sample by grid counts c (Eq. (14)) using
linear binning, citing Wand (1994, Sec. 3).  Linear binning gives each point
unit mass, split over the 2^d nodes of its grid cell with tensor-product
linear weights.  This project fixes the arithmetic so that counts are
reproducible bit for bit on any device:

  per point i and axis k:
    t = (X_ik - lo_k) / delta_k            (IEEE subtract then divide, no FMA)
    point is skipped (counted as out of grid) unless 0 <= t <= M_k - 1
    j = floor(t);  if j == M_k - 1: j = M_k - 2
    f = t - j;     w0 = 1 - f;  w1 = f
  per corner b in {0,1}^d (corner number sum_k b_k 2^k):
    w_b = ((w_{b_0,0} * w_{b_1,1}) * w_{b_2,2}) * ...     (left to right)
    q_b = round_half_even(w_b * 2^40)                       (int64)
  the corner with the largest q_b (lowest corner number on ties) instead gets
    q_{b*} = 2^40 - sum_{b != b*} q_b,
  so every point adds exactly 2^40.  q_b is added to the int64 count of node
  j + b.  Counts as reals: c = float64(count) * 2^-40.

Binning of n < 2^23 points cannot overflow an int64 node.
"""
from __future__ import annotations

import numpy as np

QBITS = 40
ONE = np.int64(1) << QBITS


def linbin(X, g):
    """Return (int64 counts of shape M, number of skipped points)."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    M = [int(m) for m in g["M"]]
    lo = g["lo"]
    delta = g["delta"]
    t = np.empty((n, d))
    for k in range(d):
        t[:, k] = (X[:, k] - lo[k]) / delta[k]
    inside = np.all((t >= 0.0) & (t <= np.array(M, dtype=np.float64) - 1.0), axis=1)
    t = t[inside]
    m = t.shape[0]
    j = np.floor(t).astype(np.int64)
    for k in range(d):
        j[j[:, k] == M[k] - 1, k] = M[k] - 2
    f = t - j.astype(np.float64)
    w = np.stack([1.0 - f, f], axis=0)          # [2, m, d]
    ncorner = 1 << d
    q = np.empty((ncorner, m), dtype=np.int64)
    for b in range(ncorner):
        wb = w[b & 1, :, 0].copy()
        for k in range(1, d):
            wb = wb * w[(b >> k) & 1, :, k]
        q[b] = np.rint(wb * float(ONE)).astype(np.int64)
    best = np.argmax(q, axis=0)                  # first maximum = lowest corner
    rest = q.sum(axis=0) - q[best, np.arange(m)]
    q[best, np.arange(m)] = ONE - rest
    counts = np.zeros(M, dtype=np.int64)
    flat = counts.reshape(-1)
    strides = np.ones(d, dtype=np.int64)
    for k in range(d - 2, -1, -1):
        strides[k] = strides[k + 1] * M[k + 1]
    for b in range(ncorner):
        idx = np.zeros(m, dtype=np.int64)
        for k in range(d):
            idx += (j[:, k] + ((b >> k) & 1)) * strides[k]
        np.add.at(flat, idx, q[b])
    return counts, int(n - m)


def counts_to_real(counts):
    return counts.astype(np.float64) * (2.0 ** -QBITS)
