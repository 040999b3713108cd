"""Direct (unbinned) double sums, O(n^2) (Sec. 4, Eq. (12)-(13); Sec. 6.3 'direct').

psi_alpha(G) = n^-2 sum_i sum_j D^alpha phi_G(X_i - X_j)                 (Eq. (13))
            = n^-2 [ n D^alpha phi_G(0) + 2 sum_{i<j} D^alpha phi_G(X_i - X_j) ]

(the summand is even in X_i - X_j for even |alpha|).  Pairs are summed in row
blocks: NumPy's pairwise summation inside a block, math.fsum across blocks.
Row blocks can be spread over worker processes.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import gauss, multiindex

BLOCK = 1024


def _block_pairs(X, a, b, fn):
    """Sum over i in [a,b), j > i of fn(X_i - X_j) -> array [k]."""
    xi = X[a:b]
    acc = None
    parts = []
    for c in range(a, X.shape[0], BLOCK):
        xj = X[c:c + BLOCK]
        diff = xi[:, None, :] - xj[None, :, :]
        vals = fn(diff)                                  # [k, bi, bj]
        ii = np.arange(a, b)[:, None]
        jj = np.arange(c, c + xj.shape[0])[None, :]
        mask = jj > ii
        parts.append(np.where(mask[None], vals, 0.0).reshape(vals.shape[0], -1).sum(axis=1))
    if parts:
        acc = np.stack(parts)                            # [nblocks, k]
    return acc


class _PairFn:
    """Picklable function of pair differences -> [k, ...] values."""

    def __init__(self, S, alphas, weights=None):
        self.S = np.asarray(S, dtype=np.float64)
        self.alphas = [tuple(a) for a in alphas]
        self.weights = weights

    def __call__(self, diff):
        return gauss.dphi_many(diff, self.S, self.alphas)


class _ComboFn:
    """Linear combination of derivative families: sum_t coef_t D^{alpha} phi_{S_t}."""

    def __init__(self, terms, alphas):
        self.terms = [(float(c), np.asarray(S, dtype=np.float64)) for c, S in terms]
        self.alphas = [tuple(a) for a in alphas]

    def __call__(self, diff):
        out = None
        for c, S in self.terms:
            v = c * gauss.dphi_many(diff, S, self.alphas)
            out = v if out is None else out + v
        return out


def _worker(args):
    X, a, b, fn = args
    return _block_pairs(X, a, b, fn)


def pair_sum_upper(X, fn, k, workers=None):
    """sum_{i<j} fn(X_i - X_j) for a k-vector-valued fn, exactly summed across blocks."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    jobs = [(X, a, min(a + BLOCK, n), fn) for a in range(0, n, BLOCK)]
    if workers is None:
        workers = 1
    if workers > 1 and len(jobs) > 1:
        with ProcessPoolExecutor(max_workers=workers) as ex:
            res = list(ex.map(_worker, jobs))
    else:
        res = [_worker(j) for j in jobs]
    res = [r for r in res if r is not None]
    allp = np.concatenate(res, axis=0) if res else np.zeros((0, k))
    return np.array([math.fsum(allp[:, t]) for t in range(k)])


def psi(X, G, r, workers=None):
    """All unique entries of psi_r(G) (order of multiindex.unique_tuples)."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    alphas = multiindex.unique_alphas(d, r)
    fn = _PairFn(G, alphas)
    off = pair_sum_upper(X, fn, len(alphas), workers)
    diag = gauss.dphi_many(np.zeros(d), G, alphas)
    return (n * diag + 2.0 * off) / float(n) ** 2


def vstat(X, terms, alphas, workers=None):
    """n^-2 sum_i sum_j sum_t coef_t D^alpha phi_{S_t}(X_i - X_j) for each alpha."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    fn = _ComboFn(terms, alphas)
    off = pair_sum_upper(X, fn, len(alphas), workers)
    diag = fn(np.zeros((d,)))
    return (n * diag + 2.0 * off) / float(n) ** 2


def default_workers():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1
