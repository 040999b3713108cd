"""The binned double sum evaluated directly, without an FFT (Sec. 4, Eq. (14), (17)-(18)).

Eq. (14) replaces the n^2 pairs by grid counts:

    psi~ = n^-2 sum_i sum_j T(g_i - g_j) c_i c_j ,

and Eq. (17)-(18) regroup it by the lag l = i - j with k_l = T(delta o l) on the
full symmetric lag range l in [-(M-1), M-1]^d.  Writing the inner sums out,

    psi~ = n^-2 sum_l k_l A_l,    A_l = sum_i c_i c_{i+l}

(A is the autocorrelation of the counts; only i with both i and i+l on the grid
contribute).  That is the plain definition the FFT route must reproduce up to
rounding; here A is built from shifted-slice dot products and the final sum
is taken with math.fsum.  ``autocorr_gemm`` computes the same A for large
grids (matrix products of shifted slabs, still no FFT); ``autocorr_fft``
(numpy.fft) is a test-only cross check.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import gauss, multiindex


def autocorr_direct(c):
    """A_l for l in [-(M_k-1), M_k-1] per axis; array index l + (M-1)."""
    c = np.asarray(c, dtype=np.float64)
    M = c.shape
    d = c.ndim
    A = np.zeros(tuple(2 * m - 1 for m in M))
    for lag in itertools.product(*[range(-(m - 1), m) for m in M]):
        # A_{-l} = A_l: compute the lexicographically non-negative half only
        neg = tuple(-x for x in lag)
        if neg < lag:
            continue
        s1 = tuple(slice(max(0, -s), m - max(0, s)) for s, m in zip(lag, M))
        s2 = tuple(slice(max(0, s), m + min(0, s)) for s, m in zip(lag, M))
        v = float(np.dot(c[s1].ravel(), c[s2].ravel()))
        A[tuple(x + m - 1 for x, m in zip(lag, M))] = v
        A[tuple(x + m - 1 for x, m in zip(neg, M))] = v
    assert d == len(M)
    return A


def autocorr_gemm(c):
    """The same A_l = sum_i c_i c_{i+l} as ``autocorr_direct`` (same layout),
    arranged for large grids and still FFT-free.  The axes are split into
    leading axes a and trailing axes t (the last axis for d <= 3, the last two
    for d = 4).  For one trailing lag l_t the two overlapping slabs S1 = c[:, i_t]
    and S2 = c[:, i_t + l_t] give, by one matrix product (library primitive),
    G[a, b] = sum_{i_t} c[a, i_t] c[b, i_t + l_t]; then
    A(l_a, l_t) = sum_a G[a, a + l_a], i.e. the entries of G summed by their
    leading-axes lag b - a (np.bincount).  Trailing lags with l_t < 0
    (lexicographically) follow from A_{-l} = A_l."""
    c = np.asarray(c, dtype=np.float64)
    M = c.shape
    d = c.ndim
    if d == 1:
        return autocorr_direct(c)
    t = 1 if d <= 3 else 2
    lead, trail = M[:d - t], M[d - t:]
    nlead = int(np.prod(lead))
    coords = np.indices(lead).reshape(d - t, -1)
    key = np.zeros((nlead, nlead), dtype=np.int64)
    for k in range(d - t):
        diff = coords[k][None, :] - coords[k][:, None] + (lead[k] - 1)
        key = key * (2 * lead[k] - 1) + diff
    key = key.ravel()
    nkey = int(np.prod([2 * m - 1 for m in lead]))
    tshape = tuple(2 * m - 1 for m in trail)
    A = np.zeros((nkey,) + tshape)
    zero = (0,) * t
    for lt in itertools.product(*[range(-(m - 1), m) for m in trail]):
        if lt < zero:
            continue
        s1 = tuple(slice(max(0, -l), m - max(0, l)) for l, m in zip(lt, trail))
        s2 = tuple(slice(max(0, l), m + min(0, l)) for l, m in zip(lt, trail))
        S1 = c[(Ellipsis,) + s1].reshape(nlead, -1)
        S2 = c[(Ellipsis,) + s2].reshape(nlead, -1)
        col = np.bincount(key, weights=(S1 @ S2.T).ravel(), minlength=nkey)
        if lt == zero:
            # A_{-l} = A_l within this column: keep the half with l_a >= 0
            half = nkey // 2
            col[:half] = col[::-1][:half]
        A[(slice(None),) + tuple(l + m - 1 for l, m in zip(lt, trail))] = col
        A[(slice(None),) + tuple(-l + m - 1 for l, m in zip(lt, trail))] = col[::-1]
    return A.reshape(tuple(2 * m - 1 for m in M))


def autocorr_fft(c):
    """Same A via numpy.fft with zero padding to 2M (test-only cross check)."""
    c = np.asarray(c, dtype=np.float64)
    M = c.shape
    P = tuple(2 * m for m in M)
    F = np.fft.rfftn(c, s=P, axes=tuple(range(len(P))))
    a = np.fft.irfftn(F * np.conj(F), s=P, axes=tuple(range(len(P))))
    idx = [np.r_[np.arange(P[k] - (M[k] - 1), P[k]), np.arange(0, M[k])] for k in range(len(M))]
    return a[np.ix_(*idx)]


def lag_coords(g, k, M=None):
    m = int(g["M"][k]) if M is None else M
    return np.arange(-(m - 1), m) * g["delta"][k]


def lag_values(g, fn, chunk_axis0=None):
    """Evaluate fn(x) [K, ...] on the full lag grid, chunked over axis 0."""
    d = g["d"]
    axes = [lag_coords(g, k) for k in range(d)]
    L0 = len(axes[0])
    step = L0 if chunk_axis0 is None else chunk_axis0
    out = []
    for a in range(0, L0, step):
        mesh = np.meshgrid(axes[0][a:a + step], *axes[1:], indexing="ij")
        x = np.stack(mesh, axis=-1)
        out.append(fn(x))
    return np.concatenate(out, axis=1)


def _chunked_dot(g, A, fn, K):
    """fsum_l fn(delta o l)[t] * A_l for each t, chunked along axis 0."""
    d = g["d"]
    axes = [lag_coords(g, k) for k in range(d)]
    L0 = len(axes[0])
    per_row = int(np.prod([len(a) for a in axes[1:]])) if d > 1 else 1
    step = max(1, min(L0, 2_000_000 // max(1, per_row)))
    parts = [[] for _ in range(K)]
    for a in range(0, L0, step):
        mesh = np.meshgrid(axes[0][a:a + step], *axes[1:], indexing="ij")
        x = np.stack(mesh, axis=-1)
        v = fn(x)                              # [K, ...]
        Ab = A[a:a + step]
        for t in range(K):
            parts[t].append(v[t] * Ab)
    return np.array([math.fsum(np.concatenate([p.ravel() for p in parts[t]])) for t in range(K)])


def psi(A, n, g, G, r):
    """Binned psi_r(G): all unique entries, from the count autocorrelation A."""
    d = g["d"]
    alphas = multiindex.unique_alphas(d, r)
    tot = _chunked_dot(g, A, lambda x: gauss.dphi_many(x, G, alphas), len(alphas))
    return tot / float(n) ** 2


def vstat(A, n, g, terms, alphas):
    """Binned n^-2 sum sum sum_t coef_t D^alpha phi_{S_t} for each alpha."""
    def fn(x):
        out = None
        for c, S in terms:
            v = c * gauss.dphi_many(x, S, alphas)
            out = v if out is None else out + v
        return out
    return _chunked_dot(g, A, fn, len(alphas)) / float(n) ** 2


def abs_scale(A, n, g, G, alphas):
    """S_abs = n^-2 sum_l |k_l| A_l per entry: scale for near-zero entries."""
    return _chunked_dot(g, A, lambda x: np.abs(gauss.dphi_many(x, G, alphas)), len(alphas)) / float(n) ** 2


def vstat_abs(A, n, g, terms, alphas):
    """n^-2 sum_l |sum_t coef_t D^alpha phi_{S_t}(delta o l)| |A_l| for each alpha:
    the absolute-value sum that scales the comparison of near-zero entries."""
    def fn(x):
        out = None
        for c, S in terms:
            v = c * gauss.dphi_many(x, S, alphas)
            out = v if out is None else out + v
        return np.abs(out)
    return _chunked_dot(g, np.abs(A), fn, len(alphas)) / float(n) ** 2
