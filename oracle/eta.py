"""Scalar Gaussian-derivative V-statistics (Sec. 5) and LSCV_r (Sec. 3, Sec. 5).

Sec. 5 contracts the 2r-th derivative vector with the r-th Kronecker power of
vec I (Eq. (30)-(31)):

    eta_r(x; S) = (vec^T I_d)^{(x)r} D^{(x)2r} phi_S(x),

and the V-statistic of Eq. (32) is Q_r(S) = n^-2 sum_i sum_j eta_r(X_i - X_j; S).
Written out, the contraction picks from D^{(x)2r} the entries whose index
tuple is (i_1, i_1, i_2, i_2, ..., i_r, i_r) and sums them over all d^r
choices of (i_1, ..., i_r); ``eta_terms`` enumerates exactly those choices and
groups equal multi-indices (mixed partials commute).

LSCV_r.  Eq. (35) is the leave-one-out form and Eq. (36) the form with
n - 1 replaced by n.  Eq. (36) prints K_H(0) for the diagonal correction at
every r; that is only the r = 0 value, so this project reads it as
eta_r(0; H), which is what removing the i = j terms of the H-sum produces.

  exact=False (Eq. (36)):  (-1)^r { V(2H) - 2 V(H) + 2 n^-1 eta_r(0; H) }
  exact=True  (Eq. (35)):  (-1)^r { V(2H) - 2 n/(n-1) V(H) + 2 (n-1)^-1 eta_r(0; H) }

with V(S) = n^-2 sum_i sum_j eta_r(X_i - X_j; S) over all pairs.  In binned form
the pairs are the lag sum of the count autocorrelation, so subtracting the
diagonal is itself an approximation (the binned self-pairs are smeared).

The r = 0 criterion is the paper's LSCV (Eq. (8)-(11)).  Its gradient follows
from the heat identity d phi_S = tr(1/2 D^2 phi_S dS):

  grad_H = n^-2 sum sum D^2 phi_{2H} - (a/2) n^-2 sum sum D^2 phi_H - (b/2) phi_H(0) H^-1,

with a = 2 (or 2n/(n-1)) the weight of V(H) and b = 2/n (or 2/(n-1)) the weight
of phi_H(0); chained to vech(chol H) as for SCV.
"""
from __future__ import annotations

import itertools
from collections import Counter

import numpy as np

from . import binned, direct, gauss, multiindex, scv


def eta_terms(d, r):
    """[(alpha, count)]: multi-indices 2*(counts of i_1..i_r) over all d^r tuples."""
    cnt = Counter()
    for tup in itertools.product(range(d), repeat=r):
        a = [0] * d
        for i in tup:
            a[i] += 2
        cnt[tuple(a)] += 1
    return sorted(cnt.items())


def eta(x, S, r):
    """eta_r(x; S) at points x [..., d]."""
    S = np.asarray(S, dtype=np.float64)
    d = S.shape[0]
    terms = eta_terms(d, r)
    vals = gauss.dphi_many(np.asarray(x, dtype=np.float64), S, [a for a, _ in terms])
    return sum(c * vals[k] for k, (_, c) in enumerate(terms))


def _lag_fn(terms_S, r, absval=False):
    def fn(x):
        v = 0.0
        for coef, S in terms_S:
            v = v + coef * eta(x, S, r)
        v = np.abs(v) if absval else v
        return v[None]
    return fn


def vstat_binned(A, n, g, terms_S, r, absval=False):
    """n^-2 sum_l [sum_t coef_t eta_r(delta o l; S_t)] A_l (absval: |.| inside)."""
    return binned._chunked_dot(g, A, _lag_fn(terms_S, r, absval), 1)[0] / float(n) ** 2


class _EtaPairs:
    def __init__(self, terms_S, r):
        self.terms_S = terms_S
        self.r = r

    def __call__(self, x):
        v = 0.0
        for coef, S in self.terms_S:
            v = v + coef * eta(x, S, self.r)
        return np.asarray(v)[None]


def vstat_direct(X, terms_S, r, workers=None):
    """n^-2 sum_i sum_j sum_t coef_t eta_r(X_i - X_j; S_t), all pairs."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    fn = _EtaPairs(terms_S, r)
    off = direct.pair_sum_upper(X, fn, 1, workers)[0]
    diag = float(fn(np.zeros((d,)))[0])
    return (n * diag + 2.0 * off) / float(n) ** 2


def qr_binned(A, n, g, S, r):
    """Binned Q_r(S) (Eq. (32))."""
    return vstat_binned(A, n, g, [(1.0, S)], r)


def qr_direct(X, S, r, workers=None):
    """Unbinned Q_r(S) (Eq. (32))."""
    return vstat_direct(X, [(1.0, S)], r, workers)


def _lscv_weights(n, exact):
    a = 2.0 * n / (n - 1.0) if exact else 2.0
    b = 2.0 / (n - 1.0) if exact else 2.0 / n
    return a, b


def lscv_r_binned(A, n, g, H, r, exact=False):
    a, b = _lscv_weights(n, exact)
    d = g["d"]
    V = vstat_binned(A, n, g, [(1.0, 2 * H), (-a, H)], r)
    return (-1) ** r * (V + b * float(eta(np.zeros(d), H, r)))


def lscv_r_direct(X, H, r, exact=False, workers=None):
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    a, b = _lscv_weights(n, exact)
    V = vstat_direct(X, [(1.0, 2 * H), (-a, H)], r, workers)
    return (-1) ** r * (V + b * float(eta(np.zeros(d), H, r)))


def lscv_abs_scale(A, n, g, H, r, exact=False):
    """n^-2 sum_l |k_l| A_l for the LSCV_r lag kernel (scale for near-zero values)."""
    a, _ = _lscv_weights(n, exact)
    return vstat_binned(A, n, g, [(1.0, 2 * H), (-a, H)], r, absval=True)


def _grad_from_hess(hv_2H, hv_H, H, n, exact):
    d = H.shape[0]
    a, b = _lscv_weights(n, exact)
    gH = scv._hess_from_unique(hv_2H, d) - 0.5 * a * scv._hess_from_unique(hv_H, d)
    gH = gH - 0.5 * b * float(gauss.phi(np.zeros(d), H)) * np.linalg.inv(H)
    return scv.vech_grad_from_matrix_grad(gH, H)


def lscv_binned(A, n, g, H, exact=False, with_grad=True):
    """LSCV (r = 0) and its gradient w.r.t. vech(chol H), binned form."""
    obj = lscv_r_binned(A, n, g, H, 0, exact)
    if not with_grad:
        return obj, None
    al = multiindex.unique_alphas(g["d"], 2)
    h2 = binned.vstat(A, n, g, [(1.0, 2 * H)], al)
    h1 = binned.vstat(A, n, g, [(1.0, H)], al)
    return obj, _grad_from_hess(h2, h1, H, n, exact)


def lscv_binned_scales(A, n, g, H, exact=False):
    """Absolute-value scales of the binned LSCV (r = 0) and of each entry of its
    vech gradient: the objective's |lag kernel| sum plus the diagonal term,
    and for the gradient |D^2 phi_{2H}| and (a/2)|D^2 phi_H| summed against A
    plus (b/2) phi_H(0) |H^-1|, carried through dLSCV/dL = lower(2 grad_H L)
    with absolute values.  Used to judge entries that nearly cancel."""
    d = g["d"]
    a, b = _lscv_weights(n, exact)
    phi0 = float(gauss.phi(np.zeros(d), H))
    s_obj = lscv_abs_scale(A, n, g, H, 0, exact) + b * phi0
    al = multiindex.unique_alphas(d, 2)
    h2 = binned.vstat_abs(A, n, g, [(1.0, 2 * H)], al)
    h1 = binned.vstat_abs(A, n, g, [(1.0, H)], al)
    sH = (scv._hess_from_unique(h2, d) + 0.5 * a * scv._hess_from_unique(h1, d)
          + 0.5 * b * phi0 * np.abs(np.linalg.inv(H)))
    L = np.abs(np.linalg.cholesky(H))
    sL = np.tril(2.0 * sH @ L)
    return s_obj, np.concatenate([sL[j:, j] for j in range(d)])


def lscv_direct(X, H, exact=False, with_grad=True, workers=None):
    """LSCV (r = 0) and its gradient, unbinned pairs."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    obj = lscv_r_direct(X, H, 0, exact, workers)
    if not with_grad:
        return obj, None
    al = multiindex.unique_alphas(d, 2)
    h2 = direct.vstat(X, [(1.0, 2 * H)], al, workers)
    h1 = direct.vstat(X, [(1.0, H)], al, workers)
    return obj, _grad_from_hess(h2, h1, H, n, exact)
