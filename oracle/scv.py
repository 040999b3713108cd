"""Smoothed cross-validation (SCV) objective and its exact gradient.

The paper lists SCV among the selectors its FFT route serves (Sec. 3, Sec. 5:
the PI and SCV criteria are double sums of Gaussian derivative functions) but
prints no formula.  This project reads it as the standard Gaussian-kernel SCV
criterion in V-statistic form (all pairs, diagonal included, as the paper's
V-statistics Eq. (28)-(29)), with pilot bandwidth G:

  SCV(H) = n^-1 (4 pi)^{-d/2} |H|^{-1/2}
         + n^-2 sum_i sum_j [phi_{2H+2G} - 2 phi_{H+2G} + phi_{2G}](X_i - X_j).

Gradient.  For a symmetric matrix argument, d phi_S = tr(1/2 D^2 phi_S dS)
(the heat equation of the normal density), and d|H|^{-1/2} =
-1/2 |H|^{-1/2} tr(H^{-1} dH), so with dSCV = tr(grad_H dH):

  grad_H = -1/2 n^-1 (4 pi)^{-d/2} |H|^{-1/2} H^{-1}
         + n^-2 sum_i sum_j [D^2 phi_{2H+2G} - D^2 phi_{H+2G}](X_i - X_j),

where D^2 phi is the Hessian matrix.  For H = L L^T (L lower, Cholesky),
dSCV/dL = lower(2 grad_H L), returned as vech (columns of the lower triangle).

Both the unbinned sums (``objective_direct``) and the binned sums evaluated
through the count autocorrelation (``objective_binned``) are provided.
"""
from __future__ import annotations

import numpy as np

from . import binned, direct, multiindex


def first_term(H, n):
    d = H.shape[0]
    return (4 * np.pi) ** (-d / 2) * np.linalg.det(H) ** -0.5 / n


def first_term_grad(H, n):
    return -0.5 * first_term(H, n) * np.linalg.inv(H)


def _terms_obj(H, G):
    return [(1.0, 2 * H + 2 * G), (-2.0, H + 2 * G), (1.0, 2 * G)]


def _terms_hess(H, G):
    return [(1.0, 2 * H + 2 * G), (-1.0, H + 2 * G)]


def _hess_from_unique(vals, d):
    Hm = np.empty((d, d))
    for k, (i, j) in enumerate(multiindex.unique_tuples(d, 2)):
        Hm[i, j] = Hm[j, i] = vals[k]
    return Hm


def vech_grad_from_matrix_grad(gH, H):
    """dSCV/d vech(L) from the symmetric gradient grad_H, H = L L^T."""
    L = np.linalg.cholesky(H)
    gL = np.tril(2.0 * gH @ L)
    d = H.shape[0]
    return np.concatenate([gL[j:, j] for j in range(d)])


def objective_direct(X, H, G, workers=None, with_grad=True):
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    zero = [(0,) * d]
    obj = first_term(H, n) + direct.vstat(X, _terms_obj(H, G), zero, workers)[0]
    if not with_grad:
        return obj, None
    alphas2 = multiindex.unique_alphas(d, 2)
    hv = direct.vstat(X, _terms_hess(H, G), alphas2, workers)
    gH = first_term_grad(H, n) + _hess_from_unique(hv, d)
    return obj, vech_grad_from_matrix_grad(gH, H)


def objective_binned(A, n, g, H, G, with_grad=True):
    d = g["d"]
    zero = [(0,) * d]
    obj = first_term(H, n) + binned.vstat(A, n, g, _terms_obj(H, G), zero)[0]
    if not with_grad:
        return obj, None
    alphas2 = multiindex.unique_alphas(d, 2)
    hv = binned.vstat(A, n, g, _terms_hess(H, G), alphas2)
    gH = first_term_grad(H, n) + _hess_from_unique(hv, d)
    return obj, vech_grad_from_matrix_grad(gH, H)


def objective_binned_parts(A, n, g, H, G):
    """Binned pieces: (first term, H-dependent double sum, constant phi_{2G} sum)."""
    d = g["d"]
    zero = [(0,) * d]
    var = binned.vstat(A, n, g, [(1.0, 2 * H + 2 * G), (-2.0, H + 2 * G)], zero)[0]
    const = binned.vstat(A, n, g, [(1.0, 2 * G)], zero)[0]
    return first_term(H, n), var, const


def objective_binned_scales(A, n, g, H, G):
    """Absolute-value scales of the binned objective and of each entry of its
    vech gradient: |closed-form term| + n^-2 sum_l |kernel_l| A_l for the
    objective and for every Hessian entry, carried through the chain rule
    dSCV/dL = lower(2 grad_H L) with absolute values.  Used to judge entries
    that nearly cancel (relative error against this scale)."""
    d = g["d"]
    zero = [(0,) * d]
    s_obj = abs(first_term(H, n)) + binned.vstat_abs(A, n, g, _terms_obj(H, G), zero)[0]
    alphas2 = multiindex.unique_alphas(d, 2)
    hv = binned.vstat_abs(A, n, g, _terms_hess(H, G), alphas2)
    sH = np.abs(first_term_grad(H, n)) + _hess_from_unique(hv, d)
    L = np.abs(np.linalg.cholesky(H))
    sL = np.tril(2.0 * sH @ L)
    return s_obj, np.concatenate([sL[j:, j] for j in range(d)])
