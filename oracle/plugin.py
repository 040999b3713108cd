"""Plug-in (PI) objective for an unconstrained bandwidth and its gradient.

Sec. 5 names the plug-in selector among those whose main cost is a double sum
of Gaussian derivatives (its r = 4 functional psi_4 of Eq. (13)), and leaves
the criterion itself to the literature.  This project reads it as the usual
asymptotic MISE of the normal-kernel estimator with the fourth-derivative
functional replaced by its estimate psi_4(G) at a pilot bandwidth G:

  PI(H) = n^-1 (4 pi)^{-d/2} |H|^{-1/2} + 1/4 (vec H (x) vec H)^T psi_4,

where psi_4 is the d^4 Kronecker-ordered vector of Sec. 5 (first index
slowest; filled from the unique entries by multiset lookup) and vec stacks the
columns of H.  For the normal kernel the second moment is the identity, so no
further constant appears.

Gradient.  The quadratic term is 1/4 sum_{ijkl} H_ij H_kl psi_ijkl with psi
symmetric in all four indices, so its derivative in H_ij is
1/2 sum_kl psi_ijkl H_kl; the first term gives -1/2 (first term) H^{-1}.
With dPI = tr(grad_H dH) for symmetric dH and H = L L^T,
dPI/dL = lower(2 grad_H L), returned as vech (columns of the lower triangle).
"""
from __future__ import annotations

import numpy as np

from . import multiindex, scv


def psi4_tensor(psi4_unique, d):
    """[d, d, d, d] array of the fourth-derivative functional."""
    return multiindex.expand_full(np.asarray(psi4_unique, dtype=np.float64), d, 4).reshape((d,) * 4)


def objective(psi4_unique, n, H, with_grad=True):
    """PI(H) and dPI/d vech(chol H) from the unique entries of psi_4."""
    H = np.asarray(H, dtype=np.float64)
    d = H.shape[0]
    T = psi4_tensor(psi4_unique, d)
    vecH = H.reshape(-1, order="F")
    quad = 0.25 * float(np.kron(vecH, vecH) @ T.reshape(-1))
    obj = scv.first_term(H, n) + quad
    if not with_grad:
        return obj, None
    gH = scv.first_term_grad(H, n) + 0.5 * np.einsum("ijkl,kl->ij", T, H)
    return obj, scv.vech_grad_from_matrix_grad(gH, H)


def objective_scales(psi4_scale, n, H):
    """Absolute-value scales of PI(H) and of each entry of its vech gradient,
    from per-entry bounds psi4_scale >= |psi_4| (its absolute values, or the
    absolute-value lag sums of an estimate): the first term's magnitude plus
    1/4 sum |H_ij| |H_kl| psi4_scale_ijkl, and for the gradient
    |d first term / dH| + 1/2 sum_kl psi4_scale_ijkl |H_kl|, carried through
    dPI/dL = lower(2 grad_H L) with absolute values."""
    H = np.asarray(H, dtype=np.float64)
    d = H.shape[0]
    T = psi4_tensor(np.abs(np.asarray(psi4_scale, dtype=np.float64)), d)
    aH = np.abs(H)
    s_obj = abs(scv.first_term(H, n)) + 0.25 * float(np.einsum("ijkl,ij,kl->", T, aH, aH))
    sH = np.abs(scv.first_term_grad(H, n)) + 0.5 * np.einsum("ijkl,kl->ij", T, aH)
    L = np.abs(np.linalg.cholesky(H))
    sL = np.tril(2.0 * sH @ L)
    return s_obj, np.concatenate([sL[j:, j] for j in range(d)])


def normal_psi4(Sigma):
    """psi_4 of the normal density N(mu, Sigma), integrated exactly:
    int D^{(x)4} f(x) f(x) dx = D^{(x)4} phi_{2 Sigma}(0) (four integrations by
    parts turn it into the convolution of f with itself at zero)."""
    from . import gauss

    Sigma = np.asarray(Sigma, dtype=np.float64)
    d = Sigma.shape[0]
    alphas = multiindex.unique_alphas(d, 4)
    return gauss.dphi_many(np.zeros(d), 2 * Sigma, alphas)
