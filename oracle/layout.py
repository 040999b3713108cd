"""The paper's four steps, literally, with its zero-padded layout (Sec. 4, Eq. (17)-(24)).

Step 2 puts the kernel on the full symmetric lag grid (Eq. (18)); step 3 pads
k and c to P_1 x ... x P_d with P_k = 2^ceil(log2(3 M_k - 1)) (Eq. (21)),
k in the leading corner (Eq. (19)) and c shifted to start at index M_k - 1
(0-based; Eq. (20)), multiplies their transforms (Eq. (22)) and keeps the
block starting at index 2M_k - 2 of the inverse transform (Eq. (23)); step 4
contracts it with the counts and scales by n^-2 (Eq. (24)).

The display of k_zp in Eq. (19) writes lags -M..M, but the sum in Eq. (17)
runs over -(M-1)..(M-1); the latter is used.  numpy.fft serves as the FFT
primitive (its inverse already divides by prod P).  ``psi_wrap`` is the same
computation with the smaller circular layout P_k = 2 M_k (kernel lag l stored
at index l mod P_k, counts at [0, M_k)), which the HIP library uses.
"""
from __future__ import annotations

import math

import numpy as np

from . import gauss, multiindex


def paper_P(M):
    return 1 << math.ceil(math.log2(3 * M - 1))


def _lag_mesh(g):
    d = g["d"]
    axes = [np.arange(-(int(m) - 1), int(m)) * g["delta"][k] for k, m in enumerate(g["M"])]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack(mesh, axis=-1)


def psi_paper(c, n, g, G, r):
    d = g["d"]
    M = [int(m) for m in g["M"]]
    P = [paper_P(m) for m in M]
    alphas = multiindex.unique_alphas(d, r)
    kvals = gauss.dphi_many(_lag_mesh(g), G, alphas)      # [A, 2M-1, ...]
    czp = np.zeros(P)
    czp[tuple(slice(m - 1, 2 * m - 1) for m in M)] = c
    C = np.fft.fftn(czp)
    out = []
    for a in range(len(alphas)):
        kzp = np.zeros(P)
        kzp[tuple(slice(0, 2 * m - 1) for m in M)] = kvals[a]
        s = np.fft.ifftn(C * np.fft.fftn(kzp)).real
        conv = s[tuple(slice(2 * m - 2, 3 * m - 2) for m in M)]
        out.append(np.sum(c * conv) / float(n) ** 2)
    return np.array(out)


def psi_wrap(c, n, g, G, r):
    d = g["d"]
    M = [int(m) for m in g["M"]]
    P = [2 * m for m in M]
    alphas = multiindex.unique_alphas(d, r)
    kvals = gauss.dphi_many(_lag_mesh(g), G, alphas)
    czp = np.zeros(P)
    czp[tuple(slice(0, m) for m in M)] = c
    C = np.fft.rfftn(czp)
    idx = [np.r_[np.arange(0, m), np.arange(p - (m - 1), p)] for m, p in zip(M, P)]
    out = []
    for a in range(len(alphas)):
        kzp = np.zeros(P)
        # lag l (array position l + M - 1) goes to index l mod P
        lag_order = [np.r_[np.arange(m - 1, 2 * m - 1), np.arange(0, m - 1)] for m in M]
        kzp[np.ix_(*idx)] = kvals[a][np.ix_(*lag_order)]
        s = np.fft.irfftn(C * np.fft.rfftn(kzp), s=P, axes=tuple(range(len(P))))
        conv = s[tuple(slice(0, m) for m in M)]
        out.append(np.sum(c * conv) / float(n) ** 2)
    return np.array(out)


def psi_wand_quadrant(c, n, g, G, r):
    """Negative control: a kernel grid built from one quadrant and mirrored
    (k_l := k_{|l|} per axis), the layout that is only valid for diagonal G
    (Sec. 2, Sec. 4).  Must disagree with psi_wrap for a full G."""
    d = g["d"]
    M = [int(m) for m in g["M"]]
    P = [2 * m for m in M]
    alphas = multiindex.unique_alphas(d, r)
    mesh = np.abs(_lag_mesh(g))
    kvals = gauss.dphi_many(mesh, G, alphas)
    czp = np.zeros(P)
    czp[tuple(slice(0, m) for m in M)] = c
    C = np.fft.rfftn(czp)
    idx = [np.r_[np.arange(0, m), np.arange(p - (m - 1), p)] for m, p in zip(M, P)]
    lag_order = [np.r_[np.arange(m - 1, 2 * m - 1), np.arange(0, m - 1)] for m in M]
    out = []
    for a in range(len(alphas)):
        kzp = np.zeros(P)
        kzp[np.ix_(*idx)] = kvals[a][np.ix_(*lag_order)]
        s = np.fft.irfftn(C * np.fft.rfftn(kzp), s=P, axes=tuple(range(len(P))))
        out.append(np.sum(c * s[tuple(slice(0, m) for m in M)]) / float(n) ** 2)
    return np.array(out)
