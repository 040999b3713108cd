"""Unique entries of the r-th derivative vector D^{(x)r} (Sec. 5).

D^{(x)r} f stacks all d^r partial derivatives of order r in Kronecker order
(first index slowest).  Because mixed partials commute, only the multisets of
indices matter; the unique entries are listed as sorted tuples
i_1 <= ... <= i_r in lexicographic order.  For d=2, r=4 that is
(0,0,0,0), (0,0,0,1), (0,0,1,1), (0,1,1,1), (1,1,1,1).
"""
from __future__ import annotations

import itertools
from math import comb

import numpy as np


def unique_tuples(d: int, r: int):
    return list(itertools.combinations_with_replacement(range(d), r))


def n_unique(d: int, r: int) -> int:
    return comb(d + r - 1, r)


def tuple_to_alpha(t, d):
    """Multiset of axis indices -> multi-index alpha (count per axis)."""
    a = [0] * d
    for i in t:
        a[i] += 1
    return tuple(a)


def unique_alphas(d: int, r: int):
    return [tuple_to_alpha(t, d) for t in unique_tuples(d, r)]


def expand_full(vals, d: int, r: int):
    """Unique-entry vector -> the d^r Kronecker-ordered vector (first index slowest)."""
    pos = {t: k for k, t in enumerate(unique_tuples(d, r))}
    out = np.empty(d ** r, dtype=np.float64)
    for flat, idx in enumerate(itertools.product(range(d), repeat=r)):
        out[flat] = vals[pos[tuple(sorted(idx))]]
    return out
