"""Shared helpers of the GPU parity tests: seeded inputs, the oracle side of
each comparison (computed on the CPU from the oracle only), and the
tolerance rule for floating-point entries."""
import functools
import sys

import numpy as np

from oracle import binned, eta, grid, linbin, scv

RTOL_PSI = 1e-11     # FFT route vs direct binned sum, relative


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def mixture_sample(n, d, seed, ncomp=3):
    rng = np.random.default_rng(seed)
    means = rng.standard_normal((ncomp, d)) * 1.2
    X = np.empty((n, d))
    lab = rng.integers(0, ncomp, size=n)
    for l in range(ncomp):
        A = rng.standard_normal((d, d)) * 0.5 + np.eye(d) * 0.6
        idx = lab == l
        X[idx] = means[l] + rng.standard_normal((idx.sum(), d)) @ A.T
    return X


def spd(d, seed, scale=0.1):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((d, d))
    S = A @ A.T / d + 0.5 * np.eye(d)
    return scale * 0.5 * (S + S.T)


@functools.lru_cache(maxsize=32)
def _oracle_counts_cached(key):
    X, G, M, pad = _REG[key]
    g = grid.plan_auto(X, G, list(M), pad)
    counts, skipped = linbin.linbin(X, g)
    return g, counts, skipped


_REG = {}


def oracle_counts(X, G, M, pad=4.0):
    key = (id(X), X.shape, tuple(M), float(pad), G.tobytes())
    _REG[key] = (X, G, tuple(M), pad)
    return _oracle_counts_cached(key)


def oracle_autocorr(c, direct_limit=70_000):
    """The oracle's FFT-free autocorrelation of the counts: shifted-slice dot
    products when affordable, else slab products summed by lag (pinned equal
    to the shifted-slice form)."""
    if c.size <= direct_limit:
        return binned.autocorr_direct(c)
    return binned.autocorr_gemm(c)


def assert_psi_close(got, want, scale_abs, rtol=RTOL_PSI, what=""):
    """Per entry |a-b| <= rtol*|b|; near-zero entries (|b| < 1e-3 S_abs) are
    compared against S_abs = n^-2 sum |k| A instead."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    for k, (a, b, s) in enumerate(zip(got, want, scale_abs)):
        ref = abs(b) if abs(b) >= 1e-3 * s else s
        err = abs(a - b) / ref
        assert err <= rtol, f"{what} entry {k}: got {a!r} want {b!r} rel err {err:.3e}"


def z16_errors(got, want, scale):
    """Per-entry relative errors under the near-zero rule: |a - b| / |b|, or
    |a - b| / S when |b| < 1e-3 S (S the entry's absolute-value scale)."""
    want = np.asarray(want, dtype=np.float64)
    got = np.asarray(got, dtype=np.float64).reshape(want.shape).ravel()
    scale = np.broadcast_to(np.asarray(scale, dtype=np.float64), want.shape).ravel()
    want = want.ravel()
    ref = np.where(np.abs(want) >= 1e-3 * scale, np.abs(want), scale)
    return np.abs(got - want) / ref


def assert_z16(got, want, scale, rtol=1e-11, what=""):
    """Every entry within rtol under the near-zero rule (z16_errors)."""
    err = z16_errors(got, want, scale)
    k = int(np.argmax(err))
    log(f"  {what}: worst entry {k} rel err {err[k]:.2e} (bar {rtol:.0e})")
    assert err[k] <= rtol, (f"{what} entry {k}: got {np.ravel(got)[k]!r} want {np.ravel(want)[k]!r} "
                            f"rel err {err[k]:.3e}")


def check_z16(got, want, scale, rtol=1e-11, what=""):
    """As assert_z16, logging only on failure (for per-candidate loops)."""
    err = z16_errors(got, want, scale)
    k = int(np.argmax(err))
    assert err[k] <= rtol, (f"{what} entry {k}: got {np.ravel(got)[k]!r} want {np.ravel(want)[k]!r} "
                            f"rel err {err[k]:.3e}")


def check_scv(obj_b, grad_b, A, n, g, H, G, rtol=1e-11, what=""):
    """One candidate's SCV objective (and gradient, if given) against the
    oracle's binned values, per entry under the near-zero rule."""
    o, gr = scv.objective_binned(A, n, g, H, G, with_grad=grad_b is not None)
    so, sg = scv.objective_binned_scales(A, n, g, H, G)
    check_z16([obj_b], [o], [so], rtol, what + " objective")
    if grad_b is not None:
        check_z16(grad_b, gr, sg, rtol, what + " gradient")


def check_lscv(obj_b, grad_b, A, n, g, H, exact=False, rtol=1e-11, what=""):
    """One candidate's LSCV (r = 0) objective and gradient against the oracle."""
    o, gr = eta.lscv_binned(A, n, g, H, exact, with_grad=grad_b is not None)
    so, sg = eta.lscv_binned_scales(A, n, g, H, exact)
    check_z16([obj_b], [o], [so], rtol, what + " objective")
    if grad_b is not None:
        check_z16(grad_b, gr, sg, rtol, what + " gradient")
