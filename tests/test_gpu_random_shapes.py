"""Seeded random shapes against the oracle: dimension, node count per axis,
sample size and bandwidth scale drawn at random (kernels from a fraction of a
grid step to wider than the grid), for psi_r (plain, fused, batched), the SCV
objective + gradient, LSCV_r and Q_r.  Same tolerances as the other parity
tests (1e-11 relative per entry; near-zero values against the absolute-value
lag sums).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import binned, eta, grid, linbin, multiindex, scv

from _gpu_util import check_scv, assert_psi_close, log, mixture_sample, oracle_autocorr

pytestmark = pytest.mark.gpu

# largest node count per axis, per d (keeps the oracle's direct autocorrelation quick)
MMAX = {1: 200, 2: 48, 3: 11, 4: 6}


def _spd_scaled(d, rng, scale):
    A = rng.standard_normal((d, d))
    S = A @ A.T / d + 0.3 * np.eye(d)
    S = 0.5 * (S + S.T)
    return scale * S / np.sqrt(np.trace(S) / d)


def _config(seed):
    rng = np.random.default_rng(151107482 + 4000 + seed)
    d = int(rng.integers(1, 5))
    M = [int(rng.integers(2, MMAX[d] + 1)) for _ in range(d)]
    n = int(rng.choice([1, 2, 17, 300, 2500]))
    X = mixture_sample(n, d, 9000 + seed)
    # bandwidth scale relative to the data spread: narrow to wide
    Gp = _spd_scaled(d, rng, float(10 ** rng.uniform(-3.0, 0.0)))
    G = _spd_scaled(d, rng, float(10 ** rng.uniform(-2.5, 0.0)))
    H = np.stack([_spd_scaled(d, rng, float(10 ** rng.uniform(-3.0, 0.3))) for _ in range(3)])
    r_psi = int(rng.choice([0, 2, 4] if d == 4 else [0, 2, 4, 6]))
    r_eta = int(rng.integers(0, 9))
    return d, M, n, X, Gp, G, H, r_psi, r_eta


@pytest.mark.parametrize("seed", range(32))
def test_random_shape(kf, gpu, seed):
    d, M, n, X, Gp, G, H, r_psi, r_eta = _config(seed)
    log(f"[random] seed={seed} d={d} M={M} n={n} r_psi={r_psi} r_eta={r_eta}")
    Xd = torch.from_numpy(X).to(gpu)
    # psi_r, single calls (grid padded by the kernel's own bandwidth)
    g_o = grid.plan_auto(X, G, M)
    co, sk = linbin.linbin(X, g_o)
    assert sk == 0
    A = oracle_autocorr(linbin.counts_to_real(co))
    al = multiindex.unique_alphas(d, r_psi)
    want = binned.psi(A, n, g_o, G, r_psi)
    sabs = binned.abs_scale(A, n, g_o, G, al)
    for mode in ("plain", "fused"):
        got = kf.psi(Xd, G, r_psi, M=M, mode=mode).cpu().numpy()
        assert_psi_close(got, want, sabs, what=f"seed {seed} psi_{r_psi} {mode}")
    # dataset on the pilot's grid: batched psi_r, SCV, LSCV_r, Q_r
    ds = kf.Dataset(Xd, Gp, M=M)
    gp_o = grid.plan_auto(X, Gp, M)
    cp, _ = linbin.linbin(X, gp_o)
    Ap = oracle_autocorr(linbin.counts_to_real(cp))
    got_b = kf.psi_batch([ds], [G], r_psi).cpu().numpy()[0]
    assert_psi_close(got_b, binned.psi(Ap, n, gp_o, G, r_psi), binned.abs_scale(Ap, n, gp_o, G, al),
                     what=f"seed {seed} psi_{r_psi} batch")
    v = torch.from_numpy(synth.vech_chol(H)).to(gpu)
    obj, gr = kf.scv([ds], v)
    obj, gr = obj.cpu().numpy(), gr.cpu().numpy()
    lr = kf.crit([ds], v, "lscv", r_eta, grad=False).cpu().numpy() if r_eta > 0 else None
    qr = kf.crit([ds], v, "qr", r_eta, grad=False).cpu().numpy()
    for b in range(H.shape[0]):
        check_scv(obj[b], gr[b], Ap, n, gp_o, H[b], Gp, what=f"seed {seed} b={b}")
        if lr is not None:
            w = eta.lscv_r_binned(Ap, n, gp_o, H[b], r_eta)
            s = eta.lscv_abs_scale(Ap, n, gp_o, H[b], r_eta)
            ref = abs(w) if abs(w) >= 1e-3 * s else s
            assert abs(lr[b] - w) <= 1e-11 * ref, (seed, b, r_eta, lr[b], w)
        w = eta.qr_binned(Ap, n, gp_o, H[b], r_eta)
        s = eta.vstat_binned(Ap, n, gp_o, [(1.0, H[b])], r_eta, absval=True)
        ref = abs(w) if abs(w) >= 1e-3 * s else s
        assert abs(qr[b] - w) <= 1e-11 * ref, (seed, b, r_eta, qr[b], w)
