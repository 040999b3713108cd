"""Grids with a different node count on every axis (so the padded lengths P_k,
the row decomposition and the last-axis length all differ between axes), on
the GPU vs the oracle on the same per-axis grid:

* psi_r (plain and fused single calls, and the batched launch), r = 2, 4;
* the SCV objective + gradient (batched lag-domain launch);
* LSCV_2 and Q_2 (the scalar eta_r kernels).

Tolerances as in the other parity tests: 1e-11 relative per entry for
objectives, gradients and psi entries (near-zero entries against the
absolute-value lag sums).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import binned, eta, grid, linbin, multiindex, scv

from _gpu_util import check_scv, assert_psi_close, log, mixture_sample, oracle_autocorr, spd

pytestmark = pytest.mark.gpu

CASES = {
    "d2": [37, 16],
    "d2_long_last": [9, 70],
    "d3": [12, 20, 9],
    "d4": [6, 9, 5, 8],
}


def _data(name):
    M = CASES[name]
    d = len(M)
    X = mixture_sample(1500, d, 40 + d)
    Gp = spd(d, 50 + d, 0.05)
    rng = np.random.default_rng(60 + d)
    H = synth.random_H_2d(4, rng) if d == 2 else synth.random_H_haar(4, d, rng)
    return d, M, X, Gp, H


def _oracle(X, G, M):
    g = grid.plan_auto(X, G, M)
    co, sk = linbin.linbin(X, g)
    assert sk == 0
    return g, oracle_autocorr(linbin.counts_to_real(co))


def _close(got, want, scale, rtol=1e-11, what=""):
    ref = abs(want) if abs(want) >= 1e-3 * scale else scale
    err = abs(got - want) / ref
    assert err <= rtol, f"{what}: got {got!r} want {want!r} rel err {err:.3e}"


@pytest.mark.parametrize("name", list(CASES))
def test_psi_anisotropic(kf, gpu, name):
    d, M, X, Gp, _ = _data(name)
    n = X.shape[0]
    Xd = torch.from_numpy(X).to(gpu)
    G = spd(d, 70 + d, 0.08)
    g_o, A = _oracle(X, G, M)
    ds = kf.Dataset(Xd, Gp, M=M)
    gp_o, Ap = _oracle(X, Gp, M)
    for r in (2, 4):
        log(f"[aniso] psi {name} M={M} r={r}")
        want = binned.psi(A, n, g_o, G, r)
        sabs = binned.abs_scale(A, n, g_o, G, multiindex.unique_alphas(d, r))
        for mode in ("plain", "fused"):
            got = kf.psi(Xd, G, r, M=M, mode=mode).cpu().numpy()
            assert_psi_close(got, want, sabs, what=f"{name} r={r} {mode}")
        # batched: the dataset's grid is planned from its pilot bandwidth
        got_b = kf.psi_batch([ds], [G], r).cpu().numpy()[0]
        want_b = binned.psi(Ap, n, gp_o, G, r)
        sabs_b = binned.abs_scale(Ap, n, gp_o, G, multiindex.unique_alphas(d, r))
        assert_psi_close(got_b, want_b, sabs_b, what=f"{name} r={r} batch")


@pytest.mark.parametrize("name", list(CASES))
def test_criteria_anisotropic(kf, gpu, name):
    d, M, X, Gp, H = _data(name)
    n = X.shape[0]
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    g_o, A = _oracle(X, Gp, M)
    v = torch.from_numpy(synth.vech_chol(H)).to(gpu)
    log(f"[aniso] scv / lscv_2 / q_2 {name} M={M}")
    obj, gr = kf.scv([ds], v)
    obj, gr = obj.cpu().numpy(), gr.cpu().numpy()
    l2 = kf.crit([ds], v, "lscv", 2, grad=False).cpu().numpy()
    q2 = kf.crit([ds], v, "qr", 2, grad=False).cpu().numpy()
    for b in range(H.shape[0]):
        check_scv(obj[b], gr[b], A, n, g_o, H[b], Gp, what=f"{name} b={b}")
        _close(l2[b], eta.lscv_r_binned(A, n, g_o, H[b], 2), eta.lscv_abs_scale(A, n, g_o, H[b], 2),
               what=f"lscv_2 {name} b={b}")
        _close(q2[b], eta.qr_binned(A, n, g_o, H[b], 2),
               eta.vstat_binned(A, n, g_o, [(1.0, H[b])], 2, absval=True), what=f"Q_2 {name} b={b}")


@pytest.mark.parametrize("launch", [(3, 0), (3, -1), (4, 0), (4, -1), (5, 0), (5, -1), (6, 0), (6, -1)])
def test_long_last_axis_all_launches(kf, gpu, launch):
    """d2_long_last (last-axis P = 256: 16-lag runs walked in 32-lag segments,
    several runs per segment) with 256 candidates in each lag-domain launch:
    objective and every gradient entry per entry (near-zero rule, 1e-11)."""
    from _gpu_util import assert_z16
    name = "d2_long_last"
    d, M, X, Gp, _ = _data(name)
    n = X.shape[0]
    H = synth.random_H_2d(256, np.random.default_rng(65))
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    N = ds.grid.P[d - 1]
    assert N == 256
    g_o, A = _oracle(X, Gp, M)
    v = torch.from_numpy(synth.vech_chol(H)).to(gpu)
    log(f"[aniso] {name} 256 candidates, launch {launch}")
    with kf.row_launch((kf.FUN_SCV_OBJ, kf.FUN_SCV_OBJGRAD, kf.FUN_SCV_GRAD), d, 2, N, *launch):
        obj, gr = kf.scv([ds], v)
    obj, gr = obj.cpu().numpy(), gr.cpu().numpy()
    want = [scv.objective_binned(A, n, g_o, H[b], Gp) for b in range(256)]
    scales = [scv.objective_binned_scales(A, n, g_o, H[b], Gp) for b in range(256)]
    assert_z16(obj, [o for o, _ in want], [s for s, _ in scales], what=f"objective {launch}")
    assert_z16(gr, np.array([g for _, g in want]), np.array([s for _, s in scales]), what=f"gradient {launch}")
