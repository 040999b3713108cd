"""The batched quasi-Newton minimiser (kdefft_minimize) on the GPU against
reference minimisers computed on the CPU from the oracle (scipy's BFGS over
vech(chol H) on the oracle objective with its exact gradient):

* PI with the exact psi_4 of a normal density (d = 2, 3): every start lands on
  the normal-scale bandwidth, the closed-form minimiser (pinned on the CPU
  side in test_oracle_minimizer.py);
* PI with psi_4 estimated on the GPU from a mixture sample (d = 2);
* SCV and LSCV (binned, d = 2, M = 64) from several starts;
* outcome codes: a singular start, evaluations running out.

Minimisers are compared as H = L L^T (the sign of each column of L is free):
1e-6 of max|H| (the criterion is flat at its minimum: its values, accurate to
about 1e-12, fix the minimiser to about their square root), and the minimum
values to 1e-11 relative.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import binned, eta, grid, linbin, plugin, scv

from _gpu_util import log, mixture_sample
from _minref import H_of, argmin_vech, normal_scale_H

pytestmark = pytest.mark.gpu

H_TOL = 1e-6
F_TOL = 1e-11


def _spd(d, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((d, d))
    return A @ A.T / d + 0.3 * np.eye(d)


def _starts(S, scales, seed):
    d = S.shape[0]
    rng = np.random.default_rng(seed)
    out = []
    for s in scales:
        Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
        E = np.diag(np.exp(rng.uniform(-0.5, 0.5, size=d)))
        out.append(s * (S + 0.3 * np.trace(S) / d * Q @ E @ Q.T))
    return np.array(out)


def _check(kf, x, f, info, H_ref, f_ref, what):
    d = H_ref.shape[0]
    x, f, info = x.cpu().numpy(), f.cpu().numpy(), info.cpu().numpy()
    for b in range(x.shape[0]):
        H = H_of(x[b], d)
        eh = np.abs(H - H_ref).max() / np.abs(H_ref).max()
        ef = abs(f[b] - f_ref) / abs(f_ref)
        log(f"  {what} start {b}: outcome {info[b, 0]}, {info[b, 1]} steps, H err {eh:.2e}, value err {ef:.2e}")
        assert info[b, 0] in (kf.MIN_CONVERGED, kf.MIN_STALLED), (what, b, info[b])
        assert eh <= H_TOL, (what, b, H, H_ref)
        assert ef <= F_TOL, (what, b, f[b], f_ref)


@pytest.mark.parametrize("d", [2, 3])
def test_pi_normal_scale(kf, gpu, d):
    Sigma = _spd(d, 7 + d)
    n = 1000
    psi4 = plugin.normal_psi4(Sigma)
    Hns = normal_scale_H(Sigma, n)
    f_ref = plugin.objective(psi4, n, Hns, with_grad=False)[0]
    H0 = _starts(Hns, (0.2, 0.7, 1.5, 4.0), 11 + d)
    log(f"[min] PI d={d} exact normal psi_4, {len(H0)} starts")
    x, f, info = kf.minimize(torch.from_numpy(synth.vech_chol(H0)).to(gpu), "pi",
                             psi4=torch.from_numpy(psi4[None]).to(gpu), ns=[n], evals=120)
    _check(kf, x, f, info, Hns, f_ref, f"PI d={d}")


def test_pi_estimated_psi4(kf, gpu):
    d, n, M = 2, 4000, 48
    X = mixture_sample(n, d, 31)
    G = 0.2 * np.cov(X.T)
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), G, M=M)
    psi4_gpu = kf.psi_batch([ds], [G], 4)
    psi4 = psi4_gpu.cpu().numpy()[0]
    fun = lambda H: plugin.objective(psi4, n, H)
    S = np.cov(X.T) * n ** (-1 / 3)
    v_ref, f_ref = argmin_vech(fun, synth.vech_chol(S), d)
    H0 = _starts(S, (0.3, 1.0, 3.0), 41)
    log("[min] PI d=2 psi_4 estimated on the GPU, 3 starts")
    x, f, info = kf.minimize(torch.from_numpy(synth.vech_chol(H0)).to(gpu), "pi", psi4=psi4_gpu, ns=[n],
                             evals=120)
    _check(kf, x, f, info, H_of(v_ref, d), f_ref, "PI estimated psi_4")


@pytest.fixture(scope="module")
def small2d(kf, gpu):
    n, d, M = 2000, 2, 64
    X = mixture_sample(n, d, 23)
    G = 0.05 * np.cov(X.T)
    g = grid.plan_auto(X, G, [M, M])
    co, sk = linbin.linbin(X, g)
    assert sk == 0
    A = binned.autocorr_direct(linbin.counts_to_real(co))
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), G, M=M)
    return X, G, g, A, ds


@pytest.mark.parametrize("crit", ["scv", "lscv"])
def test_selector_minimiser(kf, gpu, small2d, crit):
    X, G, g, A, ds = small2d
    n, d = X.shape
    if crit == "scv":
        fun = lambda H: scv.objective_binned(A, n, g, H, G)
    else:
        fun = lambda H: eta.lscv_binned(A, n, g, H)
    S = np.cov(X.T) * n ** (-1 / 3)
    v_ref, f_ref = argmin_vech(fun, synth.vech_chol(S), d)
    H0 = _starts(S, (0.6, 1.0, 1.6), 17)
    log(f"[min] {crit} d=2 n={n} M=64, 3 starts")
    x, f, info = kf.minimize(torch.from_numpy(synth.vech_chol(H0)).to(gpu), crit, datasets=[ds], evals=150)
    _check(kf, x, f, info, H_of(v_ref, d), f_ref, crit)


def test_outcomes(kf, gpu, small2d):
    X, G, g, A, ds = small2d
    S = np.cov(X.T) * X.shape[0] ** (-1 / 3)
    v = synth.vech_chol(np.array([S, S]))
    v[1, 0] = 0.0    # L11 = 0: H singular, the criterion is NaN there
    log("[min] outcome codes: singular start, evaluations running out")
    x, f, info = kf.minimize(torch.from_numpy(v).to(gpu), "scv", datasets=[ds], evals=2)
    info = info.cpu().numpy()
    assert info[0, 0] == kf.MIN_RUNNING and info[1, 0] == kf.MIN_BAD_START, info
    assert np.array_equal(x.cpu().numpy()[1], v[1])
    assert np.isnan(f.cpu().numpy()[1])


def test_minimise_in_graph(kf, gpu, small2d):
    """The whole minimisation (its evaluations and updates) captured in a HIP
    graph: every replay, with unrelated eager work in between, reproduces the
    eager result bit for bit."""
    X, G, g, A, ds = small2d
    S = np.cov(X.T) * X.shape[0] ** (-1 / 3)
    v0 = torch.from_numpy(synth.vech_chol(_starts(S, (0.6, 1.6), 5))).to(gpu)
    log("[min] SCV minimisation captured in a graph, 3 replays")
    want = [t.clone() for t in kf.minimize(v0, "scv", datasets=[ds], evals=40)]
    side = torch.cuda.Stream(gpu)
    side.wait_stream(torch.cuda.current_stream(gpu))
    with torch.cuda.stream(side):
        kf.minimize(v0, "scv", datasets=[ds], evals=40)
    torch.cuda.current_stream(gpu).wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        outs = kf.minimize(v0, "scv", datasets=[ds], evals=40)
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip(outs, want)):
            assert torch.equal(a, b), (rep, k)
        kf.scv([ds], v0)   # unrelated eager work between replays
        torch.cuda.synchronize()
