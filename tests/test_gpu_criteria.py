"""LSCV, LSCV_r, Q_r and the plug-in criterion on the GPU vs the oracle.

* LSCV (r = 0, Eq. (10) / Eq. (35) weights) objective and gradient from the
  batched launch vs the oracle's binned LSCV from its own counts (1e-11 per
  entry under the near-zero rule, for the objective and every gradient
  entry), d = 1..4;
* the LSCV adjoint and its autograd.Function;
* LSCV_r (r = 1..8) and Q_r (r = 0..8) from the scalar eta_r kernels vs the
  oracle's binned sums (<= 1e-11, near-zero values against the absolute-value
  lag sum, the rule used for psi_r), uneven multi-dataset batches;
* Q_r against the contraction of the GPU's own psi_{2r} (r <= 4);
* PI objective and gradient vs the oracle's plug-in criterion on the same
  psi_4 (<= 1e-12) and on the oracle's own binned psi_4 (<= 1e-11); PI
  autograd; singular candidates report status 1 and NaN;
* the full case-4 shape (n = 1e5, M = 256, 256 candidates) on sampled
  candidates.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import binned, eta, grid, linbin, multiindex, plugin

from _gpu_util import check_lscv, check_z16, log, mixture_sample, oracle_autocorr, spd

pytestmark = pytest.mark.gpu

CASES = {
    "d1": (1, 3000, 64, 6),
    "d2": (2, 3000, 40, 8),
    "d2_ragged": (2, 2500, 29, 5),
    "d3": (3, 3000, 16, 5),
    "d4": (4, 2000, 8, 4),
    "d2_tiny": (2, 400, 5, 4),   # coarse grid: runs rising by more than e^600 along 8 lags
}
_AC = {}


def _data(name):
    d, n, M, B = CASES[name]
    X = mixture_sample(n, d, 500 + d)
    Gp = spd(d, 600 + d, 0.05)
    rng = np.random.default_rng(700 + d)
    H = synth.random_H_2d(B, rng) if d == 2 else synth.random_H_haar(B, d, rng)
    return d, X, Gp, M, H


def _oracle(name, X, Gp, M):
    if name not in _AC:
        g = grid.plan_auto(X, Gp, [M] * X.shape[1])
        co, sk = linbin.linbin(X, g)
        assert sk == 0
        _AC[name] = (g, oracle_autocorr(linbin.counts_to_real(co)))
    return _AC[name]


def _close(got, want, scale, rtol=1e-11, what=""):
    ref = abs(want) if abs(want) >= 1e-3 * scale else scale
    err = abs(got - want) / ref
    assert err <= rtol, f"{what}: got {got!r} want {want!r} rel err {err:.3e}"


@pytest.mark.parametrize("exact", [False, True])
@pytest.mark.parametrize("name", list(CASES))
def test_lscv_vs_oracle(kf, gpu, name, exact):
    d, X, Gp, M, H = _data(name)
    crit = "lscv_exact" if exact else "lscv"
    log(f"[lscv] case={name} crit={crit}")
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    v = torch.from_numpy(synth.vech_chol(H)).to(gpu)
    obj, g = kf.crit([ds], v, crit)
    obj2 = kf.crit([ds], v, crit, grad=False)
    obj, g, obj2 = obj.cpu().numpy(), g.cpu().numpy(), obj2.cpu().numpy()
    np.testing.assert_allclose(obj2, obj, rtol=1e-13)
    g_o, A = _oracle(name, X, Gp, M)
    n = X.shape[0]
    for b in range(H.shape[0]):
        check_lscv(obj[b], g[b], A, n, g_o, H[b], exact, what=f"{name} b={b}")


def test_lscv_adjoint_and_autograd(kf, gpu):
    d, X, Gp, M, H = _data("d3")
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    v = torch.from_numpy(synth.vech_chol(H)).to(gpu)
    obj, g = kf.crit([ds], v, "lscv")
    w = torch.linspace(-1.0, 2.0, H.shape[0], dtype=torch.float64, device=gpu)
    adj = kf.crit_adjoint([ds], v, w, "lscv")
    np.testing.assert_allclose(adj.cpu().numpy(), (w[:, None] * g).cpu().numpy(), rtol=1e-13, atol=1e-300)
    vv = v.clone().requires_grad_(True)
    out = kf.Criterion.apply(vv, ds, "lscv")
    (out * w).sum().backward()
    np.testing.assert_array_equal(vv.grad.cpu().numpy(), adj.cpu().numpy())
    np.testing.assert_allclose(out.detach().cpu().numpy(), obj.cpu().numpy(), rtol=1e-13)


RS = {"d1": [1, 2, 4, 8], "d2": [1, 2, 3, 6, 7, 8], "d2_ragged": [2, 5], "d3": [1, 2, 4], "d4": [1, 2, 3],
      "d2_tiny": [1, 2, 4]}


@pytest.mark.parametrize("name", list(RS))
def test_lscv_r_and_qr_vs_oracle(kf, gpu, name):
    d, X, Gp, M, H = _data(name)
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    v = torch.from_numpy(synth.vech_chol(H)).to(gpu)
    g_o, A = _oracle(name, X, Gp, M)
    n = X.shape[0]
    nb = min(3, H.shape[0])
    for r in RS[name]:
        log(f"[lscv_r/qr] case={name} r={r}")
        lo = kf.crit([ds], v, "lscv", r, grad=False).cpu().numpy()
        qo = kf.crit([ds], v, "qr", r, grad=False).cpu().numpy()
        for b in range(nb):
            want = eta.lscv_r_binned(A, n, g_o, H[b], r)
            _close(lo[b], want, eta.lscv_abs_scale(A, n, g_o, H[b], r), what=f"lscv_{r} {name} b={b}")
            wq = eta.qr_binned(A, n, g_o, H[b], r)
            _close(qo[b], wq, eta.vstat_binned(A, n, g_o, [(1.0, H[b])], r, absval=True),
                   what=f"Q_{r} {name} b={b}")
    q0 = kf.crit([ds], v, "qr", 0, grad=False).cpu().numpy()
    for b in range(nb):
        _close(q0[b], eta.qr_binned(A, n, g_o, H[b], 0), 1.0, what=f"Q_0 {name} b={b}")


def test_criteria_uneven_datasets(kf, gpu):
    d, M = 2, 24
    Xs = [mixture_sample(n, d, 800 + j) for j, n in enumerate((700, 4000, 1500))]
    Gps = [spd(d, 810 + j, 0.05) for j in range(3)]
    dss = [kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M) for X, Gp in zip(Xs, Gps)]
    per = [3, 1, 4]
    H = synth.random_H_2d(sum(per), np.random.default_rng(5))
    v = torch.from_numpy(synth.vech_chol(H)).to(gpu)
    for crit, r in (("lscv", 0), ("lscv_exact", 0), ("lscv", 4), ("qr", 2)):
        obj = kf.crit(dss, v, crit, r, per_ds=per, grad=False).cpu().numpy()
        b = 0
        for j in range(3):
            g_o = grid.plan_auto(Xs[j], Gps[j], [M, M])
            co, _ = linbin.linbin(Xs[j], g_o)
            A = binned.autocorr_direct(linbin.counts_to_real(co))
            n = Xs[j].shape[0]
            for _ in range(per[j]):
                if crit == "qr":
                    want = eta.qr_binned(A, n, g_o, H[b], r)
                    sc = eta.vstat_binned(A, n, g_o, [(1.0, H[b])], r, absval=True)
                else:
                    ex = crit == "lscv_exact"
                    want = eta.lscv_r_binned(A, n, g_o, H[b], r, ex)
                    sc = eta.lscv_abs_scale(A, n, g_o, H[b], r, ex)
                _close(obj[b], want, sc, what=f"{crit} r={r} ds={j} b={b}")
                b += 1


def test_qr_is_contraction_of_psi(kf, gpu):
    d, X, Gp, M, H = _data("d2")
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    S = H[0]
    v = torch.from_numpy(synth.vech_chol(S[None])).to(gpu)
    g_o, A = _oracle("d2", X, Gp, M)
    n = X.shape[0]
    for r in (1, 2, 3, 4):
        q = kf.crit([ds], v, "qr", r, grad=False).cpu().numpy()[0]
        p = kf.psi_batch([ds], [S], 2 * r).cpu().numpy()[0]
        alphas = multiindex.unique_alphas(d, 2 * r)
        tot = sum(c * p[alphas.index(a)] for a, c in eta.eta_terms(d, r))
        # each psi entry is within 1e-11 of its absolute-value lag sum, so the
        # contraction is judged against sum |c| S_abs(alpha)
        sabs = binned.abs_scale(A, n, g_o, S, alphas)
        scale = sum(abs(c) * sabs[alphas.index(a)] for a, c in eta.eta_terms(d, r))
        check_z16([q], [tot], [scale], 1e-11, what=f"Q_{r} as a contraction of psi_{2 * r}")


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_pi_vs_oracle(kf, gpu, d):
    name = {1: "d1", 2: "d2", 3: "d3", 4: "d4"}[d]
    _, X, Gp, M, H = _data(name)
    log(f"[pi] d={d}")
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    G4 = spd(d, 900 + d, 0.08)
    p4 = kf.psi_batch([ds], [G4], 4)
    v = torch.from_numpy(synth.vech_chol(H)).to(gpu)
    n = X.shape[0]
    obj, g = kf.pi(p4, [n], v)
    obj, g, p4h = obj.cpu().numpy(), g.cpu().numpy(), p4.cpu().numpy()[0]
    g_o, A = _oracle(name, X, Gp, M)
    p4o = binned.psi(A, n, g_o, G4, 4)
    p4s = binned.abs_scale(A, n, g_o, G4, multiindex.unique_alphas(d, 4))
    for b in range(H.shape[0]):
        o, gr = plugin.objective(p4h, n, H[b])
        assert obj[b] == pytest.approx(o, rel=1e-12)
        np.testing.assert_allclose(g[b], gr, rtol=1e-11, atol=1e-12 * np.abs(gr).max())
        # against the oracle's PI from its own psi_4: the psi_4 entries agree to
        # 1e-11 of their absolute-value lag sums, so PI is judged against the
        # scales built from those sums
        o2, gr2 = plugin.objective(p4o, n, H[b])
        so, sg = plugin.objective_scales(p4s, n, H[b])
        check_z16([obj[b]], [o2], [so], 1e-11, what=f"PI d={d} b={b} objective")
        check_z16(g[b], gr2, sg, 1e-11, what=f"PI d={d} b={b} gradient")


def test_pi_batches_autograd_and_singular(kf, gpu):
    d = 3
    rng = np.random.default_rng(17)
    p4 = torch.from_numpy(np.stack([plugin.normal_psi4(spd(d, 30 + j, 1.0)) for j in range(2)])).to(gpu)
    H = synth.random_H_haar(5, d, rng)
    L = synth.vech_chol(H)
    L[3, 0] = 0.0   # zero diagonal entry of L: singular
    v = torch.from_numpy(L).to(gpu)
    ns = [500, 2000]
    obj, g, st = kf.pi(p4, ns, v, per_ds=[2, 3], status=True)
    st = st.cpu().numpy()
    assert st.tolist() == [0, 0, 0, 1, 0]
    assert np.isnan(obj[3].item()) and np.isnan(g[3].cpu().numpy()).all()
    for b, j in ((0, 0), (1, 0), (2, 1), (4, 1)):
        o, gr = plugin.objective(p4[j].cpu().numpy(), ns[j], H[b])
        assert obj[b].item() == pytest.approx(o, rel=1e-12)
        np.testing.assert_allclose(g[b].cpu().numpy(), gr, rtol=1e-11, atol=1e-12 * np.abs(gr).max())
    keep = [0, 1, 2, 4]
    vv = v[keep].clone().requires_grad_(True)
    out = kf.PI.apply(vv, p4, ns, [2, 2])
    w = torch.linspace(0.5, 2.0, 4, dtype=torch.float64, device=gpu)
    (out * w).sum().backward()
    _, g2 = kf.pi(p4, ns, v[keep], per_ds=[2, 2])
    np.testing.assert_allclose(vv.grad.cpu().numpy(), (w[:, None] * g2).cpu().numpy(), rtol=1e-14)


def test_case4_full_lscv_sampled(kf, gpu):
    w = synth.case4()
    X, Gp, H = w.X[0], w.G_pilot[0], w.H[0]
    log("[lscv] case4 full")
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=w.M)
    obj, g = kf.crit([ds], torch.from_numpy(synth.vech_chol(H)).to(gpu), "lscv")
    obj, g = obj.cpu().numpy(), g.cpu().numpy()
    g_o, A = _oracle("case4", X, Gp, w.M)
    n = X.shape[0]
    for b in (0, 131, 255):
        check_lscv(obj[b], g[b], A, n, g_o, H[b], what=f"case4 b={b}")
