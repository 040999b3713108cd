"""SCV objective, gradient, adjoint and batching on the GPU vs the oracle.

* batched objective and gradient (one persistent launch) vs the oracle's
  binned SCV evaluated from its own counts (1e-11 per entry, near-zero entries
  against the oracle's absolute-value scales);
* paper-literal plain path vs the same oracle;
* adjoint = grad_out * gradient; autograd.Function backward;
* central differences with Richardson extrapolation of the GPU objective
  (<= 1e-7 relative);
* uneven multi-dataset batches, every compiled launch variant, a singular
  candidate (status 1, NaN), bitwise repeatability;
* the full case-4 workload (d=2, n=1e5, M=256, 256 candidates) on sampled
  candidates; a case-5-shaped dataset (d=4, n=2e5, M=32) against the
  oracle's objective and the paper-literal path's gradient.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import binned, grid, linbin, multiindex, scv

from _gpu_util import assert_psi_close, assert_z16, check_scv, log, mixture_sample, oracle_autocorr, spd

pytestmark = pytest.mark.gpu

_AC = {}


def _oracle(name, X, G, M):
    if name not in _AC:
        g = grid.plan_auto(X, G, [M] * X.shape[1])
        co, sk = linbin.linbin(X, g)
        assert sk == 0
        _AC[name] = (g, oracle_autocorr(linbin.counts_to_real(co)))
    return _AC[name]


def _golden(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"{name}.json")) as fh:
        return json.load(fh)


def _vech(H):
    return synth.vech_chol(H)


def _Hs(d, B, seed):
    if d == 2:
        return synth.random_H_2d(B, np.random.default_rng(seed))
    return synth.random_H_haar(B, d, np.random.default_rng(seed))


CASES = {
    "d1": (1, 3000, 64, 6),
    "d2": (2, 3000, 40, 12),
    "d2_ragged": (2, 2500, 29, 7),
    "d3": (3, 3000, 16, 6),
    "d4": (4, 2000, 8, 5),
}


def _setup(name, gpu):
    d, n, M, B = CASES[name]
    X = mixture_sample(n, d, 100 + d)
    Gp = spd(d, 200 + d, 0.05)
    H = _Hs(d, B, 300 + d)
    ds = None
    return d, X, Gp, M, H, ds


def _check_against_oracle(kf, name, d, X, Gp, M, H, obj, gradv):
    """Objective and gradient of each candidate against the oracle's binned
    values: 1e-11 per entry under the near-zero rule."""
    g_o, A = _oracle(name, X, Gp, M)
    n = X.shape[0]
    for b in range(H.shape[0]):
        check_scv(obj[b], None if gradv is None else gradv[b], A, n, g_o, H[b], Gp, what=f"{name} b={b}")


@pytest.mark.parametrize("name", list(CASES))
def test_scv_batch_vs_oracle(kf, gpu, name):
    d, X, Gp, M, H, _ = _setup(name, gpu)
    log(f"[scv] case={name} B={H.shape[0]}")
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    assert ds.out_of_grid() == 0
    v = torch.from_numpy(_vech(H)).to(gpu)
    obj, g = kf.scv([ds], v)
    obj_only = kf.scv([ds], v, grad=False)
    obj, g, obj_only = obj.cpu().numpy(), g.cpu().numpy(), obj_only.cpu().numpy()
    _check_against_oracle(kf, name, d, X, Gp, M, H, obj, g)
    np.testing.assert_allclose(obj_only, obj, rtol=1e-13)


@pytest.mark.parametrize("B", [1, 4097])
def test_batch_sizes(kf, gpu, B):
    """One candidate, and 4097 candidates (several waves of items over the
    resident grid, a ragged last wave): the first, last and a random sample of
    candidates against the oracle."""
    name = "d2_ragged"
    d, X, Gp, M, _, _ = _setup(name, gpu)
    H = _Hs(d, B, 900 + B)
    log(f"[scv] batch B={B}")
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    obj, g = kf.scv([ds], torch.from_numpy(_vech(H)).to(gpu))
    obj, g = obj.cpu().numpy(), g.cpu().numpy()
    idx = sorted(set([0, B - 1] + list(np.random.default_rng(B).integers(0, B, size=min(B, 12)))))
    _check_against_oracle(kf, name, d, X, Gp, M, H[idx], obj[idx], g[idx])


@pytest.mark.parametrize("name", ["d1", "d2_ragged", "d3", "d4"])
def test_scv_plain_vs_oracle(kf, gpu, name):
    d, X, Gp, M, H, _ = _setup(name, gpu)
    log(f"[scv-plain] case={name}")
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    res = np.stack([kf.scv_plain(ds, H[b]).cpu().numpy() for b in range(min(3, H.shape[0]))])
    _check_against_oracle(kf, name, d, X, Gp, M, H[:len(res)], res[:, 0], res[:, 1:])


def test_adjoint_and_autograd(kf, gpu):
    d, X, Gp, M, H, _ = _setup("d3", gpu)
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    v = torch.from_numpy(_vech(H)).to(gpu)
    obj, g = kf.scv([ds], v)
    w = torch.linspace(-1.0, 2.0, H.shape[0], dtype=torch.float64, device=gpu)
    adj = kf.scv_adjoint([ds], v, w)
    np.testing.assert_allclose(adj.cpu().numpy(), (w[:, None] * g).cpu().numpy(), rtol=1e-13, atol=1e-300)
    vv = v.clone().requires_grad_(True)
    out = kf.SCV.apply(vv, ds)
    (out * w).sum().backward()
    np.testing.assert_allclose(vv.grad.cpu().numpy(), adj.cpu().numpy(), rtol=0, atol=0)
    np.testing.assert_allclose(out.detach().cpu().numpy(), obj.cpu().numpy(), rtol=1e-13)


@pytest.mark.parametrize("name", ["d2", "d4"])
def test_gradient_finite_differences(kf, gpu, name):
    d, X, Gp, M, H, _ = _setup(name, gpu)
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    v0 = _vech(H[:2])
    q = v0.shape[1]
    _, g = kf.scv([ds], torch.from_numpy(v0).to(gpu))
    g = g.cpu().numpy()
    h = 1e-3
    pts = []
    for b in range(2):
        for k in range(q):
            for s in (h, -h, h / 2, -h / 2):
                w = v0[b].copy()
                w[k] += s
                pts.append(w)
    obj = kf.scv([ds], torch.from_numpy(np.array(pts)).to(gpu), grad=False).cpu().numpy().reshape(2, q, 4)
    d1 = (obj[..., 0] - obj[..., 1]) / (2 * h)
    d2 = (obj[..., 2] - obj[..., 3]) / h
    fd = (4 * d2 - d1) / 3
    err = np.abs(fd - g).max() / np.abs(g).max()
    assert err <= 1e-7, (fd, g, err)


def test_uneven_multi_dataset(kf, gpu):
    d, M = 2, 32
    sets = []
    for j, n in enumerate((800, 5000, 2300)):
        X = mixture_sample(n, d, 400 + j)
        Gp = spd(d, 500 + j, 0.04)
        H = _Hs(d, (5, 3, 7)[j], 600 + j)
        sets.append((X, Gp, H))
    dss = [kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M) for X, Gp, _ in sets]
    v = torch.from_numpy(np.concatenate([_vech(H) for _, _, H in sets])).to(gpu)
    obj, g = kf.scv(dss, v, per_ds=[5, 3, 7])
    obj, g = obj.cpu().numpy(), g.cpu().numpy()
    s = 0
    for j, (X, Gp, H) in enumerate(sets):
        _check_against_oracle(kf, f"multi{j}", d, X, Gp, M, H, obj[s:s + len(H)], g[s:s + len(H)])
        s += len(H)


def test_launch_variants_agree(kf, gpu):
    d, X, Gp, M, H, _ = _setup("d2", gpu)
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    v = torch.from_numpy(_vech(H)).to(gpu)
    N = ds.grid.P[d - 1]
    ref = None
    for var in range(7):
        for gb in (0, -1, 7):
            with kf.row_launch(kf.FUN_SCV_OBJGRAD, d, 2, N, var, gb):
                obj, g = kf.scv([ds], v)
            cur = np.concatenate([obj.cpu().numpy(), g.cpu().numpy().ravel()])
            if ref is None:
                ref = cur
            np.testing.assert_allclose(cur, ref, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("d,M", [(1, 2), (1, 3), (2, 2), (2, 3), (3, 2), (2, 5)])
def test_tiny_grids(kf, gpu, d, M):
    """Grids of 2-5 nodes per axis (last-axis rows of 4-16 positions: runs
    shorter than the nominal 8 lags) in both lag-domain launches."""
    X = mixture_sample(400, d, 40 + d)
    Gp = spd(d, 41 + d, 0.05)
    H = _Hs(d, 3, 42 + d)
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    v = torch.from_numpy(_vech(H)).to(gpu)
    N = ds.grid.P[d - 1]
    log(f"[scv-tiny] d={d} M={M} P={N}")
    for var in (3, 4, 5, 6):
        with kf.row_launch(kf.FUN_SCV_OBJGRAD, d, 2, N, var, 0):
            obj, g = kf.scv([ds], v)
        _check_against_oracle(kf, f"tiny{d}_{M}", d, X, Gp, M, H, obj.cpu().numpy(), g.cpu().numpy())


@pytest.mark.parametrize("d,M", [(2, 3), (2, 5), (3, 4), (1, 6)])
@pytest.mark.parametrize("r", [0, 2, 4])
def test_psi_batch_coarse_grids(kf, gpu, d, M, r):
    """psi_r from the batched lag kernel on coarse grids with narrow G (the
    Gaussian changes by many orders of magnitude from one lag to the next)."""
    from oracle import multiindex
    X = mixture_sample(500, d, 60 + d)
    Gp = spd(d, 61 + d, 0.05)
    G = spd(d, 62 + d, 0.01)
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    got = kf.psi_batch([ds], [G], r).cpu().numpy()[0]
    g_o = grid.plan_auto(X, Gp, [M] * d)
    co, _ = linbin.linbin(X, g_o)
    A = binned.autocorr_direct(linbin.counts_to_real(co))
    want = binned.psi(A, X.shape[0], g_o, G, r)
    sabs = binned.abs_scale(A, X.shape[0], g_o, G, multiindex.unique_alphas(d, r))
    assert_psi_close(got, want, sabs, what=f"d={d} M={M} r={r}")


@pytest.mark.parametrize("scale", [1e-3, 30.0])
def test_extreme_candidates(kf, gpu, scale):
    """Candidates far narrower and far wider than the pilot on an ordinary
    grid, in both lag-domain launches."""
    d, X, Gp, M, H, _ = _setup("d2", gpu)
    Hs = H * scale
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    v = torch.from_numpy(_vech(Hs)).to(gpu)
    N = ds.grid.P[d - 1]
    log(f"[scv-extreme] H x {scale}")
    for var in (3, 4, 5, 6):
        with kf.row_launch(kf.FUN_SCV_OBJGRAD, d, 2, N, var, 0):
            obj, g = kf.scv([ds], v)
        _check_against_oracle(kf, "d2", d, X, Gp, M, Hs, obj.cpu().numpy(), g.cpu().numpy())


def test_singular_candidate_and_determinism(kf, gpu):
    d, X, Gp, M, H, _ = _setup("d2", gpu)
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    vn = _vech(H)
    vn[1, 0] = 0.0                      # zero diagonal of L: H singular
    v = torch.from_numpy(vn).to(gpu)
    obj, g, st = kf.scv([ds], v, status=True)
    st = st.cpu().numpy()
    assert st[1] == 1 and st[0] == 0 and st[2:].max() == 0
    assert np.isnan(obj[1].item()) and np.isnan(g[1].cpu().numpy()).all()
    assert np.isfinite(obj.cpu().numpy()[[0] + list(range(2, len(vn)))]).all()
    obj2, g2 = kf.scv([ds], v)
    assert np.array_equal(obj.cpu().numpy(), obj2.cpu().numpy(), equal_nan=True)
    assert np.array_equal(g.cpu().numpy(), g2.cpu().numpy(), equal_nan=True)


def test_case4_full_sampled(kf, gpu):
    """Case 4 at full size in the benchmark's launch: d=2, n=1e5, M=256, 256 H."""
    w = synth.case4()
    X, Gp, H = w.X[0], w.G_pilot[0], w.H[0]
    log("[scv-full] case4")
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=256)
    obj, g = kf.scv([ds], torch.from_numpy(_vech(H)).to(gpu))
    obj, g = obj.cpu().numpy(), g.cpu().numpy()
    idx = [0, 77, 255]
    _check_against_oracle(kf, "case4", 2, X, Gp, 256, H[idx], obj[idx], g[idx])
    # the paper-literal path (one candidate, per-grid FFTs) against the values
    # the oracle wrote for the same candidate
    gold = _golden("case4")["scv"]
    pl = kf.scv_plain(ds, H[77]).cpu().numpy()
    assert_z16(pl[0], gold["obj"][77], gold["obj_scale"][77], 1e-11, what="case4 plain objective")
    assert_z16(pl[1:], gold["grad"][77], gold["grad_scale"][77], 1e-11, what="case4 plain gradient")


def test_case5_shape_sampled(kf, gpu):
    """A case-5-shaped dataset (d=4, n=2e5, M=32, P=64): thousands of row
    chunks per candidate; two candidates (batched and paper-literal paths)
    against the oracle's binned objective and gradient."""
    w = synth.case5(n_datasets=1, B=2, n_lo=200_000, n_hi=200_000)
    X, Gp, H = w.X[0], w.G_pilot[0], w.H[0]
    log("[scv-full] case5 shape d=4 n=2e5 M=32")
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=32)
    obj, g = kf.scv([ds], torch.from_numpy(_vech(H)).to(gpu))
    obj, g = obj.cpu().numpy(), g.cpu().numpy()
    # objective and gradient of both candidates, and the paper-literal path for
    # the second, against the values the oracle wrote (tests/golden)
    gold = _golden("case5_shape")["scv"]
    for b in range(2):
        assert_z16(obj[b], gold["obj"][b], gold["obj_scale"][b], 1e-11, what=f"case5 shape objective {b}")
        assert_z16(g[b], gold["grad"][b], gold["grad_scale"][b], 1e-11, what=f"case5 shape gradient {b}")
    pl = kf.scv_plain(ds, H[1]).cpu().numpy()
    assert_z16(pl[0], gold["obj"][1], gold["obj_scale"][1], 1e-11, what="case5 shape plain objective")
    assert_z16(pl[1:], gold["grad"][1], gold["grad_scale"][1], 1e-11, what="case5 shape plain gradient")


def test_psi_batch(kf, gpu):
    d, M, r = 2, 24, 4
    dss, Gs, Xs = [], [], []
    for j, n in enumerate((700, 3000)):
        X = mixture_sample(n, d, 700 + j)
        Gp = spd(d, 800 + j, 0.05)
        Xs.append(X)
        Gs.append(spd(d, 900 + j, 0.08))
        dss.append(kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M))
    out = kf.psi_batch(dss, Gs, r).cpu().numpy()
    for j in range(2):
        # the dataset grid is planned from its pilot; the oracle uses the same grid
        g_o = grid.plan_auto(Xs[j], spd(d, 800 + j, 0.05), [M, M])
        co, _ = linbin.linbin(Xs[j], g_o)
        A = binned.autocorr_direct(linbin.counts_to_real(co))
        want = binned.psi(A, Xs[j].shape[0], g_o, Gs[j], r)
        sabs = binned.abs_scale(A, Xs[j].shape[0], g_o, Gs[j], multiindex.unique_alphas(d, r))
        assert_psi_close(out[j], want, sabs, what=f"psi batch dataset {j}")


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("name", ["d1", "d2_ragged", "d3", "d4"])
def test_every_variant_vs_oracle(kf, gpu, name, variant):
    """Each compiled launch variant (three spectral, two lag-domain) against the
    oracle, for the objective+gradient, objective-only and adjoint families."""
    d, X, Gp, M, H, _ = _setup(name, gpu)
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    N = ds.grid.P[d - 1]
    v = torch.from_numpy(_vech(H)).to(gpu)
    kinds = (kf.FUN_SCV_OBJ, kf.FUN_SCV_OBJGRAD, kf.FUN_SCV_GRAD)
    with kf.row_launch(kinds, d, 2, N, variant, 0):
        obj, g = kf.scv([ds], v)
        obj_only = kf.scv([ds], v, grad=False)
        w = torch.ones(H.shape[0], dtype=torch.float64, device=gpu)
        adj = kf.scv_adjoint([ds], v, w)
    obj, g = obj.cpu().numpy(), g.cpu().numpy()
    _check_against_oracle(kf, name, d, X, Gp, M, H, obj, g)
    np.testing.assert_allclose(obj_only.cpu().numpy(), obj, rtol=1e-13)
    np.testing.assert_allclose(adj.cpu().numpy(), g, rtol=1e-11, atol=1e-12 * np.abs(g).max())


@pytest.mark.parametrize("variant", [0, 3])
def test_psi_batch_variants(kf, gpu, variant):
    d, M, r = 3, 14, 4
    X = mixture_sample(2500, d, 950)
    Gp = spd(d, 951, 0.05)
    Gpsi = spd(d, 952, 0.08)
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    N = ds.grid.P[d - 1]
    with kf.row_launch(kf.FUN_PSI, d, r, N, variant, 0):
        out = kf.psi_batch([ds], [Gpsi], r).cpu().numpy()[0]
    g_o = grid.plan_auto(X, Gp, [M] * d)
    co, _ = linbin.linbin(X, g_o)
    A = binned.autocorr_direct(linbin.counts_to_real(co))
    want = binned.psi(A, X.shape[0], g_o, Gpsi, r)
    sabs = binned.abs_scale(A, X.shape[0], g_o, Gpsi, multiindex.unique_alphas(d, r))
    assert_psi_close(out, want, sabs, what=f"psi batch variant {variant}")


@pytest.mark.parametrize("variant", [3, 4, 5, 6])
def test_narrow_kernels_recurrence_fallback(kf, gpu, variant):
    """Kernels much narrower than the bins: the far lags underflow, so the
    lag-domain kernel's recurrence falls back to direct evaluation (variant 3)
    or walks scaled values (variant 4) there."""
    d, M = 2, 48
    X = mixture_sample(1500, d, 990)
    Gp = np.diag([2e-4, 3e-4])
    H = np.stack([np.diag([1e-4, 2e-4]), np.array([[3e-4, 1e-4], [1e-4, 2e-4]]), np.eye(2) * 0.3])
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    v = torch.from_numpy(_vech(H)).to(gpu)
    N = ds.grid.P[d - 1]
    with kf.row_launch(kf.FUN_SCV_OBJGRAD, d, 2, N, variant, 0):
        obj, g = kf.scv([ds], v)
    _check_against_oracle(kf, "narrow", d, X, Gp, M, H, obj.cpu().numpy(), g.cpu().numpy())


def test_timing_hook_records_row_launches(kf, gpu):
    """The row-kernel timer brackets exactly the batched row launches, tags
    them by family and r, and leaves the results unchanged."""
    name = "d2"
    d, n, M, B = CASES[name]
    X = mixture_sample(n, d, 100 + d)
    Gp = spd(d, 200 + d, 0.05)
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    v = torch.from_numpy(_vech(_Hs(d, B, 5))).to(gpu)
    o0, g0 = kf.scv([ds], v)
    kf.timing_start(8)
    o1, g1 = kf.scv([ds], v)
    kf.psi_batch([ds], [spd(d, 300, 0.08)], 4)
    kf.scv([ds], v, grad=False)
    torch.cuda.synchronize()
    recs = kf.timing_stop()
    log(f"timing records {recs}")
    assert [(f, r) for _, f, r in recs] == [(kf.FUN_SCV_OBJGRAD, 2), (kf.FUN_PSI, 4), (kf.FUN_SCV_OBJ, 2)]
    assert all(0.0 < ms < 1000.0 for ms, _, _ in recs)
    assert torch.equal(o0, o1) and torch.equal(g0, g1)
    assert kf.timing_stop() == []
    # a full timer records no more than it was armed for
    kf.timing_start(1)
    kf.scv([ds], v)
    kf.scv([ds], v)
    assert len(kf.timing_stop()) == 1


def test_walk_runs_count(kf, gpu):
    """kdefft_scv_walk_runs: the compacted walk's live runs -- at least one per
    candidate and row band around lag 0, at most every run of every row, and
    more for wider bandwidths (longer live intervals)."""
    d, X, Gp, M, H, _ = _setup("d2", gpu)
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=M)
    N = ds.grid.P[d - 1]
    RL = kf.lag_layout(N, True)[0]
    B = H.shape[0]
    v = torch.from_numpy(_vech(H)).to(gpu)
    runs = kf.scv_walk_runs([ds], v)
    log(f"[walk runs] d=2 M={M} N={N}: {runs} of {(B + 1) * M * (N // RL)} runs")
    assert B + 1 <= runs <= (B + 1) * M * (N // RL)
    wide = kf.scv_walk_runs([ds], torch.from_numpy(_vech(4.0 * H)).to(gpu))
    narrow = kf.scv_walk_runs([ds], torch.from_numpy(_vech(0.25 * H)).to(gpu))
    assert narrow <= runs <= wide and narrow < wide
