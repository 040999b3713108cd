"""Full-size parity at the benchmark cases' shapes, in the launches the
benchmark times, against values the oracle wrote (tests/golden/make_golden.py:
FFT-free binned sums of Eq. (17)-(18) on the same seeded inputs).

* case 4 (d=2, n=1e5, M=256, P=512): grid bits and counts (SHA-256) of the
  device-planned dataset; psi_4 at the psi pilot on that grid through the
  batched lag launch that completes inside the kernel; the SCV objective and
  every gradient entry of all 256 candidates in each lag-domain launch
  (variants 3-6, resident and one-block-per-item grids) and each spectral
  launch (variants 0-2): 1e-11 per entry under the near-zero rule;
* case 4: the GPU gradient against central differences of the GPU objective
  with Richardson extrapolation, 8 candidates, 1e-7;
* case 3 (d=3, n=2e5, M=64): psi_2 (plain, fused and batched routes) and the
  SCV objective + gradient at four bandwidths;
* case-5 shape (d=4, n=2e5, M=32, P=64): the 35-entry psi_4 batch launch, the
  SCV objective + gradient of two candidates in every lag-domain launch, and
  the gradient against central differences (Richardson) of the GPU objective;
* case-5 uneven batch: four d=4 datasets of uneven n in one SCV launch and one
  psi_4 launch.
"""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

import synth

from _gpu_util import assert_z16, log

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
RTOL = 1e-11


def _golden(name):
    with open(os.path.join(GOLDEN, f"{name}.json")) as fh:
        return json.load(fh)


def _check_grid_counts(ds, gold):
    g = ds.grid
    d = g.d
    assert [float(v).hex() for v in g.lo[:d]] == gold["lo_hex"]
    assert [float(v).hex() for v in g.delta[:d]] == gold["delta_hex"]
    assert list(g.P[:d]) == gold["P"]


def _sha(counts):
    return hashlib.sha256(np.ascontiguousarray(counts.cpu().numpy(), dtype="<i8").tobytes()).hexdigest()


def _check_scv(obj, grad, gold, what):
    assert_z16(obj, gold["obj"], gold["obj_scale"], RTOL, what=f"{what} objective")
    assert_z16(grad, gold["grad"], gold["grad_scale"], RTOL, what=f"{what} gradient")


def _fd_check(kf, ds, v0, h, what):
    """Central differences of the GPU objective with Richardson extrapolation
    against the GPU gradient (all perturbed candidates in one launch)."""
    B, q = v0.shape
    _, g = kf.scv([ds], torch.from_numpy(v0).to(ds.device))
    g = g.cpu().numpy()
    pts = []
    for b in range(B):
        for k in range(q):
            for s in (h, -h, h / 2, -h / 2):
                w = v0[b].copy()
                w[k] += s
                pts.append(w)
    obj = kf.scv([ds], torch.from_numpy(np.array(pts)).to(ds.device), grad=False).cpu().numpy().reshape(B, q, 4)
    d1 = (obj[..., 0] - obj[..., 1]) / (2 * h)
    d2 = (obj[..., 2] - obj[..., 3]) / h
    fd = (4 * d2 - d1) / 3
    err = np.abs(fd - g).max(axis=1) / np.abs(g).max(axis=1)
    log(f"  {what}: finite differences, worst candidate rel err {err.max():.2e} (bar 1e-7)")
    assert err.max() <= 1e-7, (what, err)


# ------------------------------------------------------------------ case 4

@pytest.fixture(scope="module")
def case4(kf, gpu):
    w = synth.case4()
    gold = _golden("case4")
    X = torch.from_numpy(w.X[0]).to(gpu)
    ds = kf.Dataset(X, w.G_pilot[0], M=w.M)
    v = torch.from_numpy(synth.vech_chol(w.H[0])).to(gpu)
    return w, gold, ds, v


def test_case4_grid_counts_psi4(kf, gpu, case4):
    w, gold, ds, _ = case4
    log("[full] case4 grid, counts, psi_4 (P=512, completion inside the lag launch)")
    _check_grid_counts(ds, gold["grid"])
    assert _sha(ds.counts()) == gold["counts_sha256"]
    N = gold["grid"]["P"][1]
    for var in (3, 4):
        with kf.row_launch(kf.FUN_PSI, 2, 4, N, var, 0):
            got = kf.psi_batch([ds], [w.G_psi[0]], 4).cpu().numpy()[0]
        assert_z16(got, gold["psi4"]["values"], gold["psi4"]["scales"], RTOL, what=f"case4 psi_4 variant {var}")


@pytest.mark.parametrize("launch", [(3, 0), (3, -1), (4, 0), (4, -1), (5, 0), (5, -1), (6, 0), (6, -1),
                                    (0, 0), (1, 0), (2, 0)])
def test_case4_all_candidates(kf, gpu, case4, launch):
    w, gold, ds, v = case4
    N = gold["grid"]["P"][1]
    log(f"[full] case4 SCV obj+grad, all 256 candidates, launch variant {launch[0]} grid {launch[1]}")
    kinds = (kf.FUN_SCV_OBJ, kf.FUN_SCV_OBJGRAD, kf.FUN_SCV_GRAD)
    with kf.row_launch(kinds, 2, 2, N, *launch):
        obj, g = kf.scv([ds], v)
        adj = kf.scv_adjoint([ds], v, torch.ones(v.shape[0], dtype=torch.float64, device=gpu))
    _check_scv(obj.cpu().numpy(), g.cpu().numpy(), gold["scv"], f"case4 launch {launch}")
    assert_z16(adj.cpu().numpy(), gold["scv"]["grad"], gold["scv"]["grad_scale"], RTOL,
               what=f"case4 adjoint launch {launch}")


def test_case4_default_launch_and_tuned(kf, gpu, case4):
    """The untuned default and the autotuner's choice (the benchmark's launch)."""
    w, gold, ds, v = case4
    obj, g = kf.scv([ds], v)
    _check_scv(obj.cpu().numpy(), g.cpu().numpy(), gold["scv"], "case4 default launch")
    N = gold["grid"]["P"][1]
    kinds = (kf.FUN_SCV_OBJ, kf.FUN_SCV_OBJGRAD, kf.FUN_SCV_GRAD)
    saved = [(k, kf.get_row_launch(k, 2, 2, N)) for k in kinds]
    P = gold["grid"]["P"]
    saved_fft = kf.get_fft_schedule(P)
    saved_psi = kf.get_row_launch(kf.FUN_PSI, 2, 4, N)
    try:
        log("[full] case4 autotune " + kf.autotune(ds).replace("\n", "; "))
        obj, g = kf.scv([ds], v)
        _check_scv(obj.cpu().numpy(), g.cpu().numpy(), gold["scv"], "case4 tuned launch")
        # the tuner re-ran the dataset's transform under the chosen schedule;
        # a dataset prepared afresh uses it too
        for dd in (ds, kf.Dataset(torch.from_numpy(w.X[0]).to(gpu), w.G_pilot[0], M=w.M)):
            got = kf.psi_batch([dd], [w.G_psi[0]], 4).cpu().numpy()[0]
            assert_z16(got, gold["psi4"]["values"], gold["psi4"]["scales"], RTOL, what="case4 psi_4 tuned")
    finally:
        for k, (var, gb) in saved:
            kf.set_row_launch(k, 2, 2, N, var, gb)
        kf.set_row_launch(kf.FUN_PSI, 2, 4, N, *saved_psi)
        kf.set_fft_schedule(P, saved_fft)


def test_case4_finite_differences(kf, gpu, case4):
    w, gold, ds, _ = case4
    idx = [0, 31, 64, 100, 128, 177, 200, 255]
    log("[full] case4 gradient vs central differences (Richardson), 8 candidates")
    _fd_check(kf, ds, synth.vech_chol(w.H[0][idx]), 1e-3, "case4")


# ------------------------------------------------------------------ case 3

def test_case3_psi2_and_scv(kf, gpu):
    w = synth.case3()
    gold = _golden("case3")
    X = torch.from_numpy(w.X[0]).to(gpu)
    G = w.G_psi[0]
    log("[full] case3 d=3 n=2e5 M=64: psi_2 plain / fused / batched, SCV obj+grad")
    g = kf.grid_auto(X, G, w.M)
    assert [float(x).hex() for x in g.lo[:3]] == gold["grid"]["lo_hex"]
    assert [float(x).hex() for x in g.delta[:3]] == gold["grid"]["delta_hex"]
    for mode in ("plain", "fused"):
        got = kf.psi(X, G, 2, grid=g, mode=mode).cpu().numpy()
        assert_z16(got, gold["psi2"]["values"], gold["psi2"]["scales"], RTOL, what=f"case3 psi_2 {mode}")
    ds = kf.Dataset(X, w.G_pilot[0], M=w.M)
    _check_grid_counts(ds, gold["grid"])
    assert _sha(ds.counts()) == gold["counts_sha256"]
    got = kf.psi_batch([ds], [G], 2).cpu().numpy()[0]
    assert_z16(got, gold["psi2"]["values"], gold["psi2"]["scales"], RTOL, what="case3 psi_2 batched")
    H = np.array(gold["H"])
    obj, gr = kf.scv([ds], torch.from_numpy(synth.vech_chol(H)).to(gpu))
    _check_scv(obj.cpu().numpy(), gr.cpu().numpy(), gold["scv"], "case3")


# ------------------------------------------------------------------ case 5

@pytest.fixture(scope="module")
def case5_shape(kf, gpu):
    w = synth.case5(n_datasets=1, B=2, n_lo=200_000, n_hi=200_000)
    gold = _golden("case5_shape")
    ds = kf.Dataset(torch.from_numpy(w.X[0]).to(gpu), w.G_pilot[0], M=w.M)
    return w, gold, ds


def test_case5_shape_psi4_batch(kf, gpu, case5_shape):
    w, gold, ds = case5_shape
    log("[full] case5 shape d=4 n=2e5 M=32: grid, counts, psi_4 (35 entries, N=64)")
    _check_grid_counts(ds, gold["grid"])
    assert _sha(ds.counts()) == gold["counts_sha256"]
    got = kf.psi_batch([ds], [w.G_psi[0]], 4).cpu().numpy()[0]
    assert_z16(got, gold["psi4"]["values"], gold["psi4"]["scales"], RTOL, what="case5 shape psi_4")


@pytest.mark.parametrize("variant", [3, 4, 5, 6])
def test_case5_shape_scv(kf, gpu, case5_shape, variant):
    w, gold, ds = case5_shape
    log(f"[full] case5 shape SCV obj+grad, launch variant {variant}")
    v = torch.from_numpy(synth.vech_chol(w.H[0])).to(gpu)
    kinds = (kf.FUN_SCV_OBJ, kf.FUN_SCV_OBJGRAD, kf.FUN_SCV_GRAD)
    with kf.row_launch(kinds, 4, 2, 64, variant, 0):
        obj, g = kf.scv([ds], v)
    _check_scv(obj.cpu().numpy(), g.cpu().numpy(), gold["scv"], f"case5 shape variant {variant}")


def test_case5_shape_finite_differences(kf, gpu, case5_shape):
    w, gold, ds = case5_shape
    log("[full] case5 shape gradient vs central differences (Richardson)")
    _fd_check(kf, ds, synth.vech_chol(w.H[0]), 1e-3, "case5 shape")


def test_case5_uneven_batch(kf, gpu):
    gold = _golden("case5_uneven")
    w = synth.case5(**gold["args"])
    log(f"[full] case5 uneven: {len(w.X)} datasets, n = {gold['n']}")
    dss = [kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=w.M) for X, Gp in zip(w.X, w.G_pilot)]
    for j, ds in enumerate(dss):
        _check_grid_counts(ds, gold["grid"][j])
        assert _sha(ds.counts()) == gold["counts_sha256"][j]
    per = [H.shape[0] for H in w.H]
    v = torch.from_numpy(np.concatenate([synth.vech_chol(H) for H in w.H])).to(gpu)
    obj, g = kf.scv(dss, v, per_ds=per)
    obj, g = obj.cpu().numpy(), g.cpu().numpy()
    psi = kf.psi_batch(dss, w.G_psi, 4).cpu().numpy()
    s = 0
    for j in range(len(dss)):
        _check_scv(obj[s:s + per[j]], g[s:s + per[j]], gold["scv"][j], f"case5 uneven dataset {j}")
        assert_z16(psi[j], gold["psi4"][j]["values"], gold["psi4"][j]["scales"], RTOL,
                   what=f"case5 uneven psi_4 dataset {j}")
        s += per[j]
