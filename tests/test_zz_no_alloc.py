"""kdefft_scv_batch_noalloc (the batched SCV call with the library's fixed
device scratch as workspace) against kdefft_scv_batch (caller workspace) and
the oracle, through the C ABI:

* two calls in a row, the second with a smaller input (fewer candidates, a
  smaller grid in another dimension), each equal to the workspace call bit for
  bit and to the oracle's binned objective and gradient (1e-11 per entry,
  near-zero rule);
* an uneven two-dataset batch, objective only;
* a batch whose workspace exceeds the scratch is refused (KDEFFT_E_WORKSPACE)
  and leaves the outputs untouched.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import grid, linbin, scv

from _gpu_util import assert_z16, log, mixture_sample, oracle_autocorr, spd

pytestmark = pytest.mark.gpu


def _oracle_check(X, Gp, M, H, obj, grad, what):
    d = X.shape[1]
    g = grid.plan_auto(X, Gp, [M] * d)
    counts, _ = linbin.linbin(X, g)
    A = oracle_autocorr(linbin.counts_to_real(counts))
    n = X.shape[0]
    want = [scv.objective_binned(A, n, g, H[b], Gp) for b in range(H.shape[0])]
    sc = [scv.objective_binned_scales(A, n, g, H[b], Gp) for b in range(H.shape[0])]
    assert_z16(obj, [o for o, _ in want], [s for s, _ in sc], what=f"{what} objective")
    if grad is not None:
        assert_z16(grad, np.array([gr for _, gr in want]), np.array([s for _, s in sc]), what=f"{what} gradient")


def _call_both(kf, dss, v, per_ds, with_grad=True):
    dev = v.device
    B, q = v.shape
    obj = torch.full((B,), -1.0, dtype=torch.float64, device=dev)
    grad = torch.full((B, q), -1.0, dtype=torch.float64, device=dev) if with_grad else None
    st = torch.full((B,), 7, dtype=torch.int32, device=dev)
    kf.scv_batch_noalloc(dss, v, obj, grad, st, per_ds=per_ds)
    ref = kf.scv(dss, v, per_ds=per_ds, grad=with_grad, status=True)
    torch.cuda.synchronize()
    assert torch.equal(obj, ref[0])
    if with_grad:
        assert torch.equal(grad, ref[1])
    assert torch.equal(st, ref[2]) and int(st.max()) == 0
    return obj.cpu().numpy(), None if grad is None else grad.cpu().numpy()


def test_noalloc_two_calls_second_smaller(kf, gpu):
    X1 = mixture_sample(3000, 2, 81)
    Gp1 = spd(2, 82, 0.05)
    H1 = synth.random_H_2d(300, np.random.default_rng(83))
    ds1 = kf.Dataset(torch.from_numpy(X1).to(gpu), Gp1, M=40)
    log("[noalloc] call 1: d=2 M=40 B=300")
    obj, grad = _call_both(kf, [ds1], torch.from_numpy(synth.vech_chol(H1)).to(gpu), None)
    _oracle_check(X1, Gp1, 40, H1[::37], obj[::37], grad[::37], "call 1")

    X2 = mixture_sample(1200, 3, 84)
    Gp2 = spd(3, 85, 0.05)
    H2 = synth.random_H_haar(17, 3, np.random.default_rng(86))
    ds2 = kf.Dataset(torch.from_numpy(X2).to(gpu), Gp2, M=12)
    log("[noalloc] call 2: d=3 M=12 B=17")
    obj, grad = _call_both(kf, [ds2], torch.from_numpy(synth.vech_chol(H2)).to(gpu), None)
    _oracle_check(X2, Gp2, 12, H2, obj, grad, "call 2")


def test_noalloc_uneven_datasets_objective_only(kf, gpu):
    sets = []
    for j, n in enumerate((900, 4000)):
        X = mixture_sample(n, 2, 90 + j)
        Gp = spd(2, 92 + j, 0.04)
        H = synth.random_H_2d((5, 9)[j], np.random.default_rng(94 + j))
        sets.append((X, Gp, H))
    dss = [kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=32) for X, Gp, _ in sets]
    v = torch.from_numpy(np.concatenate([synth.vech_chol(H) for _, _, H in sets])).to(gpu)
    log("[noalloc] two datasets, objective only")
    obj, _ = _call_both(kf, dss, v, [5, 9], with_grad=False)
    _oracle_check(*sets[1][:2], 32, sets[1][2], obj[5:], None, "dataset 1")


def test_noalloc_rejects_oversized_batch(kf, gpu):
    X = mixture_sample(500, 2, 96)
    Gp = spd(2, 97, 0.05)
    ds = kf.Dataset(torch.from_numpy(X).to(gpu), Gp, M=16)
    B = 40_000    # about 30 MiB of parameter blocks and partial sums
    v = torch.from_numpy(synth.vech_chol(synth.random_H_2d(B, np.random.default_rng(98)))).to(gpu)
    obj = torch.full((B,), -1.0, dtype=torch.float64, device=gpu)
    with pytest.raises(kf.KdefftError) as ei:
        kf.scv_batch_noalloc([ds], v, obj)
    assert ei.value.code == kf._lib.E_WORKSPACE
    torch.cuda.synchronize()
    assert bool((obj == -1.0).all())
