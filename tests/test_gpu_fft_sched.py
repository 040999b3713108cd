"""Every FFT-stage schedule the tuner can pick (kdefft_set_fft_schedule) on
the count transform, against the oracle:

* the prepared lag array vs the oracle's FFT-free autocorrelation of the same
  counts (1e-12 of its largest entry; exact zeros beyond the last-axis
  support) on small grids d = 1..4 (ragged M, one-wavefront and 256-thread
  shapes, P from 16 to 2048);
* the counts are bit-identical under every schedule, and re-running a dataset's
  transform from its counts reproduces its arrays bit for bit;
* at the benchmark shapes -- d=2, n=1e5, P=512 and the d=4, n=2e5, P=64 case-5
  dataset -- psi_4 of the dataset prepared under each schedule against the
  values the oracle wrote (tests/golden), 1e-11 per entry (near-zero rule).
"""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

import synth
from oracle import grid, linbin

from _gpu_util import assert_z16, log, mixture_sample, oracle_autocorr, spd

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

SMALL = {
    "d1_m900": lambda: (mixture_sample(6000, 1, 61), spd(1, 61, 0.05), 900),
    "d1_m100": lambda: (mixture_sample(3000, 1, 62), spd(1, 62, 0.05), 100),
    "d2_m37": lambda: (mixture_sample(2000, 2, 63), spd(2, 63), 37),
    "d2_m120": lambda: (mixture_sample(4000, 2, 64), spd(2, 64, 0.05), 120),
    "d3_m20": lambda: (mixture_sample(3000, 3, 65), spd(3, 65), 20),
    "d4_m8": lambda: (mixture_sample(2000, 4, 66), spd(4, 66, 0.2), 8),
}

_OR = {}


def _oracle(name, X, G, M):
    if name not in _OR:
        g = grid.plan_auto(X, G, [M] * X.shape[1])
        counts, skipped = linbin.linbin(X, g)
        assert skipped == 0
        _OR[name] = (g, oracle_autocorr(linbin.counts_to_real(counts)))
    return _OR[name]


def _sha(t):
    return hashlib.sha256(np.ascontiguousarray(t.cpu().numpy(), dtype="<i8").tobytes()).hexdigest()


@pytest.mark.parametrize("name", list(SMALL))
def test_every_schedule_lag_array(kf, gpu, name):
    X, G, M = SMALL[name]()
    d = X.shape[1]
    g_o, A = _oracle(name, X, G, M)
    Xd = torch.from_numpy(X).to(gpu)
    g = kf.grid_auto(Xd, G, M)
    P = [int(p) for p in g.P[:d]]
    Mv = [int(m) for m in g.M[:d]]
    idx = [np.arange(-(m - 1), m) % p for m, p in zip(Mv, P)]
    zero = np.arange(P[-1])
    zero = zero[(zero > Mv[-1] - 1) & (zero < P[-1] - (Mv[-1] - 1))]
    shas = set()
    for sched in range(kf.FFT_SCHEDULES):
        log(f"[fft schedule] {name} P={P} schedule {sched}")
        with kf.fft_schedule(P, sched):
            ds = kf.Dataset(Xd, G, grid=g)
            al = ds.lag_array().cpu().numpy()
            shas.add(_sha(ds.counts()))
            # the count transform re-run from the counts (kdefft_dataset_transform)
            # reproduces the prepared arrays bit for bit
            ds.transform()
            assert np.array_equal(ds.lag_array().cpu().numpy(), al)
        got = al[np.ix_(*idx)] / float(np.prod(P))
        np.testing.assert_allclose(got, A, rtol=0, atol=1e-12 * np.abs(A).max(), err_msg=f"schedule {sched}")
        assert np.all(al[..., zero] == 0.0)
    assert len(shas) == 1


def _golden(name):
    with open(os.path.join(GOLDEN, f"{name}.json")) as fh:
        return json.load(fh)


@pytest.mark.parametrize("which", ["case4", "case5_shape"])
def test_every_schedule_full_size_psi4(kf, gpu, which):
    gold = _golden(which)
    if which == "case4":
        w = synth.case4()
    else:
        w = synth.case5(n_datasets=1, B=2, n_lo=200_000, n_hi=200_000)
    X = torch.from_numpy(w.X[0]).to(gpu)
    P = gold["grid"]["P"]
    for sched in range(kf.FFT_SCHEDULES):
        log(f"[fft schedule] {which} P={P} schedule {sched}: psi_4 vs the oracle's values")
        with kf.fft_schedule(P, sched):
            ds = kf.Dataset(X, w.G_pilot[0], M=w.M)
            got = kf.psi_batch([ds], [w.G_psi[0]], 4).cpu().numpy()[0]
        assert_z16(got, gold["psi4"]["values"], gold["psi4"]["scales"], 1e-11,
                   what=f"{which} psi_4 FFT schedule {sched}")
