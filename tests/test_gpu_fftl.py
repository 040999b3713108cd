"""fft-L (Eq. (25)-(27)) on the GPU vs the oracle.

* psi_r by the truncated-support route vs the oracle's binned sum over the
  same lag box (<= 1e-11 relative, near-zero entries against the sum of
  |kernel|), d = 1..4, r = 0, 2, 4; the L and P the library used equal the
  oracle's Eq. (26)-(27) values;
* the paper's speed-experiment shape (d = 2, N(0, I), n = 4000, M = 160) and
  the case-2 shape (n = 1e5, M = 256, r = 4); the truncation error against the
  full sum is logged (a property of the method, not a tolerance).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import binned, fftl, grid, linbin, multiindex

from _gpu_util import assert_psi_close, log, mixture_sample, oracle_autocorr, spd

pytestmark = pytest.mark.gpu

CASES = [(1, 3000, 200, 0), (1, 3000, 200, 4), (2, 3000, 60, 0), (2, 3000, 45, 2), (2, 3000, 60, 4),
         (3, 4000, 24, 2), (4, 3000, 10, 0), (4, 3000, 9, 2)]


@pytest.mark.parametrize("d,n,M,r", CASES)
def test_psi_fftl_vs_oracle(kf, gpu, d, n, M, r):
    X = mixture_sample(n, d, 40 + d)
    G = spd(d, 50 + d, 0.03)
    g = kf.grid_auto(torch.from_numpy(X).to(gpu), G, M)
    log(f"[fftl] d={d} n={n} M={M} r={r}")
    out, L, P = kf.psi_fftl(torch.from_numpy(X).to(gpu), G, r, grid=g)
    gd = g.to_dict()
    Lo = fftl.plan_L(gd, G)
    assert L == Lo and P == fftl.plan_P(gd["M"], Lo)
    co, sk = linbin.linbin(X, gd)
    assert sk == 0
    A = oracle_autocorr(linbin.counts_to_real(co))
    want = fftl.psi_truncated(A, n, gd, G, r, Lo)
    sc = fftl.psi_truncated(A, n, gd, G, r, Lo, absval=True)
    assert_psi_close(out.cpu().numpy(), want, sc, what=f"fftl d={d} M={M} r={r}")
    full = binned.psi(A, n, gd, G, r)
    log(f"   L={L} P={P} grid P={list(gd['P'])} truncation rel diff "
        f"{np.max(np.abs(want - full) / np.maximum(np.abs(full), 1e-300)):.2e}")


def test_paper_speed_shape(kf, gpu):
    rng = np.random.default_rng(151107482 + 60)
    n, M = 4000, 160
    X = rng.standard_normal((n, 2))
    Sh = np.cov(X.T)
    G = n ** (-2.0 / 6.0) * Sh
    Xt = torch.from_numpy(X).to(gpu)
    g = kf.grid_auto(Xt, G, M)
    out, L, P = kf.psi_fftl(Xt, G, 0, grid=g)
    gd = g.to_dict()
    co, _ = linbin.linbin(X, gd)
    A = oracle_autocorr(linbin.counts_to_real(co))
    want = fftl.psi_truncated(A, n, gd, G, 0, L)
    assert out.item() == pytest.approx(want[0], rel=1e-11)
    full = kf.psi(Xt, G, 0, grid=g, mode="plain").item()
    log(f"[fftl] paper shape L={L} P={P} (fft-M P={list(gd['P'])}) psi0 fftL={out.item():.15e} "
        f"full={full:.15e} rel diff {abs(out.item() - full) / full:.2e}")


def test_case2_shape(kf, gpu):
    w = synth.case2()
    X, G = w.X[0], w.G_psi[0]
    Xt = torch.from_numpy(X).to(gpu)
    g = kf.grid_auto(Xt, G, w.M)
    out, L, P = kf.psi_fftl(Xt, G, 4, grid=g)
    gd = g.to_dict()
    co, _ = linbin.linbin(X, gd)
    A = oracle_autocorr(linbin.counts_to_real(co))
    want = fftl.psi_truncated(A, X.shape[0], gd, G, 4, L)
    sc = fftl.psi_truncated(A, X.shape[0], gd, G, 4, L, absval=True)
    assert_psi_close(out.cpu().numpy(), want, sc, what="fftl case2")
    full = kf.psi(Xt, G, 4, grid=g, mode="plain").cpu().numpy()
    log(f"[fftl] case2 L={L} P={P} max rel diff to full {np.max(np.abs(out.cpu().numpy() - full) / np.abs(full)):.2e}")
