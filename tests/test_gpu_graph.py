"""The whole hot-path step (device-planned grid, binning, count transform,
psi_4, SCV objective + gradient and adjoint, LSCV, LSCV_4, Q_2, PI, and the
single-call psi_2 routes) captured in a HIP graph.

Every replay must reproduce the eager results bit for bit; replays are
interleaved with unrelated eager work on the same device (the capture must not
depend on state that eager calls change), and all replays are checked.
"""
import numpy as np
import pytest
import torch

import synth

from _gpu_util import log, mixture_sample, spd

pytestmark = pytest.mark.gpu


def test_step_graph_replays_match_eager(kf, gpu):
    d, n, M, B = 2, 3000, 40, 16
    X = torch.from_numpy(mixture_sample(n, d, 4242)).to(gpu)
    Gp, Gpsi = spd(d, 4243, 0.05), spd(d, 4244, 0.08)
    v = torch.from_numpy(synth.vech_chol(synth.random_H_2d(B, np.random.default_rng(4245)))).to(gpu)

    g = kf.grid_auto(X, Gpsi, M)   # reads the bounds back: planned outside the capture
    w = torch.linspace(0.5, 1.5, B, dtype=torch.float64, device=gpu)

    def step():
        ds = kf.Dataset(X, Gp, M=M)
        p4 = kf.psi_batch([ds], [Gpsi], 4)
        so, sg = kf.scv([ds], v)
        lo, lg = kf.crit([ds], v, "lscv")
        po, pg = kf.pi(p4, [n], v)
        adj = kf.scv_adjoint([ds], v, w)
        l4 = kf.crit([ds], v, "lscv", 4, grad=False)
        q2 = kf.crit([ds], v, "qr", 2, grad=False)
        p2f = kf.psi(X, Gpsi, 2, grid=g, mode="fused")
        p2p = kf.psi(X, Gpsi, 2, grid=g, mode="plain")
        return p4, so, sg, lo, lg, po, pg, adj, l4, q2, p2f, p2p

    want = [t.clone() for t in step()]
    side = torch.cuda.Stream(gpu)
    side.wait_stream(torch.cuda.current_stream(gpu))
    with torch.cuda.stream(side):
        for _ in range(2):
            step()
    torch.cuda.current_stream(gpu).wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        outs = step()
    other = torch.from_numpy(mixture_sample(1500, d, 77)).to(gpu)
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip(outs, want)):
            assert torch.equal(a, b), (rep, k)
        # unrelated eager work between replays
        ds2 = kf.Dataset(other, Gp, M=24)
        kf.scv([ds2], v[:3])
        torch.cuda.synchronize()
        log(f"[graph] replay {rep} matches eager")
