"""The whole hot-path step (device-planned grid, binning, count transform,
psi_4, SCV objective + gradient, LSCV, PI) captured in a HIP graph.

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

    def step():
        ds = kf.Dataset(X, Gp, M=M)
        p4 = kf.psi_batch([ds], [Gpsi], 4)
        so, sg = kf.scv([ds], v)
        lo, lg = kf.crit([ds], v, "lscv")
        po, pg = kf.pi(p4, [n], v)
        return p4, so, sg, lo, lg, po, pg

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
