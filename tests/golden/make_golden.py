"""Write the expected values of the full-size GPU parity tests.

Every value in the files written here comes from ``oracle/`` alone (the
FFT-free binned sums: count autocorrelation by shifted slices or slab
products, then the lag-domain sums of Eq. (17)-(18)), on the seeded inputs of
``synth``.  The GPU tests regenerate the same inputs, run the HIP library and
compare against these numbers; nothing here reads the library.

    python tests/golden/make_golden.py [case4] [case3] [case5_shape] [case5_uneven]

Each JSON file records the command, the workload, the oracle's grid (float64
bits as hex), a SHA-256 of the oracle's int64 counts, and for every expected
value its absolute-value scale (the Z16 reading: an entry whose magnitude is
below 1e-3 of its scale is judged against the scale).
"""
from __future__ import annotations

import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import binned, grid, linbin, multiindex, scv  # noqa: E402

_DS = {}   # dataset key -> (A, n, g); filled before the pool forks


def _grid_json(g):
    return {"M": [int(m) for m in g["M"]], "P": [int(p) for p in g["P"]],
            "lo_hex": [float(v).hex() for v in g["lo"]], "delta_hex": [float(v).hex() for v in g["delta"]]}


def _prepare(key, X, Gp, M):
    d = X.shape[1]
    g = grid.plan_auto(X, Gp, [M] * d)
    counts, skipped = linbin.linbin(X, g)
    assert skipped == 0
    c = linbin.counts_to_real(counts)
    A = binned.autocorr_direct(c) if c.size <= 70_000 else binned.autocorr_gemm(c)
    _DS[key] = (A, X.shape[0], g)
    sha = hashlib.sha256(np.ascontiguousarray(counts, dtype="<i8").tobytes()).hexdigest()
    return g, sha


def _task(t):
    kind, key, mat, extra = t
    A, n, g = _DS[key]
    if kind == "psi":
        r = extra
        alphas = multiindex.unique_alphas(g["d"], r)
        return binned.psi(A, n, g, mat, r).tolist(), binned.abs_scale(A, n, g, mat, alphas).tolist()
    Gp = extra
    obj, gr = scv.objective_binned(A, n, g, mat, Gp)
    s_obj, s_gr = scv.objective_binned_scales(A, n, g, mat, Gp)
    return float(obj), gr.tolist(), float(s_obj), s_gr.tolist()


def _run(tasks, workers):
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        return pool.map(_task, tasks, chunksize=1)


def _scv_block(res):
    return {"obj": [r[0] for r in res], "grad": [r[1] for r in res],
            "obj_scale": [r[2] for r in res], "grad_scale": [r[3] for r in res]}


def case4(workers):
    w = synth.case4()
    X, Gpsi, Gp, H = w.X[0], w.G_psi[0], w.G_pilot[0], w.H[0]
    g, sha = _prepare("c4", X, Gp, w.M)
    tasks = [("psi", "c4", Gpsi, 4)] + [("scv", "c4", H[b], Gp) for b in range(H.shape[0])]
    res = _run(tasks, workers)
    return {"workload": "synth.case4(): d=2, n=1e5, M=256, pilot grid n^{-2/8} S_hat; psi_4 at n^{-2/10} S_hat "
                        "on that grid; SCV objective + gradient for all 256 candidates",
            "grid": _grid_json(g), "counts_sha256": sha,
            "psi4": {"values": res[0][0], "scales": res[0][1]}, "scv": _scv_block(res[1:])}


def case3(workers):
    w = synth.case3()
    X, G, Gp, HNS = w.X[0], w.G_psi[0], w.G_pilot[0], w.H[0]
    H = np.concatenate([HNS, synth.random_H_haar(3, 3, synth.rng_for(3, salt=7))])
    g, sha = _prepare("c3", X, Gp, w.M)
    tasks = [("psi", "c3", G, 2)] + [("scv", "c3", H[b], Gp) for b in range(H.shape[0])]
    res = _run(tasks, workers)
    return {"workload": "synth.case3(): d=3, n=2e5, M=64, grid from the pilot n^{-2/9} S_hat; psi_2 at that "
                        "bandwidth; SCV objective + gradient at the normal-scale H and 3 Haar-rotated H "
                        "(synth.random_H_haar(3, 3, synth.rng_for(3, salt=7)))",
            "grid": _grid_json(g), "counts_sha256": sha, "H": H.tolist(),
            "psi2": {"values": res[0][0], "scales": res[0][1]}, "scv": _scv_block(res[1:])}


def case5_shape(workers):
    w = synth.case5(n_datasets=1, B=2, n_lo=200_000, n_hi=200_000)
    X, Gpsi, Gp, H = w.X[0], w.G_psi[0], w.G_pilot[0], w.H[0]
    g, sha = _prepare("c5", X, Gp, w.M)
    tasks = [("psi", "c5", Gpsi, 4)] + [("scv", "c5", H[b], Gp) for b in range(H.shape[0])]
    res = _run(tasks, workers)
    return {"workload": "synth.case5(n_datasets=1, B=2, n_lo=200000, n_hi=200000): d=4, n=2e5, M=32 (P=64), "
                        "grid from the pilot n^{-2/10} S_hat; psi_4 (35 entries) at n^{-2/12} S_hat; SCV "
                        "objective + gradient of both candidates",
            "grid": _grid_json(g), "counts_sha256": sha,
            "psi4": {"values": res[0][0], "scales": res[0][1]}, "scv": _scv_block(res[1:])}


CASE5_UNEVEN = dict(n_datasets=4, B=2, n_lo=2_000, n_hi=40_000)


def case5_uneven(workers):
    w = synth.case5(**CASE5_UNEVEN)
    grids, shas, tasks = [], [], []
    for j, (X, Gp, H) in enumerate(zip(w.X, w.G_pilot, w.H)):
        g, sha = _prepare(f"u{j}", X, Gp, w.M)
        grids.append(_grid_json(g))
        shas.append(sha)
        tasks += [("scv", f"u{j}", H[b], Gp) for b in range(H.shape[0])]
    tasks += [("psi", f"u{j}", w.G_psi[j], 4) for j in range(len(w.X))]
    res = _run(tasks, workers)
    nds, B = len(w.X), CASE5_UNEVEN["B"]
    return {"workload": f"synth.case5(**{CASE5_UNEVEN}): d=4, M=32, {nds} datasets of uneven n, {B} candidates "
                        "each: SCV objective + gradient of every candidate and psi_4 of every dataset",
            "args": CASE5_UNEVEN, "n": [int(X.shape[0]) for X in w.X], "grid": grids, "counts_sha256": shas,
            "scv": [_scv_block(res[j * B:(j + 1) * B]) for j in range(nds)],
            "psi4": [{"values": r[0], "scales": r[1]} for r in res[nds * B:]]}


CASES = {"case4": case4, "case3": case3, "case5_shape": case5_shape, "case5_uneven": case5_uneven}


def main(argv):
    names = argv or list(CASES)
    workers = len(os.sched_getaffinity(0))
    for name in names:
        t0 = time.time()
        out = CASES[name](workers)
        out = {"command": f"python tests/golden/make_golden.py {name}", **out}
        path = os.path.join(HERE, f"{name}.json")
        with open(path, "w") as fh:
            json.dump(out, fh, indent=1)
            fh.write("\n")
        print(f"{name}: {time.time() - t0:.1f} s -> {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
