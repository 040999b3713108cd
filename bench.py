#!/usr/bin/env python3
"""Throughput of the FFT-based psi_r / SCV hot path on one MI355X.

Workload (synthetic, seeded; see synth.case4): d = 2, n = 100,000 points from
a four-component normal mixture, grid M = 256 per axis (padded P = 512),
pilot G = n^{-2/8} S_hat, 256 candidate bandwidths H (random rotations,
log-eigenvalues U[-3, 0]).

One step = the whole hot path over that batch, inputs already in HBM:
  grid plan (data bounds) -> linear binning -> count transform (R2C, |C|^2,
  leading-axis transform, lag array) -> psi_4 at the psi pilot -> SCV
  objective + gradient w.r.t. vech(chol H) for all 256 candidates (and the
  constant phi_{2G} term) in one persistent launch.
value = 256 / (seconds per step)  [SCV objective+gradient evaluations/s].

Also reported (outside the timed loop): the paper-literal plain path one H at
a time (with and without per-call binning and count transform), the
autograd (forward + adjoint) form, psi_4 evals/s, the dominant kernel's
roofline figures and the CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "psi_r evals/s and SCV objective+grad evals/s, batched+adjoint vs plain, FP64"
PEAK_FP64_VECTOR = 78.6e12          # MI355X FP64 vector FLOP/s (256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz)
EXP_FLOPS = 20                      # flops charged per exp (the device exp is ~13 FMA + 4 other FP64 ops)
ROW_KERNEL_SOURCES = ["rows_impl.h", "dev_kernels.h", "dev_common.h", "finish.h", "rows_dispatch.h", "rows_d2.hip",
                      "rows.hip", "params.h"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-h", type=int, default=16, help="candidates timed on the plain path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch", default=None, metavar="VARIANT,GRID",
                    help="pin the SCV row launch (e.g. 3,-1) instead of tuning; used for counter runs")
    ap.add_argument("--cpu-h", type=int, default=256, help="candidates in the CPU oracle sample")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB device copy (counter calibration for rocprofv3 --pmc runs)")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch autotuner (library defaults)")
    ap.add_argument("--no-graph", action="store_true",
                    help="time the eager step only (default: the step is also captured in a HIP graph and replayed)")
    ap.add_argument("--case5", action="store_true",
                    help="measure the d=4 uneven multi-dataset workload instead (extra line, not the headline)")
    return ap.parse_args()


def row_kernel_hash():
    h = hashlib.sha256()
    for f in ROW_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1511_07482_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def gen_flops_per_lag(d=2):
    """Kernel generation at one lag for the objective+gradient family: two
    Gaussians (matrix-vector 2d^2, quadratic form 2d, scale 2, one exp each),
    the objective combination (2) and d(d+1)/2 Hessian entries (7 each)."""
    return 2 * (2 * d * d + 2 * d + 2 + EXP_FLOPS) + 2 + 7 * d * (d + 1) // 2


def moment_walk_layout(N):
    """Run length and runs per segment of the lag moment kernel for rows of
    N positions, as the library was compiled (kdefft_lag_layout; 16-lag runs
    in 32-lag segments for N >= 256, else single runs of up to 8)."""
    import paper_1511_07482_amd as kf
    run, seg, _ = kf.lag_layout(N, True)
    return run, seg


def flops_per_run(N, d=2):
    """FP64 flops of one run of the moment walk (see algorithmic_flops_per_candidate)."""
    q = d * (d + 1) // 2
    RL, SEG = moment_walk_layout(N)
    return (RL * (2 * 8 + 1) + (3 + 25 * q) + 4 * d * (SEG - 1) / SEG
            + 2 * (2 * d * d + 2 * d + 4 + 2 * EXP_FLOPS) / SEG)


def algorithmic_flops_per_candidate(M, N, d=2, variant=0, rows=None):
    """FP64 flops of one candidate in the batched objective+gradient kernel
    over `rows` rows of the half lag set, N positions each (default M rows,
    l_0 = 0..M-1, the d = 2 set; in general M_0 prod_{0<k<d-1} (2 M_k - 1)).

    Lag form (variants 3, 4), the algorithm as designed: per position, per
    Gaussian, the walk e*A, the three moment sums (1 add + 2 FMA) and the two
    recurrence products = 8 flops, plus the row weight (1); per run of RL
    positions the fold of the moments into the objective (3) and the q
    Hessian sums (25 each), and the advance of z (4d); per segment a fresh
    start per Gaussian: S^-1 x (2d^2), x^T S^-1 x (2d), exponent arguments
    (4), two exponentials (EXP_FLOPS each).  Runs whose Gaussians are all
    below the float64 cut-off are skipped by the kernel and still counted here
    (case 4 has almost none).
    Spectral form (variants 0-2), per row: generation at direct-evaluation cost
    at the 2M-1 nonzero lags, two complex FFTs of length N (the 4 real grids
    packed two per transform) at 5 N log2 N flops each and the contraction,
    8 flops per complex multiply-add per transform."""
    q = d * (d + 1) // 2
    rows = M if rows is None else rows
    if variant >= 3:
        RL, SEG = moment_walk_layout(N)
        per_run = (RL * (2 * 8 + 1) + (3 + 25 * q) + 4 * d * (SEG - 1) / SEG
                   + 2 * (2 * d * d + 2 * d + 4 + 2 * EXP_FLOPS) / SEG)
        return rows * (N // RL) * per_run
    gen = (2 * M - 1) * gen_flops_per_lag(d)
    log2n = int(np.log2(N))
    fft = 2 * 5 * N * log2n
    contraction = 2 * N * 8
    return rows * (fft + contraction + gen)


def direct_equivalent_flops_per_candidate(M, d=2):
    """The same sums evaluated lag by lag (kernel generation at its direct
    cost at each of the (2M-1) lags of the M rows, then 2 flops per grid):
    the work the walk replaces."""
    return M * (2 * M - 1) * (gen_flops_per_lag(d) + 2 * (1 + d * (d + 1) // 2))


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported "
              "(the path shards by candidates or datasets with no exchange between GPUs)", file=sys.stderr)
        sys.exit(2)
    if a.case5:
        return main_case5(a)
    import torch
    import paper_1511_07482_amd as kf
    import synth

    dev = torch.device("cuda:0")
    w = synth.case4()
    X_h, Gpsi, Gp, H = w.X[0], w.G_psi[0], w.G_pilot[0], w.H[0]
    n, d = X_h.shape
    B = H.shape[0]
    M = w.M
    X = torch.from_numpy(X_h).to(dev)
    vechL = torch.from_numpy(synth.vech_chol(H)).to(dev)
    tuned = None
    variant, grid_blocks = 4, 0   # library default for untuned shapes
    if a.launch:
        variant, grid_blocks = (int(x) for x in a.launch.split(","))
        kf.set_row_launch(kf.FUN_SCV_OBJGRAD, d, 2, max(4, 1 << (2 * M - 2).bit_length()), variant, grid_blocks)
    elif not a.no_tune:
        ds0 = kf.Dataset(X, Gp, M=M)
        tuned = kf.autotune(ds0)
        for line in tuned.splitlines():
            if line.startswith("best: variant"):
                variant, grid_blocks = int(line.split()[2]), int(line.split()[4])

    def step(ev=None):
        # grid planned, data binned and counts transformed on the device
        main = torch.cuda.current_stream(dev)
        ds = kf.Dataset(X, Gp, M=M)
        psi = kf.psi_batch([ds], [Gpsi], 4)
        if ev is not None:
            ev[0].record(main)
        obj, grad = kf.scv([ds], vechL)
        if ev is not None:
            ev[1].record(main)
        return ds, psi, obj, grad

    stream = torch.cuda.current_stream(dev)
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()

    # ---- timed region: exactly `steps` whole steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(a.steps)]
    # the library brackets each row-kernel launch with HIP events on its stream
    kf.timing_start(4 * a.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(a.steps):
        ds, psi, obj, grad = step(ev[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    recs = kf.timing_stop()
    sec_per_step = (t1 - t0) / a.steps
    g = ds.grid   # the device-planned grid, read back after the timed region
    value = B / sec_per_step
    scv_call_ms = float(np.mean([s.elapsed_time(e) for s, e in ev]))
    scv_k = [ms for ms, fam, r in recs if fam == kf.FUN_SCV_OBJGRAD]
    psi_k = [ms for ms, fam, r in recs if fam == kf.FUN_PSI]
    assert len(scv_k) == a.steps and len(psi_k) == a.steps, recs
    scv_ms = float(np.mean(scv_k))
    assert torch.isfinite(obj).all() and torch.isfinite(grad).all()
    eager = {"value": value, "ms_per_step": sec_per_step * 1e3}

    # ---- the same step captured once in a HIP graph and replayed: every
    # kernel of the step runs on every replay; only the host-side launch work
    # is recorded once.  Replays are checked against the eager results.
    graph_info = None
    if not a.no_graph:
        side = torch.cuda.Stream(dev)
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            for _ in range(2):
                step()
        stream.wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            _, g_psi, g_obj, g_grad = step()
        for _ in range(max(a.warmup, 1)):
            graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(g_obj, obj) and torch.equal(g_grad, grad) and torch.equal(g_psi, psi)
        t0 = time.perf_counter()
        for k in range(a.steps):
            graph.replay()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        assert torch.equal(g_obj, obj) and torch.equal(g_grad, grad)
        sec_per_step = (t1 - t0) / a.steps
        value = B / sec_per_step
        graph_info = {"mode": "whole step captured once in a HIP graph (torch.cuda.CUDAGraph), replayed",
                      "value": value, "ms_per_step": sec_per_step * 1e3,
                      "replays_equal_eager": True}
        del graph

    # ---- components outside the timed loop
    def timed(fn, reps, warm=2):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        s = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - s) / reps, out

    t_prep, ds = timed(lambda: kf.Dataset(X, Gp, M=M), 5)
    t_psi_batched, _ = timed(lambda: kf.psi_batch([ds], [Gpsi], 4), 10)
    t_psi_plain, _ = timed(lambda: kf.psi(X, Gpsi, 4, grid=g, mode="plain"), 5)
    t_scv_only, _ = timed(lambda: kf.scv([ds], vechL), 10)

    # binning alone (the standalone entry: zero fill of one int64 grid, then the
    # points), HIP events on the stream: n points x 2^d lane atomics each
    kf.linbin(X, g)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(20):
        kf.linbin(X, g)
    e1.record(stream)
    torch.cuda.synchronize()
    t_bin = e0.elapsed_time(e1) / 20 * 1e-3
    binning = {"call_ms": t_bin * 1e3, "points_per_s": n / t_bin, "lane_atomics_per_s": n * 2 ** d / t_bin,
               "x_read_GB_per_s": n * d * 8 / t_bin / 1e9,
               "what": "kdefft_linbin on the case-4 grid: fill of the 256^2 int64 grid plus binning of the "
                       "1e5 points (the step's own binning adds into corner slots cleared by the bounds pass)"}

    def autograd_step():
        v = vechL.clone().requires_grad_(True)
        o = kf.SCV.apply(v, ds)
        o.sum().backward()
        return v.grad

    t_autograd, _ = timed(autograd_step, 5)

    # the per-candidate FFT route (spectral kernel, best of its variants in the
    # tuner's list, else variant 1), timed with HIP events like the step's launch
    N = int(g.P[d - 1])
    spec_variant = 1
    if tuned:
        best_us = None
        for line in tuned.splitlines():
            p = line.split()
            if p and p[0] == "variant" and int(p[1]) < 3:
                us = float(p[4])
                if best_us is None or us < best_us:
                    best_us, spec_variant = us, int(p[1])
    kf.set_row_launch(kf.FUN_SCV_OBJGRAD, d, 2, N, spec_variant, 0)
    kf.scv([ds], vechL)
    kf.timing_start(5)
    for _ in range(5):
        kf.scv([ds], vechL)
    torch.cuda.synchronize()
    spec_ms = float(np.mean([ms for ms, fam, r in kf.timing_stop()]))
    kf.set_row_launch(kf.FUN_SCV_OBJGRAD, d, 2, N, variant, grid_blocks)
    # the paper's literal steps one H at a time.  The device-planned grid is read
    # back once here (ds.grid keeps it in the descriptor), so no plain call waits
    # on the device; "with binning" re-bins the data and re-transforms the counts
    # on that same grid before every call (as the paper's timings include binning)
    hp = min(a.plain_h, B)
    assert ds.grid.d == d
    kf.scv_plain(ds, H[0])
    torch.cuda.synchronize()
    s = time.perf_counter()
    for b in range(hp):
        kf.scv_plain(ds, H[b])
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - s) / hp
    kf.scv_plain(kf.Dataset(X, Gp, grid=g), H[0])
    torch.cuda.synchronize()
    s = time.perf_counter()
    for b in range(hp):
        dsb = kf.Dataset(X, Gp, grid=g)
        kf.scv_plain(dsb, H[b])
    torch.cuda.synchronize()
    t_plain_prep = (time.perf_counter() - s) / hp

    if a.calib_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    # ---- roofline of the dominant kernel (batched SCV objective+gradient launch)
    # work of the launch: the compacted walk (variants 5, 6) visits only the
    # runs with a lag above 1e-30 of some Gaussian's peak, counted on the device
    # for these candidates (and the constant term's pseudo-candidate); the
    # other lag-domain variants walk every run of every row
    RL = moment_walk_layout(N)[0]
    all_runs = (B + 1) * M * (N // RL)
    walked_runs = kf.scv_walk_runs([ds], vechL) if variant >= 5 else all_runs
    flops = (walked_runs * flops_per_run(N, d) if variant >= 3
             else algorithmic_flops_per_candidate(M, N, d, variant) * B)
    achieved = flops / (scv_ms * 1e-3)
    spec_flops = algorithmic_flops_per_candidate(M, N, d, spec_variant) * B
    traffic = None
    prof = os.path.join(ROOT, "profiles", "scv_rows_case4_counters.json")
    if os.path.exists(prof):
        with open(prof) as fh:
            rec = json.load(fh)
        # counters are kept per launch configuration (variant, grid) and only
        # for the row-kernel sources they were taken on
        if rec.get("row_kernel_hash") == row_kernel_hash():
            ent = rec.get("launches", {}).get(f"{variant},{grid_blocks}")
            if ent:
                traffic = ent["hbm_bytes_per_launch"]
    kname = (f"k_lag_mom<2,{N},ScvFun<2,1>,256,{RL},{'true' if variant in (4, 6) else 'false'},"
             f"{'true' if variant >= 5 else 'false'}> variant {variant}"
             if variant >= 3 else f"k_rows<2,{N},ScvFun<2,1>> variant {variant}")
    kname += " (grid: one block per work item)" if grid_blocks < 0 else " (grid: resident blocks)"
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VECTOR / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR, "traffic": traffic,
                "kernel": kname, "launch_ms": scv_ms, "call_ms": scv_call_ms,
                "flops_per_launch": flops, "variant": variant,
                "walk": {"runs_walked": walked_runs, "runs_all": all_runs, "lags_per_run": RL,
                         "flops_per_run": flops_per_run(N, d)},
                "direct_evaluation_equivalent": {
                    "flops_per_launch": direct_equivalent_flops_per_candidate(M, d) * B,
                    "rate_tflops": direct_equivalent_flops_per_candidate(M, d) * B / (scv_ms * 1e-3) / 1e12}}
    fft_route = {"kernel": f"k_rows<2,512,ScvFun<2,1>> variant {spec_variant} (per-candidate last-axis FFTs in LDS)",
                 "launch_ms": spec_ms, "evals_per_s": B / (spec_ms * 1e-3), "flops_per_launch": spec_flops,
                 "achieved_tflops": spec_flops / (spec_ms * 1e-3) / 1e12,
                 "frac": spec_flops / (spec_ms * 1e-3) / PEAK_FP64_VECTOR}

    crit_out = criteria_section(kf, torch, ds, vechL, Gpsi, n, B)
    fftl_out = fftl_section(kf, torch, dev, X, Gpsi, g)
    fft_stage = fft_stage_section(kf, torch, dev, stream, tune=not a.no_tune)

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(X_h, Gp, H, M, a.cpu_h)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "SCV objective+gradient evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": sec_per_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "case4: d=2 n=1e5 4-comp mixture, M=256 (P=512), psi_4 at pilot + SCV obj+grad "
                               "for 256 H per step (binning and count transform included)",
                   "d": d, "n": n, "M": M, "P": int(g.P[d - 1]), "candidates": B, "psi_r": 4},
        "step_timing": {"timed": "graph replays" if graph_info else "eager steps", "eager": eager,
                        "graph": graph_info,
                        "kernel_times_from": "eager timed steps (library HIP events around each row-kernel launch)"},
        "roofline": roofline,
        "fft_route_batched": fft_route,
        "fft_stage": fft_stage,
        "cpu_baseline": cpu,
        "row_kernels_in_timed_steps_ms": {"scv_objgrad_256": scv_ms, "psi4": float(np.mean(psi_k)),
                                          "scv_call_with_setup_final": scv_call_ms},
        "binning": binning,
        "components_ms": {"dataset_prepare": t_prep * 1e3, "psi4_batched": t_psi_batched * 1e3,
                          "scv_objgrad_batched_256": t_scv_only * 1e3, "scv_autograd_fwd_adjoint_256": t_autograd * 1e3,
                          "psi4_plain_with_binning": t_psi_plain * 1e3, "scv_plain_per_H": t_plain * 1e3,
                          "scv_plain_per_H_with_binning": t_plain_prep * 1e3},
        "psi4_evals_per_s": {"batched_on_prepared": 1.0 / t_psi_batched, "plain_with_binning": 1.0 / t_psi_plain},
        "scv_evals_per_s": {"step": value, "batched_only": B / t_scv_only, "autograd_fwd_adjoint": B / t_autograd,
                            "plain": 1.0 / t_plain, "plain_with_binning": 1.0 / t_plain_prep},
        "batched_over_plain": {"step_vs_plain": value * t_plain,
                               "batched_vs_plain": (B / t_scv_only) * t_plain,
                               "autograd_vs_plain": (B / t_autograd) * t_plain,
                               "step_vs_plain_with_binning": value * t_plain_prep},
        "criteria_256": crit_out,
        "fftl": fftl_out,
        "tuned": tuned,
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(out))


def _kernel_and_call(kf, torch, fn, reps=10):
    """(mean row-kernel ms from the library's HIP events, mean wall ms per call)."""
    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    kf.timing_start(4 * reps)
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps * 1e3
    recs = kf.timing_stop()
    kern = float(np.mean([ms for ms, _, _ in recs])) if recs else None
    return kern, wall


def criteria_section(kf, torch, ds, vechL, Gpsi, n, B):
    """The other criteria on the same prepared case-4 dataset and candidates:
    LSCV (paper's objective) with gradient, LSCV_4 and Q_4 (scalar eta_r
    kernels), and PI (psi_4 at the psi pilot + closed-form contraction)."""
    out = {}
    for name, fn in (
        ("lscv_objgrad", lambda: kf.crit([ds], vechL, "lscv", 0)),
        ("lscv_exact_objgrad", lambda: kf.crit([ds], vechL, "lscv_exact", 0)),
        ("lscv4_obj", lambda: kf.crit([ds], vechL, "lscv", 4, grad=False)),
        ("qr4", lambda: kf.crit([ds], vechL, "qr", 4, grad=False)),
        ("qr8", lambda: kf.crit([ds], vechL, "qr", 8, grad=False)),
    ):
        kern, wall = _kernel_and_call(kf, torch, fn)
        out[name] = {"row_kernel_ms": kern, "call_ms": wall, "evals_per_s": B / (wall * 1e-3)}

    def pi_step():
        p4 = kf.psi_batch([ds], [Gpsi], 4)
        return kf.pi(p4, [n], vechL)
    kern, wall = _kernel_and_call(kf, torch, pi_step)
    out["pi_objgrad_with_psi4"] = {"psi4_row_kernel_ms": kern, "call_ms": wall, "evals_per_s": B / (wall * 1e-3)}
    return out


def fftl_section(kf, torch, dev, X, Gpsi, g):
    """The paper's fft-L variant against the full-support plain route (fft-M),
    binning included as in the paper's timing: its speed-experiment shape
    (d = 2, N(0, I), n = 4000, M = 160, psi_0) and the case-2 shape (psi_4)."""
    rng = np.random.default_rng(151107482 + 60)
    Xs = rng.standard_normal((4000, 2))
    Gs = 4000 ** (-2.0 / 6.0) * np.cov(Xs.T)
    Xt = torch.from_numpy(Xs).to(dev)
    gs = kf.grid_auto(Xt, Gs, 160)
    res = {}
    for label, XX, G, gg, r in (("paper_shape_n4000_M160_psi0", Xt, Gs, gs, 0), ("case2_shape_psi4", X, Gpsi, g, 4)):
        def full():
            return kf.psi(XX, G, r, grid=gg, mode="plain")

        def trunc():
            return kf.psi_fftl(XX, G, r, grid=gg)
        t = {}
        for nm, fn in (("fft_M_ms", full), ("fft_L_ms", trunc)):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(5):
                fn()
            torch.cuda.synchronize()
            t[nm] = (time.perf_counter() - t0) / 5 * 1e3
        vf = full().cpu().numpy()
        vt, L, P = trunc()
        vt = vt.cpu().numpy()
        t.update({"L": L, "P_fft_L": P, "P_fft_M": [int(p) for p in gg.P[:gg.d]],
                  "max_rel_diff": float(np.max(np.abs(vt - vf) / np.abs(vf))),
                  "max_diff_over_max_abs": float(np.max(np.abs(vt - vf)) / np.max(np.abs(vf)))})
        res[label] = t
    return res


def fft_stage_bytes(P, M, d):
    """Algorithmic HBM bytes of one dataset's count transform as the passes are
    built (d >= 2, f = M/P the live fraction of a leading axis): the last-axis
    R2C reads the int64 counts (prod M) and writes the rows of the half
    spectrum that can be nonzero (a fraction f^(d-1) of its 16 L Q bytes, L =
    prod of the leading P, Q = P/2 + 1); the forward pass along axis a
    (a = d-2..1) reads the fraction f^(a+1) of it and writes f^a; the axis-0
    pass reads f and writes C and the mixed spectrum |C|^2 transformed forward;
    axes 1..d-2 of the mixed spectrum read and write it; the last-axis C2R
    reads it and writes the real lag array (8 prod P)."""
    half = 16 * P ** (d - 1) * (P // 2 + 1)
    f = M / P
    fwd = f ** (d - 1) + sum(f ** (a + 1) + f ** a for a in range(1, d - 1)) + f + 2
    return int(round(8 * M ** d + 8 * P ** d + half * (fwd + 2 * (d - 2) + 1)))


def fft_stage_section(kf, torch, dev, stream, tune=True):
    """The count transform alone at the case-5 dataset shape (d=4, M=32,
    P=64: 418 MB touched per transform) over 4 datasets back to back (1.7 GB
    cycled, well above the 256 MB last-level cache), under the FFT schedule
    the tuner picks for that shape (kdefft_autotune on the first dataset, as
    the case-5 line does): algorithmic bytes per transform over the HIP-event
    time per transform."""
    import synth
    w = synth.case5(n_datasets=4, B=1, n_lo=200_000, n_hi=200_000)
    dss = [kf.Dataset(torch.from_numpy(X).to(dev), Gp, M=w.M) for X, Gp in zip(w.X, w.G_pilot)]
    d, M, P = w.d, w.M, int(dss[0].shape_grid.P[0])
    if tune:
        kf.autotune(dss[0])
    for ds in dss:
        ds.transform()
    torch.cuda.synchronize()
    reps = 3
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        for ds in dss:
            ds.transform()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / (reps * len(dss))
    nbytes = fft_stage_bytes(P, M, d)
    half = 16 * P ** (d - 1) * (P // 2 + 1)
    touched = 8 * M ** d + 2 * half + 8 * P ** d
    return {"workload": f"count transform of {len(dss)} case-5-shaped datasets back to back (d={d}, M={M}, "
                        f"P={P}), re-run from their counts",
            "bytes_per_transform": nbytes, "ms_per_transform": ms,
            "achieved_GBps": nbytes / (ms * 1e-3) / 1e9, "peak_GBps": 8000.0,
            "frac": nbytes / (ms * 1e-3) / 8e12, "touched_bytes_per_dataset": touched,
            "cycled_bytes": touched * len(dss), "schedule": kf.get_fft_schedule([P] * d),
            "schedule_from": "kdefft_autotune" if tune else "untuned default"}


def main_case5(a):
    import torch
    import paper_1511_07482_amd as kf
    import synth
    dev = torch.device("cuda:0")
    w = synth.case5()
    d, M = w.d, w.M
    Xs = [torch.from_numpy(X).to(dev) for X in w.X]
    ns = [X.shape[0] for X in w.X]
    per = [H.shape[0] for H in w.H]
    B = sum(per)
    vech = torch.from_numpy(np.concatenate([synth.vech_chol(H) for H in w.H])).to(dev)
    torch.cuda.synchronize()

    def prepare():
        return [kf.Dataset(X, Gp, M=M) for X, Gp in zip(Xs, w.G_pilot)]

    dss = prepare()
    tuned = None if a.no_tune else kf.autotune(dss[0])
    stream = torch.cuda.current_stream(dev)

    def ev_time(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            out = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, out

    t_prep, dss = ev_time(prepare, 2)
    t_psi, _ = ev_time(lambda: kf.psi_batch(dss, w.G_psi, 4), 3)
    t_scv, (obj, grad) = ev_time(lambda: kf.scv(dss, vech, per_ds=per), 3)
    assert torch.isfinite(obj).all() and torch.isfinite(grad).all()
    # the lag kernel of the SCV launch alone (library HIP events), against the
    # walk's algorithmic flops over every run (all runs of these grids are above
    # the 1e-290 cut, so the kernel walks each one)
    kf.timing_start(16)
    for _ in range(3):
        kf.scv(dss, vech, per_ds=per)
    torch.cuda.synchronize()
    lag_ms = float(np.mean([ms for ms, fam, r in kf.timing_stop() if fam == kf.FUN_SCV_OBJGRAD]))
    variant = 4
    for line in (tuned or "").splitlines():
        if line.startswith("best: variant"):
            variant = int(line.split()[2])
    P_last = int(dss[0].grid.P[d - 1])
    roofline = None
    if variant >= 3:
        rows = M * (2 * M - 1) ** (d - 2)
        if variant >= 5:   # the compacted walk: the runs it visits, counted on the device
            flops = kf.scv_walk_runs(dss, vech, per_ds=per) * flops_per_run(P_last, d)
        else:
            flops = B * algorithmic_flops_per_candidate(M, P_last, d=d, variant=variant, rows=rows)
        roofline = {"bound": "alu", "kernel": f"k_lag_mom<{d},{P_last},ScvFun<{d},1>> variant {variant}",
                    "launch_ms": lag_ms, "flops_per_launch": flops, "achieved": flops / (lag_ms * 1e-3) / 1e12,
                    "peak": 78.6, "unit": "TFLOP/s", "frac": flops / (lag_ms * 1e-3) / 1e12 / 78.6}
    # one large dataset: binning alone vs full preparation -> count-transform time
    big = int(np.argmax(ns))
    gbig = dss[big].grid
    t_bin, _ = ev_time(lambda: kf.linbin(Xs[big], gbig), 3)
    t_prep1, _ = ev_time(lambda: kf.Dataset(Xs[big], w.G_pilot[big], grid=gbig), 3)
    P = int(gbig.P[0])
    if a.calib_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    out = {"metric": "case5 (extra line): d=4, 32 datasets n~U[1e4,1e6], M=32 (P=64), 64 H each",
           "n_total": int(sum(ns)), "candidates": B,
           "prepare_all_ms": t_prep, "psi4_batch_ms": t_psi, "scv_objgrad_batch_ms": t_scv,
           "scv_evals_per_s": B / (t_scv * 1e-3), "psi4_evals_per_s": len(dss) / (t_psi * 1e-3),
           "largest_n": ns[big], "linbin_largest_ms": t_bin, "prepare_largest_ms": t_prep1,
           "fft_stage_bytes_per_dataset": fft_stage_bytes(P, M, d), "scv_roofline": roofline, "tuned": tuned}
    print(json.dumps(out))


def cpu_model():
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_CPU = {}   # oracle inputs shared with the forked workers


def _cpu_candidate(b):
    from threadpoolctl import threadpool_limits
    from oracle import scv
    A, n, g, H, Gp = _CPU["args"]
    with threadpool_limits(limits=1):
        scv.objective_binned(A, n, g, H[b], Gp)
    return b


def cpu_baseline(X, Gp, H, M, nh):
    """The oracle's binned SCV (objective + gradient) on the host: counts and
    their direct autocorrelation once (one process), then nh candidates spread
    over one worker process per core of this process's affinity set (BLAS
    threads = 1 each); evals/s over the whole sample (autocorrelation included)."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    from oracle import binned, grid, linbin, scv
    cores = len(os.sched_getaffinity(0))
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        g = grid.plan_auto(X, Gp, [M, M])
        counts, _ = linbin.linbin(X, g)
        A = binned.autocorr_direct(linbin.counts_to_real(counts))
        t_a = time.perf_counter() - t0
    nh = min(nh, H.shape[0])
    _CPU["args"] = (A, X.shape[0], g, H, Gp)
    t1 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        done = pool.map(_cpu_candidate, range(nh), chunksize=1)
    t_h = time.perf_counter() - t1
    assert sorted(done) == list(range(nh))
    # the unbinned double sum (the direct method the paper compares against) on
    # a fixed subsample, its row blocks over the same workers, extrapolated to n by n^2
    n_sub = 6000
    sub = X[np.random.default_rng(151107482).choice(X.shape[0], n_sub, replace=False)]
    t2 = time.perf_counter()
    with threadpool_limits(limits=1):
        scv.objective_direct(sub, H[0], Gp, workers=cores, with_grad=True)
    t_d = (time.perf_counter() - t2) * (X.shape[0] / n_sub) ** 2
    return {"value": nh / (t_a + t_h), "unit": "SCV objective+gradient evals/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"case4 data: binning + direct autocorrelation of the 256^2 counts in one process "
                      f"({t_a:.1f} s), then {nh} of the 256 candidates over {cores} worker processes "
                      f"({t_h:.1f} s wall)",
            "per_candidate_core_s": t_h * cores / nh, "autocorrelation_s": t_a,
            "direct_unbinned": {"per_candidate_s_extrapolated": t_d, "evals_per_s_extrapolated": 1.0 / t_d,
                                "sample": f"unbinned O(n^2) objective+gradient of one candidate on a {n_sub}-point "
                                          f"subsample, row blocks over {cores} workers, scaled by (n/{n_sub})^2"}}


if __name__ == "__main__":
    main()
