"""The benchmark's work model (CPU): the algorithmic flop and byte counts that
the roofline figures divide by, pinned to hand counts of the same formulas."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_walk_flops_case4():
    # d = 2, N = 512: runs of 16 lags in segments of 2 runs; per run
    # 16 * (2 * 8 + 1) walk flops, 3 + 25 * 3 fold flops, z advance 4d / 2,
    # and a fresh start per segment: 2 * (2 d^2 + 2 d + 4 + 2 * 20) / 2
    assert bench.moment_walk_layout(512) == (16, 2)
    per_run = 16 * 17 + (3 + 75) + 8 / 2 + 2 * (8 + 4 + 4 + 40) / 2
    assert per_run == 410.0
    per_cand = bench.algorithmic_flops_per_candidate(256, 512, d=2, variant=3)
    assert per_cand == 256 * 32 * per_run
    assert per_cand * 256 == 859_832_320


def test_direct_equivalent_flops_case4():
    # generation at a lag: 2 * (2 d^2 + 2 d + 2 + 20) + 2 + 7 * 3 = 91 at d = 2,
    # plus 2 flops for each of the 4 grids' sums: 99 per lag
    assert bench.gen_flops_per_lag(2) == 2 * (8 + 4 + 2 + 20) + 2 + 21 == 91
    assert bench.direct_equivalent_flops_per_candidate(256, 2) == 256 * 511 * (91 + 8)
    assert bench.direct_equivalent_flops_per_candidate(256, 2) * 256 == 3_315_400_704


@pytest.mark.parametrize("N,layout", [(4, (2, 1, 128)), (8, (4, 1, 128)), (64, (8, 1, 32)), (128, (8, 1, 16)),
                                      (256, (16, 2, 32)), (512, (16, 2, 16)), (1024, (16, 2, 8))])
def test_walk_layout(N, layout):
    """The compiled layout the model reads from the library (runs of up to 8
    lags below N = 256, runs of 16 in segments of 2 from there; a 256-thread
    block covers 256 * run * seg / N rows per pass)."""
    assert bench.moment_walk_layout(N) == layout[:2]
    import paper_1511_07482_amd as kf
    assert kf.lag_layout(N, True) == layout
    assert layout[2] == 256 * layout[0] * layout[1] // N


def test_lag_layout_rejects_bad_length():
    import paper_1511_07482_amd as kf
    for N in (2, 3, 96, 4096):
        with pytest.raises(RuntimeError):
            kf.lag_layout(N)


def test_fft_stage_bytes():
    # case 5 (M = 32, P = 64, d = 4): int64 counts 8 M^4 read by the R2C pass,
    # half spectrum 16 P^3 (P/2 + 1), real lag array 8 P^4 written by the C2R
    # pass.  The counts fill [0, 32)^4 of the 64^4 grid, so the forward passes
    # touch only the part that can be nonzero: R2C writes the rows with all
    # three leading indices < 32 (1/8 of half); the axis-2 pass reads those
    # (1/8) and writes columns with i0, i1 < 32 (1/4); axis 1 reads 1/4 and
    # writes 1/2; axis 0 reads 1/2 and writes C and the mixed spectrum (2 half);
    # axes 1, 2 of the mixed spectrum are dense (2 half each); C2R reads half.
    counts, real, half = 8 * 32 ** 4, 8 * 64 ** 4, 16 * 64 ** 3 * 33
    want = (counts + half // 8) + (half // 8 + half // 4) + (half // 4 + half // 2) + (half // 2 + 2 * half) \
        + 2 * 2 * half + (half + real)
    assert bench.fft_stage_bytes(64, 32, 4) == want == 1_353_711_616
    # d = 2 (M = 256, P = 512): R2C writes half the rows, axis 0 reads them
    counts, real, half = 8 * 256 ** 2, 8 * 512 ** 2, 16 * 512 * 257
    assert bench.fft_stage_bytes(512, 256, 2) == (counts + half // 2) + (half // 2 + 2 * half) + (half + real)