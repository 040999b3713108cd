// Compile-time instantiation of the batched row kernels for one dimension D.
// Included once per dimension (and per kernel family group) so the many
// template instances compile in parallel translation units.
#pragma once

#include "rows_impl.h"

namespace kdefft {

template <int N, class Fun>
constexpr bool rows_fits() {
    return ((Fun::NG + 1) / 2) * N * 16 <= 61440;
}

template <int D, int N, class Fun>
hipError_t rows_var(int var, const double* prm, RowGeom geo, int64_t nitems, double* partial, int grid_blocks,
                    const double2* tw, hipStream_t s) {
    if constexpr (!rows_fits<N, Fun>()) {
        return hipErrorInvalidValue;
    } else {
        switch (var) {
            case 0: return run_rows_t<D, N, Fun, 0>(prm, geo, nitems, partial, grid_blocks, tw, s);
            case 1: return run_rows_t<D, N, Fun, 1>(prm, geo, nitems, partial, grid_blocks, tw, s);
            case 2: return run_rows_t<D, N, Fun, 2>(prm, geo, nitems, partial, grid_blocks, tw, s);
            case 3:
            case 4:
            case 5:
            case 6: return run_lag_t<D, N, Fun>(prm, geo, nitems, partial, grid_blocks, s, var);
            default: return hipErrorInvalidValue;
        }
    }
}

// Rows one block transforms per pass (rows per wavefront x wavefronts).
template <int D, int N, class Fun>
constexpr int rows_per_iter_t(int var) {
    return var >= 3 ? (HasMoments<Fun>::value ? mom_rows_per_pass<N>() : lag_rows_per_pass<N>()) : var == 1 ? rows_for<N, Fun::NG, 1>() * waves_for<N, Fun::NG, rows_for<N, Fun::NG, 1>()>()
                    : rows_for<N, Fun::NG, 0>() * waves_for<N, Fun::NG, rows_for<N, Fun::NG, 0>()>();
}

}  // namespace kdefft
