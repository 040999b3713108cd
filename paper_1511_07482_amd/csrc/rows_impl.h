// Batched evaluation of binned double sums by the FFT route in Parseval form.
//
// For a real, centrally symmetric kernel grid k on the circular P^d layout and
// the count spectrum C = R2C(c_zp), the paper's steps 3-4 (Eq. (22)-(24)) give
//     sum_i c_i (c * k)_i = (prod P)^-1 sum_w |C(w)|^2 K(w),   K = DFT(k).
// Moving the DFT along the leading axes 0..d-2 onto |C|^2 (done once per
// dataset, giving the mixed spectrum What(l', w_last)), each kernel grid only
// needs its last-axis DFT, row by row:
//     sum_w |C|^2 K = sum_{l'} sum_{w_last} What(l', w_last) DFT_last(k)(l', w_last).
// Rows l' and -l' contribute equally (k(-l) = k(l)), so only rows with
// l_0 >= 0 are formed, the others counted twice, and rows that fall in the
// zero slots of the layout are skipped.  Two real grids share one complex
// transform: with Z = DFT(k_a + i k_b), sum_w What Z over the full last axis
// has real part = grid a's sum and imaginary part = grid b's sum.
//
// One work item = one candidate bandwidth x one chunk of rows.  A block
// generates ROWS rows of all NG grids in LDS, transforms them, contracts with
// the What rows (read once for all grids) and keeps NG running sums in
// registers.  Blocks loop over items (persistent grid); per-item partial sums
// are written out and summed later in a fixed order.
#pragma once

#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "dev_kernels.h"
#include "internal.h"

namespace kdefft {

template <int D, int N, class Fun, int ROWS, int NT, int SCHED>
__global__ __launch_bounds__(NT) void k_rows(const double* __restrict__ prm, RowGeom geo, int64_t nitems,
                                             double* __restrict__ partial, const double2* __restrict__ tw) {
    constexpr int NG = Fun::NG;
    constexpr int NPEN = (NG + 1) / 2;
    constexpr int NPT = ROWS * NPEN;
    constexpr int PS = N + 1;
    constexpr int Q = N / 2 + 1;
    __shared__ double2 pen[NPT * PS];
    __shared__ double red[(NT / 64) * NG];
    __shared__ double xlead[ROWS][4];
    __shared__ int64_t wrow_s[ROWS];
    __shared__ double rw_s[ROWS];

    for (int64_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int64_t h = item / geo.nchunks;
        const int64_t ch = item - h * geo.nchunks;
        const double* pr = prm + h * PRM;
        Fun f;
        f.load(pr);
        double delta[D];
#pragma unroll
        for (int k = 0; k < D; ++k) delta[k] = pr[S_DELTA + k];
        const double2* __restrict__ W =
            reinterpret_cast<const double2*>(static_cast<uintptr_t>(__double_as_longlong(pr[S_WMIX])));
        double acc[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) acc[g] = 0.0;
        const int64_t rbeg = ch * geo.chunk;
        const int64_t rend = rbeg + geo.chunk < geo.nrows ? rbeg + geo.chunk : geo.nrows;

        for (int64_t r0 = rbeg; r0 < rend; r0 += ROWS) {
            // row decode: lead lags, What row index, weight (rows with l_0 > 0 stand
            // for their mirror images too)
            if (threadIdx.x < ROWS) {
                const int rr = threadIdx.x;
                int64_t rem = r0 + rr;
                int64_t wr = 0;
                double w = 0.0;
                if (r0 + rr < rend) {
                    if constexpr (D == 1) {
                        w = 1.0;
                    } else {
                        int lag[4] = {0, 0, 0, 0};
#pragma unroll
                        for (int k = D - 2; k >= 1; --k) {
                            const int64_t E = 2 * geo.M[k] - 1;
                            const int64_t c = rem % E;
                            rem /= E;
                            lag[k] = (int)c - (geo.M[k] - 1);
                        }
                        lag[0] = (int)rem;
#pragma unroll
                        for (int k = 0; k < D - 1; ++k) {
                            const int idx = lag[k] >= 0 ? lag[k] : lag[k] + geo.P[k];
                            wr = wr * geo.P[k] + idx;
                            xlead[rr][k] = delta[k] * (double)lag[k];
                        }
                        w = lag[0] == 0 ? 1.0 : 2.0;
                    }
                }
                wrow_s[rr] = wr;
                rw_s[rr] = w;
            }
            __syncthreads();
            // generation of ROWS rows x NG grids, packed two grids per pencil
            for (int e = threadIdx.x; e < ROWS * N; e += NT) {
                const int rr = e / N, p = e - rr * N;
                double vals[NG];
                int lag = 0;
                const bool nz = rw_s[rr] != 0.0 && lag_of(p, geo.M[D - 1], N, &lag);
                if (nz) {
                    double x[D];
#pragma unroll
                    for (int k = 0; k < D - 1; ++k) x[k] = xlead[rr][k];
                    x[D - 1] = delta[D - 1] * (double)lag;
                    f.eval(x, vals);
                } else {
#pragma unroll
                    for (int g = 0; g < NG; ++g) vals[g] = 0.0;
                }
#pragma unroll
                for (int gp = 0; gp < NPEN; ++gp)
                    pen[(rr * NPEN + gp) * PS + p] =
                        make_double2(vals[2 * gp], (2 * gp + 1 < NG) ? vals[2 * gp + 1] : 0.0);
            }
            __syncthreads();
            fft_lds<N, NPT, NT, -1, SCHED>(pen, PS, tw);
            // contraction with the mixed spectrum over the full last axis
            for (int e = threadIdx.x; e < ROWS * Q; e += NT) {
                const int rr = e / Q, w = e - rr * Q;
                const double rw = rw_s[rr];
                if (rw == 0.0) continue;
                const double2 Wv = W[wrow_s[rr] * Q + w];
                const bool two = (w != 0) && (w != N / 2);
                const double2 Wc = two ? c_conj(Wv) : make_double2(0.0, 0.0);
#pragma unroll
                for (int gp = 0; gp < NPEN; ++gp) {
                    const double2* pp = pen + (rr * NPEN + gp) * PS;
                    double2 cz = c_mul(Wv, pp[w]);
                    if (two) cz = c_add(cz, c_mul(Wc, pp[N - w]));
                    acc[2 * gp] += rw * cz.x;
                    if (2 * gp + 1 < NG) acc[2 * gp + 1] += rw * cz.y;
                }
            }
            __syncthreads();
        }
        double outv[NG];
        block_sum<NG, NT>(acc, red, outv);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int g = 0; g < NG; ++g) partial[item * NG + g] = outv[g];
        }
    }
}

// Rows per block iteration: about 32 KiB of pencils (variant 0/2) or 64 KiB (1).
template <int N, int NG, int VAR>
constexpr int rows_for() {
    constexpr int npen = (NG + 1) / 2;
    constexpr int bytes = (VAR == 1 ? 65536 : 32768) - 2048;
    constexpr int r = bytes / (npen * (N + 1) * 16);
    return r >= 16 ? 16 : (r >= 8 ? 8 : (r >= 4 ? 4 : (r >= 2 ? 2 : 1)));
}

// Persistent grid: grid_blocks > 0 as given, 0 = resident blocks per CU x CUs,
// -1 = one block per work item.
template <int D, int N, class Fun, int VAR>
hipError_t run_rows_t(const double* prm, RowGeom geo, int64_t nitems, double* partial, int grid_blocks,
                      const double2* tw, hipStream_t s) {
    constexpr int ROWS = rows_for<N, Fun::NG, VAR>();
    constexpr int SCHED = VAR == 2 ? 1 : 0;
    auto kern = k_rows<D, N, Fun, ROWS, 256, SCHED>;
    int64_t blocks = nitems;
    if (grid_blocks > 0) {
        blocks = grid_blocks;
    } else if (grid_blocks == 0) {
        static int resident = -1;  // per instantiation, per process
        if (resident < 0) {
            int per_cu = 0, dev = 0, cus = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0) != hipSuccess) per_cu = 1;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
                cus = 256;
            resident = (per_cu < 1 ? 1 : per_cu) * cus;
        }
        blocks = resident;
    }
    if (blocks > nitems) blocks = nitems;
    if (blocks < 1) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, s, prm, geo, nitems, partial, tw);
    return hipGetLastError();
}

template <int N, class Fun, int VAR>
constexpr int rows_of() { return rows_for<N, Fun::NG, VAR>(); }

}  // namespace kdefft
