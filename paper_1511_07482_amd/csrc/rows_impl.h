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
// has real part = grid a's sum and imaginary part = grid b's sum (What is
// conjugate-symmetric along the last axis).
//
// Work decomposition: one work item = one candidate bandwidth x one chunk of
// rows; a block of WPB wavefronts takes items in a persistent loop, and each
// wavefront transforms its own rows (RPW at a time) in a private LDS region,
// synchronising only at wavefront scope.  The first radix stage is fused with
// the kernel-grid generation (values go from registers straight into the
// butterfly) when the registers allow it, and the last stage is fused with
// the contraction against What (its outputs are never written back).  Each
// lane keeps NG running sums; a block reduction at the end of an item writes
// the item's partial sums, which a later kernel adds in a fixed order.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "dev_common.h"
#include "dev_kernels.h"
#include "finish.h"
#include "internal.h"
#include "params.h"

namespace kdefft {

// LDS written and read by the same wavefront: order the accesses without a
// block-wide barrier.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A value that is the same in every lane (read from LDS at a uniform address),
// moved to scalar registers so that it takes no vector register.
__device__ __forceinline__ double wave_uniform(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Position of element e of a pencil in LDS: the low four index bits are XORed
// with a function of the next bits, so that 16 consecutive lanes hit 16
// different 16-byte bank groups for contiguous reads, stride-8 writes (first
// radix-8 stage) and the grouped writes of later stages alike.
__device__ __forceinline__ constexpr int swz(int e) {
    return e ^ (((e >> 4) & 7) | (((e >> 4) & 4) << 1));
}

template <int N, int SCHED>
constexpr int last_L() {
    int L = 1;
    while (L * next_radix(N / L, SCHED) < N) L *= next_radix(N / L, SCHED);
    return L;
}

// Middle Stockham stages [L, LEND) of NPW pencils, executed by one wavefront.
// Butterflies are taken in groups that cover whole pencils (one pencil, or
// several short ones, per group), each group read, transformed and written
// back before the next, so only one group's values are live in registers.
template <int N, int L, int LEND, int NPW, int SCHED>
__device__ __forceinline__ void wave_mid_stages(double2* buf, int lane, const double2* __restrict__ tw) {
    if constexpr (L < LEND) {
        constexpr int R = next_radix(N / L, SCHED);
        constexpr int NB = N / R;
        constexpr int TOT = NB * NPW;
        constexpr int PER = (TOT + 63) / 64;
        constexpr int G = NB >= 64 ? NB / 64 : 1;     // butterfly sets per group
        constexpr int NGRP = (PER + G - 1) / G;
        constexpr int TWS = TWN / (R * L);
#pragma unroll 1
        for (int grp = 0; grp < NGRP; ++grp) {
            double2 v[G][R];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int b = lane + (grp * G + g) * 64;
                if ((TOT % 64) == 0 || b < TOT) {
                    const int p = b / NB, i = b - p * NB;
                    const int k = i & (L - 1);
                    const double2* src = buf + p * N;
#pragma unroll
                    for (int m = 0; m < R; ++m) v[g][m] = src[swz(i + m * NB)];
#pragma unroll
                    for (int m = 1; m < R; ++m) v[g][m] = c_mul(v[g][m], tw[m * k * TWS]);
                    dft<R, -1>(v[g]);
                }
            }
            wave_sync();
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int b = lane + (grp * G + g) * 64;
                if ((TOT % 64) == 0 || b < TOT) {
                    const int p = b / NB, i = b - p * NB;
                    const int k = i & (L - 1);
                    double2* dst = buf + p * N;
                    const int base = (i - k) * R + k;
#pragma unroll
                    for (int m = 0; m < R; ++m) dst[swz(base + m * L)] = v[g][m];
                }
            }
            wave_sync();
        }
        wave_mid_stages<N, L * R, LEND, NPW, SCHED>(buf, lane, tw);
    }
}

struct RowInfo {
    double x[4];      // lead lag coordinates
    const double2* w;  // What row
    int64_t wr;       // flat index of the row over the leading axes
    double rw;        // row weight (0 = no row)
};

template <int D>
__device__ __forceinline__ RowInfo row_info(int64_t row, int64_t rend, const RowGeom& geo, const double* delta,
                                            const double2* W) {
    RowInfo ri;
    ri.x[0] = ri.x[1] = ri.x[2] = ri.x[3] = 0.0;
    ri.w = W;
    ri.wr = 0;
    ri.rw = 0.0;
    if (row >= rend) return ri;
    if constexpr (D == 1) {
        ri.rw = 1.0;
    } else {
        int rem = (int)row;  // rows < 2^31 for every supported grid
        int lag[4] = {0, 0, 0, 0};
#pragma unroll
        for (int k = D - 2; k >= 1; --k) {
            const int E = 2 * geo.M[k] - 1;
            const int c = rem % E;
            rem /= E;
            lag[k] = c - (geo.M[k] - 1);
        }
        lag[0] = rem;
        int64_t wr = 0;
#pragma unroll
        for (int k = 0; k < D - 1; ++k) {
            const int idx = lag[k] >= 0 ? lag[k] : lag[k] + geo.P[k];
            wr = wr * geo.P[k] + idx;
            ri.x[k] = delta[k] * (double)lag[k];
        }
        ri.w = W + wr * geo.Q;
        ri.wr = wr;
        ri.rw = lag[0] == 0 ? 1.0 : 2.0;
    }
    return ri;
}

// Kernel values of all NG grids at last-axis index p of a row.
template <int D, int N, class Fun>
__device__ __forceinline__ void gen_point(const Fun& f, const RowInfo& ri, int p, int M_last, const double* delta,
                                          double* vals) {
    int lag = 0;
    if (ri.rw != 0.0 && lag_of(p, M_last, N, &lag)) {
        double x[D];
#pragma unroll
        for (int k = 0; k < D - 1; ++k) x[k] = ri.x[k];
        x[D - 1] = delta[D - 1] * (double)lag;
        f.eval(x, vals);
    } else {
#pragma unroll
        for (int g = 0; g < Fun::NG; ++g) vals[g] = 0.0;
    }
}

template <int D, int N, class Fun, int RPW, int WPB, int SCHED>
__global__ __launch_bounds__(WPB * 64) void k_rows(const double* __restrict__ prm, RowGeom geo, int64_t nitems,
                                                   double* __restrict__ partial, const double2* __restrict__ tw) {
    constexpr int NG = Fun::NG;
    constexpr int NPEN = (NG + 1) / 2;
    constexpr int NPW = RPW * NPEN;
    constexpr int PS = N;
    constexpr int R1 = next_radix(N, SCHED);
    constexpr int NB1 = N / R1;
    constexpr bool FUSE1 = NPEN * R1 <= 16;
    constexpr int LL = last_L<N, SCHED>();
    constexpr int RL = N / LL;
    constexpr bool ONE_STAGE = (R1 == N);
    __shared__ double2 pen_all[WPB * NPW * PS];
    __shared__ double red[WPB * NG];
    __shared__ RowInfo rtab_all[WPB * RPW];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double2* pen = pen_all + wave * NPW * PS;
    RowInfo* rtab = rtab_all + wave * RPW;

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
        const int M_last = geo.M[D - 1];
        double acc[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) acc[g] = 0.0;
        const int64_t rbeg = ch * geo.chunk;
        const int64_t rend = rbeg + geo.chunk < geo.nrows ? rbeg + geo.chunk : geo.nrows;

        for (int64_t r0 = rbeg + wave * RPW; r0 < rend; r0 += WPB * RPW) {
            if (lane < RPW) rtab[lane] = row_info<D>(r0 + lane, rend, geo, delta, W);
            wave_sync();

            if constexpr (ONE_STAGE) {
                // whole transform in registers: generate, DFT, contract
                constexpr int TOT = RPW;
                for (int b = lane; b < TOT; b += 64) {
                    const RowInfo rinf = rtab[b];
                    if (rinf.rw == 0.0) continue;
                    double2 a[NPEN][N];
#pragma unroll
                    for (int m = 0; m < N; ++m) {
                        double vals[NG];
                        gen_point<D, N>(f, rinf, m, M_last, delta, vals);
#pragma unroll
                        for (int gp = 0; gp < NPEN; ++gp)
                            a[gp][m] = make_double2(vals[2 * gp], (2 * gp + 1 < NG) ? vals[2 * gp + 1] : 0.0);
                    }
#pragma unroll
                    for (int gp = 0; gp < NPEN; ++gp) dft<N, -1>(a[gp]);
#pragma unroll
                    for (int m = 0; m < N; ++m) {
                        const bool lo = m <= N / 2;
                        double2 wv = rinf.w[lo ? m : N - m];
                        if (!lo) wv = c_conj(wv);
#pragma unroll
                        for (int gp = 0; gp < NPEN; ++gp) {
                            const double2 cz = c_mul(wv, a[gp][m]);
                            acc[2 * gp] += rinf.rw * cz.x;
                            if (2 * gp + 1 < NG) acc[2 * gp + 1] += rinf.rw * cz.y;
                        }
                    }
                }
                wave_sync();
            } else {
                // ---- stage 1 (L = 1, no twiddles), generation fused when registers allow
                if constexpr (FUSE1) {
                    constexpr int TOT = RPW * NB1;
                    constexpr int PER = (TOT + 63) / 64;
#pragma unroll
                    for (int u = 0; u < PER; ++u) {
                        const int b = lane + u * 64;
                        if ((TOT % 64) == 0 || b < TOT) {
                            const int rr = b / NB1, i = b - rr * NB1;
                            double2 a[NPEN][R1];
#pragma unroll
                            for (int m = 0; m < R1; ++m) {
                                double vals[NG];
                                gen_point<D, N>(f, rtab[rr], i + m * NB1, M_last, delta, vals);
#pragma unroll
                                for (int gp = 0; gp < NPEN; ++gp)
                                    a[gp][m] =
                                        make_double2(vals[2 * gp], (2 * gp + 1 < NG) ? vals[2 * gp + 1] : 0.0);
                            }
#pragma unroll
                            for (int gp = 0; gp < NPEN; ++gp) {
                                dft<R1, -1>(a[gp]);
                                double2* dst = pen + (rr * NPEN + gp) * PS;
#pragma unroll
                                for (int m = 0; m < R1; ++m) dst[swz(i * R1 + m)] = a[gp][m];
                            }
                        }
                    }
                    wave_sync();
                    wave_mid_stages<N, R1, LL, NPW, SCHED>(pen, lane, tw);
                } else {
                    for (int e = lane; e < RPW * N; e += 64) {
                        const int rr = e / N, p = e - rr * N;
                        double vals[NG];
                        gen_point<D, N>(f, rtab[rr], p, M_last, delta, vals);
#pragma unroll
                        for (int gp = 0; gp < NPEN; ++gp)
                            pen[(rr * NPEN + gp) * PS + swz(p)] =
                                make_double2(vals[2 * gp], (2 * gp + 1 < NG) ? vals[2 * gp + 1] : 0.0);
                    }
                    wave_sync();
                    wave_mid_stages<N, 1, LL, NPW, SCHED>(pen, lane, tw);
                }
                // ---- last stage fused with the contraction against What
                {
                    constexpr int NB = N / RL;  // == LL
                    constexpr int TOT = RPW * NB;
                    constexpr int PER = (TOT + 63) / 64;
                    constexpr int TWS = TWN / N;
#pragma unroll
                    for (int u = 0; u < PER; ++u) {
                        const int b = lane + u * 64;
                        if ((TOT % 64) == 0 || b < TOT) {
                            const int rr = b / NB, i = b - rr * NB;
                            const RowInfo rinf = rtab[rr];
                            if (rinf.rw != 0.0) {
                                double2 wv[RL];
#pragma unroll
                                for (int m = 0; m < RL; ++m) {
                                    const int w = i + m * NB;
                                    const bool lo = w <= N / 2;
                                    wv[m] = rinf.w[lo ? w : N - w];
                                    if (!lo) wv[m] = c_conj(wv[m]);
                                }
#pragma unroll
                                for (int gp = 0; gp < NPEN; ++gp) {
                                    const double2* src = pen + (rr * NPEN + gp) * PS;
                                    double2 a[RL];
#pragma unroll
                                    for (int m = 0; m < RL; ++m) a[m] = src[swz(i + m * NB)];
#pragma unroll
                                    for (int m = 1; m < RL; ++m) a[m] = c_mul(a[m], tw[m * i * TWS]);
                                    dft<RL, -1>(a);
                                    double sre = 0.0, sim = 0.0;
#pragma unroll
                                    for (int m = 0; m < RL; ++m) {
                                        const double2 cz = c_mul(wv[m], a[m]);
                                        sre += cz.x;
                                        sim += cz.y;
                                    }
                                    acc[2 * gp] += rinf.rw * sre;
                                    if (2 * gp + 1 < NG) acc[2 * gp + 1] += rinf.rw * sim;
                                }
                            }
                        }
                    }
                }
                wave_sync();
            }
        }
        double outv[NG];
        block_sum<NG, WPB * 64>(acc, red, outv);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int g = 0; g < NG; ++g) partial[item * NG + g] = outv[g];
        }
    }
}

// Lag-domain evaluation of the same sums (variant 3): with the prepared
// count autocorrelation A (times prod P, circular layout),
//     sum_w |C|^2 K = prod P * sum_l k(l) A(l),
// so each candidate needs no transform at all.  The same half set of rows
// (l_0 >= 0, mirror rows counted twice) is used.  Each thread walks a run of
// RUN consecutive lags of one row.  Along the last axis every Gaussian's
// exponent is quadratic in the lag, so with x advancing by dl = delta_last:
//     z(l+1) = z(l) + dl S^{-1} e_last,
//     e(l+1) = e(l) rho(l),  rho(l) = exp(-(dl z_last(l) + dl^2 P_ll / 2)),
//     rho(l+1) = rho(l) sigma,  sigma = exp(-dl^2 P_ll),
// which replaces RUN exponentials per Gaussian by two (each step adds a few
// ulps of rounding).  A run whose start underflows or whose ratio is huge is
// evaluated directly instead.
template <int D, int N, class Fun, int NT, int RUN>
__global__ __launch_bounds__(NT) void k_lag(const double* __restrict__ prm, RowGeom geo, int64_t nitems,
                                            double* __restrict__ partial) {
    constexpr int NG = Fun::NG;
    constexpr int NGS = Fun::NGAUSS;
    __shared__ double red[(NT / 64) * NG];
    const int M_last = geo.M[D - 1];
    const int nrun = (2 * M_last - 1 + RUN - 1) / RUN;
    // thread t takes the (row, run) pairs t, t + NT, ... of its item in row-major
    // order; the pair is advanced incrementally (no division in the loop)
    const int step_ro = NT / nrun, step_j = NT % nrun;
    const int ro0 = (int)threadIdx.x / nrun, j0 = (int)threadIdx.x % nrun;
    for (int64_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int64_t h = item / geo.nchunks;
        const int64_t ch = item - h * geo.nchunks;
        const double* pr = prm + h * PRM;
        Fun f;
        f.load(pr);
        double delta[D];
#pragma unroll
        for (int k = 0; k < D; ++k) delta[k] = pr[S_DELTA + k];
        const double* __restrict__ A =
            reinterpret_cast<const double*>(static_cast<uintptr_t>(__double_as_longlong(pr[S_ALAG])));
        const double dl = delta[D - 1];
        double dz[NGS][D], sig[NGS], hpl[NGS], lcut[NGS];
#pragma unroll
        for (int k = 0; k < NGS; ++k) {
            const double* P = f.Pm(k);
#pragma unroll
            for (int i = 0; i < D; ++i) dz[k][i] = dl * P[i * D + D - 1];
            hpl[k] = 0.5 * dl * dl * P[(D - 1) * D + D - 1];
            sig[k] = exp(-2.0 * hpl[k]);
            lcut[k] = -667.74967696827317 - log(f.cn(k));   // c e^x < 1e-290 below
        }
        double acc[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) acc[g] = 0.0;
        const int64_t rbeg = ch * geo.chunk;
        const int64_t rend = rbeg + geo.chunk < geo.nrows ? rbeg + geo.chunk : geo.nrows;
        const int nro = (int)(rend - rbeg);   // rows of one item < 2^31
        for (int ro = ro0, j = j0; ro < nro; ro += step_ro + (j + step_j >= nrun ? 1 : 0),
                 j = j + step_j >= nrun ? j + step_j - nrun : j + step_j) {
            const RowInfo ri = row_info<D>(rbeg + ro, rend, geo, delta, nullptr);
            const double* __restrict__ Arow = A + ri.wr * N;
            const int lag0 = -(M_last - 1) + j * RUN;
            double x[D];
#pragma unroll
            for (int k = 0; k < D - 1; ++k) x[k] = ri.x[k];
            x[D - 1] = dl * (double)lag0;
            double z[NGS][D], ev[NGS], rho[NGS];
            bool direct = false, alive = false;
#pragma unroll
            for (int k = 0; k < NGS; ++k) {
                const double* P = f.Pm(k);
                double q = 0.0;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    double s = 0.0;
#pragma unroll
                    for (int jj = 0; jj < D; ++jj) s += P[i * D + jj] * x[jj];
                    z[k][i] = s;
                    q += x[i] * s;
                }
                const double ea = -0.5 * q;
                const double lr = -(dl * z[k][D - 1] + hpl[k]);
                ev[k] = f.cn(k) * exp(ea);
                rho[k] = exp(lr);
                // ratios along the run are rho, rho sig, ... with sig < 1, so the
                // exponent stays below ea + (RUN - 1) max(lr, 0): when that is
                // under the 1e-290 cut the run adds nothing a float64 sum can
                // hold next to the lag-0 term
                if (!(ev[k] >= 1e-290) && (rho[k] <= 1.0 || ea + (double)(RUN - 1) * lr < lcut[k])) {
                    ev[k] = 0.0;
                } else {
                    direct = direct || !(ev[k] >= 1e-290) || !(rho[k] <= 1e200);
                    alive = true;
                }
            }
            if (!alive) continue;
#pragma unroll
            for (int t = 0; t < RUN; ++t) {
                const int lag = lag0 + t;
                if (lag <= M_last - 1) {
                    double vals[NG];
                    if (direct) {
                        x[D - 1] = dl * (double)lag;
                        eval_direct<Fun, D>(f, x, vals);
                    } else {
                        f.combine(z, ev, vals);
                    }
                    const double a = ri.rw * Arow[lag >= 0 ? lag : lag + N];
#pragma unroll
                    for (int g = 0; g < NG; ++g) acc[g] += vals[g] * a;
                }
#pragma unroll
                for (int k = 0; k < NGS; ++k) {
                    ev[k] *= rho[k];
                    rho[k] *= sig[k];
#pragma unroll
                    for (int i = 0; i < D; ++i) z[k][i] += dz[k][i];
                }
            }
        }
        double outv[NG];
        block_sum<NG, NT>(acc, red, outv);
        if (threadIdx.x == 0) store_item<NG>(pr, partial + item * NG, outv);
        fused_finish<D>(pr, partial, geo.nchunks, h);
    }
}

constexpr int LAG_RUN = 8;

// Moment families: long rows use runs of 16 lags (one fold per 16 lags) ...
template <int N>
constexpr int mom_run_of() { return N >= 256 ? 16 : LAG_RUN; }
// ... walked in segments of 32 lags per thread; short rows one run per
// thread, so that a row's few live runs are spread over several threads.
template <int N, int RL>
constexpr int mom_seg_of() { return N >= 256 && RL <= 32 && (N / 2) % 32 == 0 ? 32 / RL : 1; }

// Relative cut of the compacted lag walk: a run is walked only if some of its
// lags x has c_k exp(-x^T S_k^{-1} x / 2) >= 1e-30 c_k for some Gaussian k of
// the family (log 1e-30 below).  The dropped values are each below 1e-30 of
// their Gaussian's peak, so all of them together (times the moment-form
// polynomial factors, at most a few hundred times P) stay below 1e-30 x (number
// of lags) x (largest autocorrelation) x 10^3 -- more than ten orders of
// magnitude under float64 rounding of the lag-0 term alone.
constexpr double LOG_REL_CUT = -69.077552789821368;

// Live runs of one row: for every Gaussian of the family the lags l with
// exponent above LOG_REL_CUT form an interval (the exponent is a concave
// quadratic in l along the row); their hull, widened by one lag each side and
// clipped to |l| <= M - 1, as runs of RL array positions on the two sides of
// the circular row: pn runs from run pf (lags >= 0), nn runs from run nf
// (lags < 0).
struct LiveRuns {
    int pf, pn, nf, nn;
};

template <int D, class Fun>
__device__ __forceinline__ LiveRuns row_live(const Fun& f, const RowInfo& ri, int M_last, int N, int RL, double dl) {
    double la = INFINITY, lb = -INFINITY;
#pragma unroll
    for (int k = 0; k < Fun::NGAUSS; ++k) {
        const double* P = f.Pm(k);
        double b = 0.0, ql = 0.0;
#pragma unroll
        for (int i = 0; i < D - 1; ++i) {
            b += P[(D - 1) * D + i] * ri.x[i];
#pragma unroll
            for (int jj = 0; jj < D - 1; ++jj) ql += ri.x[i] * P[i * D + jj] * ri.x[jj];
        }
        const double pll = P[(D - 1) * D + D - 1];
        const double emax = -0.5 * (ql - b * b / pll);   // largest exponent along the row
        if (emax > LOG_REL_CUT) {
            const double ls = -b / (dl * pll);
            const double w = sqrt(2.0 * (emax - LOG_REL_CUT) / (dl * dl * pll));
            la = fmin(la, ls - w);
            lb = fmax(lb, ls + w);
        }
    }
    LiveRuns lr{0, 0, 0, 0};
    const double lim = (double)(M_last - 1);
    const double fa = fmax(floor(la) - 1.0, -lim), fb = fmin(ceil(lb) + 1.0, lim);
    if (fa <= fb) {   // false for an empty (or NaN) interval
        const int ia = (int)fa, ib = (int)fb;
        if (ib >= 0) {
            lr.pf = (ia > 0 ? ia : 0) / RL;
            lr.pn = ib / RL - lr.pf + 1;
        }
        if (ia <= -1) {
            lr.nf = (ia + N) / RL;
            lr.nn = ((ib < -1 ? ib : -1) + N) / RL - lr.nf + 1;
        }
    }
    return lr;
}

// Segments (of up to SEG runs) of a row's live runs.
template <int SEG>
__device__ __forceinline__ int live_units(const LiveRuns& lr) {
    return (lr.pn + SEG - 1) / SEG + (lr.nn + SEG - 1) / SEG;
}

// Exclusive block scan of v (all NT threads); *total receives the sum.  Ends
// with a barrier, so s_wsum can be reused right away.
template <int NT>
__device__ __forceinline__ int block_scan_excl(int v, int* s_wsum, int* total) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) s_wsum[wave] = x;
    __syncthreads();
    int pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        pre += w < wave ? s_wsum[w] : 0;
        tot += s_wsum[w];
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}

// Unit word of the per-item segment lists: row << 16 | first run << 8 | runs.
__device__ __forceinline__ uint32_t unit_word(int row, int run, int nruns) {
    return (uint32_t)row << 16 | (uint32_t)run << 8 | (uint32_t)nruns;
}

// Append the segments of a row with live runs lr to the list (positive side,
// then negative side), numbered from first; only those with numbers in
// [lo, hi) are written, at s_unit[number - lo].
template <int SEG>
__device__ __forceinline__ void write_units(uint32_t* s_unit, int row, const LiveRuns& lr, int first, int lo, int hi) {
    int o = first;
    for (int a = 0; a < lr.pn; a += SEG, ++o)
        if (o >= lo && o < hi) s_unit[o - lo] = unit_word(row, lr.pf + a, lr.pn - a < SEG ? lr.pn - a : SEG);
    for (int a = 0; a < lr.nn; a += SEG, ++o)
        if (o >= lo && o < hi) s_unit[o - lo] = unit_word(row, lr.nf + a, lr.nn - a < SEG ? lr.nn - a : SEG);
}

// Largest number of segments one item's list holds in LDS, and of candidates
// in a balanced plan.
constexpr int UNIT_CAP = 4096;
constexpr int MAX_PLAN = 1024;

// Compacted dealing of an item's rows row0, row0 + rstride, ... (count rows):
// the rows are taken RB at a time; thread t finds row t's live runs
// (row_live), a block scan numbers their segments, the segments are listed in
// LDS (rows in order, runs in order within a row, so neighbouring lanes read
// neighbouring blocks of the autocorrelation), and the threads walk segments
// t, t + NT, ... of the list with seg_walk(ri, first run, runs).
template <int D, int N, int RL, int SEG, int NT, class Fun, class Walk>
__device__ __forceinline__ void live_segments(const Fun& f, const RowGeom& geo, int64_t row0, int64_t rstride,
                                              int64_t count, const double* delta, Walk&& seg_walk) {
    constexpr int NRUN = N / RL;                               // runs per row
    constexpr int UPR = 2 * ((NRUN / 2 + SEG - 1) / SEG);     // segments per row, at most (both sides)
    constexpr int RB = NT < UNIT_CAP / UPR ? NT : UNIT_CAP / UPR;   // rows per pass
    static_assert(NRUN <= 256 && NT <= 256 && RB >= 1, "unit word layout");
    __shared__ uint32_t s_unit[RB * UPR];
    __shared__ int s_wsum[NT / 64];
    const int M_last = geo.M[D - 1];
    for (int64_t jb = 0; jb < count; jb += RB) {
        const int nb = count - jb < RB ? (int)(count - jb) : RB;
        LiveRuns lr{0, 0, 0, 0};
        if ((int)threadIdx.x < nb)
            lr = row_live<D>(f, row_info<D>(row0 + (jb + threadIdx.x) * rstride, geo.nrows, geo, delta, nullptr),
                             M_last, N, RL, delta[D - 1]);
        int total = 0;
        const int first = block_scan_excl<NT>(live_units<SEG>(lr), s_wsum, &total);
        if ((int)threadIdx.x < nb) write_units<SEG>(s_unit, (int)threadIdx.x, lr, first, 0, total);
        __syncthreads();
        for (int k = threadIdx.x; k < total; k += NT) {
            const uint32_t u = s_unit[k];
            seg_walk(row_info<D>(row0 + (jb + (u >> 16)) * rstride, geo.nrows, geo, delta, nullptr),
                     (int)((u >> 8) & 255u), (int)(u & 255u));
        }
        __syncthreads();
    }
}

// Balanced dealing: the item is the window [k W / parts, (k + 1) W / parts) of
// its candidate's list of W live segments over all nrows rows (rows in order).
// The rows are scanned in passes of NT (a first sweep counts W when the rows
// span several passes); the window's segments are listed in LDS, UNIT_CAP at a
// time, and walked as in live_segments.
template <int D, int N, int RL, int SEG, int NT, class Fun, class Walk>
__device__ __forceinline__ void live_window(const Fun& f, const RowGeom& geo, int k, int parts,
                                            const double* delta, Walk&& seg_walk) {
    static_assert(N / RL <= 256 && NT <= 256, "unit word layout");
    __shared__ uint32_t s_unit[UNIT_CAP];
    __shared__ int s_wsum[NT / 64];
    const int M_last = geo.M[D - 1];
    const int64_t nrows = geo.nrows;
    int64_t wtot = -1;
    if (nrows > NT) {
        wtot = 0;
        for (int64_t rb = 0; rb < nrows; rb += NT) {
            LiveRuns lr{0, 0, 0, 0};
            if (rb + threadIdx.x < nrows)
                lr = row_live<D>(f, row_info<D>(rb + threadIdx.x, nrows, geo, delta, nullptr), M_last, N, RL,
                                 delta[D - 1]);
            int total = 0;
            (void)block_scan_excl<NT>(live_units<SEG>(lr), s_wsum, &total);
            wtot += total;
        }
    }
    int64_t lo = -1, hi = -1;
    for (int64_t sub = 0;; sub += UNIT_CAP) {
        int64_t seen = 0, sl = 0, sh = 0;
        for (int64_t rb = 0; rb < nrows; rb += NT) {
            LiveRuns lr{0, 0, 0, 0};
            if (rb + threadIdx.x < nrows)
                lr = row_live<D>(f, row_info<D>(rb + threadIdx.x, nrows, geo, delta, nullptr), M_last, N, RL,
                                 delta[D - 1]);
            int total = 0;
            const int first = block_scan_excl<NT>(live_units<SEG>(lr), s_wsum, &total);
            if (wtot < 0) wtot = total;   // all rows in this one pass
            if (lo < 0) {
                lo = (int64_t)k * wtot / parts;
                hi = (int64_t)(k + 1) * wtot / parts;
            }
            sl = lo + sub;
            sh = hi < sl + UNIT_CAP ? hi : sl + UNIT_CAP;
            if (rb + threadIdx.x < nrows && seen + first < sh)
                write_units<SEG>(s_unit, (int)(rb + threadIdx.x), lr, (int)(seen + first - sl), 0, (int)(sh - sl));
            seen += total;
            if (seen >= sh) break;   // block-uniform
        }
        __syncthreads();
        for (int u = threadIdx.x; u < sh - sl; u += NT) {
            const uint32_t w = s_unit[u];
            seg_walk(row_info<D>(w >> 16, nrows, geo, delta, nullptr), (int)((w >> 8) & 255u), (int)(w & 255u));
        }
        __syncthreads();
        if (sh >= hi) break;
    }
}

// Items of the balanced plan (every block computes the same plan from the
// candidates' live segment counts wc): with W the total, the smallest U (from
// ceil(W / slots), raised by 1/16 steps) for which giving candidate c
// max(1, ceil(wc / U)) items keeps the total within max(slots, candidates) (the
// loop ends: once U exceeds every count each candidate has one item);
// s_off[c] is candidate c's first item, s_off[nplan] the number of items.
// Block 0 also stores the offsets for the final kernel.
template <int NT>
__device__ __forceinline__ int balanced_plan(const RowGeom& geo, int slots, int* s_off, int* s_wsum) {
    const int nc = geo.nplan;
    const int target = slots > nc ? slots : nc;
    int64_t wl = 0;
    for (int c = threadIdx.x; c < nc; c += NT) wl += geo.wc[c];
    int wtot = 0;
    (void)block_scan_excl<NT>((int)wl, s_wsum, &wtot);
    int64_t U = (wtot + (int64_t)slots - 1) / slots;
    if (U < 1) U = 1;
    for (;;) {
        int tl = 0;
        for (int c = threadIdx.x; c < nc; c += NT) {
            const int64_t n = (geo.wc[c] + U - 1) / U;
            tl += n > 1 ? (int)n : 1;
        }
        int t = 0;
        (void)block_scan_excl<NT>(tl, s_wsum, &t);
        if (t <= target) break;   // block-uniform
        U += U / 16 > 1 ? U / 16 : 1;
    }
    // offsets: thread t takes candidates [t * per, (t + 1) * per)
    const int per = (nc + NT - 1) / NT;
    int cnt = 0;
    for (int c = threadIdx.x * per; c < nc && c < (int)(threadIdx.x + 1) * per; ++c) {
        const int64_t n = (geo.wc[c] + U - 1) / U;
        cnt += n > 1 ? (int)n : 1;
    }
    int total = 0;
    int o = block_scan_excl<NT>(cnt, s_wsum, &total);
    for (int c = threadIdx.x * per; c < nc && c < (int)(threadIdx.x + 1) * per; ++c) {
        const int64_t n = (geo.wc[c] + U - 1) / U;
        s_off[c] = o;
        o += n > 1 ? (int)n : 1;
    }
    if (threadIdx.x == 0) s_off[nc] = total;
    __syncthreads();
    if (blockIdx.x == 0)
        for (int c = threadIdx.x; c <= nc; c += NT) geo.item_off[c] = s_off[c];
    return total;
}

// Lag-domain evaluation for the families with a moment form (SCV / LSCV):
// runs of RL consecutive array positions of the circular row (see below),
// their RL autocorrelation values loaded as one aligned block, and per run
// only the moments sum_t t^p e(t) A(t) of each Gaussian (Fun::fold).  A thread
// walks a segment of SEG consecutive runs of one row: the values e and ratios
// rho reached at the end of a run are those of the next run's start, so only
// the segment's first run (or a run after one that needed special handling)
// evaluates exponentials.
template <int D, int N, class Fun, int NT, int RUN, bool SCALED, bool COMPACT>
__global__ __launch_bounds__(NT, D <= 2 ? (COMPACT ? 3 : 1) : 2) void k_lag_mom(const double* __restrict__ prm, RowGeom geo, int64_t nitems,
                                            double* __restrict__ partial) {
    constexpr int NG = Fun::NG;
    constexpr int NGS = Fun::NGAUSS;
    // Runs of RL consecutive array positions of the circular row: p in [0, N/2)
    // holds lags p, p in [N/2, N) lags p - N; N/2 is a multiple of RL * SEG, so
    // neither a run nor a segment mixes the two sides, their lags are
    // consecutive, and a run's RL values of the autocorrelation form one
    // aligned block that is loaded at once.  Positions outside |lag| <= M-1
    // (the zero slots) get weight 0.
    constexpr int RL = RUN < N / 2 ? RUN : N / 2;
    constexpr int SEG = mom_seg_of<N, RL>();
    constexpr int nseg = N / (RL * SEG);
    __shared__ double red[(NT / 64) * NG];
    const int M_last = geo.M[D - 1];
    // thread t takes the (row, segment) pairs t, t + NT, ... of its item in
    // row-major order; the pair is advanced incrementally (no division in the loop)
    constexpr int step_ro = NT / nseg, step_j = NT % nseg;
    const int ro0 = (int)threadIdx.x / nseg, j0 = (int)threadIdx.x % nseg;
    // balanced plan (compacted walk, geo.nplan candidates): items are windows of
    // the candidates' live segment lists, numbered by the plan
    __shared__ int s_off[COMPACT ? MAX_PLAN + 1 : 1];
    __shared__ int s_pw[NT / 64];
    int64_t nit = nitems;
    if constexpr (COMPACT) {
        if (geo.nplan > 0) nit = balanced_plan<NT>(geo, (int)gridDim.x, s_off, s_pw);
    }
    // parameter blocks built in the launch (one block per work item, no plan):
    // thread 0 computes the block's candidate's parameters into LDS before
    // anything else is live, and the block of the candidate's first item also
    // stores them for the final kernel
    __shared__ double s_prm[COMPACT && !SCALED ? PRM : 1];
    if constexpr (COMPACT && !SCALED) {
        if (geo.setup.on) {
            const int64_t h0 = blockIdx.x / geo.nchunks, ch0 = blockIdx.x - h0 * geo.nchunks;
            if (threadIdx.x == 0) {
                if (h0 < geo.setup.ncand)
                    scv_params<D, false>(geo.setup.vechL, geo.setup.a, h0, geo.setup.ncand, geo.setup.npseudo, s_prm,
                                         ch0 == 0 ? geo.setup.status : nullptr);
                else
                    pseudo_params<D>(geo.setup.a, (int)(h0 - geo.setup.ncand), s_prm);
                if (ch0 == 0)
                    for (int i = 0; i < PRM; ++i) geo.setup.prm_out[h0 * PRM + i] = s_prm[i];
            }
            __syncthreads();
        }
    }
    for (int64_t item = blockIdx.x; item < nit; item += gridDim.x) {
        int64_t h, ch = 0;
        int part = 0, parts = 1;
        if (COMPACT && geo.nplan > 0) {
            int lo = 0, hi = geo.nplan - 1;   // the last candidate whose first item is <= item
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_off[mid] <= item)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            h = lo;
            part = (int)(item - s_off[lo]);
            parts = s_off[lo + 1] - s_off[lo];
        } else {
            h = item / geo.nchunks;
            ch = item - h * geo.nchunks;
        }
        // the parameter block, uniform over the block: loaded from the
        // parameter array (scalar loads), or taken from LDS into scalar
        // registers when the launch built it
        double pv[PRM];
        if (COMPACT && !SCALED && geo.setup.on) {
#pragma unroll
            for (int i = 0; i < PRM; ++i) pv[i] = wave_uniform(s_prm[i]);
        } else {
#pragma unroll
            for (int i = 0; i < PRM; ++i) pv[i] = prm[h * PRM + i];
        }
        const double* pr = pv;
        Fun f;
        f.load(pr);
        double delta[D];
#pragma unroll
        for (int k = 0; k < D; ++k) delta[k] = pr[S_DELTA + k];
        const double* __restrict__ A =
            reinterpret_cast<const double*>(static_cast<uintptr_t>(__double_as_longlong(pr[S_ALAG])));
        const double dl = delta[D - 1];
        double dz[NGS][D], sig[NGS], hpl[NGS], lcut[NGS];
#pragma unroll
        for (int k = 0; k < NGS; ++k) {
            const double* P = f.Pm(k);
#pragma unroll
            for (int i = 0; i < D; ++i) dz[k][i] = dl * P[i * D + D - 1];
            hpl[k] = 0.5 * dl * dl * P[(D - 1) * D + D - 1];
            lcut[k] = -667.74967696827317 - log(f.cn(k));   // c e^x < 1e-290 below
        }
        // The ratio update rho <- rho sigma, sigma = exp(-2 hpl), compounds the
        // representation error of sigma t(t-1)/2 times by lag t of a walk, the
        // same way for every run.  sig holds sigma - 1 (expm1) and the update is
        // rho + rho (sigma - 1), one FMA, so the compounded error is that of the
        // small number sigma - 1.  That needs sigma near 1: with some sigma below
        // 1/2 (kernels narrower than about a grid step, whose values fall by half
        // a decade per lag or faster and cover only a few lags of a row) every
        // run of the item is evaluated lag by lag instead.
        bool near1 = true;
#pragma unroll
        for (int k = 0; k < NGS; ++k) {
            near1 = near1 && 2.0 * hpl[k] < 0.69314718055994531;
            sig[k] = expm1(-2.0 * hpl[k]);
        }
        double acc[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) acc[g] = 0.0;
        const int64_t rbeg = ch * geo.chunk;
        const int64_t rend = rbeg + geo.chunk < geo.nrows ? rbeg + geo.chunk : geo.nrows;
        const int nro = (int)(rend - rbeg);   // rows of one item < 2^31
        // One segment of a row: nruns consecutive runs from run index j (runs
        // of RL array positions, j < N / RL; all on one side of the row),
        // carrying the walk state from run to run.
        auto seg_walk = [&](const RowInfo& ri, int j, int nruns) {
            // walk state carried from run to run: z at the run start, e, rho
            double z[NGS][D], ev[NGS], rho[NGS];
            bool carried = false;
#pragma unroll 1
            for (int c = 0; c < nruns; ++c) {
                const int p0 = (j + c) * RL;
                const bool pos = p0 < N / 2;
                const int lag0 = pos ? p0 : p0 - N;
                // runs that lie wholly in the zero slots
                if (pos ? lag0 > M_last - 1 : lag0 + RL - 1 < -(M_last - 1)) {
                    carried = false;
                    continue;
                }
                const double* __restrict__ Arow = A + ri.wr * N + p0;
                // the run's autocorrelation values, one aligned block, loaded
                // first so that their latency overlaps the run start; the lag
                // array is exactly zero at |lag| > M - 1 (stored so by the
                // preparation), so no position needs masking here
                double av[RL];
                if constexpr (RL % 2 == 0) {
                    const double2* a2 = reinterpret_cast<const double2*>(Arow);
#pragma unroll
                    for (int t = 0; t < RL / 2; ++t) {
                        const double2 v = a2[t];
                        av[2 * t] = v.x;
                        av[2 * t + 1] = v.y;
                    }
                } else {
#pragma unroll
                    for (int t = 0; t < RL; ++t) av[t] = Arow[t];
                }
                bool scl[NGS];
                bool direct = false, alive = false, rising = false;
                if (carried) {
                    // continue the walk: values at or above 1e-290 go on, values
                    // below it that decrease are dropped; a Gaussian rising from
                    // below restarts the run with exponentials (the ratios only
                    // decrease along a walk, so none can newly exceed 1e200)
                    bool rise = false;
#pragma unroll
                    for (int k = 0; k < NGS; ++k) {
                        scl[k] = false;
#pragma unroll
                        for (int i = 0; i < D; ++i) z[k][i] += (double)RL * dz[k][i];
                        const bool low = !(ev[k] >= 1e-290);
                        rise = rise || (low && rho[k] > 1.0);
                        ev[k] = low ? 0.0 : ev[k];
                        alive = alive || !low;
                    }
                    carried = !rise;
                }
                if (!carried) {
                    double x[D];
#pragma unroll
                    for (int k = 0; k < D - 1; ++k) x[k] = ri.x[k];
                    x[D - 1] = dl * (double)lag0;
                    direct = false;
                    alive = false;
#pragma unroll
                    for (int k = 0; k < NGS; ++k) {
                        const double* P = f.Pm(k);
                        double q = 0.0;
#pragma unroll
                        for (int i = 0; i < D; ++i) {
                            double s = 0.0;
#pragma unroll
                            for (int jj = 0; jj < D; ++jj) s += P[i * D + jj] * x[jj];
                            z[k][i] = s;
                            q += x[i] * s;
                        }
                        // A run starting below 1e-290 with ratios rho, rho sig, ... <= 1
                        // (sig < 1) stays there and adds nothing a float64 sum can hold
                        // next to the lag-0 term.  A run that rises from there is walked
                        // with values scaled by e^600 (kept in the normal range) and its
                        // moments scaled back at the end (SCALED), or evaluated lag by lag.
                        const double ea = -0.5 * q;
                        const double lr = -(dl * z[k][D - 1] + hpl[k]);
                        rho[k] = exp(lr);
                        // a run below the cut that rises: its exponent stays below
                        // ea + (RL - 1) lr (the log-ratios only decrease); if that
                        // bound is below the cut too, the run is negligible
                        const bool low = ea < lcut[k];
                        const bool negl = low && ea + (double)(RL - 1) * lr < lcut[k];
                        if constexpr (SCALED) {
                            scl[k] = low;
                            if (low && (rho[k] <= 1.0 || negl)) {
                                ev[k] = 0.0;
                                rising = rising || rho[k] > 1.0;
                            } else {
                                const double es = low ? ea + 600.0 : ea;
                                ev[k] = f.cn(k) * exp(es);
                                // a start still below 1e-290 after the e^600 scaling
                                // (the values rise by more than that along the run,
                                // and would start from zero): lag by lag instead
                                direct = direct || !(rho[k] <= 1e200) || !(es >= lcut[k]);
                                alive = true;
                            }
                        } else {
                            scl[k] = false;
                            ev[k] = f.cn(k) * exp(ea);
                            if (!(ev[k] >= 1e-290) && (rho[k] <= 1.0 || negl)) {
                                ev[k] = 0.0;
                                rising = rising || rho[k] > 1.0;
                            } else {
                                direct = direct || !(ev[k] >= 1e-290) || !(rho[k] <= 1e200);
                                alive = true;
                            }
                        }
                    }
                }
                direct = direct || !near1;
                if (!alive) {
                    // every Gaussian below 1e-290 and decreasing: so are the
                    // rest of the segment's runs (further along the same
                    // direction); one still rising is looked at again next run
                    if (!rising) break;
                    carried = false;
                    continue;
                }
                // the next run continues this one's walk unless this one is
                // evaluated directly or walked scaled
                carried = !direct;
#pragma unroll
                for (int k = 0; k < NGS; ++k) carried = carried && !scl[k];
                if (direct) {
                    // exact evaluation lag by lag (values near the float64 range
                    // limits; rare): a rolled loop keeps one copy of the evaluation
                    double x[D];
#pragma unroll
                    for (int k = 0; k < D - 1; ++k) x[k] = ri.x[k];
#pragma unroll 1
                    for (int t = 0; t < RL; ++t) {
                        const int lag = lag0 + t;
                        const bool ok = pos ? lag <= M_last - 1 : lag >= -(M_last - 1);
                        if (ok) {
                            double vals[NG];
                            x[D - 1] = dl * (double)lag;
                            eval_direct<Fun, D>(f, x, vals);
                            const double a = ri.rw * Arow[t];
#pragma unroll
                            for (int g = 0; g < NG; ++g) acc[g] += vals[g] * a;
                        }
                    }
                    continue;
                }
                {
                    constexpr int NM = Fun::NMOM;
                    double m[NGS][3];
#pragma unroll
                    for (int k = 0; k < NGS; ++k) m[k][0] = m[k][1] = m[k][2] = 0.0;
#pragma unroll
                    for (int t = 0; t < RL; ++t) {
#pragma unroll
                        for (int k = 0; k < NGS; ++k) {
                            const double w = ev[k] * av[t];
                            m[k][0] += w;
                            if constexpr (NM > 1) {
                                m[k][1] += (double)t * w;
                                m[k][2] += (double)(t * t) * w;
                            }
                            ev[k] *= rho[k];
                            rho[k] = fma(rho[k], sig[k], rho[k]);   // rho sigma, sig = sigma - 1
                        }
                    }
                    // row weight (mirror rows count twice), and the e^600 scaling undone
#pragma unroll
                    for (int k = 0; k < NGS; ++k) {
                        constexpr double E_M600 = 2.6503965530043108e-261;   // e^-600
                        const double wk = (SCALED && scl[k]) ? ri.rw * E_M600 : ri.rw;
                        m[k][0] *= wk;
                        m[k][1] *= wk;
                        m[k][2] *= wk;
                    }
                    f.fold(z, dz, m, acc);
                }
            }
        };
        if constexpr (!COMPACT) {
            for (int ro = ro0, sg = j0; ro < nro; ro += step_ro + (sg + step_j >= nseg ? 1 : 0),
                     sg = sg + step_j >= nseg ? sg + step_j - nseg : sg + step_j)
                seg_walk(row_info<D>(rbeg + ro, rend, geo, delta, nullptr), sg * SEG, SEG);
        } else {
            if (geo.nplan > 0)
                live_window<D, N, RL, SEG, NT>(f, geo, part, parts, delta, seg_walk);
            else   // the item's rows interleaved with its candidate's other items' (ch, ch + nchunks, ...):
                   // every item gets a like share of the rows near the kernels' peaks
                live_segments<D, N, RL, SEG, NT>(f, geo, ch, geo.nchunks, (geo.nrows - ch + geo.nchunks - 1) / geo.nchunks,
                                                 delta, seg_walk);
        }
        double outv[NG];
        block_sum<NG, NT>(acc, red, outv);
        if (threadIdx.x == 0) store_item<NG>(pr, partial + item * NG, outv);
        fused_finish<D>(pr, partial, geo.nchunks, h);
    }
}

// Families whose combine step dominates (many Hermite outputs) gain nothing
// from the exponential recurrence and lose registers to it: runs of one lag.
template <class Fun>
constexpr int lag_run_of() { return Fun::NG > 12 ? 1 : LAG_RUN; }


template <int D, int N, class Fun, int NT, bool SCALED, bool COMPACT>
constexpr auto select_lag() {
    if constexpr (HasMoments<Fun>::value)
        return k_lag_mom<D, N, Fun, NT, mom_run_of<N>(), SCALED, COMPACT>;
    else
        return k_lag<D, N, Fun, NT, lag_run_of<Fun>()>;
}

// variant 3: lag walk, runs that rise from below the float64 range evaluated
// lag by lag; 4: the same runs walked scaled by e^600; 5, 6: as 3, 4 with the
// live runs of each row dealt to the threads (compacted).  The psi and eta
// families (no moment form) run one lag-walk kernel for all four.
template <int D, int N, class Fun>
hipError_t run_lag_t(const double* prm, RowGeom geo, int64_t nitems, double* partial, int grid_blocks,
                     hipStream_t s, int variant) {
    constexpr int NT = 256;
    auto kern = variant == 4   ? select_lag<D, N, Fun, NT, true, false>()
                : variant == 5 ? select_lag<D, N, Fun, NT, false, true>()
                : variant == 6 ? select_lag<D, N, Fun, NT, true, true>()
                               : select_lag<D, N, Fun, NT, false, false>();
    int64_t blocks = nitems;
    if (grid_blocks > 0) {
        blocks = grid_blocks;
    } else if (grid_blocks == 0) {
        static int resident = -1;
        if (resident < 0) {
            int per_cu = 0, dev = 0, cus = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NT, 0) != hipSuccess) per_cu = 1;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
                cus = 256;
            resident = (per_cu < 1 ? 1 : per_cu) * cus;
        }
        blocks = resident;
    }
    if (blocks > nitems) blocks = nitems;
    if (blocks < 1) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(NT), 0, s, prm, geo, nitems, partial);
    return hipGetLastError();
}

// rows covered by one pass of a 256-thread block (runs of LAG_RUN lags, or
// for the moment families segments of mom_seg_of x mom_run_of lags)
template <int N>
constexpr int lag_rows_per_pass() { return (256 * LAG_RUN) / N >= 1 ? (256 * LAG_RUN) / N : 1; }
template <int N>
constexpr int mom_rows_per_pass() {
    constexpr int RL = mom_run_of<N>() < N / 2 ? mom_run_of<N>() : N / 2;
    constexpr int per = 256 * RL * mom_seg_of<N, RL>() / N;
    return per >= 1 ? per : 1;
}

// Rows per wavefront per pass: enough butterflies for one per lane in a radix-8
// stage (variant 0, 2) or twice that (variant 1); at most 8.
template <int N, int NG, int VAR>
constexpr int rows_for() {
    constexpr int npen = (NG + 1) / 2;
    constexpr int bfly = npen * (N / 8 > 0 ? N / 8 : 1);
    constexpr int base = bfly >= 64 ? 1 : (64 / bfly >= 8 ? 8 : (64 / bfly >= 4 ? 4 : (64 / bfly >= 2 ? 2 : 1)));
    constexpr int r = VAR == 1 ? (base * 2 > 8 ? 8 : base * 2) : base;
    return r;
}

// Wavefronts per block: as many (<= 4) as fit 96 KiB of pencils.
template <int N, int NG, int RPW>
constexpr int waves_for() {
    constexpr int per = RPW * ((NG + 1) / 2) * N * 16;
    return per * 4 <= 98304 ? 4 : (per * 2 <= 98304 ? 2 : 1);
}

// Persistent grid: grid_blocks > 0 as given, 0 = resident blocks per CU x CUs,
// -1 = one block per work item.
template <int D, int N, class Fun, int VAR>
hipError_t run_rows_t(const double* prm, RowGeom geo, int64_t nitems, double* partial, int grid_blocks,
                      const double2* tw, hipStream_t s) {
    constexpr int RPW = rows_for<N, Fun::NG, VAR>();
    constexpr int WPB = waves_for<N, Fun::NG, RPW>();
    constexpr int SCHED = VAR == 2 ? 1 : 0;
    auto kern = k_rows<D, N, Fun, RPW, WPB, SCHED>;
    int64_t blocks = nitems;
    if (grid_blocks > 0) {
        blocks = grid_blocks;
    } else if (grid_blocks == 0) {
        static int resident = -1;  // per instantiation, per process
        if (resident < 0) {
            int per_cu = 0, dev = 0, cus = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, WPB * 64, 0) != hipSuccess) per_cu = 1;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
                cus = 256;
            resident = (per_cu < 1 ? 1 : per_cu) * cus;
        }
        blocks = resident;
    }
    if (blocks > nitems) blocks = nitems;
    if (blocks < 1) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(WPB * 64), 0, s, prm, geo, nitems, partial, tw);
    return hipGetLastError();
}

}  // namespace kdefft
