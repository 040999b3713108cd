// Host dispatch of the batched row kernels, and the small per-candidate
// kernels around them: SCV parameter setup (Cholesky factors of 2H+2G and
// H+2G) and the final assembly of psi / SCV objective / gradient from the
// per-item partial sums (fixed summation order).
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "dev_kernels.h"
#include "eta_fun.h"
#include "finish.h"
#include "internal.h"
#include "params.h"
#include "rows_impl.h"

namespace kdefft {

hipError_t launch_rows_d1(int, int, int, int, const double*, RowGeom, int64_t, double*, int, const double2*,
                          hipStream_t);
hipError_t launch_rows_d2(int, int, int, int, const double*, RowGeom, int64_t, double*, int, const double2*,
                          hipStream_t);
hipError_t launch_rows_d3(int, int, int, int, const double*, RowGeom, int64_t, double*, int, const double2*,
                          hipStream_t);
hipError_t launch_rows_d4(int, int, int, int, const double*, RowGeom, int64_t, double*, int, const double2*,
                          hipStream_t);
hipError_t launch_rows_eta_d1(int, int, int, int, const double*, RowGeom, int64_t, double*, int, hipStream_t);
hipError_t launch_rows_eta_d2(int, int, int, int, const double*, RowGeom, int64_t, double*, int, hipStream_t);
hipError_t launch_rows_eta_d3(int, int, int, int, const double*, RowGeom, int64_t, double*, int, hipStream_t);
hipError_t launch_rows_eta_d4(int, int, int, int, const double*, RowGeom, int64_t, double*, int, hipStream_t);
int rows_iter_eta_d1(int, int, int);
int rows_iter_eta_d2(int, int, int);
int rows_iter_eta_d3(int, int, int);
int rows_iter_eta_d4(int, int, int);
int rows_iter_d1(int, int, int, int);
int rows_iter_d2(int, int, int, int);
int rows_iter_d3(int, int, int, int);
int rows_iter_d4(int, int, int, int);

static int binom_h(int n, int k) {
    int r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

template <int N>
static int layout_of(int moments, int* run_len, int* runs_per_seg, int* rows_per_pass) {
    if (moments) {
        constexpr int RL = mom_run_of<N>() < N / 2 ? mom_run_of<N>() : N / 2;
        *run_len = RL;
        *runs_per_seg = mom_seg_of<N, RL>();
        *rows_per_pass = mom_rows_per_pass<N>();
    } else {
        *run_len = LAG_RUN;
        *runs_per_seg = 1;
        *rows_per_pass = lag_rows_per_pass<N>();
    }
    return 1;
}

int lag_layout(int N, int moments, int* run_len, int* runs_per_seg, int* rows_per_pass) {
    switch (N) {
        case 4: return layout_of<4>(moments, run_len, runs_per_seg, rows_per_pass);
        case 8: return layout_of<8>(moments, run_len, runs_per_seg, rows_per_pass);
        case 16: return layout_of<16>(moments, run_len, runs_per_seg, rows_per_pass);
        case 32: return layout_of<32>(moments, run_len, runs_per_seg, rows_per_pass);
        case 64: return layout_of<64>(moments, run_len, runs_per_seg, rows_per_pass);
        case 128: return layout_of<128>(moments, run_len, runs_per_seg, rows_per_pass);
        case 256: return layout_of<256>(moments, run_len, runs_per_seg, rows_per_pass);
        case 512: return layout_of<512>(moments, run_len, runs_per_seg, rows_per_pass);
        case 1024: return layout_of<1024>(moments, run_len, runs_per_seg, rows_per_pass);
        case 2048: return layout_of<2048>(moments, run_len, runs_per_seg, rows_per_pass);
        default: return 0;
    }
}

int ng_of(int kind, int d, int r) {
    const int q = d * (d + 1) / 2;
    switch (kind) {
        case FUN_PSI: return binom_h(d + r - 1, r);
        case FUN_SCV_OBJ: return 1;
        case FUN_SCV_OBJGRAD: return 1 + q;
        case FUN_SCV_GRAD: return q;
        case FUN_ETA1:
        case FUN_ETA2: return 1;
        default: return 0;
    }
}

int rows_per_iter(int kind, int d, int r, int N, int variant) {
    if (kind == FUN_ETA1 || kind == FUN_ETA2) {
        switch (d) {
            case 1: return rows_iter_eta_d1(kind, N, variant);
            case 2: return rows_iter_eta_d2(kind, N, variant);
            case 3: return rows_iter_eta_d3(kind, N, variant);
            case 4: return rows_iter_eta_d4(kind, N, variant);
            default: return 0;
        }
    }
    switch (d) {
        case 1: return rows_iter_d1(kind, r, N, variant);
        case 2: return rows_iter_d2(kind, r, N, variant);
        case 3: return rows_iter_d3(kind, r, N, variant);
        case 4: return rows_iter_d4(kind, r, N, variant);
        default: return 0;
    }
}

// Resident blocks of the compacted lag kernels on the current device: their
// launch bounds ask for 3 blocks of 256 threads per CU at d <= 2, 2 above.
static int compact_slots(int d) {
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (cus[dev] <= 0) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1) c = 256;
        cus[dev] = c;
    }
    return cus[dev] * (d <= 2 ? 3 : 2);
}

RowGeom make_geom(const kdefft_grid& g, int kind, int r, int64_t ncand, int variant) {
    RowGeom geo{};
    geo.d = g.d;
    for (int k = 0; k < 4; ++k) {
        geo.M[k] = k < g.d ? g.M[k] : 1;
        geo.P[k] = k < g.d ? g.P[k] : 1;
    }
    int64_t nrows = 1;
    if (g.d >= 2) {
        nrows = g.M[0];
        for (int k = 1; k + 1 < g.d; ++k) nrows *= (2 * g.M[k] - 1);
    }
    geo.nrows = nrows;
    geo.Q = g.P[g.d - 1] / 2 + 1;
    int ri = rows_per_iter(kind, g.d, r, g.P[g.d - 1], variant);
    if (ri < 1) ri = 1;
    const bool mom = kind == FUN_SCV_OBJ || kind == FUN_SCV_OBJGRAD || kind == FUN_SCV_GRAD;
    if (variant >= 5 && mom && nrows <= 4096 && ncand <= 1024) {
        // compacted walk with a balanced plan (items numbered on the device,
        // at most one per resident block): candidates x nchunks covers the
        // resident blocks; the launch without a plan takes the same number of
        // items per candidate, each with every nchunks-th row of its candidate
        const int64_t slots = (int64_t)compact_slots(g.d);
        int64_t per = (slots + ncand - 1) / ncand;
        // more items than resident slots by more than an eighth of them would
        // start a large second round of blocks: one round of fewer, larger
        // items instead (a small overflow is absorbed by the blocks that
        // finish early)
        if (per > 1 && ncand * per > slots + slots / 8) per = slots / ncand > 1 ? slots / ncand : 1;
        if (per > nrows) per = nrows;
        const int64_t chunk = (nrows + per - 1) / per;
        geo.chunk = chunk;
        geo.nchunks = (nrows + chunk - 1) / chunk;
        return geo;
    }
    if (variant >= 5 && mom) {
        // compacted walk: the live runs of a whole item are dealt over the
        // block at once, so items are sized to the resident blocks instead:
        // the fewest whole rounds of items over the resident slots that keep an
        // item at most 4096 rows, the items split evenly over the candidates
        const int64_t slots = (int64_t)compact_slots(g.d);
        const int64_t maxrows = 4096;
        int64_t rounds = (nrows * ncand + slots * maxrows - 1) / (slots * maxrows);
        if (rounds < 1) rounds = 1;
        int64_t per = slots * rounds / ncand;
        if (per < 1) per = 1;
        if (per > nrows) per = nrows;
        const int64_t chunk = (nrows + per - 1) / per;
        geo.chunk = chunk;
        geo.nchunks = (nrows + chunk - 1) / chunk;
        return geo;
    }
    // lag kernel: larger items amortise the per-item set-up and block reduction
    const int64_t target = variant >= 3 ? 2048 : 8192;
    int64_t iters = (nrows * ncand + (int64_t)ri * target - 1) / ((int64_t)ri * target);
    if (iters < 1) iters = 1;
    int64_t chunk = iters * ri;
    if (chunk > nrows) chunk = ((nrows + ri - 1) / ri) * ri;
    geo.chunk = chunk;
    geo.nchunks = (nrows + chunk - 1) / chunk;
    return geo;
}

hipError_t launch_rows(int kind, int d, int r, const RowGeom& geo, const double* prm, int64_t ncand,
                       double* partial, const RowLaunch& rl, hipStream_t s) {
    // only the spectral variants read the twiddle table (set up on first use)
    const double2* tw = nullptr;
    if (rl.variant < 3 && kind != FUN_ETA1 && kind != FUN_ETA2) {
        hipError_t e = twiddles(&tw);
        if (e != hipSuccess) return e;
    }
    const int64_t nitems = ncand * geo.nchunks;
    const int N = geo.P[d - 1];
    if (kind == FUN_ETA1 || kind == FUN_ETA2) {
        switch (d) {
            case 1: return launch_rows_eta_d1(kind, r, N, rl.variant, prm, geo, nitems, partial, rl.grid_blocks, s);
            case 2: return launch_rows_eta_d2(kind, r, N, rl.variant, prm, geo, nitems, partial, rl.grid_blocks, s);
            case 3: return launch_rows_eta_d3(kind, r, N, rl.variant, prm, geo, nitems, partial, rl.grid_blocks, s);
            case 4: return launch_rows_eta_d4(kind, r, N, rl.variant, prm, geo, nitems, partial, rl.grid_blocks, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (d) {
        case 1: return launch_rows_d1(kind, r, N, rl.variant, prm, geo, nitems, partial, rl.grid_blocks, tw, s);
        case 2: return launch_rows_d2(kind, r, N, rl.variant, prm, geo, nitems, partial, rl.grid_blocks, tw, s);
        case 3: return launch_rows_d3(kind, r, N, rl.variant, prm, geo, nitems, partial, rl.grid_blocks, tw, s);
        case 4: return launch_rows_d4(kind, r, N, rl.variant, prm, geo, nitems, partial, rl.grid_blocks, tw, s);
        default: return hipErrorInvalidValue;
    }
}

// One wavefront per candidate (real ones, then npseudo constant-term
// candidates): lane 0 writes the parameter block; with wc set, the wavefront
// then counts the candidate's live segments over all rows of the half lag set
// (row_live with the moment walk's run length rl and segment length seg) into
// wc[c] for the balanced plan of the compacted walk (with seg = 1: its live
// runs, the work the compacted walk does).
template <int D>
__global__ __launch_bounds__(256) void k_scv_setup(const double* __restrict__ vechL, ScvBatchArgs a, int64_t ncand,
                                                   int npseudo, double* __restrict__ prm,
                                                   int32_t* __restrict__ status, RowGeom geo, int rl, int seg,
                                                   int32_t* __restrict__ wc) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * 4 + wave;
    const bool active = c < ncand + npseudo;
    if (active && lane == 0) {
        if (c < ncand)
            scv_params<D>(vechL, a, c, ncand, npseudo, prm + c * PRM, status);
        else
            pseudo_params<D>(a, (int)(c - ncand), prm + c * PRM);
    }
    if (!wc) return;   // grid-uniform
    __syncthreads();   // the blocks written by lane 0 are visible to the block
    if (!active) return;
    const double* p = prm + c * PRM;
    ScvFun<D, 1> f;
    f.load(p);
    double delta[D];
#pragma unroll
    for (int k = 0; k < D; ++k) delta[k] = p[S_DELTA + k];
    const int M_last = geo.M[D - 1], N = geo.P[D - 1];
    int units = 0;
    for (int64_t row = lane; row < geo.nrows; row += 64) {
        const LiveRuns lr = row_live<D>(f, row_info<D>(row, geo.nrows, geo, delta, nullptr), M_last, N, rl, delta[D - 1]);
        units += (lr.pn + seg - 1) / seg + (lr.nn + seg - 1) / seg;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) units += __shfl_xor(units, off, 64);
    if (lane == 0) wc[c] = units;
}

hipError_t launch_scv_setup(const double* vechL, const ScvBatchArgs& a, int64_t ncand, int npseudo, double* prm,
                            int32_t* status, const RowGeom& geo, int32_t* wc, hipStream_t s, bool count_runs) {
    const int64_t blocks = (ncand + npseudo + 3) / 4;
    int rl = 1, seg = 1, rows = 1;
    if (wc && !lag_layout(geo.P[geo.d - 1], 1, &rl, &seg, &rows)) return hipErrorInvalidValue;
    if (count_runs) seg = 1;   // one run per unit: wc counts the live runs
    switch (a.d) {
        case 1: hipLaunchKernelGGL(k_scv_setup<1>, dim3((unsigned)blocks), dim3(256), 0, s, vechL, a, ncand, npseudo, prm, status, geo, rl, seg, wc); break;
        case 2: hipLaunchKernelGGL(k_scv_setup<2>, dim3((unsigned)blocks), dim3(256), 0, s, vechL, a, ncand, npseudo, prm, status, geo, rl, seg, wc); break;
        case 3: hipLaunchKernelGGL(k_scv_setup<3>, dim3((unsigned)blocks), dim3(256), 0, s, vechL, a, ncand, npseudo, prm, status, geo, rl, seg, wc); break;
        case 4: hipLaunchKernelGGL(k_scv_setup<4>, dim3((unsigned)blocks), dim3(256), 0, s, vechL, a, ncand, npseudo, prm, status, geo, rl, seg, wc); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// One thread per dataset: the psi_r parameter block at its bandwidth
// (validated SPD on the host).
template <int D>
__global__ void k_psi_setup(PsiBatchArgs a, double* __restrict__ prm) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n_ds) return;
    const DsDev* dsp = a.rec[0];
    double gv[10];
    for (int t = 0; t < 10; ++t) gv[t] = a.Gv[0][t];
#pragma unroll
    for (int jj = 1; jj < KDEFFT_MAX_PSI_DS; ++jj)
        if (jj == j) {
            dsp = a.rec[jj];
#pragma unroll
            for (int t = 0; t < 10; ++t) gv[t] = a.Gv[jj][t];
        }
    psi_params<D>(gv, *dsp, a.prodP, prm + (int64_t)j * PRM);
    put_finish(prm + (int64_t)j * PRM, a.fin, j);
}

hipError_t launch_psi_setup(const PsiBatchArgs& a, double* prm, hipStream_t s) {
    switch (a.d) {
        case 1: hipLaunchKernelGGL(k_psi_setup<1>, dim3(1), dim3(64), 0, s, a, prm); break;
        case 2: hipLaunchKernelGGL(k_psi_setup<2>, dim3(1), dim3(64), 0, s, a, prm); break;
        case 3: hipLaunchKernelGGL(k_psi_setup<3>, dim3(1), dim3(64), 0, s, a, prm); break;
        case 4: hipLaunchKernelGGL(k_psi_setup<4>, dim3(1), dim3(64), 0, s, a, prm); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// The preparation header (one block: the reduction of the bound partials uses
// all its threads, the rest one thread): grid origin and spacing from the data
// bounds (same IEEE steps and order as the host planner; non-finite data give
// a NaN spacing, so every point counts as out of the grid), the record, the
// cleared counter and scalar block, and the constant-term parameter block.
template <int D>
__global__ __launch_bounds__(256) void k_ds_header(HeaderArgs h) {
#pragma clang fp contract(off)
    __shared__ double scratch[32], red[8];
    if (h.partial) reduce_bounds(h.partial, h.nblk, D, scratch, red);   // uniform branch
    if (threadIdx.x != 0) return;
    DsDev v = h.val;
    if (h.partial) {
        const double nan = __longlong_as_double(0x7ff8000000000000LL);
        for (int k = 0; k < D; ++k) {
            const double lo = red[k] - h.pad[k];
            double hi = red[4 + k] + h.pad[k];
            if (!isfinite(lo) || !isfinite(hi)) {
                v.lo[k] = nan;
                v.delta[k] = nan;
                continue;
            }
            if (!(hi > lo)) hi = lo + 1.0;
            v.lo[k] = lo;
            v.delta[k] = (hi - lo) / (double)(h.g.M[k] - 1);
        }
    }
    *h.rec = v;
    if (h.n_out) *h.n_out = 0;
    for (int k = 0; k < 4; ++k) h.scal[k] = 0.0;
    if (h.prm) {
        psi_params<D>(h.Gv2, v, h.prodP, h.prm);
        put_finish(h.prm, h.fin, 0);
    }
}

hipError_t launch_ds_header(const HeaderArgs& h, hipStream_t s) {
    switch (h.g.d) {
        case 1: hipLaunchKernelGGL(k_ds_header<1>, dim3(1), dim3(256), 0, s, h); break;
        case 2: hipLaunchKernelGGL(k_ds_header<2>, dim3(1), dim3(256), 0, s, h); break;
        case 3: hipLaunchKernelGGL(k_ds_header<3>, dim3(1), dim3(256), 0, s, h); break;
        case 4: hipLaunchKernelGGL(k_ds_header<4>, dim3(1), dim3(256), 0, s, h); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Criterion assembly, one wavefront per candidate (see crit_finish); the
// npseudo constant-term candidates after the real ones store their term in
// their dataset's scalar block.  Work items of candidate c: item_off[c] ..
// item_off[c + 1] (balanced plan) or c * nchunks + [0, nchunks).
template <int D>
__global__ __launch_bounds__(64) void k_scv_final(int kind, const double* __restrict__ partial, int64_t nchunks,
                                                  const int32_t* __restrict__ item_off, int ng,
                                                  const double* __restrict__ prm, int64_t ncand, int npseudo,
                                                  const double* __restrict__ grad_out, double* __restrict__ obj,
                                                  double* __restrict__ grad) {
    const int64_t h = blockIdx.x;
    if (h >= ncand + npseudo) return;
    auto first_of = [&](int64_t c) { return item_off ? (int64_t)item_off[c] : c * nchunks; };
    auto count_of = [&](int64_t c) { return item_off ? (int64_t)(item_off[c + 1] - item_off[c]) : nchunks; };
    const double* p = prm + h * PRM;
    if (h >= ncand) {
        const double v = item_sum(partial, first_of(h), count_of(h), ng, 0) * p[S_SCALE];
        if (threadIdx.x == 0) static_cast<double*>(slot_ptr(p[S_FIN_SCAL]))[0] = v;
        return;
    }
    double cst = 0.0;
    if (p[S_PSEUDO] >= 0.0) {
        const int64_t c = (int64_t)p[S_PSEUDO];
        cst = item_sum(partial, first_of(c), count_of(c), ng, 0) * prm[c * PRM + S_SCALE];
    }
    crit_finish<D>(kind, partial, first_of(h), count_of(h), ng, p, h, cst, grad_out, obj, grad);
}

hipError_t launch_scv_final(int kind, const double* partial, const RowGeom& geo, const double* prm, int64_t ncand,
                            int npseudo, const double* grad_out, double* obj, double* grad, hipStream_t s) {
    const int ng = ng_of(kind, geo.d, 2);
    const dim3 grid((unsigned)(ncand + npseudo));
    const int32_t* off = geo.nplan > 0 ? geo.item_off : nullptr;
    switch (geo.d) {
        case 1: hipLaunchKernelGGL(k_scv_final<1>, grid, dim3(64), 0, s, kind, partial, geo.nchunks, off, ng, prm, ncand, npseudo, grad_out, obj, grad); break;
        case 2: hipLaunchKernelGGL(k_scv_final<2>, grid, dim3(64), 0, s, kind, partial, geo.nchunks, off, ng, prm, ncand, npseudo, grad_out, obj, grad); break;
        case 3: hipLaunchKernelGGL(k_scv_final<3>, grid, dim3(64), 0, s, kind, partial, geo.nchunks, off, ng, prm, ncand, npseudo, grad_out, obj, grad); break;
        case 4: hipLaunchKernelGGL(k_scv_final<4>, grid, dim3(64), 0, s, kind, partial, geo.nchunks, off, ng, prm, ncand, npseudo, grad_out, obj, grad); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Position of each Kronecker-ordered 4-index (i, j, k, l) (first slowest)
// among the unique entries: sorted tuples in lexicographic order (Sec. 5).
template <int D>
struct Kron4 {
    int u[D * D * D * D];
    static constexpr Kron4 make() {
        Kron4 t{};
        int code[256] = {};
        int cnt = 0;
        for (int a = 0; a < D; ++a)
            for (int b = a; b < D; ++b)
                for (int c = b; c < D; ++c)
                    for (int e = c; e < D; ++e) code[((a * D + b) * D + c) * D + e] = cnt++;
        for (int f = 0; f < D * D * D * D; ++f) {
            int v[4] = {f / (D * D * D), (f / (D * D)) % D, (f / D) % D, f % D};
            for (int x = 0; x < 4; ++x)
                for (int y = 0; y + 1 < 4 - x; ++y)
                    if (v[y] > v[y + 1]) { const int tmp = v[y]; v[y] = v[y + 1]; v[y + 1] = tmp; }
            t.u[f] = code[((v[0] * D + v[1]) * D + v[2]) * D + v[3]];
        }
        return t;
    }
};

// Plug-in criterion, one thread per candidate:
//   PI(H) = n^-1 (4 pi)^{-d/2} |H|^{-1/2} + 1/4 sum_{ijkl} H_ij H_kl psi_ijkl,
//   grad_H = -1/2 (first term) H^{-1} + 1/2 sum_kl psi_ijkl H_kl,
// chained to vech(L) by dPI/dL = lower(2 grad_H L).
template <int D>
__global__ void k_pi(PiArgs a, const double* __restrict__ psi4, const double* __restrict__ vechL, int64_t ncand,
                     double* __restrict__ obj, double* __restrict__ grad, int32_t* __restrict__ status) {
    const int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (h >= ncand) return;
    constexpr int d = D, q = D * (D + 1) / 2, NU = (D + 3) * (D + 2) * (D + 1) * D / 24;
    constexpr Kron4<D> K = Kron4<D>::make();
    int ds = 0;
    double n = a.n[0];
#pragma unroll
    for (int jj = 1; jj < KDEFFT_MAX_BATCH_DS; ++jj)
        if (jj < a.n_ds && h >= a.off[jj]) { ds = jj; n = a.n[jj]; }
    const double* ps = psi4 + (int64_t)ds * NU;
    double L[16], H[16];
    for (int i = 0; i < 16; ++i) L[i] = 0.0;
    int t = 0;
    bool sing = false;
    for (int jj = 0; jj < d; ++jj)
        for (int i = jj; i < d; ++i) {
            const double v = vechL[h * q + t++];
            L[i * 4 + jj] = v;
            if (!isfinite(v) || (i == jj && v == 0.0)) sing = true;
        }
    for (int i = 0; i < d; ++i)
        for (int k2 = 0; k2 < d; ++k2) {
            double s = 0.0;
            for (int k = 0; k < d; ++k) s += L[i * 4 + k] * L[k2 * 4 + k];
            H[i * 4 + k2] = s;
        }
    double ldet = 1.0;
    for (int k = 0; k < d; ++k) ldet *= fabs(L[k * 4 + k]);
    double c4 = 1.0;  // (4 pi)^{-d/2}
    for (int k = 0; k < d; ++k) c4 *= 0.28209479177387814347;
    const double first = sing ? 0.0 : c4 / (n * ldet);
    // M_ij = sum_kl psi_ijkl H_kl
    double Mq[16];
    double quad = 0.0;
#pragma unroll
    for (int i = 0; i < d; ++i)
#pragma unroll
        for (int j = 0; j < d; ++j) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < d; ++k)
#pragma unroll
                for (int l = 0; l < d; ++l) s += ps[K.u[((i * D + j) * D + k) * D + l]] * H[k * 4 + l];
            Mq[i * 4 + j] = s;
            quad += H[i * 4 + j] * s;
        }
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    if (status) status[h] = sing ? 1 : 0;
    if (obj) obj[h] = sing ? nan : first + 0.25 * quad;
    if (!grad) return;
    double Hinv[16];
    if (!sing) {
        chol_inv4<D>(L, Hinv);
    } else {
        for (int i = 0; i < 16; ++i) Hinv[i] = 0.0;
    }
    double gH[16];
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) gH[i * 4 + j] = -0.5 * first * Hinv[i * 4 + j] + 0.5 * Mq[i * 4 + j];
    int o = 0;
    for (int j = 0; j < d; ++j)
        for (int i = j; i < d; ++i) {
            double s = 0.0;
            for (int k = 0; k < d; ++k) s += gH[i * 4 + k] * L[k * 4 + j];
            grad[h * q + o++] = sing ? nan : 2.0 * s;
        }
}

hipError_t launch_pi(const PiArgs& a, const double* psi4, const double* vechL, int64_t ncand, double* obj,
                     double* grad, int32_t* status, hipStream_t s) {
    const int64_t blocks = (ncand + 63) / 64;
    switch (a.d) {
        case 1: hipLaunchKernelGGL(k_pi<1>, dim3((unsigned)blocks), dim3(64), 0, s, a, psi4, vechL, ncand, obj, grad, status); break;
        case 2: hipLaunchKernelGGL(k_pi<2>, dim3((unsigned)blocks), dim3(64), 0, s, a, psi4, vechL, ncand, obj, grad, status); break;
        case 3: hipLaunchKernelGGL(k_pi<3>, dim3((unsigned)blocks), dim3(64), 0, s, a, psi4, vechL, ncand, obj, grad, status); break;
        case 4: hipLaunchKernelGGL(k_pi<4>, dim3((unsigned)blocks), dim3(64), 0, s, a, psi4, vechL, ncand, obj, grad, status); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// psi[h, g] = scale_h * sum over chunks (fixed order), one wavefront per
// (candidate, grid); scal_out (if set) receives psi[0, 0] (the constant SCV
// term of a dataset).
__global__ __launch_bounds__(64) void k_psi_final(const double* __restrict__ partial, int64_t nchunks, int ng,
                                                  const double* __restrict__ prm, int64_t ncand,
                                                  double* __restrict__ psi, double* __restrict__ scal_out) {
    const int64_t e = blockIdx.x;
    if (e >= ncand * ng) return;
    const int64_t h = e / ng;
    psi_finish(partial, nchunks, ng, prm + h * PRM, h, (int)(e - h * ng), psi, scal_out);
}

hipError_t launch_psi_final(const double* partial, const RowGeom& geo, int ng, const double* prm, int64_t ncand,
                            double* psi, double* scal_out, hipStream_t s) {
    hipLaunchKernelGGL(k_psi_final, dim3((unsigned)(ncand * ng)), dim3(64), 0, s, partial, geo.nchunks, ng, prm,
                       ncand, psi, scal_out);
    return hipGetLastError();
}

}  // namespace kdefft
