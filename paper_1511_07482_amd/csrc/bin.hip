// Step 1 of Sec. 4: data bounds, linear binning into int64 fixed-point counts,
// and the zero-padded real count array of the circular layout.
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "internal.h"
#include "params.h"

namespace kdefft {

// ------------------------------------------------------------------ bounds
// Per-block min/max of each column of X [n, D] into partial[block * 8 + k]
// (min) and partial[block * 8 + 4 + k] (max); min/max are exact, so the
// result does not depend on the reduction order.  Also clears zero16 16-byte
// words at zero_ptr (the binning's scratch), so the preparation needs no
// separate clearing launch.
template <int D>
__global__ __launch_bounds__(256) void k_bounds(const double* __restrict__ X, int64_t n,
                                                double* __restrict__ partial, uint4* __restrict__ zero_ptr,
                                                int64_t zero16, int32_t* __restrict__ n_out,
                                                double* __restrict__ scal) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < zero16; i += stride) zero_ptr[i] = make_uint4(0, 0, 0, 0);
    if (blockIdx.x == 0 && threadIdx.x < 4) {   // the dataset's out-of-grid counter and scalar block
        if (n_out && threadIdx.x == 0) *n_out = 0;
        if (scal) scal[threadIdx.x] = 0.0;
    }
    double mn[D], mx[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        mn[k] = INFINITY;
        mx[k] = -INFINITY;
    }
    // unrolled so that a thread's loads are in flight together
#pragma unroll 4
    for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += stride) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double v = X[i * D + k];
            mn[k] = fmin(mn[k], v);
            mx[k] = fmax(mx[k], v);
        }
    }
    __shared__ double sw[4][8];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < D; ++k) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            mn[k] = fmin(mn[k], __shfl_xor(mn[k], off, 64));
            mx[k] = fmax(mx[k], __shfl_xor(mx[k], off, 64));
        }
        if (lane == 0) {
            sw[wid][k] = mn[k];
            sw[wid][4 + k] = mx[k];
        }
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)D) {
        const int k = threadIdx.x;
        double a = sw[0][k], b = sw[0][4 + k];
        for (int w = 1; w < 4; ++w) {
            a = fmin(a, sw[w][k]);
            b = fmax(b, sw[w][4 + k]);
        }
        partial[blockIdx.x * 8 + k] = a;
        partial[blockIdx.x * 8 + 4 + k] = b;
    }
}

// Reduction of the per-block partials into out (min[4], max[4]); one block.
__global__ __launch_bounds__(256) void k_bounds_final(const double* __restrict__ partial, int nblk, int d,
                                                      double* __restrict__ out) {
    __shared__ double scratch[32], red[8];
    reduce_bounds(partial, nblk, d, scratch, red);
    if (threadIdx.x < (unsigned)d) {
        out[threadIdx.x] = red[threadIdx.x];
        out[4 + threadIdx.x] = red[4 + threadIdx.x];
    }
}

hipError_t launch_bounds_partial(const double* X, int64_t n, int d, double* partial, int nblk, hipStream_t s,
                                 void* zero_ptr, size_t zero_bytes, int32_t* n_out, double* scal) {
    if (zero_bytes % 16 || (reinterpret_cast<uintptr_t>(zero_ptr) & 15)) return hipErrorInvalidValue;
    uint4* z = static_cast<uint4*>(zero_ptr);
    const int64_t z16 = (int64_t)(zero_bytes / 16);
    switch (d) {
        case 1: hipLaunchKernelGGL(k_bounds<1>, dim3(nblk), dim3(256), 0, s, X, n, partial, z, z16, n_out, scal); break;
        case 2: hipLaunchKernelGGL(k_bounds<2>, dim3(nblk), dim3(256), 0, s, X, n, partial, z, z16, n_out, scal); break;
        case 3: hipLaunchKernelGGL(k_bounds<3>, dim3(nblk), dim3(256), 0, s, X, n, partial, z, z16, n_out, scal); break;
        case 4: hipLaunchKernelGGL(k_bounds<4>, dim3(nblk), dim3(256), 0, s, X, n, partial, z, z16, n_out, scal); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_bounds(const double* X, int64_t n, int d, double* partial, int nblk, double* out,
                         hipStream_t s) {
    hipError_t e = launch_bounds_partial(X, n, d, partial, nblk, s, nullptr, 0, nullptr, nullptr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bounds_final, dim3(1), dim3(256), 0, s, partial, nblk, d, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ zero fill
// Zero `bytes` bytes (a multiple of 4) with 32-bit vector stores.
__global__ void k_zero(uint32_t* __restrict__ p, int64_t words) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    if (bytes % 4) return hipErrorInvalidValue;
    const int64_t words = (int64_t)(bytes / 4);
    if (words == 0) return hipSuccess;
    int64_t blocks = (words + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<uint32_t*>(p), words);
    return hipGetLastError();
}

// ------------------------------------------------------------------ linear binning
// Fixed-point contract (one thread per point):
//   t_k = (x_k - lo_k) / delta_k; skip unless 0 <= t_k <= M_k - 1
//   j_k = floor(t_k) (M_k - 1 -> M_k - 2); f_k = t_k - j_k; weights (1 - f_k, f_k)
//   corner weight = left-to-right product over axes; q = rint(w * 2^40)
//   the largest corner (lowest number on ties) takes 2^40 - sum of the others.
// Floating-point contraction is disabled so that every step is one IEEE
// operation, as on the host.
// slots != 0: the increments go to the corner slots of the last min(D, 3)
// axes (a record of 2^min(D, 3) int64 per cell), so that a point's 2^D
// increments fall in 2^max(D-3, 0) contiguous records; the count transform's
// first pass gathers the counts from the slots (exactly, in integers) while
// it reads them.  slots == 0: straight into the count grid.
//
// Scattered 64-bit atomics cost one memory-side request per distinct cache
// line per instruction, so after the per-point arithmetic the wavefront's
// 64 x 2^D corner increments are re-dealt through LDS: instruction `it` gives
// lane l the increment number it * 64 + l, i.e. point (it * 64 + l) / 2^D and
// corner (it * 64 + l) % 2^D in an order whose consecutive corners differ in
// the last (contiguous) axis, so neighbouring lanes add to adjacent bins of
// the grid (2^(D-1) cache lines per point), or, with the corner slots, to one
// record per 2^min(D, 3) lanes (one cache line per point, two for D = 4).
// Grid origin and spacing from the data bounds (per-block partials of the
// bounds kernel), by the same IEEE steps and order as the host planner:
// lo = min - pad, hi = max + pad, hi = lo + 1 for a degenerate axis,
// delta = (hi - lo) / (M - 1); non-finite data give a NaN spacing, so every
// point counts as out of the grid.  Called by all threads of a block.
template <int D>
__device__ __forceinline__ void grid_from_bounds(const HeaderArgs& h, double* lo, double* delta) {
#pragma clang fp contract(off)
    __shared__ double scratch[32], red[8], sg[8];
    reduce_bounds(h.partial, h.nblk, D, scratch, red);
    if (threadIdx.x < (unsigned)D) {
        const int k = threadIdx.x;
        const double nan = __longlong_as_double(0x7ff8000000000000LL);
        const double l = red[k] - h.pad[k];
        double hi = red[4 + k] + h.pad[k];
        if (!isfinite(l) || !isfinite(hi)) {
            sg[k] = nan;
            sg[4 + k] = nan;
        } else {
            if (!(hi > l)) hi = l + 1.0;
            sg[k] = l;
            sg[4 + k] = (hi - l) / (double)(h.g.M[k] - 1);
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < D; ++k) {
        lo[k] = sg[k];
        delta[k] = sg[4 + k];
    }
}

// hdr.partial set: the dataset header is computed here, not by a separate
// launch: every block derives the grid origin and spacing from the bound
// partials (grid_from_bounds), and block 0 writes the dataset record and the
// parameter block of the constant SCV term for the later launches.
template <int D>
__global__ __launch_bounds__(256) void k_linbin(const double* __restrict__ X, int64_t n, kdefft_grid g,
                                                const double* __restrict__ gdev,
                                                unsigned long long* __restrict__ counts,
                                                int32_t* __restrict__ n_out, int slots, HeaderArgs hdr) {
#pragma clang fp contract(off)
    constexpr int NC = 1 << D;
    __shared__ long long qs[256 * NC];   // increments, per wavefront in issue order
    __shared__ int64_t fbs[256];         // flat index of each point's lowest corner
    if (gdev) {   // origin and spacing computed on the device
#pragma unroll
        for (int k = 0; k < D; ++k) {
            g.lo[k] = gdev[k];
            g.delta[k] = gdev[4 + k];
        }
    }
    if (hdr.partial) {   // block-uniform
        grid_from_bounds<D>(hdr, g.lo, g.delta);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            DsDev v = hdr.val;
            for (int k = 0; k < D; ++k) {
                v.lo[k] = g.lo[k];
                v.delta[k] = g.delta[k];
            }
            *hdr.rec = v;
            if (hdr.prm) {
                psi_params<D>(hdr.Gv2, v, hdr.prodP, hdr.prm);
                put_finish(hdr.prm, hdr.fin, 0);
            }
        }
    }
    int64_t stride[D];
    stride[D - 1] = 1;
#pragma unroll
    for (int k = D - 2; k >= 0; --k) stride[k] = stride[k + 1] * g.M[k + 1];
    const int lane = threadIdx.x & 63, w0ff = threadIdx.x & ~63;
    const double one_q = 1099511627776.0;  // 2^40
    for (int64_t i0 = blockIdx.x * 256LL; i0 < n; i0 += (int64_t)gridDim.x * 256) {   // block-uniform
        const int64_t i = i0 + threadIdx.x;
        long long q[NC];
#pragma unroll
        for (int b = 0; b < NC; ++b) q[b] = 0;
        int64_t fb = 0;
        if (i < n) {
            double w0[D], w1[D];
            int64_t j[D];
            bool ok = true;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double t = (X[i * D + k] - g.lo[k]) / g.delta[k];
                ok = ok && (t >= 0.0) && (t <= (double)(g.M[k] - 1));
                double jf = floor(t);
                if (jf == (double)(g.M[k] - 1)) jf = (double)(g.M[k] - 2);
                const double f = t - jf;
                w0[k] = 1.0 - f;
                w1[k] = f;
                j[k] = (int64_t)jf;
            }
            if (!ok) {
                if (n_out) atomicAdd(n_out, 1);
            } else {
                // corner b: bit k set = upper node along axis k
                int best = 0;
#pragma unroll
                for (int b = 0; b < NC; ++b) {
                    double w = (b & 1) ? w1[0] : w0[0];
#pragma unroll
                    for (int k = 1; k < D; ++k) w = w * (((b >> k) & 1) ? w1[k] : w0[k]);
                    q[b] = (long long)rint(w * one_q);
                    if (q[b] > q[best]) best = b;
                }
                long long rest = 0;
#pragma unroll
                for (int b = 0; b < NC; ++b)
                    if (b != best) rest += q[b];
                q[best] = (1LL << 40) - rest;
#pragma unroll
                for (int k = 0; k < D; ++k) fb += j[k] * stride[k];
            }
        }
        // issue order c = bit-reversed b: bit 0 of c is the last axis
#pragma unroll
        for (int b = 0; b < NC; ++b) {
            int c = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) c |= ((b >> k) & 1) << (D - 1 - k);
            qs[w0ff * NC + lane * NC + c] = q[b];
        }
        fbs[threadIdx.x] = fb;
        __syncthreads();
#pragma unroll
        for (int it = 0; it < NC; ++it) {
            const int a = it * 64 + lane;
            const int pnt = a / NC, c = a % NC;
            const long long v = qs[w0ff * NC + a];
            if (v != 0) {
                if (slots) {
                    // record: the lowest corner moved along the unslotted
                    // leading axes of corner c; slot: c's bits of the slotted axes
                    constexpr int NSA = slot_axes(D), NS = corner_slots(D);
                    int64_t off = 0;
#pragma unroll
                    for (int k = 0; k + NSA < D; ++k) off += ((c >> (D - 1 - k)) & 1) * stride[k];
                    atomicAdd(counts + (fbs[w0ff + pnt] + off) * NS + (c & (NS - 1)), (unsigned long long)v);
                } else {
                    int64_t off = 0;
#pragma unroll
                    for (int k = 0; k < D; ++k) off += ((c >> (D - 1 - k)) & 1) * stride[k];
                    atomicAdd(counts + fbs[w0ff + pnt] + off, (unsigned long long)v);
                }
            }
        }
        __syncthreads();
    }
}

hipError_t launch_linbin_slots(const double* X, int64_t n, const kdefft_grid& g, int64_t* slots, int32_t* n_out,
                               hipStream_t s, const double* gdev, bool slots_zeroed, const HeaderArgs* hdr) {
    int64_t prodM = 1;
    for (int k = 0; k < g.d; ++k) prodM *= g.M[k];
    hipError_t e = hipSuccess;
    if (!slots_zeroed) {
        e = launch_zero(slots, (size_t)(corner_slots(g.d) * prodM) * sizeof(int64_t), s);
        if (e != hipSuccess) return e;
    }
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    auto* c = reinterpret_cast<unsigned long long*>(slots);
    HeaderArgs h{};
    if (hdr) h = *hdr;
    switch (g.d) {
        case 1: hipLaunchKernelGGL(k_linbin<1>, dim3((unsigned)blocks), dim3(256), 0, s, X, n, g, gdev, c, n_out, 1, h); break;
        case 2: hipLaunchKernelGGL(k_linbin<2>, dim3((unsigned)blocks), dim3(256), 0, s, X, n, g, gdev, c, n_out, 1, h); break;
        case 3: hipLaunchKernelGGL(k_linbin<3>, dim3((unsigned)blocks), dim3(256), 0, s, X, n, g, gdev, c, n_out, 1, h); break;
        case 4: hipLaunchKernelGGL(k_linbin<4>, dim3((unsigned)blocks), dim3(256), 0, s, X, n, g, gdev, c, n_out, 1, h); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_linbin(const double* X, int64_t n, const kdefft_grid& g, int64_t* counts, int32_t* n_out,
                         hipStream_t s, const double* gdev) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    auto* c = reinterpret_cast<unsigned long long*>(counts);
    const HeaderArgs h{};
    switch (g.d) {
        case 1: hipLaunchKernelGGL(k_linbin<1>, dim3((unsigned)blocks), dim3(256), 0, s, X, n, g, gdev, c, n_out, 0, h); break;
        case 2: hipLaunchKernelGGL(k_linbin<2>, dim3((unsigned)blocks), dim3(256), 0, s, X, n, g, gdev, c, n_out, 0, h); break;
        case 3: hipLaunchKernelGGL(k_linbin<3>, dim3((unsigned)blocks), dim3(256), 0, s, X, n, g, gdev, c, n_out, 0, h); break;
        case 4: hipLaunchKernelGGL(k_linbin<4>, dim3((unsigned)blocks), dim3(256), 0, s, X, n, g, gdev, c, n_out, 0, h); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ counts -> c_zp
// Real array of the circular layout: c at [0, M)^d, zero elsewhere in P^d.
template <int D>
__global__ void k_fill_czp(const int64_t* __restrict__ counts, kdefft_grid g, int64_t total,
                           double* __restrict__ czp) {
    const double quantum = 9.094947017729282379150390625e-13;  // 2^-40
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int64_t rem = e, cflat = 0;
        bool in = true;
        int idx[D];
#pragma unroll
        for (int k = D - 1; k >= 0; --k) {
            idx[k] = (int)(rem % g.P[k]);
            rem /= g.P[k];
            in = in && idx[k] < g.M[k];
        }
        if (in) {
#pragma unroll
            for (int k = 0; k < D; ++k) cflat = cflat * g.M[k] + idx[k];
            czp[e] = (double)counts[cflat] * quantum;
        } else {
            czp[e] = 0.0;
        }
    }
}

hipError_t launch_fill_czp(const int64_t* counts, const kdefft_grid& g, double* czp, hipStream_t s) {
    int64_t total = 1;
    for (int k = 0; k < g.d; ++k) total *= g.P[k];
    int64_t blocks = (total + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    switch (g.d) {
        case 1: hipLaunchKernelGGL(k_fill_czp<1>, dim3((unsigned)blocks), dim3(256), 0, s, counts, g, total, czp); break;
        case 2: hipLaunchKernelGGL(k_fill_czp<2>, dim3((unsigned)blocks), dim3(256), 0, s, counts, g, total, czp); break;
        case 3: hipLaunchKernelGGL(k_fill_czp<3>, dim3((unsigned)blocks), dim3(256), 0, s, counts, g, total, czp); break;
        case 4: hipLaunchKernelGGL(k_fill_czp<4>, dim3((unsigned)blocks), dim3(256), 0, s, counts, g, total, czp); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace kdefft
