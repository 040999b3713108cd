// Step 1 of Sec. 4: data bounds, linear binning into int64 fixed-point counts,
// and the zero-padded real count array of the circular layout.
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "internal.h"

namespace kdefft {

// ------------------------------------------------------------------ bounds
// Per-block min/max of each column of X [n, d]; min/max are exact, so the
// result does not depend on the reduction order.
// Also clears zero_words 32-bit words at zero_ptr (the binning's scratch), so
// the preparation needs no separate clearing launch.
__global__ __launch_bounds__(256) void k_bounds(const double* __restrict__ X, int64_t n, int d,
                                                double* __restrict__ partial, uint32_t* __restrict__ zero_ptr,
                                                int64_t zero_words) {
    for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < zero_words; i += (int64_t)gridDim.x * 256)
        zero_ptr[i] = 0u;
    __shared__ double smin[4][256], smax[4][256];
    double mn[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
    double mx[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        for (int k = 0; k < d; ++k) {
            const double v = X[i * d + k];
            mn[k] = fmin(mn[k], v);
            mx[k] = fmax(mx[k], v);
        }
    }
    for (int k = 0; k < 4; ++k) {
        smin[k][threadIdx.x] = mn[k];
        smax[k][threadIdx.x] = mx[k];
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int k = 0; k < 4; ++k) {
                smin[k][threadIdx.x] = fmin(smin[k][threadIdx.x], smin[k][threadIdx.x + s]);
                smax[k][threadIdx.x] = fmax(smax[k][threadIdx.x], smax[k][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x < (unsigned)d) {
        partial[blockIdx.x * 8 + threadIdx.x] = smin[threadIdx.x][0];
        partial[blockIdx.x * 8 + 4 + threadIdx.x] = smax[threadIdx.x][0];
    }
}

__global__ __launch_bounds__(256) void k_bounds_final(const double* __restrict__ partial, int nblk, int d,
                                                      double* __restrict__ out) {
    __shared__ double smin[4][256], smax[4][256];
    for (int k = 0; k < 4; ++k) {
        double mn = INFINITY, mx = -INFINITY;
        if (k < d)
            for (int b = threadIdx.x; b < nblk; b += 256) {
                mn = fmin(mn, partial[b * 8 + k]);
                mx = fmax(mx, partial[b * 8 + 4 + k]);
            }
        smin[k][threadIdx.x] = mn;
        smax[k][threadIdx.x] = mx;
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int k = 0; k < 4; ++k) {
                smin[k][threadIdx.x] = fmin(smin[k][threadIdx.x], smin[k][threadIdx.x + s]);
                smax[k][threadIdx.x] = fmax(smax[k][threadIdx.x], smax[k][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x < (unsigned)d) {
        out[threadIdx.x] = smin[threadIdx.x][0];
        out[4 + threadIdx.x] = smax[threadIdx.x][0];
    }
}

hipError_t launch_bounds(const double* X, int64_t n, int d, double* partial, int nblk, double* out,
                         hipStream_t s, void* zero_ptr, size_t zero_bytes) {
    if (zero_bytes % 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bounds, dim3(nblk), dim3(256), 0, s, X, n, d, partial, static_cast<uint32_t*>(zero_ptr),
                       (int64_t)(zero_bytes / 4));
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
// Index of the accelerator complex die (XCD) the wavefront runs on.
__device__ __forceinline__ unsigned xcd_id() {
    unsigned v;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(v));
    return v;
}

// copy_stride > 0: the counts are accumulated into XCD_COPIES grids of
// copy_stride bins, one per XCD (chosen by the die the block runs on), so the
// atomics of different dies never meet; k_sum_copies adds them afterwards.
template <int D>
__global__ __launch_bounds__(256) void k_linbin(const double* __restrict__ X, int64_t n, kdefft_grid g,
                                                const double* __restrict__ gdev,
                                                unsigned long long* __restrict__ counts,
                                                int32_t* __restrict__ n_out, int64_t copy_stride) {
#pragma clang fp contract(off)
    constexpr int NC = 1 << D;
    if (copy_stride > 0) counts += (int64_t)(xcd_id() % XCD_COPIES) * copy_stride;
    if (gdev) {   // origin and spacing computed on the device
#pragma unroll
        for (int k = 0; k < D; ++k) {
            g.lo[k] = gdev[k];
            g.delta[k] = gdev[4 + k];
        }
    }
    const double one_q = 1099511627776.0;  // 2^40
    for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
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
            continue;
        }
        long long q[NC];
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
        for (int b = 0; b < NC; ++b) {
            if (q[b] == 0) continue;
            int64_t flat = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) flat = flat * g.M[k] + j[k] + ((b >> k) & 1);
            atomicAdd(counts + flat, (unsigned long long)q[b]);
        }
    }
}

__global__ __launch_bounds__(256) void k_sum_copies(const unsigned long long* __restrict__ copies, int64_t stride,
                                                    unsigned long long* __restrict__ counts) {
    for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < stride; i += (int64_t)gridDim.x * 256) {
        unsigned long long t = 0;
#pragma unroll
        for (int c = 0; c < XCD_COPIES; ++c) t += copies[c * stride + i];
        counts[i] = t;
    }
}

hipError_t launch_linbin_xcd(const double* X, int64_t n, const kdefft_grid& g, int64_t* counts, int64_t* copies,
                             int32_t* n_out, hipStream_t s, const double* gdev, bool copies_zeroed) {
    int64_t prodM = 1;
    for (int k = 0; k < g.d; ++k) prodM *= g.M[k];
    hipError_t e = hipSuccess;
    if (!copies_zeroed) {
        e = launch_zero(copies, (size_t)(XCD_COPIES * prodM) * sizeof(int64_t), s);
        if (e != hipSuccess) return e;
    }
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    auto* c = reinterpret_cast<unsigned long long*>(copies);
    switch (g.d) {
        case 1: hipLaunchKernelGGL(k_linbin<1>, dim3((unsigned)blocks), dim3(256), 0, s, X, n, g, gdev, c, n_out, prodM); break;
        case 2: hipLaunchKernelGGL(k_linbin<2>, dim3((unsigned)blocks), dim3(256), 0, s, X, n, g, gdev, c, n_out, prodM); break;
        case 3: hipLaunchKernelGGL(k_linbin<3>, dim3((unsigned)blocks), dim3(256), 0, s, X, n, g, gdev, c, n_out, prodM); break;
        case 4: hipLaunchKernelGGL(k_linbin<4>, dim3((unsigned)blocks), dim3(256), 0, s, X, n, g, gdev, c, n_out, prodM); break;
        default: return hipErrorInvalidValue;
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    int64_t sb = (prodM + 255) / 256;
    if (sb > 4096) sb = 4096;
    hipLaunchKernelGGL(k_sum_copies, dim3((unsigned)sb), dim3(256), 0, s, c, prodM,
                       reinterpret_cast<unsigned long long*>(counts));
    return hipGetLastError();
}

hipError_t launch_linbin(const double* X, int64_t n, const kdefft_grid& g, int64_t* counts, int32_t* n_out,
                         hipStream_t s, const double* gdev) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    auto* c = reinterpret_cast<unsigned long long*>(counts);
    switch (g.d) {
        case 1: hipLaunchKernelGGL(k_linbin<1>, dim3((unsigned)blocks), dim3(256), 0, s, X, n, g, gdev, c, n_out, (int64_t)0); break;
        case 2: hipLaunchKernelGGL(k_linbin<2>, dim3((unsigned)blocks), dim3(256), 0, s, X, n, g, gdev, c, n_out, (int64_t)0); break;
        case 3: hipLaunchKernelGGL(k_linbin<3>, dim3((unsigned)blocks), dim3(256), 0, s, X, n, g, gdev, c, n_out, (int64_t)0); break;
        case 4: hipLaunchKernelGGL(k_linbin<4>, dim3((unsigned)blocks), dim3(256), 0, s, X, n, g, gdev, c, n_out, (int64_t)0); break;
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
