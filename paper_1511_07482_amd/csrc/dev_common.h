// Device-side building blocks shared by the kdefft kernels (gfx950, wave64).
//
// * double2 complex helpers;
// * an LDS-resident Stockham FFT (radix 8/4/2 stages, unnormalised, sign -1
//   forward / +1 inverse) over a batch of pencils, with twiddles read from a
//   table e^{-2 pi i m / TWN}, m < TWN (plus contiguous copies of its
//   N-point subsets), computed once per device on the host;
// * deterministic block reductions (wave64 xor-shuffles then a fixed-order
//   pass over the waves).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kdefft {

constexpr int TWN = 4096;  // twiddle table length = largest supported transform

// ------------------------------------------------------------------ complex
__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 c_mul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ double2 c_mulc(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ double2 c_conj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 c_scale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// multiply by -i (DIR < 0) or +i (DIR > 0)
template <int DIR>
__device__ __forceinline__ double2 c_rot(double2 a) {
    return DIR < 0 ? make_double2(a.y, -a.x) : make_double2(-a.y, a.x);
}

// ------------------------------------------------------------------ small DFTs
template <int DIR>
__device__ __forceinline__ void dft2(double2* v) {
    double2 t = v[0];
    v[0] = c_add(t, v[1]);
    v[1] = c_sub(t, v[1]);
}

template <int DIR>
__device__ __forceinline__ void dft4(double2& a0, double2& a1, double2& a2, double2& a3) {
    double2 t0 = c_add(a0, a2), t1 = c_sub(a0, a2);
    double2 t2 = c_add(a1, a3), t3 = c_rot<DIR>(c_sub(a1, a3));
    a0 = c_add(t0, t2);
    a2 = c_sub(t0, t2);
    a1 = c_add(t1, t3);
    a3 = c_sub(t1, t3);
}

template <int DIR>
__device__ __forceinline__ void dft4(double2* v) { dft4<DIR>(v[0], v[1], v[2], v[3]); }

template <int DIR>
__device__ __forceinline__ void dft8(double2* v) {
    constexpr double c = 0.70710678118654752440;  // sqrt(1/2)
    double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    double2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<DIR>(e0, e1, e2, e3);
    dft4<DIR>(o0, o1, o2, o3);
    // o_k *= e^{DIR 2 pi i k / 8}
    double2 w1, w3;
    if (DIR < 0) {
        w1 = make_double2(c * (o1.x + o1.y), c * (o1.y - o1.x));
        w3 = make_double2(c * (o3.y - o3.x), -c * (o3.x + o3.y));
    } else {
        w1 = make_double2(c * (o1.x - o1.y), c * (o1.x + o1.y));
        w3 = make_double2(-c * (o3.x + o3.y), c * (o3.x - o3.y));
    }
    double2 w2 = c_rot<DIR>(o2);
    v[0] = c_add(e0, o0);
    v[4] = c_sub(e0, o0);
    v[1] = c_add(e1, w1);
    v[5] = c_sub(e1, w1);
    v[2] = c_add(e2, w2);
    v[6] = c_sub(e2, w2);
    v[3] = c_add(e3, w3);
    v[7] = c_sub(e3, w3);
}

template <int R, int DIR>
__device__ __forceinline__ void dft(double2* v) {
    if constexpr (R == 2) dft2<DIR>(v);
    else if constexpr (R == 4) dft4<DIR>(v);
    else dft8<DIR>(v);
}

// ------------------------------------------------------------------ radix plan
__host__ __device__ constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n >> 1); }

// Radix of the next Stockham stage when `rem` points remain to be combined.
// SCHED 0: as many radix-8 stages as possible (4x4 instead of 8x2);
// SCHED 1: radix-4 stages, one radix-8 (or 2) when log2 is odd.
__host__ __device__ constexpr int next_radix(int rem, int sched) {
    return sched == 0
               ? (rem == 2 ? 2 : (ilog2c(rem) % 3 == 0 ? 8 : 4))
               : (rem == 2 ? 2 : (ilog2c(rem) % 2 == 0 ? 4 : 8));
}

// One radix-R Stockham stage, in place in LDS, on NPEN pencils of length N
// (pencil p starts at buf + p * ps).  L = length of the sub-transforms
// already formed.  Every thread first reads all its butterflies into
// registers, then the block synchronises and writes them back.  tw holds
// e^{-2 pi i j / TL} for j < TL (the device table, TL = TWN, or a copy of the
// N-point subset in LDS, TL = N or a multiple of it).
template <int N, int R, int L, int NPEN, int NT, int DIR, int TL = TWN>
__device__ __forceinline__ void stockham_stage(double2* buf, int ps, const double2* __restrict__ tw) {
    constexpr int NB = N / R;
    constexpr int TOT = NB * NPEN;
    constexpr int PER = (TOT + NT - 1) / NT;
    constexpr int TWS = TL / (R * L);
    double2 v[PER][R];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int b = threadIdx.x + u * NT;
        if ((TOT % NT) == 0 || b < TOT) {
            const int p = b / NB, i = b - p * NB;
            const int k = i & (L - 1);
            const double2* src = buf + p * ps + i;
#pragma unroll
            for (int m = 0; m < R; ++m) v[u][m] = src[m * NB];
            if constexpr (L > 1) {
#pragma unroll
                for (int m = 1; m < R; ++m) {
                    const double2 w = tw[m * k * TWS];
                    v[u][m] = DIR < 0 ? c_mul(v[u][m], w) : c_mulc(v[u][m], w);
                }
            }
            dft<R, DIR>(v[u]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int b = threadIdx.x + u * NT;
        if ((TOT % NT) == 0 || b < TOT) {
            const int p = b / NB, i = b - p * NB;
            const int k = i & (L - 1);
            double2* dst = buf + p * ps + (i - k) * R + k;
#pragma unroll
            for (int m = 0; m < R; ++m) dst[m * L] = v[u][m];
        }
    }
    __syncthreads();
}

template <int N, int L, int NPEN, int NT, int DIR, int SCHED, int TL>
__device__ __forceinline__ void fft_stages(double2* buf, int ps, const double2* __restrict__ tw) {
    if constexpr (L < N) {
        constexpr int R = next_radix(N / L, SCHED);
        stockham_stage<N, R, L, NPEN, NT, DIR, TL>(buf, ps, tw);
        fft_stages<N, L * R, NPEN, NT, DIR, SCHED, TL>(buf, ps, tw);
    }
}

// Unnormalised DFT of NPEN pencils of length N held in LDS; ends synchronised.
// Caller must have synchronised after filling the buffer.  tw: a twiddle table
// of length TL (see stockham_stage).
template <int N, int NPEN, int NT, int DIR, int SCHED = 0, int TL = TWN>
__device__ __forceinline__ void fft_lds(double2* buf, int ps, const double2* __restrict__ tw) {
    static_assert(TL % N == 0, "twiddle table must hold the N-th roots");
    if constexpr (N > 1) fft_stages<N, 1, NPEN, NT, DIR, SCHED, TL>(buf, ps, tw);
}

// Copy of e^{-2 pi i j / N}, j < N, from the device table (its contiguous
// N-point subset at offset TWN + N) into LDS in two steps: fetch() issues the
// loads into registers (at kernel start, so their latency overlaps the data
// loads), store() writes them to LDS; the caller synchronises before use.
// Subsets of more than 8 values per thread are loaded in store() directly.
template <int N, int NT>
struct TwiddleCopy {
    static constexpr int PER = (N + NT - 1) / NT;
    static constexpr bool PRE = PER <= 8;
    double2 v[PRE ? PER : 1];
    __device__ __forceinline__ void fetch(const double2* __restrict__ tw) {
        if constexpr (PRE) {
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int j = threadIdx.x + u * NT;
                if ((N % NT) == 0 || j < N) v[u] = tw[TWN + N + j];
            }
        }
    }
    __device__ __forceinline__ void store(double2* lds_tw, const double2* __restrict__ tw) {
        if constexpr (PRE) {
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int j = threadIdx.x + u * NT;
                if ((N % NT) == 0 || j < N) lds_tw[j] = v[u];
            }
        } else {
            for (int j = threadIdx.x; j < N; j += NT) lds_tw[j] = tw[TWN + N + j];
        }
    }
};

// ------------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum of K per-thread values over the block, fixed order; result valid in
// thread 0 (out[k]).  scratch: LDS with at least (NT/64)*K doubles.  Ends
// synchronised.
template <int K, int NT>
__device__ __forceinline__ void block_sum(double* vals, double* scratch, double* out) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = wave_sum(vals[k]);
        if (lane == 0) scratch[wid * K + k] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int w = 0; w < NW; ++w) s += scratch[w * K + k];
            out[k] = s;
        }
    }
    __syncthreads();
}

// Min/max over nblk per-block bound partials (partial[b * 8 + k] = min,
// partial[b * 8 + 4 + k] = max, k < d) by a block of 256 threads; result in
// red[0..3] (min) and red[4..7] (max), valid in every thread on return.
// scratch: 32 doubles of LDS.  min/max are exact: the order does not matter.
__device__ __forceinline__ void reduce_bounds(const double* __restrict__ partial, int nblk, int d,
                                              double* scratch, double* red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double mn = INFINITY, mx = -INFINITY;
        if (k < d)
            for (int b = threadIdx.x; b < nblk; b += 256) {
                mn = fmin(mn, partial[b * 8 + k]);
                mx = fmax(mx, partial[b * 8 + 4 + k]);
            }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            mn = fmin(mn, __shfl_xor(mn, off, 64));
            mx = fmax(mx, __shfl_xor(mx, off, 64));
        }
        if (lane == 0) {
            scratch[wid * 8 + k] = mn;
            scratch[wid * 8 + 4 + k] = mx;
        }
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        const int k = threadIdx.x;
        double v = scratch[k];
        for (int w = 1; w < 4; ++w) v = k < 4 ? fmin(v, scratch[w * 8 + k]) : fmax(v, scratch[w * 8 + k]);
        red[k] = v;
    }
    __syncthreads();
}

}  // namespace kdefft
