// Assembly of the batched results from the per-item partial sums: psi
// entries, and criterion objective and gradient (fixed summation order).  Used
// by the separate final kernels and, for psi, fused into the lag kernels, where
// the block that completes a candidate's last work item assembles it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dev_common.h"
#include "internal.h"

namespace kdefft {

// ------------------------------------------------------------------ small dense linear algebra (d <= 4)
// Cholesky A = L L^T of a symmetric d x d (row stride 4); false if not positive definite.
template <int D>
__device__ __forceinline__ static bool chol4(const double* A, double* L) {
#pragma unroll
    for (int i = 0; i < 16; ++i) L[i] = 0.0;
    bool ok = true;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        double s = A[j * 4 + j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= L[j * 4 + k] * L[j * 4 + k];
        ok = ok && (s > 0.0);
        const double ljj = sqrt(s > 0.0 ? s : 1.0);
        L[j * 4 + j] = ljj;
#pragma unroll
        for (int i = j + 1; i < D; ++i) {
            double t = A[i * 4 + j];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= L[i * 4 + k] * L[j * 4 + k];
            L[i * 4 + j] = t / ljj;
        }
    }
    return ok;
}

// Inverse of L L^T from the lower factor L (row stride 4).
template <int D>
__device__ __forceinline__ static void chol_inv4(const double* L, double* Ainv) {
    double Li[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) Li[i] = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        Li[j * 4 + j] = 1.0 / L[j * 4 + j];
#pragma unroll
        for (int i = j + 1; i < D; ++i) {
            double s = 0.0;
#pragma unroll
            for (int k = j; k < i; ++k) s -= L[i * 4 + k] * Li[k * 4 + j];
            Li[i * 4 + j] = s / L[i * 4 + i];
        }
    }
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            double s = 0.0;
#pragma unroll
            for (int k = (i > j ? i : j); k < D; ++k) s += Li[k * 4 + i] * Li[k * 4 + j];
            Ainv[i * 4 + j] = s;
        }
}

// Sum of the partial sums of candidate h, grid g over its chunks, by one
// wavefront: lane t takes chunks t, t+64, ... in order, then a fixed xor tree.
// COHERENT: the partial sums were stored by other blocks of the running launch
// (agent-scope atomic stores, ordered before their counter increments by
// release); each value is read with an agent-scope atomic load after the
// reading lane's own acquire of the counter.
template <bool COHERENT = false>
__device__ static double chunk_sum(const double* __restrict__ partial, int64_t h, int64_t nchunks, int ng, int g) {
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    for (int64_t c = lane; c < nchunks; c += 64) {
        const double* q = partial + (h * nchunks + c) * ng + g;
        if constexpr (COHERENT) {
            s += __hip_atomic_load(const_cast<double*>(q), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            s += *q;
        }
    }
    return wave_sum(s);
}

// Sum of grid g of the count items from item `first` (partial sums of NG = ng
// values per item), by one wavefront in the same fixed order as chunk_sum.
__device__ static double item_sum(const double* __restrict__ partial, int64_t first, int64_t count, int ng, int g) {
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    for (int64_t c = lane; c < count; c += 64) s += partial[(first + c) * ng + g];
    return wave_sum(s);
}

// psi[h, g] = scale * chunk sum, by one wavefront; scal_out (if set) receives
// psi[0, 0] (the constant SCV term of a dataset).  p: candidate h's block.
template <bool COHERENT = false>
__device__ __forceinline__ static void psi_finish(const double* __restrict__ partial, int64_t nchunks, int ng,
                                                  const double* __restrict__ p, int64_t h, int g,
                                                  double* __restrict__ psi, double* __restrict__ scal_out) {
    const double v = chunk_sum<COHERENT>(partial, h, nchunks, ng, g) * p[S_SCALE];
    if ((threadIdx.x & 63) != 0) return;
    if (psi) psi[h * ng + g] = v;
    if (scal_out && h == 0 && g == 0) scal_out[0] = v;
}

// Criterion assembly for candidate h by one wavefront (p: its parameter
// block).  kind: FUN_SCV_OBJ or FUN_ETA* (obj only), FUN_SCV_OBJGRAD (obj +
// grad), FUN_SCV_GRAD (adjoint: grad scaled by grad_out).
// The candidate's work items are `count` items from `first`; cst is the
// constant term added to the objective (the SCV phi_{2G} sum, else 0).
template <int D>
__device__ __forceinline__ static void crit_finish(int kind, const double* __restrict__ partial, int64_t first,
                                                   int64_t count, int ng, const double* __restrict__ p, int64_t h,
                                                   double cst, const double* __restrict__ grad_out,
                                                   double* __restrict__ obj, double* __restrict__ grad) {
    constexpr int d = D;
    constexpr int q = d * (d + 1) / 2;
    double T[1 + q];
#pragma unroll
    for (int g = 0; g < 1 + q; ++g) T[g] = g < ng ? item_sum(partial, first, count, ng, g) * p[S_SCALE] : 0.0;
    if ((threadIdx.x & 63) != 0) return;
    const bool sing = p[S_SING] != 0.0;
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    const double* L = p + S_L;
    // closed-form term: proportional to |H|^{-1/2} for every criterion with a
    // gradient, so its matrix gradient is -1/2 first H^{-1}
    const double t0 = p[S_FIRST];
    if (kind != FUN_SCV_GRAD) obj[h] = sing ? nan : t0 + T[0] + cst;
    if (kind == FUN_SCV_OBJ || kind == FUN_ETA1 || kind == FUN_ETA2 || grad == nullptr) return;
    const int off = kind == FUN_SCV_OBJGRAD ? 1 : 0;
    double Hinv[16];
    chol_inv4<D>(L, Hinv);
    double gH[16];
    int t = off;
    for (int i = 0; i < d; ++i)
        for (int j = i; j < d; ++j) {
            const double v = -0.5 * t0 * Hinv[i * 4 + j] + T[t++];
            gH[i * 4 + j] = v;
            gH[j * 4 + i] = v;
        }
    const double sc = kind == FUN_SCV_GRAD ? grad_out[h] : 1.0;
    int o = 0;
    for (int j = 0; j < d; ++j)
        for (int i = j; i < d; ++i) {
            double s = 0.0;
            for (int k = 0; k < d; ++k) s += gH[i * 4 + k] * L[k * 4 + j];
            grad[h * q + o++] = sing ? nan : 2.0 * s * sc;
        }
}

__device__ __forceinline__ static void* slot_ptr(double v) {
    return reinterpret_cast<void*>(static_cast<uintptr_t>(__double_as_longlong(v)));
}

// Partial sums of one work item (thread 0).  When the launch completes fused,
// they are written with agent-scope atomic stores (write-through to the
// coherence point shared by all dies), and the same thread's release on the
// candidate's counter (fused_finish) orders them before its increment.
template <int NG>
__device__ __forceinline__ static void store_item(const double* __restrict__ p, double* dst, const double* v) {
    if ((int)p[S_FIN_MODE] == 0) {
#pragma unroll
        for (int g = 0; g < NG; ++g) dst[g] = v[g];
    } else {
#pragma unroll
        for (int g = 0; g < NG; ++g) __hip_atomic_store(dst + g, v[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Fused completion of the psi launches, called by every thread of a lag
// kernel's block after thread 0 stored the item's partial sums (store_item).
// Thread 0 counts the item on its candidate h's counter (set to zero by the
// setup kernel) with an acquire-release read-modify-write at agent scope: the
// release makes its partial-sum stores visible before the increment, and the
// increments of all items form one release sequence.  If the item was the
// candidate's last of nchunks, every lane of the first wavefront takes an
// acquire load of the counter (it reads the final value, so it synchronizes
// with every item's release) and the wavefront writes the candidate's psi
// entries.  The other wavefronts go on at once.  Does nothing when the
// parameter block asks for no fusion.
template <int D>
__device__ __forceinline__ static void fused_finish(const double* __restrict__ p, const double* partial,
                                                    int64_t nchunks, int64_t h) {
    const int mode = (int)p[S_FIN_MODE];
    if (mode == 0 || threadIdx.x >= 64) return;
    int32_t* cnt = static_cast<int32_t*>(slot_ptr(p[S_FIN_CNT]));
    int last = 0;
    if (threadIdx.x == 0)
        last = __hip_atomic_fetch_add(cnt + h, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == (int)(nchunks - 1);
    last = __shfl(last, 0, 64);
    if (!last) return;
    (void)__hip_atomic_load(cnt + h, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const int ng = (int)p[S_FIN_NG];
    double* psi = static_cast<double*>(slot_ptr(p[S_FIN_OUT]));
    double* scal = static_cast<double*>(slot_ptr(p[S_FIN_SCAL]));
    for (int g = 0; g < ng; ++g) psi_finish<true>(partial, nchunks, ng, p, h, g, psi, scal);
}

}  // namespace kdefft
