// Per-candidate parameter blocks written on the device (the slots of Slot in
// internal.h): shared by the set-up kernels and the preparation kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "finish.h"
#include "internal.h"

namespace kdefft {

__device__ __forceinline__ static double two_pi_pow(int d) {  // (2 pi)^{-d/2}
    const double c = 0.39894228040143267794;      // (2 pi)^{-1/2}
    double r = 1.0;
    for (int k = 0; k < d; ++k) r *= c;
    return r;
}

__device__ __forceinline__ static void put_ptr(double* slot, const void* p) {
    *slot = __longlong_as_double(static_cast<long long>(reinterpret_cast<uintptr_t>(p)));
}

// Completion slots of candidate h's block; clears its counter when fused.
__device__ __forceinline__ static void put_finish(double* p, const FinishArgs& f, int64_t h) {
    p[S_FIN_MODE] = (double)f.mode;
    p[S_FIN_NG] = (double)f.ng;
    put_ptr(p + S_FIN_CNT, f.counters);
    put_ptr(p + S_FIN_OUT, f.out);
    put_ptr(p + S_FIN_SCAL, f.scal);
    if (f.mode != FIN_NONE) f.counters[h] = 0;
}

// Parameter block of the psi_r family for bandwidth vech gv on dataset ds:
// P = G^{-1}, c = (-1)^r (2 pi)^{-d/2} |G|^{-1/2} (even r: the sign is +1),
// lag array, spacing, n and the scale of the lag sums.
template <int D>
__device__ __forceinline__ static void psi_params(const double* gv, const DsDev& ds, double prodP, double* p) {
    constexpr int d = D;
    double G[16], L[16];
    for (int i = 0; i < 16; ++i) G[i] = 0.0;
    int t = 0;
    for (int jj = 0; jj < d; ++jj)
        for (int i = jj; i < d; ++i) {
            G[i * 4 + jj] = gv[t];
            G[jj * 4 + i] = gv[t];
            ++t;
        }
    // every slot the psi kernels read is written here or by put_finish
    chol4<D>(G, L);
    chol_inv4<D>(L, p + S_P1);
    double det = 1.0;
    for (int k = 0; k < d; ++k) det *= L[k * 4 + k];
    p[S_C] = two_pi_pow(d) / det;
    put_ptr(p + S_WMIX, ds.wmix);
    put_ptr(p + S_ALAG, ds.alag);
    for (int k = 0; k < d; ++k) p[S_DELTA + k] = ds.delta[k];
    p[S_N] = ds.n;
    p[S_SCALE] = 1.0 / (ds.n * ds.n * prodP);
}

}  // namespace kdefft
