// Per-candidate parameter blocks written on the device (the slots of Slot in
// internal.h): shared by the set-up kernels and the preparation kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "eta_fun.h"
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

// Parameter block of candidate h: H = L L^T from vechL, then per criterion
//   SCV:          S1 = 2H + 2G, S2 = H + 2G, first = n^-1 (4 pi)^{-d/2} |H|^{-1/2},
//                 and the index of the dataset's constant-term candidate
//                 (npseudo > 0; see pseudo_params);
//   LSCV (r):     S1 = 2H, S2 = H with the S2 weight a/2 folded into c2
//                 (a = 2, or 2n/(n-1) for the leave-one-out form), sign (-1)^r,
//                 first = (-1)^r b eta_r(0; H) (b = 2/n, or 2/(n-1));
//   Q_r:          S1 = H (the candidate matrix itself), no first or constant term;
// their inverses and normal constants, grid spacing, n and the scale of the
// lag sums.  status 1 = singular candidate.
// ETA = false: the caller serves r = 0 only (the moment kernels), where the
// diagonal term's eta_r(0; H) / phi_H(0) is 1, and the eta_r code is left out.
template <int D, bool ETA = true>
__device__ static void scv_params(const double* __restrict__ vechL, const ScvBatchArgs& a, int64_t h, int64_t ncand,
                                  int npseudo, double* __restrict__ p, int32_t* __restrict__ status) {
    // dataset of candidate h: the last j with off[j] <= h (a binary search with
    // run-time indices, so the argument arrays are read where they are instead
    // of being held in registers)
    int lo = 0, hi = a.n_ds - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.off[mid] <= h)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int ds_index = lo;
    const DsDev& ds = *a.rec[ds_index];
    constexpr int d = D;
    const int q = d * (d + 1) / 2;
    double L[16], H[16], S1[16], S2[16], L1[16], L2[16];
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
    const int crit = a.crit;
    const bool scv = crit == KDEFFT_CRIT_SCV;
    const bool qr = crit == KDEFFT_CRIT_QR;
    const double gw = scv ? 2.0 : 0.0;      // weight of the pilot in S1, S2
    const double hw = qr ? 1.0 : 2.0;       // weight of H in S1
    for (int i = 0; i < 16; ++i) { S1[i] = 0.0; S2[i] = 0.0; }
    for (int i = 0; i < d; ++i)
        for (int k2 = 0; k2 < d; ++k2) {
            S1[i * 4 + k2] = hw * H[i * 4 + k2] + gw * ds.G[i * 4 + k2];
            S2[i * 4 + k2] = H[i * 4 + k2] + gw * ds.G[i * 4 + k2];
        }
    // every slot the row and final kernels read is written below; these three
    // default to zero (no closed-form or constant term, separate final kernel)
    p[S_FIRST] = 0.0;
    p[S_CONST] = 0.0;
    p[S_FIN_MODE] = 0.0;
    p[S_PSEUDO] = npseudo > 0 ? (double)(ncand + ds_index) : -1.0;
    const bool ok1 = chol4<D>(S1, L1);
    const bool ok2 = chol4<D>(S2, L2);
    const bool ok = !sing && ok1 && ok2;
    if (!ok) {
        sing = true;
        // benign parameters keep the row kernel finite; the result is set to NaN
        for (int i = 0; i < 16; ++i) { L1[i] = 0.0; L2[i] = 0.0; }
        for (int k = 0; k < d; ++k) { L1[k * 4 + k] = 1.0; L2[k * 4 + k] = 1.0; }
    }
    chol_inv4<D>(L1, p + S_P1);
    chol_inv4<D>(L2, p + S_P2);
    double det1 = 1.0, det2 = 1.0, ldet = 1.0;
    for (int k = 0; k < d; ++k) {
        det1 *= L1[k * 4 + k];
        det2 *= L2[k * 4 + k];
        ldet *= fabs(L[k * 4 + k]);
    }
    const double n = ds.n;
    const int r = a.r;
    const double sgn = (r & 1) ? -1.0 : 1.0;
    p[S_C1] = two_pi_pow(d) / det1;
    p[S_C2] = two_pi_pow(d) / det2;
    p[S_R] = (double)r;
    p[S_SIGN] = 1.0;
    if (scv) {
        double c4 = 1.0;  // (4 pi)^{-d/2}
        for (int k = 0; k < d; ++k) c4 *= 0.28209479177387814347;
        p[S_FIRST] = c4 / (n * ldet);
    } else if (!qr) {
        const bool exact = crit == KDEFFT_CRIT_LSCV_EXACT;
        const double b = exact ? 2.0 / (n - 1.0) : 2.0 / n;
        // eta_r(0; H) = phi_H(0) Y_r(kappa at x = 0); phi_H(0) = c2 before weighting
        double ratio = 1.0;
        if constexpr (ETA) {
            double P2[D * D], T2[ETA_RMAX + 1], z0[D];
            for (int i = 0; i < D * D; ++i) P2[i] = p[S_P2 + (i / D) * 4 + (i % D)];
            for (int i = 0; i < D; ++i) z0[i] = 0.0;
            eta_traces<D>(P2, T2);
            ratio = eta_ratio<D>(z0, P2, T2, r);
        }
        p[S_FIRST] = sgn * b * p[S_C2] * ratio;
        if (exact) p[S_C2] *= n / (n - 1.0);
        p[S_SIGN] = sgn;
    }
    put_ptr(p + S_WMIX, ds.wmix);
    put_ptr(p + S_ALAG, ds.alag);
    for (int k = 0; k < d; ++k) p[S_DELTA + k] = ds.delta[k];
    p[S_N] = n;
    p[S_SCALE] = 1.0 / (n * n * a.prodP);
    p[S_SING] = sing ? 1.0 : 0.0;
    for (int i = 0; i < 16; ++i) p[S_L + i] = L[i];
    if (status) status[h] = sing ? 1 : 0;
}


// Parameter block of the constant SCV term of dataset j (a candidate after
// the real ones): n^-2 sum sum phi_{2G} evaluated by the same walk as a
// candidate, with the first Gaussian phi_{2G} (its normal constant c1 > 0, as
// the walk's magnitude tests assume) and the second switched off (c2 = 0), so
// that the walk's objective sum (first minus twice the second) is the phi_{2G}
// sum.  Both carry (2G)^{-1} (the live intervals use them).  No status or first
// term; the final kernel stores the term in the dataset's scalar block (slot
// S_FIN_SCAL).
template <int D>
__device__ static void pseudo_params(const ScvBatchArgs& a, int j, double* __restrict__ p) {
    constexpr int d = D;
    const DsDev& ds = *a.rec[j];
    double S[16], L[16];
    for (int i = 0; i < 16; ++i) S[i] = 0.0;
    for (int i = 0; i < d; ++i)
        for (int k2 = 0; k2 < d; ++k2) S[i * 4 + k2] = 2.0 * ds.G[i * 4 + k2];
    chol4<D>(S, L);   // the pilot was validated positive definite when the dataset was prepared
    chol_inv4<D>(L, p + S_P1);
    chol_inv4<D>(L, p + S_P2);
    double det = 1.0;
    for (int k = 0; k < d; ++k) det *= L[k * 4 + k];
    p[S_C1] = two_pi_pow(d) / det;
    p[S_C2] = 0.0;
    p[S_FIRST] = 0.0;
    p[S_CONST] = 0.0;
    p[S_R] = 0.0;
    p[S_SIGN] = 1.0;
    p[S_PSEUDO] = -1.0;
    p[S_FIN_MODE] = 0.0;
    put_ptr(p + S_FIN_SCAL, ds.scal);
    put_ptr(p + S_WMIX, ds.wmix);
    put_ptr(p + S_ALAG, ds.alag);
    for (int k = 0; k < d; ++k) p[S_DELTA + k] = ds.delta[k];
    p[S_N] = ds.n;
    p[S_SCALE] = 1.0 / (ds.n * ds.n * a.prodP);
    p[S_SING] = 0.0;
    for (int i = 0; i < 16; ++i) p[S_L + i] = i % 5 == 0 ? 1.0 : 0.0;
}

}  // namespace kdefft
