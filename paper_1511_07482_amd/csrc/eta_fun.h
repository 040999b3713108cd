// Scalar eta_r families on the lag grid (Q_r, LSCV_r): their kernel
// functions, evaluated by the lag-domain row kernels.
#pragma once

#include "dev_kernels.h"

namespace kdefft {

// eta_r family (Sec. 5, Eq. (30)-(32)): eta_r(x; S) = (vec^T I)^{(x)r} D^{(x)2r} phi_S(x),
// the r-th power of the Laplacian of phi_S.  By the heat equation of the normal
// density, eta_r(x; S) = d^r/dt^r phi_{S + 2tI}(x) at t = 0, so eta_r / phi_S is
// the complete Bell polynomial Y_r of the t-cumulants of log phi_{S+2tI}(x):
//   kappa_m = (-1)^{m+1} (m-1)!/2 (m U_m - T_m),
//   U_m = x^T S^-1 (2 S^-1)^m x = 2^m z^T P^{m-1} z  (z = P x, P = S^-1),
//   T_m = tr (2P)^m.
// r is a run-time value in [0, ETA_RMAX]; the loops are unrolled to a
// compile-time bound on r, so every array index is a compile-time constant.
constexpr int ETA_RMAX = 8;

// T_m = tr (2P)^m, m = 1..ETA_RMAX, for a symmetric P (row stride D).
template <int D>
__device__ __forceinline__ void eta_traces(const double* P, double* T) {
    double B[D * D], Bm[D * D];
#pragma unroll
    for (int i = 0; i < D * D; ++i) { B[i] = 2.0 * P[i]; Bm[i] = B[i]; }
    T[0] = (double)D;
#pragma unroll
    for (int m = 1; m <= ETA_RMAX; ++m) {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) t += Bm[i * D + i];
        T[m] = t;
        if (m < ETA_RMAX) {
            double nx[D * D];
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    double u = 0.0;
#pragma unroll
                    for (int k = 0; k < D; ++k) u += Bm[i * D + k] * B[k * D + j];
                    nx[i * D + j] = u;
                }
#pragma unroll
            for (int i = 0; i < D * D; ++i) Bm[i] = nx[i];
        }
    }
}

// Y_r of the t-cumulants at z = P x (eta_r(x; S) = phi_S(x) * this), for
// r <= RB: kappa_m needs s_{m-1} = z^T P^{m-1} z = w_a . w_b (a = floor((m-1)/2),
// b = m-1-a) from w_0 = z, w_{c+1} = P w_c; then the Bell recursion
// Y_0 = 1, Y_{m+1} = sum_{k<=m} C(m,k) kappa_{k+1} Y_{m-k}.  Straight-line code
// (the cumulants are independent of each other) up to the bound RB.
template <int D, int RB>
__device__ __forceinline__ double eta_ratio_upto(const double* z, const double* P, const double* T, int r) {
    constexpr double C[ETA_RMAX][ETA_RMAX] = {
        {1, 0, 0, 0, 0, 0, 0, 0},    {1, 1, 0, 0, 0, 0, 0, 0},     {1, 2, 1, 0, 0, 0, 0, 0},
        {1, 3, 3, 1, 0, 0, 0, 0},    {1, 4, 6, 4, 1, 0, 0, 0},     {1, 5, 10, 10, 5, 1, 0, 0},
        {1, 6, 15, 20, 15, 6, 1, 0}, {1, 7, 21, 35, 35, 21, 7, 1}};
    constexpr double FACT[ETA_RMAX] = {1, 1, 2, 6, 24, 120, 720, 5040};  // (m-1)!
    double w[RB / 2 + 1][D];
#pragma unroll
    for (int i = 0; i < D; ++i) w[0][i] = z[i];
#pragma unroll
    for (int c = 1; c <= RB / 2; ++c)
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double u = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) u += P[i * D + k] * w[c - 1][k];
            w[c][i] = u;
        }
    double kap[RB + 1];
    kap[0] = 0.0;
    double two_m = 1.0;
#pragma unroll
    for (int m = 1; m <= RB; ++m) {
        const int j = m - 1, a = j / 2, b = j - a;
        double sj = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) sj += w[a][i] * w[b][i];
        two_m *= 2.0;
        const double U = two_m * sj;
        const double v = 0.5 * FACT[m - 1] * ((double)m * U - T[m]);
        kap[m] = (m & 1) ? v : -v;
    }
    double Y[RB + 1];
    Y[0] = 1.0;
#pragma unroll
    for (int m = 0; m < RB; ++m) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k <= m; ++k) s += C[m][k] * kap[k + 1] * Y[m - k];
        Y[m + 1] = s;
    }
    double out = Y[0];
#pragma unroll
    for (int m = 1; m <= RB; ++m)
        if (m == r) out = Y[m];
    return out;
}

// Order classes: orders 0-2, 3-4, 5-6 and 7-8 run the straight-line form of
// their bound (2, 4, 6, 8).
__host__ __device__ constexpr int eta_bound(int r) { return r <= 2 ? 2 : (r <= 4 ? 4 : (r <= 6 ? 6 : ETA_RMAX)); }

template <int D>
__device__ __forceinline__ double eta_ratio(const double* z, const double* P, const double* T, int r) {
    if (r <= 2) return eta_ratio_upto<D, 2>(z, P, T, r);
    if (r <= 4) return eta_ratio_upto<D, 4>(z, P, T, r);
    if (r <= 6) return eta_ratio_upto<D, 6>(z, P, T, r);
    return eta_ratio_upto<D, ETA_RMAX>(z, P, T, r);
}

// Scalar families on the lag grid:
//   NGS = 1 (Q_r):      eta_r(x; S1)
//   NGS = 2 (LSCV_r):   sgn [eta_r(x; S1) - 2 eta_r(x; S2)]
// with c1, c2 the normal constants (the LSCV weight of the S2 sum folded into c2).
// Parameters: P1, P2 at S_P1, S_P2; c1, c2 at S_C1, S_C2; r at S_R; sgn at S_SIGN.
// RB = eta_bound(r) is the order class the kernel is compiled for (r <= RB).
template <int D, int NGS, int RB>
struct EtaFun {
    static constexpr int NG = 1;
    static constexpr int NGAUSS = NGS;
    double P[NGS][D * D];
    double c[NGS];
    double T[NGS][ETA_RMAX + 1];
    double sgn;
    int r;
    __device__ __forceinline__ void load(const double* prm) {
#pragma unroll
        for (int k = 0; k < NGS; ++k) {
            const int base = k == 0 ? S_P1 : S_P2;
#pragma unroll
            for (int i = 0; i < D * D; ++i) P[k][i] = prm[base + (i / D) * 4 + (i % D)];
            c[k] = prm[k == 0 ? S_C1 : S_C2];
            eta_traces<D>(P[k], T[k]);
        }
        r = (int)prm[S_R];
        sgn = prm[S_SIGN];
    }
    __device__ __forceinline__ const double* Pm(int k) const { return P[k]; }
    __device__ __forceinline__ double cn(int k) const { return c[k]; }
    __device__ __forceinline__ void combine(const double (*z)[D], const double* e, double* out) const {
        double v = e[0] * eta_ratio_upto<D, RB>(z[0], P[0], T[0], r);
        if constexpr (NGS == 2) v -= 2.0 * e[1] * eta_ratio_upto<D, RB>(z[1], P[1], T[1], r);
        out[0] = sgn * v;
    }
    __device__ __forceinline__ void eval(const double* x, double* out) const;
};

template <int D, int NGS, int RB>
__device__ __forceinline__ void EtaFun<D, NGS, RB>::eval(const double* x, double* out) const {
    eval_direct<EtaFun<D, NGS, RB>, D>(*this, x, out);
}

}  // namespace kdefft
