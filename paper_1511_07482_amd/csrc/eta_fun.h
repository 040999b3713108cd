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
// The row kernels are compiled for each order r (template R), so every
// array index is a compile-time constant and a lag costs the work of its
// own order.
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

// Y_R of the t-cumulants at z = P x, divided by R! (eta_R(x; S) = phi_S(x) R! * this).
// With khat_j = kappa_j / (j-1)! = A_j s_{j-1} + B_j, where s_i = z^T P^i z,
// A_j = (-1)^{j+1} j 2^{j-1} and B_j = (-1)^j T_j / 2 (eta_offsets), and
// y_m = Y_m / m!, the Bell recursion Y_{m+1} = sum_{k<=m} C(m,k) kappa_{k+1} Y_{m-k}
// becomes y_0 = 1, (m+1) y_{m+1} = sum_{k<=m} khat_{k+1} y_{m-k}.
// s_i = w_a . w_b (a = floor(i/2), b = i - a) from w_0 = z, w_{c+1} = P w_c.
template <int D, int R>
__device__ __forceinline__ double eta_scaled(const double* z, const double* P, const double* B) {
    if constexpr (R == 0) {
        return 1.0;
    } else {
        double w[R / 2 + 1][D];
#pragma unroll
        for (int i = 0; i < D; ++i) w[0][i] = z[i];
#pragma unroll
        for (int c = 1; c <= R / 2; ++c)
#pragma unroll
            for (int i = 0; i < D; ++i) {
                double u = 0.0;
#pragma unroll
                for (int k = 0; k < D; ++k) u += P[i * D + k] * w[c - 1][k];
                w[c][i] = u;
            }
        double kh[R + 1];
#pragma unroll
        for (int j = 1; j <= R; ++j) {
            const int i = j - 1, a = i / 2, b = i - a;
            double sj = 0.0;
#pragma unroll
            for (int q = 0; q < D; ++q) sj += w[a][q] * w[b][q];
            const double A = (double)((j & 1) ? j : -j) * (double)(1 << (j - 1));
            kh[j] = A * sj + B[j];
        }
        double y[R + 1];
        y[0] = 1.0;
#pragma unroll
        for (int m = 0; m < R; ++m) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k <= m; ++k) acc += kh[k + 1] * y[m - k];
            y[m + 1] = m == 0 ? acc : acc * (1.0 / (double)(m + 1));
        }
        return y[R];
    }
}

// B_j = (-1)^j T_j / 2, j = 1..ETA_RMAX (B_0 unused).
__device__ __forceinline__ void eta_offsets(const double* T, double* B) {
    B[0] = 0.0;
#pragma unroll
    for (int j = 1; j <= ETA_RMAX; ++j) B[j] = (j & 1) ? -0.5 * T[j] : 0.5 * T[j];
}

// Y_r for a run-time r in [0, ETA_RMAX] (set-up kernels).
template <int D>
__device__ __forceinline__ double eta_ratio(const double* z, const double* P, const double* T, int r) {
    double B[ETA_RMAX + 1];
    eta_offsets(T, B);
    switch (r) {
        case 0: return 1.0;
        case 1: return eta_scaled<D, 1>(z, P, B);
        case 2: return 2.0 * eta_scaled<D, 2>(z, P, B);
        case 3: return 6.0 * eta_scaled<D, 3>(z, P, B);
        case 4: return 24.0 * eta_scaled<D, 4>(z, P, B);
        case 5: return 120.0 * eta_scaled<D, 5>(z, P, B);
        case 6: return 720.0 * eta_scaled<D, 6>(z, P, B);
        case 7: return 5040.0 * eta_scaled<D, 7>(z, P, B);
        default: return 40320.0 * eta_scaled<D, 8>(z, P, B);
    }
}

// Scalar families on the lag grid:
//   NGS = 1 (Q_r):      eta_r(x; S1)
//   NGS = 2 (LSCV_r):   sgn [eta_r(x; S1) - 2 eta_r(x; S2)]
// with c1, c2 the normal constants (the LSCV weight of the S2 sum folded into c2).
// Parameters: P1, P2 at S_P1, S_P2; c1, c2 at S_C1, S_C2; sgn at S_SIGN.  The
// kernel is compiled for the order R (the r at S_R); R! is folded into c1, c2.
template <int D, int NGS, int R>
struct EtaFun {
    static constexpr int NG = 1;
    static constexpr int NGAUSS = NGS;
    double P[NGS][D * D];
    double c[NGS];
    double B[NGS][ETA_RMAX + 1];
    double sgn;
    __device__ __forceinline__ void load(const double* prm) {
        constexpr double FACT[ETA_RMAX + 1] = {1, 1, 2, 6, 24, 120, 720, 5040, 40320};
#pragma unroll
        for (int k = 0; k < NGS; ++k) {
            const int base = k == 0 ? S_P1 : S_P2;
#pragma unroll
            for (int i = 0; i < D * D; ++i) P[k][i] = prm[base + (i / D) * 4 + (i % D)];
            c[k] = FACT[R] * prm[k == 0 ? S_C1 : S_C2];
            double T[ETA_RMAX + 1];
            eta_traces<D>(P[k], T);
            eta_offsets(T, B[k]);
        }
        sgn = prm[S_SIGN];
    }
    __device__ __forceinline__ const double* Pm(int k) const { return P[k]; }
    __device__ __forceinline__ double cn(int k) const { return c[k]; }
    __device__ __forceinline__ void combine(const double (*z)[D], const double* e, double* out) const {
        double v = e[0] * eta_scaled<D, R>(z[0], P[0], B[0]);
        if constexpr (NGS == 2) v -= 2.0 * e[1] * eta_scaled<D, R>(z[1], P[1], B[1]);
        out[0] = sgn * v;
    }
    __device__ __forceinline__ void eval(const double* x, double* out) const;
};

template <int D, int NGS, int R>
__device__ __forceinline__ void EtaFun<D, NGS, R>::eval(const double* x, double* out) const {
    eval_direct<EtaFun<D, NGS, R>, D>(*this, x, out);
}

}  // namespace kdefft
