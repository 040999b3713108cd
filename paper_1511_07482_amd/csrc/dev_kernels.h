// Gaussian kernel derivative families evaluated at a lag x = delta o l
// (Sec. 4, Eq. (18); Sec. 5 for the r-th derivative vector).
//
// D^alpha phi_S(x) = (-1)^{|alpha|} He_alpha(x) phi_S(x), with z = S^{-1} x,
// He_0 = 1 and He_{a+e_k} = z_k He_a - sum_j a_j (S^{-1})_kj He_{a-e_j}.
// The multi-indices of order <= r, the recurrence parents and coefficients
// are built at compile time, so the recurrence unrolls into registers.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "internal.h"

namespace kdefft {

__host__ __device__ constexpr int choose_c(int n, int k) {
    int r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

template <int D, int R>
struct HermTab {
    static constexpr int NB = choose_c(D + R, R);      // multi-indices with |a| <= R
    static constexpr int NU = choose_c(D + R - 1, R);  // unique entries of order R
    struct Tab {
        int a[NB][4];
        int k[NB];
        int par[NB];
        int gp[NB][4];
        int cf[NB][4];
    };
    static constexpr int find(const Tab& t, const int* q, int upto) {
        for (int b = 0; b < upto; ++b) {
            bool eq = true;
            for (int j = 0; j < D; ++j) eq = eq && t.a[b][j] == q[j];
            if (eq) return b;
        }
        return -1;
    }
    static constexpr Tab make() {
        Tab t{};
        int cnt = 0;
        for (int s = 0; s <= R; ++s) {
            // sorted index tuples i_1 <= ... <= i_s in lexicographic order
            int idx[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            while (true) {
                for (int j = 0; j < 4; ++j) t.a[cnt][j] = 0;
                for (int m = 0; m < s; ++m) t.a[cnt][idx[m]] += 1;
                ++cnt;
                int m = s - 1;
                while (m >= 0 && idx[m] == D - 1) --m;
                if (m < 0) break;
                idx[m] += 1;
                for (int q = m + 1; q < s; ++q) idx[q] = idx[m];
            }
        }
        for (int b = 1; b < NB; ++b) {
            int kk = 0;
            while (t.a[b][kk] == 0) ++kk;
            t.k[b] = kk;
            int pa[4] = {t.a[b][0], t.a[b][1], t.a[b][2], t.a[b][3]};
            pa[kk] -= 1;
            t.par[b] = find(t, pa, b);
            for (int j = 0; j < 4; ++j) {
                t.gp[b][j] = 0;
                t.cf[b][j] = 0;
                if (j < D && pa[j] > 0) {
                    int q2[4] = {pa[0], pa[1], pa[2], pa[3]};
                    q2[j] -= 1;
                    t.gp[b][j] = find(t, q2, b);
                    t.cf[b][j] = pa[j];
                }
            }
        }
        return t;
    }
    static constexpr Tab tab = make();
};

template <int D, int R, int B, int... J>
__device__ __forceinline__ double herm_one(const double* z, const double* P, const double* he,
                                           std::integer_sequence<int, J...>) {
    using T = HermTab<D, R>;
    constexpr int k = T::tab.k[B];
    double v = z[k] * he[T::tab.par[B]];
    ((T::tab.cf[B][J] != 0 ? (v -= (double)T::tab.cf[B][J] * P[k * D + J] * he[T::tab.gp[B][J]]) : 0.0), ...);
    return v;
}

template <int D, int R, int... B>
__device__ __forceinline__ void herm_all(const double* z, const double* P, double* he,
                                         std::integer_sequence<int, B...>) {
    ((he[B + 1] = herm_one<D, R, B + 1>(z, P, he, std::make_integer_sequence<int, D>{})), ...);
}

// Every family below is a combination of NGAUSS Gaussians phi_{S_k}: at a lag
// x it needs z_k = S_k^{-1} x and e_k = c_k exp(-x.z_k / 2), then combines
// them (combine()).  eval() does it directly; the lag-domain kernel instead
// walks z_k and e_k along the last axis by exact recurrences.

// psi_r family: the NU unique D^alpha phi_G, |alpha| = R, canonical order.
// Parameters: P = G^{-1} at prm[0..) (row stride 4), c = (2 pi)^{-D/2} |G|^{-1/2}
// at prm[16] (the sign (-1)^R is +1 for even R).
template <int D, int R>
struct PsiFun {
    static constexpr int NG = HermTab<D, R>::NU;
    static constexpr int NGAUSS = 1;
    double P[D * D];
    double c;
    __device__ __forceinline__ void load(const double* prm) {
#pragma unroll
        for (int i = 0; i < D * D; ++i) P[i] = prm[S_P1 + (i / D) * 4 + (i % D)];
        c = prm[S_C];
    }
    __device__ __forceinline__ const double* Pm(int) const { return P; }
    __device__ __forceinline__ double cn(int) const { return c; }
    __device__ __forceinline__ void combine(const double (*z)[D], const double* e, double* out) const {
        if constexpr (R == 0) {
            out[0] = e[0];
        } else {
            using T = HermTab<D, R>;
            double he[T::NB];
            he[0] = 1.0;
            herm_all<D, R>(z[0], P, he, std::make_integer_sequence<int, T::NB - 1>{});
#pragma unroll
            for (int u = 0; u < T::NU; ++u) out[u] = he[T::NB - T::NU + u] * e[0];
        }
    }
    __device__ __forceinline__ void eval(const double* x, double* out) const;
};

// SCV families with S1 = 2H + 2G, S2 = H + 2G (P1, P2 their inverses, c1, c2
// the normal constants):
//   MODE 0 (objective):   phi_{S1} - 2 phi_{S2}
//   MODE 1 (obj + grad):  the above, then D_ij phi_{S1} - D_ij phi_{S2}, i <= j
//   MODE 2 (gradient):    D_ij phi_{S1} - D_ij phi_{S2}, i <= j
// with D_ij phi_S = ((S^{-1}x)_i (S^{-1}x)_j - (S^{-1})_ij) phi_S.
template <int D, int MODE>
struct ScvFun {
    static constexpr int NQ = D * (D + 1) / 2;
    static constexpr int NG = MODE == 0 ? 1 : (MODE == 1 ? 1 + NQ : NQ);
    static constexpr int NGAUSS = 2;
    double P1[D * D], P2[D * D];
    double c1, c2;
    __device__ __forceinline__ void load(const double* prm) {
#pragma unroll
        for (int i = 0; i < D * D; ++i) {
            P1[i] = prm[S_P1 + (i / D) * 4 + (i % D)];
            P2[i] = prm[S_P2 + (i / D) * 4 + (i % D)];
        }
        c1 = prm[S_C1];
        c2 = prm[S_C2];
    }
    __device__ __forceinline__ const double* Pm(int k) const { return k == 0 ? P1 : P2; }
    __device__ __forceinline__ double cn(int k) const { return k == 0 ? c1 : c2; }
    // Moment form along a run of lags t = 0, 1, ...: z_k(t) = z_k + t dz_k is
    // linear in t, so with w_k(t) = e_k(t) A(t) every output is a polynomial of
    // degree <= 2 in t weighted by w_k, and the run needs only the moments
    // m_k[p] = sum_t t^p w_k(t), p < NMOM, folded in once per run:
    //   sum_t w (z_i z_j - P_ij)(t) = z_i z_j m0 + (z_i dz_j + dz_i z_j) m1 + dz_i dz_j m2 - P_ij m0.
    static constexpr int NMOM = MODE == 0 ? 1 : 3;
    __device__ __forceinline__ void fold(const double (*z)[D], const double (*dz)[D], const double (*m)[3],
                                         double* acc) const {
        int o = 0;
        if constexpr (MODE != 2) acc[o++] += m[0][0] - 2.0 * m[1][0];
        if constexpr (MODE != 0) {
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = i; j < D; ++j) {
                    double v = 0.0;
#pragma unroll
                    for (int k = 0; k < 2; ++k) {
                        const double* P = k == 0 ? P1 : P2;
                        const double t = (z[k][i] * z[k][j] - P[i * D + j]) * m[k][0] +
                                         (z[k][i] * dz[k][j] + dz[k][i] * z[k][j]) * m[k][1] +
                                         dz[k][i] * dz[k][j] * m[k][2];
                        v += k == 0 ? t : -t;
                    }
                    acc[o++] += v;
                }
        }
    }
    __device__ __forceinline__ void combine(const double (*z)[D], const double* e, double* out) const {
        int o = 0;
        if constexpr (MODE != 2) out[o++] = e[0] - 2.0 * e[1];
        if constexpr (MODE != 0) {
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = i; j < D; ++j)
                    out[o++] = e[0] * (z[0][i] * z[0][j] - P1[i * D + j]) - e[1] * (z[1][i] * z[1][j] - P2[i * D + j]);
        }
    }
    __device__ __forceinline__ void eval(const double* x, double* out) const;
};

// Families that provide the moment form (fold) along a run of lags.
template <class Fun, class = void>
struct HasMoments { static constexpr bool value = false; };
template <class Fun>
struct HasMoments<Fun, decltype((void)Fun::NMOM)> { static constexpr bool value = true; };

// Direct evaluation at one lag x.
template <class Fun, int D>
__device__ __forceinline__ void eval_direct(const Fun& f, const double* x, double* out) {
    double z[Fun::NGAUSS][D];
    double e[Fun::NGAUSS];
#pragma unroll
    for (int k = 0; k < Fun::NGAUSS; ++k) {
        const double* P = f.Pm(k);
        double q = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) s += P[i * D + j] * x[j];
            z[k][i] = s;
            q += x[i] * s;
        }
        e[k] = f.cn(k) * exp(-0.5 * q);
    }
    f.combine(z, e, out);
}

template <int D, int R>
__device__ __forceinline__ void PsiFun<D, R>::eval(const double* x, double* out) const {
    eval_direct<PsiFun<D, R>, D>(*this, x, out);
}
template <int D, int MODE>
__device__ __forceinline__ void ScvFun<D, MODE>::eval(const double* x, double* out) const {
    eval_direct<ScvFun<D, MODE>, D>(*this, x, out);
}

// Plain-path SCV grids: entry 0 is the whole objective kernel
// phi_{S1} - 2 phi_{S2} + phi_{S3} (S3 = 2G), entries 1..q the Hessian grids.
// Parameters as ScvFun plus P3 at prm[S_L..S_L+16) and c3 at prm[S_CONST].
template <int D>
struct ScvPlainFun {
    static constexpr int NQ = D * (D + 1) / 2;
    static constexpr int NG = 1 + NQ;
    ScvFun<D, 1> f;
    double P3[D * D];
    double c3;
    __device__ __forceinline__ void load(const double* prm) {
        f.load(prm);
#pragma unroll
        for (int i = 0; i < D * D; ++i) P3[i] = prm[S_L + (i / D) * 4 + (i % D)];
        c3 = prm[S_CONST];
    }
    __device__ __forceinline__ void eval(const double* x, double* out) const {
        f.eval(x, out);
        double q3 = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) s += P3[i * D + j] * x[j];
            q3 += x[i] * s;
        }
        out[0] += c3 * exp(-0.5 * q3);
    }
};

// Signed lag of array index p on an axis of the circular layout, or a flag
// for the zero slots between the positive and negative lags.
__device__ __forceinline__ bool lag_of(int p, int M, int P, int* lag) {
    if (p < M) { *lag = p; return true; }
    if (p > P - M) { *lag = p - P; return true; }
    return false;
}

}  // namespace kdefft
