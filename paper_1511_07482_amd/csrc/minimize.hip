// Batched quasi-Newton minimisation of a bandwidth criterion over vech(L),
// H = L L^T, one independent problem per candidate (Sec. 5 names the PI and
// SCV selectors, Sec. 6 minimises them numerically without derivatives; here
// the exact gradients drive a BFGS inverse-Hessian update with a backtracking
// Armijo line search).
//
// The loop is a per-candidate state machine advanced by one update launch
// after each batched criterion evaluation: the evaluation takes the trial
// points xt of all candidates, the update reads their values and gradients,
// accepts or shortens the step and writes the next trial points.  A fixed
// number of evaluations is enqueued without host synchronisation, so a whole
// minimisation can be captured in a graph; finished candidates keep their
// point as the trial point (its evaluation is repeated and ignored).
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace kdefft {

namespace {

constexpr int MQ = 10;   // q = d(d+1)/2 <= 10 for d <= 4

// double state per candidate: x[q], g[q], p[q], Hinv[q*q], f, alpha
__host__ __device__ constexpr int min_sw(int q) { return 3 * q + q * q + 2; }

enum : int { PH_START = 0, PH_LINE = 1 };

// int32 state per candidate: phase, backtracks, accepted steps, outcome, flat steps
constexpr int MIN_IS = 8;

// Armijo constant, step shrink bounds, backtracking limit, first-step cap
constexpr double C_ARMIJO = 1e-4;
constexpr int MAX_BACK = 60;
constexpr double STEP_CAP = 0.25;   // a new direction moves no entry of x by more than this x max|x|

__device__ double dot(const double* a, const double* b, int q) {
    double s = 0.0;
    for (int i = 0; i < q; ++i) s = fma(a[i], b[i], s);
    return s;
}

__device__ double amax(const double* a, int q) {
    double m = 0.0;
    for (int i = 0; i < q; ++i) m = fmax(m, fabs(a[i]));
    return m;
}

// p = -Hinv g (a steepest-descent restart if that is not a descent direction),
// first step length 1 capped so that no entry moves by more than STEP_CAP x max|x|
__device__ void new_direction(int q, const double* x, const double* g, double* p, double* Hi, double* alpha,
                              double* xt) {
    for (int i = 0; i < q; ++i) {
        double s = 0.0;
        for (int j = 0; j < q; ++j) s = fma(Hi[i * q + j], g[j], s);
        p[i] = -s;
    }
    if (!(dot(g, p, q) < 0.0)) {
        for (int i = 0; i < q; ++i) {
            for (int j = 0; j < q; ++j) Hi[i * q + j] = i == j ? 1.0 : 0.0;
            p[i] = -g[i];
        }
    }
    const double pn = amax(p, q), xn = amax(x, q);
    double a = 1.0;
    if (pn > STEP_CAP * xn && pn > 0.0) a = STEP_CAP * xn / pn;
    *alpha = a;
    for (int i = 0; i < q; ++i) xt[i] = x[i] + a * p[i];
}

__global__ void k_min_init(int64_t B, int q, const double* __restrict__ x0, double* __restrict__ xt,
                           int32_t* __restrict__ ist) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    for (int i = 0; i < q; ++i) xt[b * q + i] = x0[b * q + i];
    int32_t* is = ist + MIN_IS * b;
    is[0] = PH_START;
    is[1] = 0;                      // backtracks of the current line search
    is[2] = 0;                      // accepted steps
    is[3] = KDEFFT_MIN_RUNNING;     // outcome
    is[4] = 0;                      // accepted steps in a row without a decrease above rounding
}

__global__ void k_min_step(int64_t B, int q, double tol, double* __restrict__ st, int32_t* __restrict__ ist,
                           const double* __restrict__ ft, const double* __restrict__ gt,
                           const int32_t* __restrict__ stt, double* __restrict__ xt_all) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double* s = st + b * min_sw(q);
    double* x = s;
    double* g = s + q;
    double* p = s + 2 * q;
    double* Hi = s + 3 * q;
    double& f = s[3 * q + q * q];
    double& alpha = s[3 * q + q * q + 1];
    int32_t* is = ist + MIN_IS * b;
    double* xt = xt_all + b * q;
    if (is[3] != KDEFFT_MIN_RUNNING) {
        for (int i = 0; i < q; ++i) xt[i] = x[i];
        return;
    }
    const double fb = ft[b];
    const double* gb = gt + b * q;
    bool ok = (stt == nullptr || stt[b] == 0) && isfinite(fb);
    for (int i = 0; i < q; ++i) ok = ok && isfinite(gb[i]);
    if (is[0] == PH_START) {
        for (int i = 0; i < q; ++i) {
            x[i] = xt[i];
            g[i] = gb[i];
        }
        f = fb;
        if (!ok) {
            is[3] = KDEFFT_MIN_BAD_START;
            return;
        }
        for (int i = 0; i < q * q; ++i) Hi[i] = (i % (q + 1)) == 0 ? 1.0 : 0.0;
        new_direction(q, x, g, p, Hi, &alpha, xt);
        is[0] = PH_LINE;
        is[1] = 0;
        return;
    }
    const double gp = dot(g, p, q);
    if (ok && fb <= f + C_ARMIJO * alpha * gp) {
        // accepted: BFGS update of the inverse Hessian with s = xt - x, y = gt - g
        double sv[MQ], yv[MQ], hy[MQ];
        for (int i = 0; i < q; ++i) {
            sv[i] = xt[i] - x[i];
            yv[i] = gb[i] - g[i];
        }
        const double sy = dot(sv, yv, q), yy = dot(yv, yv, q);
        // the update needs curvature well above the rounding of s and y
        if (yy > 0.0 && sy > 1e-10 * sqrt(dot(sv, sv, q) * yy)) {
            if (is[2] == 0) {
                // first accepted step: the identity scaled to the observed curvature
                const double sc = sy / yy;
                for (int i = 0; i < q * q; ++i) Hi[i] *= sc;
            }
            for (int i = 0; i < q; ++i) {
                double t = 0.0;
                for (int j = 0; j < q; ++j) t = fma(Hi[i * q + j], yv[j], t);
                hy[i] = t;
            }
            const double rho = 1.0 / sy;
            const double c = rho * (1.0 + rho * dot(yv, hy, q));
            for (int i = 0; i < q; ++i)
                for (int j = 0; j < q; ++j)
                    Hi[i * q + j] += c * sv[i] * sv[j] - rho * (hy[i] * sv[j] + sv[i] * hy[j]);
        }
        // a decrease within a few roundings of f is no decrease: two such
        // accepted steps in a row end the search (float64 offers no more)
        is[4] = f - fb <= 8.8817841970012523e-16 * fabs(f) ? is[4] + 1 : 0;
        for (int i = 0; i < q; ++i) {
            x[i] = xt[i];
            g[i] = gb[i];
        }
        f = fb;
        is[2] += 1;
        // first-order test, invariant to the scales of f and of x
        if (amax(g, q) * amax(x, q) <= tol * fabs(f)) {
            is[3] = KDEFFT_MIN_CONVERGED;
            for (int i = 0; i < q; ++i) xt[i] = x[i];
            return;
        }
        if (is[4] >= 2) {
            is[3] = KDEFFT_MIN_STALLED;
            for (int i = 0; i < q; ++i) xt[i] = x[i];
            return;
        }
        new_direction(q, x, g, p, Hi, &alpha, xt);
        is[1] = 0;
        return;
    }
    // rejected: shorten the step to the minimiser of the quadratic through
    // f, the slope gp and the trial value, kept within [0.1, 0.5] of the step
    if (++is[1] > MAX_BACK) {
        is[3] = KDEFFT_MIN_STALLED;
        for (int i = 0; i < q; ++i) xt[i] = x[i];
        return;
    }
    double an = 0.25 * alpha;
    if (ok) {
        const double den = 2.0 * (fb - f - alpha * gp);
        an = den > 0.0 ? -gp * alpha * alpha / den : 0.5 * alpha;
        an = fmin(fmax(an, 0.1 * alpha), 0.5 * alpha);
    }
    alpha = an;
    for (int i = 0; i < q; ++i) xt[i] = x[i] + an * p[i];
}

__global__ void k_min_final(int64_t B, int q, const double* __restrict__ st, const int32_t* __restrict__ ist,
                            double* __restrict__ x_out, double* __restrict__ f_out, int32_t* __restrict__ info) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const double* s = st + b * min_sw(q);
    for (int i = 0; i < q; ++i) x_out[b * q + i] = s[i];
    if (f_out) f_out[b] = s[3 * q + q * q];
    if (info) {
        info[2 * b] = ist[MIN_IS * b + 3];
        info[2 * b + 1] = ist[MIN_IS * b + 2];
    }
}

unsigned blocks_for(int64_t B) { return (unsigned)((B + 63) / 64); }

}  // namespace

int min_state_doubles(int q) { return min_sw(q); }
int min_state_ints() { return MIN_IS; }

hipError_t launch_min_init(int64_t B, int q, const double* x0, double* xt, int32_t* ist, hipStream_t s) {
    if (q < 1 || q > MQ) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_min_init, dim3(blocks_for(B)), dim3(64), 0, s, B, q, x0, xt, ist);
    return hipGetLastError();
}

hipError_t launch_min_step(int64_t B, int q, double tol, double* st, int32_t* ist, const double* ft,
                           const double* gt, const int32_t* stt, double* xt, hipStream_t s) {
    if (q < 1 || q > MQ) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_min_step, dim3(blocks_for(B)), dim3(64), 0, s, B, q, tol, st, ist, ft, gt, stt, xt);
    return hipGetLastError();
}

hipError_t launch_min_final(int64_t B, int q, const double* st, const int32_t* ist, double* x_out, double* f_out,
                            int32_t* info, hipStream_t s) {
    if (q < 1 || q > MQ) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_min_final, dim3(blocks_for(B)), dim3(64), 0, s, B, q, st, ist, x_out, f_out, info);
    return hipGetLastError();
}

}  // namespace kdefft
