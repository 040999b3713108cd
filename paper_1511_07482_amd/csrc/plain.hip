// The paper's steps 2-4 taken literally, one kernel grid at a time (Sec. 4):
//   step 2: kernel values on the full symmetric lag grid, stored in the
//           circular zero-padded layout (lag l at index l mod P, Eq. (18));
//   step 3: K = R2C(k), S = C K, s = C2R(S) / prod P (Eq. (22)-(23));
//   step 4: n^-2 sum_i c_i s_i over the grid nodes (Eq. (24)).
// Each step is its own launch.  Reductions use a fixed block count and a fixed
// order, so results are reproducible bit for bit.
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "dev_kernels.h"
#include "internal.h"

namespace kdefft {

// ------------------------------------------------------------------ step 2
template <int D, class Fun>
__global__ __launch_bounds__(256) void k_kgrid(double* __restrict__ out, kdefft_grid g, int64_t total,
                                               ParamBlock prm, int entry) {
    Fun f;
    f.load(prm.v);
    for (int64_t e = blockIdx.x * 256LL + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        int64_t rem = e;
        double x[D];
        bool nz = true;
#pragma unroll
        for (int k = D - 1; k >= 0; --k) {
            const int p = (int)(rem % g.P[k]);
            rem /= g.P[k];
            int lag = 0;
            nz = nz && lag_of(p, g.M[k], g.P[k], &lag);
            x[k] = g.delta[k] * (double)lag;
        }
        double v = 0.0;
        if (nz) {
            double vals[Fun::NG];
            f.eval(x, vals);
            v = vals[entry];
        }
        out[e] = v;
    }
}

static int64_t prod_P(const kdefft_grid& g) {
    int64_t t = 1;
    for (int k = 0; k < g.d; ++k) t *= g.P[k];
    return t;
}

static unsigned grid_for(int64_t total) {
    int64_t b = (total + 255) / 256;
    return (unsigned)(b > 16384 ? 16384 : (b < 1 ? 1 : b));
}

template <int D, int R>
static hipError_t kgrid_psi_t(double* out, const kdefft_grid& g, const ParamBlock& prm, int entry, hipStream_t s) {
    const int64_t total = prod_P(g);
    hipLaunchKernelGGL((k_kgrid<D, PsiFun<D, R>>), dim3(grid_for(total)), dim3(256), 0, s, out, g, total, prm, entry);
    return hipGetLastError();
}

hipError_t launch_kgrid_psi(double* out, const kdefft_grid& g, int r, const ParamBlock& prm, int entry,
                            hipStream_t s) {
#define KG(DD, RR) if (g.d == DD && r == RR) return kgrid_psi_t<DD, RR>(out, g, prm, entry, s);
    KG(1, 0) KG(1, 2) KG(1, 4) KG(1, 6) KG(1, 8)
    KG(2, 0) KG(2, 2) KG(2, 4) KG(2, 6) KG(2, 8)
    KG(3, 0) KG(3, 2) KG(3, 4) KG(3, 6)
    KG(4, 0) KG(4, 2) KG(4, 4)
#undef KG
    return hipErrorInvalidValue;
}

hipError_t launch_kgrid_scv(double* out, const kdefft_grid& g, const ParamBlock& prm, int entry, hipStream_t s) {
    const int64_t total = prod_P(g);
    switch (g.d) {
        case 1: hipLaunchKernelGGL((k_kgrid<1, ScvPlainFun<1>>), dim3(grid_for(total)), dim3(256), 0, s, out, g, total, prm, entry); break;
        case 2: hipLaunchKernelGGL((k_kgrid<2, ScvPlainFun<2>>), dim3(grid_for(total)), dim3(256), 0, s, out, g, total, prm, entry); break;
        case 3: hipLaunchKernelGGL((k_kgrid<3, ScvPlainFun<3>>), dim3(grid_for(total)), dim3(256), 0, s, out, g, total, prm, entry); break;
        case 4: hipLaunchKernelGGL((k_kgrid<4, ScvPlainFun<4>>), dim3(grid_for(total)), dim3(256), 0, s, out, g, total, prm, entry); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ step 3 product
__global__ void k_cmul(double2* __restrict__ K, const double2* __restrict__ C, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        K[i] = c_mul(C[i], K[i]);
}

hipError_t launch_cmul(double2* K, const double2* C, int64_t count, hipStream_t s) {
    hipLaunchKernelGGL(k_cmul, dim3(grid_for(count)), dim3(256), 0, s, K, C, count);
    return hipGetLastError();
}

// ------------------------------------------------------------------ step 4
// partial[b] = sum over the nodes handled by block b of c_i * s_i, where
// c_i = counts_i 2^-40 and s is the circular convolution (unscaled).
template <int D>
__global__ __launch_bounds__(256) void k_dot_counts(const int64_t* __restrict__ counts,
                                                    const double* __restrict__ sreal, kdefft_grid g,
                                                    int64_t total, double* __restrict__ partial) {
    __shared__ double scratch[4];
    const double quantum = 9.094947017729282379150390625e-13;  // 2^-40
    double acc = 0.0;
    for (int64_t e = blockIdx.x * 256LL + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        int64_t rem = e, pf = 0, mul = 1;
#pragma unroll
        for (int k = D - 1; k >= 0; --k) {
            const int i = (int)(rem % g.M[k]);
            rem /= g.M[k];
            pf += i * mul;
            mul *= g.P[k];
        }
        acc += ((double)counts[e] * quantum) * sreal[pf];
    }
    double v[1] = {acc}, out[1];
    block_sum<1, 256>(v, scratch, out);
    if (threadIdx.x == 0) partial[blockIdx.x] = out[0];
}

hipError_t launch_dot_counts(const int64_t* counts, const double* sreal, const kdefft_grid& g,
                             double* partial, int nblk, hipStream_t s) {
    int64_t total = 1;
    for (int k = 0; k < g.d; ++k) total *= g.M[k];
    switch (g.d) {
        case 1: hipLaunchKernelGGL(k_dot_counts<1>, dim3(nblk), dim3(256), 0, s, counts, sreal, g, total, partial); break;
        case 2: hipLaunchKernelGGL(k_dot_counts<2>, dim3(nblk), dim3(256), 0, s, counts, sreal, g, total, partial); break;
        case 3: hipLaunchKernelGGL(k_dot_counts<3>, dim3(nblk), dim3(256), 0, s, counts, sreal, g, total, partial); break;
        case 4: hipLaunchKernelGGL(k_dot_counts<4>, dim3(nblk), dim3(256), 0, s, counts, sreal, g, total, partial); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// out[0] = scale * sum_b partial[b], fixed order.
__global__ __launch_bounds__(256) void k_sum_scale(const double* __restrict__ partial, int nblk, double scale,
                                                   double* __restrict__ out) {
    __shared__ double scratch[4];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) acc += partial[b];
    double v[1] = {acc}, o[1];
    block_sum<1, 256>(v, scratch, o);
    if (threadIdx.x == 0) out[0] = o[0] * scale;
}

hipError_t launch_sum_scale(const double* partial, int nblk, double scale, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_scale, dim3(1), dim3(256), 0, s, partial, nblk, scale, out);
    return hipGetLastError();
}

// SCV(H) and d SCV / d vech(L) from the plain-path sums.
// sums[0] = n^-2 sum sum [phi_{S1} - 2 phi_{S2} + phi_{2G}], sums[1..q] the
// Hessian sums (already scaled).  fin: H^{-1} in slots [0,16), L in [16,32)
// (row stride 4), the first term n^-1 (4 pi)^{-d/2} |H|^{-1/2} in slot 32.
__global__ void k_scv_plain_final(const double* __restrict__ sums, ParamBlock fin, int d,
                                  double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    const double* prm = fin.v;
    const double first = prm[32];
    double gH[4][4];
    int t = 1;
    for (int i = 0; i < d; ++i)
        for (int j = i; j < d; ++j) {
            const double v = -0.5 * first * prm[0 + i * 4 + j] + sums[t++];
            gH[i][j] = v;
            gH[j][i] = v;
        }
    out[0] = first + sums[0];
    // d SCV / d L = lower(2 gH L), vech by columns of the lower triangle
    int o = 1;
    for (int j = 0; j < d; ++j)
        for (int i = j; i < d; ++i) {
            double s = 0.0;
            for (int k = 0; k < d; ++k) s += gH[i][k] * prm[16 + k * 4 + j];
            out[o++] = 2.0 * s;
        }
}

hipError_t launch_scv_plain_final(const double* sums, const ParamBlock& fin, int d, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_scv_plain_final, dim3(1), dim3(64), 0, s, sums, fin, d, out);
    return hipGetLastError();
}

}  // namespace kdefft
