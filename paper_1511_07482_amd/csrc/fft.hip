// Multi-dimensional real FFT for the zero-padded grids (Sec. 4, Eq. (19)-(23)):
// LDS-staged Stockham passes along one axis at a time.
//
//  * last axis (contiguous): real-to-complex through a half-length complex
//    transform of the even/odd pairs plus the standard split step, and the
//    inverse complex-to-real;
//  * leading axes (strided): each block loads a tile of T adjacent columns for
//    the full axis length (T * 16 contiguous bytes per row: coalesced), runs T
//    pencils in LDS and writes the tile back in place.  The axis-0 pass of the
//    count transform also forms |C|^2 and transforms it forward again while the
//    tile is still in LDS.
//
// Transforms are unnormalised: forward uses e^{-2 pi i jk/N}, inverse e^{+...}.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "dev_common.h"
#include "internal.h"

namespace kdefft {

// ------------------------------------------------------------------ twiddles
// One table per device; kernels receive its device address as an argument.
// [0, TWN): e^{-2 pi i m / TWN}; then, at offset TWN + N for each power of two
// N <= TWN, the N-point subset e^{-2 pi i j / N}, j < N (the same values, stored
// contiguously so a block can copy the subset it needs in whole cache lines).
static __device__ double2 g_twiddle[3 * TWN];

hipError_t twiddles(const double2** out) {
    static std::mutex mu;
    static const double2* ptr[64] = {nullptr};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        // cos/sin of 2 pi m / TWN from the first octant in long double, so that
        // symmetric entries are exactly symmetric and each value is rounded once.
        static double2 host[3 * TWN];
        const long double pi = 3.141592653589793238462643383279502884L;
        for (int m = 0; m < TWN; ++m) {
            int q = m / (TWN / 4), rr = m % (TWN / 4);  // quadrant, remainder
            long double cs, sn;
            if (rr <= TWN / 8) {
                long double a = 2.0L * pi * rr / TWN;
                cs = cosl(a);
                sn = sinl(a);
            } else {
                long double a = 2.0L * pi * (TWN / 4 - rr) / TWN;
                cs = sinl(a);
                sn = cosl(a);
            }
            long double c2, s2;  // rotate by q quarter turns
            switch (q) {
                case 0: c2 = cs; s2 = sn; break;
                case 1: c2 = -sn; s2 = cs; break;
                case 2: c2 = -cs; s2 = -sn; break;
                default: c2 = sn; s2 = -cs; break;
            }
            host[m] = make_double2((double)c2, -(double)s2);  // e^{-i theta}
        }
        for (int N = 1; N <= TWN; N *= 2)
            for (int j = 0; j < N; ++j) host[TWN + N + j] = host[j * (TWN / N)];
        e = hipMemcpyToSymbol(HIP_SYMBOL(g_twiddle), host, sizeof(host), 0, hipMemcpyHostToDevice);
        if (e != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_twiddle));
        if (e != hipSuccess) return e;
        ptr[dev] = static_cast<const double2*>(p);
    }
    *out = ptr[dev];
    return hipSuccess;
}

// ------------------------------------------------------------------ last axis
// Optional input maps of the last-axis passes.
//  * CountSrc: the R2C input row is read straight from the int64 grid counts,
//    or gathered from the binning's corner slots (c = count 2^-40 at [0, M)^d
//    of the circular layout, zero elsewhere), so the zero-padded real array is
//    never materialised.
//  * RowFlip: the C2R pass reads input row -l' (each leading index negated
//    modulo P) for output row l'.
struct CountSrc {
    const int64_t* counts;  // nullptr: read the real input array
    int d;
    int M[4];
    int P[4];
    int slots;              // counts holds the binning's corner slots, gathered here
    int64_t* sum_out;       // the gathered counts, written when slots is set
    int prune;              // only the rows inside the counts' box: row r of the launch is the counts'
                            // row r (leading indices over M), stored at its place in the padded grid;
                            // the padding's zero rows are not written (the next pass never reads them)
};

// Count of cell i = base + p (base: the cell of the row's first position, p
// the last-axis index; bit j - 1 of lmask: the row's index along axis d-1-j
// is >= 1) gathered from the corner slots of the last NSA axes: slot s of the
// record of cell i - e(s), e(s) = the sum over the set bits j of s of the
// stride of axis d-1-j, for the slots whose lower cell exists.  Exact
// (unsigned 64-bit sums).
template <int NSA>
__device__ __forceinline__ uint64_t gather_slots(const int64_t* __restrict__ sl, int64_t i, int p, int lmask,
                                                 const int* M, int d) {
    constexpr int NS = 1 << NSA;
    const int64_t st1 = NSA > 1 ? M[d - 1] : 0;
    const int64_t st2 = NSA > 2 ? st1 * M[d - 2] : 0;
    uint64_t t = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const bool ok = (!(s & 1) || p >= 1) && (!(s & 2) || (lmask & 1)) && (!(s & 4) || (lmask & 2));
        const int64_t off = (s & 1 ? 1 : 0) + (s & 2 ? st1 : 0) + (s & 4 ? st2 : 0);
        if (ok) t += static_cast<uint64_t>(sl[(i - off) * NS + s]);
    }
    return t;
}

// Count of cell base + p: read directly, or gathered from the corner slots
// (then also stored to sum_out).
__device__ __forceinline__ int64_t load_count(const CountSrc& cs, int64_t base, int p, int lmask) {
    const int64_t i = base + p;
    if (!cs.slots) return cs.counts[i];
    uint64_t t;
    if (cs.d == 1)
        t = gather_slots<1>(cs.counts, i, p, lmask, cs.M, cs.d);
    else if (cs.d == 2)
        t = gather_slots<2>(cs.counts, i, p, lmask, cs.M, cs.d);
    else
        t = gather_slots<3>(cs.counts, i, p, lmask, cs.M, cs.d);
    cs.sum_out[i] = static_cast<int64_t>(t);
    return static_cast<int64_t>(t);
}

struct RowFlip {
    int on;
    int nlead;
    int P[3];
    int mlast;   // > 0: positions of the last axis with |lag| > mlast - 1 are written as exact zeros
};

// Row indices of the passes are below 2^31 (checked on the host), so rows
// are decoded with 32-bit divisions.
__device__ __forceinline__ int64_t flip_row(int64_t row, const RowFlip& f) {
    uint32_t r = (uint32_t)row, out = 0, mul = 1;
    for (int k = f.nlead - 1; k >= 0; --k) {
        const uint32_t p = (uint32_t)f.P[k], i = r % p;
        r /= p;
        out += (i == 0 ? 0u : p - i) * mul;
        mul *= p;
    }
    return out;
}

// Rows per block for a last-axis pass of real length N.
template <int N>
constexpr int last_rows() { return (N / 2) >= 2048 ? 1 : 2048 / (N / 2); }

template <int N, int NT, int ROWS, int RADIX>
__global__ __launch_bounds__(NT) void k_r2c_last(const double* __restrict__ in, double2* __restrict__ out,
                                                 int64_t rows, const double2* __restrict__ tw, CountSrc cs) {
    constexpr int H = N / 2, Q = H + 1;
    constexpr int PS = H + 1;
    __shared__ double2 buf[ROWS * PS];
    __shared__ double2 twl[N];
    TwiddleCopy<N, NT> twc;
    twc.fetch(tw);
    const int64_t r0 = (int64_t)blockIdx.x * ROWS;
    const double2* src = reinterpret_cast<const double2*>(in);
    if (cs.counts) {
        const double quantum = 9.094947017729282379150390625e-13;  // 2^-40
        const int Ml = cs.M[cs.d - 1];
        // offset of each row's counts (-1: a zero row of the padding), decoded
        // once per row
        __shared__ int64_t rbase[ROWS];
        __shared__ int rmask[ROWS];   // bit 0: the row's index along axis d-2 is >= 1; bit 1: along d-3
        for (int rr = threadIdx.x; rr < ROWS; rr += NT) {
            const int64_t row = r0 + rr;
            int64_t base = -1;
            int mask = 0;
            if (row < rows) {
                // the row's leading indices: digits over M (pruned launches
                // run over the counts' rows) or over P (others)
                uint32_t rem = (uint32_t)row, cf = 0, mul = 1;
                bool ok = true;
                for (int k = cs.d - 2; k >= 0; --k) {
                    const uint32_t p = (uint32_t)(cs.prune ? cs.M[k] : cs.P[k]), i = rem % p;
                    rem /= p;
                    ok = ok && i < (uint32_t)cs.M[k];
                    if (k == cs.d - 2 && i >= 1) mask |= 1;
                    if (k == cs.d - 3 && i >= 1) mask |= 2;
                    cf += i * mul;
                    mul *= (uint32_t)cs.M[k];
                }
                if (ok) base = (int64_t)cf * Ml;
            }
            rbase[rr] = base;
            rmask[rr] = mask;
        }
        __syncthreads();
        // a block of zero rows only (the padding): its spectrum is zero
        bool any = false;
        for (int rr = 0; rr < ROWS; ++rr) any = any || rbase[rr] >= 0;
        if (!any) {
            for (int e = threadIdx.x; e < ROWS * Q; e += NT) {
                const int64_t row = r0 + e / Q;
                if (row < rows) out[row * Q + (e % Q)] = make_double2(0.0, 0.0);
            }
            return;
        }
        // a thread's elements in an unrolled loop, so that their loads are in
        // flight together (these passes are bound by load latency)
        constexpr int PE = (ROWS * H + NT - 1) / NT;
#pragma unroll
        for (int u = 0; u < PE; ++u) {
            const int e = threadIdx.x + u * NT;
            if ((ROWS * H) % NT == 0 || e < ROWS * H) {
                const int rr = e / H, m = e - rr * H;
                const int64_t base = rbase[rr];
                double2 v = make_double2(0.0, 0.0);
                if (base >= 0) {
                    const int p0 = 2 * m, p1 = 2 * m + 1, lm = rmask[rr];
                    if (p0 < Ml) v.x = (double)load_count(cs, base, p0, lm) * quantum;
                    if (p1 < Ml) v.y = (double)load_count(cs, base, p1, lm) * quantum;
                }
                buf[rr * PS + m] = v;
            }
        }
    } else {
        constexpr int PE = (ROWS * H + NT - 1) / NT;
#pragma unroll
        for (int u = 0; u < PE; ++u) {
            const int e = threadIdx.x + u * NT;
            if ((ROWS * H) % NT == 0 || e < ROWS * H) {
                const int rr = e / H, m = e - rr * H;
                const int64_t row = r0 + rr;
                buf[rr * PS + m] = row < rows ? src[row * H + m] : make_double2(0.0, 0.0);
            }
        }
    }
    twc.store(twl, tw);
    __syncthreads();
    fft_lds<H, ROWS, NT, -1, RADIX, N>(buf, PS, twl);
    __shared__ int64_t rout[ROWS];   // output row of each row: its place in the padded grid when pruned
    for (int rr = threadIdx.x; rr < ROWS; rr += NT) {
        int64_t row = r0 + rr;
        if (cs.counts && cs.prune) {
            uint32_t rem = (uint32_t)row, o = 0, mul = 1;
            for (int k = cs.d - 2; k >= 0; --k) {
                const uint32_t m = (uint32_t)cs.M[k];
                o += (rem % m) * mul;
                rem /= m;
                mul *= (uint32_t)cs.P[k];
            }
            row = o;
        }
        rout[rr] = row;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ROWS * Q; e += NT) {
        const int rr = e / Q, k = e - rr * Q;
        if (r0 + rr >= rows) continue;
        const int64_t row = rout[rr];
        const double2 zk = buf[rr * PS + (k == H ? 0 : k)];
        const double2 zc = c_conj(buf[rr * PS + (k == 0 ? 0 : H - k)]);
        const double2 E = c_scale(c_add(zk, zc), 0.5);
        const double2 O = c_rot<-1>(c_scale(c_sub(zk, zc), 0.5));  // (zk - zc)/(2i)
        const double2 w = twl[k];
        out[row * Q + k] = c_add(E, c_mul(w, O));
    }
}

template <int N, int NT, int ROWS, int RADIX>
__global__ __launch_bounds__(NT) void k_c2r_last(const double2* __restrict__ in, double* __restrict__ out,
                                                 int64_t rows, const double2* __restrict__ tw, RowFlip fl) {
    constexpr int H = N / 2, Q = H + 1;
    constexpr int PS = H + 1;
    __shared__ double2 buf[ROWS * PS];
    __shared__ double2 twl[N];
    __shared__ int64_t rsrc[ROWS];   // source row of each row (-1: past the end), decoded once per row
    TwiddleCopy<N, NT> twc;
    twc.fetch(tw);
    const int64_t r0 = (int64_t)blockIdx.x * ROWS;
    for (int rr = threadIdx.x; rr < ROWS; rr += NT) {
        const int64_t row = r0 + rr;
        rsrc[rr] = row < rows ? (fl.on ? flip_row(row, fl) : row) : -1;
    }
    __syncthreads();
    {
        constexpr int PE = (ROWS * Q + NT - 1) / NT;   // unrolled: the loads in flight together
#pragma unroll
        for (int u = 0; u < PE; ++u) {
            const int e = threadIdx.x + u * NT;
            if ((ROWS * Q) % NT == 0 || e < ROWS * Q) {
                const int rr = e / Q, k = e - rr * Q;
                const int64_t src_row = rsrc[rr];
                buf[rr * PS + k] = src_row >= 0 ? in[src_row * Q + k] : make_double2(0.0, 0.0);
            }
        }
    }
    twc.store(twl, tw);
    __syncthreads();
    constexpr int PER = (ROWS * H + NT - 1) / NT;
    double2 z[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int e = threadIdx.x + u * NT;
        if (e < ROWS * H) {
            const int rr = e / H, k = e - rr * H;
            const double2 xk = buf[rr * PS + k];
            const double2 xc = c_conj(buf[rr * PS + H - k]);
            const double2 E = c_scale(c_add(xk, xc), 0.5);
            const double2 O = c_scale(c_mulc(c_sub(xk, xc), twl[k]), 0.5);  // * e^{+i..}
            z[u] = c_add(E, c_rot<1>(O));
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int e = threadIdx.x + u * NT;
        if (e < ROWS * H) {
            const int rr = e / H, k = e - rr * H;
            buf[rr * PS + k] = z[u];
        }
    }
    __syncthreads();
    fft_lds<H, ROWS, NT, 1, RADIX, N>(buf, PS, twl);
    double2* dst = reinterpret_cast<double2*>(out);
    for (int e = threadIdx.x; e < ROWS * H; e += NT) {
        const int rr = e / H, m = e - rr * H;
        const int64_t row = r0 + rr;
        if (row >= rows) continue;
        double2 v = c_scale(buf[rr * PS + m], 2.0);
        if (fl.mlast > 0) {
            // positions 2m, 2m + 1 hold lags p (p < N/2) or p - N
            const int p0 = 2 * m, p1 = 2 * m + 1;
            if (p0 > fl.mlast - 1 && p0 < N - (fl.mlast - 1)) v.x = 0.0;
            if (p1 > fl.mlast - 1 && p1 < N - (fl.mlast - 1)) v.y = 0.0;
        }
        dst[row * H + m] = v;
    }
}

// ------------------------------------------------------------------ strided axes
// Columns per tile: the largest power of two <= 16 whose padded tile fits 64 KiB.
template <int N>
constexpr int tile_cols() {
    return 4096 / (N + 1) >= 16 ? 16 : 4096 / (N + 1) >= 8 ? 8 : 4096 / (N + 1) >= 4 ? 4
         : 4096 / (N + 1) >= 2 ? 2 : 1;
}

// Zero structure of a forward count-transform pass along axis a (pruning):
// the counts fill [0, M)^d of the padded P^d grid, so before the pass a
// column (outer index i_0..i_{a-1} over the axes before a) can be nonzero only
// if every i_k < M_k, and within it only its first M_a entries.  The launch
// covers the live columns only (its outer index runs over the M_k extents and
// is placed in the P_k-extent buffer; the dead columns are neither read nor
// written: the next pass, along a - 1, reads only live columns' outputs), and
// only the first nlive entries of a column are read.  na = 0, nlive = N: the
// dense transform.
struct Prune {
    int na;       // axes before the pass's axis
    int P[3];     // their extents (outer index digits, major first)
    int M[3];     // their count extents
    int nlive;    // entries of a live column that can be nonzero
};

// MODE 0: in-place transform.  MODE 1: forward transform stored in place
// (the finished count spectrum C), then |C|^2 transformed forward again and
// stored to out2.
template <int N, int NT, int DIR, int MODE, int T, int RADIX>
__global__ __launch_bounds__(NT) void k_c2c_strided(double2* __restrict__ buf, double2* __restrict__ out2,
                                                    int64_t inner, int64_t tiles,
                                                    const double2* __restrict__ tw, Prune pr) {
    constexpr int PS = T > 1 ? N + 1 : N;
    __shared__ double2 lds[T * PS];
    __shared__ double2 twl[N];
    TwiddleCopy<N, NT> twc;
    twc.fetch(tw);
    // block indices and outer indices are below 2^32: 32-bit divisions
    const uint32_t ol = blockIdx.x / (uint32_t)tiles;
    uint32_t o = ol;
    if (pr.na > 0) {   // live column ol (extents M) -> its outer index in the buffer (extents P)
        uint32_t rem = ol, mul = 1;
        o = 0;
        for (int k = pr.na - 1; k >= 0; --k) {
            const uint32_t m = (uint32_t)pr.M[k];
            o += (rem % m) * mul;
            rem /= m;
            mul *= (uint32_t)pr.P[k];
        }
    }
    const int64_t i0 = (int64_t)(blockIdx.x - ol * (uint32_t)tiles) * T;
    double2* base = buf + (int64_t)o * N * inner + i0;
    {
        constexpr int PE = (N * T + NT - 1) / NT;   // unrolled: the loads in flight together
#pragma unroll
        for (int u = 0; u < PE; ++u) {
            const int e = threadIdx.x + u * NT;
            if ((N * T) % NT == 0 || e < N * T) {
                const int t = e % T, p = e / T;
                lds[t * PS + p] =
                    (i0 + t < inner && p < pr.nlive) ? base[(int64_t)p * inner + t] : make_double2(0.0, 0.0);
            }
        }
    }
    twc.store(twl, tw);
    __syncthreads();
    fft_lds<N, T, NT, DIR, RADIX, N>(lds, PS, twl);
    for (int e = threadIdx.x; e < N * T; e += NT) {
        const int t = e % T, p = e / T;
        if (i0 + t < inner) base[(int64_t)p * inner + t] = lds[t * PS + p];
    }
    if constexpr (MODE == 1) {
        for (int e = threadIdx.x; e < N * T; e += NT) {
            const int t = e % T, p = e / T;
            const double2 v = lds[t * PS + p];
            lds[t * PS + p] = make_double2(v.x * v.x + v.y * v.y, 0.0);
        }
        __syncthreads();
        fft_lds<N, T, NT, -1, RADIX, N>(lds, PS, twl);
        double2* b2 = out2 + (int64_t)o * N * inner + i0;
        for (int e = threadIdx.x; e < N * T; e += NT) {
            const int t = e % T, p = e / T;
            if (i0 + t < inner) b2[(int64_t)p * inner + t] = lds[t * PS + p];
        }
    }
}

// |C|^2 for d = 1 (no leading axis).
__global__ void k_abs2(const double2* __restrict__ in, double2* __restrict__ out, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double2 v = in[i];
        out[i] = make_double2(v.x * v.x + v.y * v.y, 0.0);
    }
}

// ------------------------------------------------------------------ dispatch
static int ilog2i(int n) { int k = 0; while ((1 << k) < n) ++k; return k; }

// Launch shapes.  Default: ~2048 complex values per block (256 threads).
// Small problems (fewer than ~512 blocks at the default shape) take one or a
// few pencils per block instead, so more CUs take part: the pencils of one
// wavefront's shape on 256 threads, whose extra lanes shorten the loads and
// stores that bound these passes (part of them idle in the stages).
constexpr int64_t kMinBlocks = 512;

// pencils of one wavefront (at most 16, ~512 values), and half of them (at
// least one) for the 256-thread small shape
template <int N>
constexpr int small_rows() { return (N / 2) >= 512 ? 1 : ((512 / (N / 2)) > 16 ? 16 : 512 / (N / 2)); }
template <int N>
constexpr int deep_rows() { return small_rows<N>() > 1 ? small_rows<N>() / 2 : 1; }

// FFT-stage schedules (the tuner's choices, per grid shape):
//   FS_AUTO    the shape rule above, radix-8 stages first;
//   FS_RADIX4  the same shapes, radix-4 stages (one radix-8 or 2 when log2 is odd);
//   FS_WIDE    256-thread blocks of the default shape for every pass;
//   FS_NARROW  one-wavefront blocks for every pass that has them;
//   FS_HALF    strided passes on T/2-column tiles (twice the blocks), last axis as FS_AUTO;
//   FS_DEEP    the small problems' 256-thread shapes for every pass that has them.
enum { FS_AUTO = 0, FS_RADIX4 = 1, FS_WIDE = 2, FS_NARROW = 3, FS_HALF = 4, FS_DEEP = 5 };

// Radix-4 stages for schedule FS_RADIX4, and under the default schedule for
// 64-point passes (4 x 4 x 4 measured up to 6% faster than 8 x 8 over a
// d = 4, P = 64 transform streaming from HBM; other lengths keep radix 8 first).
template <int N>
constexpr bool radix4_for_default() { return N == 64; }
template <int N>
static bool radix4_for(int fs) { return fs == FS_RADIX4 || (fs == FS_AUTO && radix4_for_default<N>()); }

// Last-axis launch shapes: ROWS rows on 256 threads, small_rows on one
// wavefront, deep_rows on 256 threads.
enum { SH_WIDE = 0, SH_NARROW = 1, SH_DEEP = 2 };

template <int N, int RADIX>
static void launch_r2c_shape(int sh, const double* in, double2* out, int64_t rows, const double2* tw,
                             hipStream_t s, CountSrc cs) {
    constexpr int ROWS = last_rows<N>();
    constexpr int RS = small_rows<N>();
    constexpr int RD = deep_rows<N>();
    if (sh == SH_NARROW && RS < ROWS)
        hipLaunchKernelGGL((k_r2c_last<N, 64, RS, RADIX>), dim3((unsigned)((rows + RS - 1) / RS)), dim3(64), 0, s,
                           in, out, rows, tw, cs);
    else if (sh == SH_DEEP && RS < ROWS)
        hipLaunchKernelGGL((k_r2c_last<N, 256, RD, RADIX>), dim3((unsigned)((rows + RD - 1) / RD)), dim3(256), 0,
                           s, in, out, rows, tw, cs);
    else
        hipLaunchKernelGGL((k_r2c_last<N, 256, ROWS, RADIX>), dim3((unsigned)((rows + ROWS - 1) / ROWS)), dim3(256),
                           0, s, in, out, rows, tw, cs);
}

template <int N, int RADIX>
static void launch_c2r_shape(int sh, const double2* in, double* out, int64_t rows, const double2* tw,
                             hipStream_t s, RowFlip fl) {
    constexpr int ROWS = last_rows<N>();
    constexpr int RS = small_rows<N>();
    constexpr int RD = deep_rows<N>();
    if (sh == SH_NARROW && RS < ROWS)
        hipLaunchKernelGGL((k_c2r_last<N, 64, RS, RADIX>), dim3((unsigned)((rows + RS - 1) / RS)), dim3(64), 0, s,
                           in, out, rows, tw, fl);
    else if (sh == SH_DEEP && RS < ROWS)
        hipLaunchKernelGGL((k_c2r_last<N, 256, RD, RADIX>), dim3((unsigned)((rows + RD - 1) / RD)), dim3(256), 0,
                           s, in, out, rows, tw, fl);
    else
        hipLaunchKernelGGL((k_c2r_last<N, 256, ROWS, RADIX>), dim3((unsigned)((rows + ROWS - 1) / ROWS)), dim3(256),
                           0, s, in, out, rows, tw, fl);
}

// last-axis launch shape for schedule fs
template <int N>
static int last_shape(int64_t rows, int fs) {
    constexpr int ROWS = last_rows<N>();
    if (fs == FS_WIDE) return SH_WIDE;
    if (fs == FS_NARROW) return SH_NARROW;
    if (fs == FS_DEEP) return SH_DEEP;
    return (rows + ROWS - 1) / ROWS < kMinBlocks ? SH_DEEP : SH_WIDE;
}

template <int N>
static hipError_t run_r2c_last(const double* in, double2* out, int64_t rows, const double2* tw, hipStream_t s,
                               CountSrc cs, int fs) {
    const int sh = last_shape<N>(rows, fs);
    if (radix4_for<N>(fs))
        launch_r2c_shape<N, 1>(sh, in, out, rows, tw, s, cs);
    else
        launch_r2c_shape<N, 0>(sh, in, out, rows, tw, s, cs);
    return hipGetLastError();
}
template <int N>
static hipError_t run_c2r_last(const double2* in, double* out, int64_t rows, const double2* tw, hipStream_t s,
                               RowFlip fl, int fs) {
    const int sh = last_shape<N>(rows, fs);
    if (radix4_for<N>(fs))
        launch_c2r_shape<N, 1>(sh, in, out, rows, tw, s, fl);
    else
        launch_c2r_shape<N, 0>(sh, in, out, rows, tw, s, fl);
    return hipGetLastError();
}

template <int N, int NT, int T, int RADIX>
static void launch_c2c_t(double2* buf, double2* out2, int64_t outer, int64_t inner, int dir, int mode,
                         const double2* tw, hipStream_t s, const Prune& pr) {
    const int64_t tiles = (inner + T - 1) / T;
    const dim3 grid((unsigned)(outer * tiles));
    if (mode == 1)
        hipLaunchKernelGGL((k_c2c_strided<N, NT, -1, 1, T, RADIX>), grid, dim3(NT), 0, s, buf, out2, inner, tiles,
                           tw, pr);
    else if (dir < 0)
        hipLaunchKernelGGL((k_c2c_strided<N, NT, -1, 0, T, RADIX>), grid, dim3(NT), 0, s, buf, out2, inner, tiles,
                           tw, pr);
    else
        hipLaunchKernelGGL((k_c2c_strided<N, NT, 1, 0, T, RADIX>), grid, dim3(NT), 0, s, buf, out2, inner, tiles,
                           tw, pr);
}

// Slab tiles: when the axis is the last leading one its inner extent is the
// half-spectrum length Q = P/2 + 1 (17, 33, 65, ...), which T-column tiles
// cover raggedly (33 = 16 + 16 + 1).  For Q = 17 and 33 one block takes the
// whole contiguous [N][Q] slab instead (fully coalesced, no partial tile)
// while it fits 80 KiB of LDS.
template <int N, int Q>
constexpr bool slab_fits() { return N >= 8 && Q * (N + 1) * 16 <= 81920; }

template <int N, int RADIX>
static void run_c2c_r(double2* buf, double2* out2, int64_t outer, int64_t inner, int dir, int mode,
                      const double2* tw, hipStream_t s, int fs, const Prune& pr) {
    constexpr int T = tile_cols<N>();
    constexpr int TS = N >= 64 ? 1 : (64 / N > 16 ? 16 : 64 / N);  // one radix pass per lane
    constexpr int TH = T > 1 ? T / 2 : 1;
    const bool small = outer * ((inner + T - 1) / T) < kMinBlocks;
    if (fs != FS_NARROW && fs != FS_HALF && fs != FS_DEEP) {
        if constexpr (slab_fits<N, 33>()) {
            if (inner == 33 && (outer >= kMinBlocks || fs == FS_WIDE)) {
                launch_c2c_t<N, 256, 33, RADIX>(buf, out2, outer, inner, dir, mode, tw, s, pr);
                return;
            }
        }
        if constexpr (slab_fits<N, 17>()) {
            if (inner == 17 && (outer >= kMinBlocks || fs == FS_WIDE)) {
                launch_c2c_t<N, 256, 17, RADIX>(buf, out2, outer, inner, dir, mode, tw, s, pr);
                return;
            }
        }
    }
    if constexpr (TS < T) {
        // one-wavefront blocks (FS_NARROW), or the same tiles on 256 threads
        if (fs == FS_NARROW) {
            launch_c2c_t<N, 64, TS, RADIX>(buf, out2, outer, inner, dir, mode, tw, s, pr);
            return;
        }
        if (fs == FS_DEEP || (fs != FS_WIDE && small)) {
            launch_c2c_t<N, 256, TS, RADIX>(buf, out2, outer, inner, dir, mode, tw, s, pr);
            return;
        }
    }
    if constexpr (RADIX == 0 && TH < T) {
        if (fs == FS_HALF) {
            launch_c2c_t<N, 256, TH, 0>(buf, out2, outer, inner, dir, mode, tw, s, pr);
            return;
        }
    }
    launch_c2c_t<N, 256, T, RADIX>(buf, out2, outer, inner, dir, mode, tw, s, pr);
}

template <int N>
static hipError_t run_c2c(double2* buf, double2* out2, int64_t outer, int64_t inner, int dir, int mode,
                          const double2* tw, hipStream_t s, int fs, const Prune& pr) {
    if (radix4_for<N>(fs))
        run_c2c_r<N, 1>(buf, out2, outer, inner, dir, mode, tw, s, fs, pr);
    else
        run_c2c_r<N, 0>(buf, out2, outer, inner, dir, mode, tw, s, fs, pr);
    return hipGetLastError();
}

#define KDEFFT_SWITCH_N(LOGN, CALL)                           \
    switch (LOGN) {                                          \
        case 1: return CALL(2);                              \
        case 2: return CALL(4);                              \
        case 3: return CALL(8);                              \
        case 4: return CALL(16);                             \
        case 5: return CALL(32);                             \
        case 6: return CALL(64);                             \
        case 7: return CALL(128);                            \
        case 8: return CALL(256);                            \
        case 9: return CALL(512);                            \
        case 10: return CALL(1024);                          \
        case 11: return CALL(2048);                          \
        case 12: return CALL(4096);                          \
        default: return hipErrorInvalidValue;                \
    }

static hipError_t r2c_last(const double* in, double2* out, int64_t rows, int N, const double2* tw, hipStream_t s,
                           CountSrc cs = CountSrc{nullptr, 0, {0, 0, 0, 0}, {0, 0, 0, 0}, 0, nullptr, 0},
                           int fs = FS_AUTO) {
#define CALL(NN) run_r2c_last<NN>(in, out, rows, tw, s, cs, fs)
    if (N < 4) return hipErrorInvalidValue;
    KDEFFT_SWITCH_N(ilog2i(N), CALL)
#undef CALL
}
static hipError_t c2r_last(const double2* in, double* out, int64_t rows, int N, const double2* tw, hipStream_t s,
                           RowFlip fl = RowFlip{0, 0, {1, 1, 1}, 0}, int fs = FS_AUTO) {
#define CALL(NN) run_c2r_last<NN>(in, out, rows, tw, s, fl, fs)
    if (N < 4) return hipErrorInvalidValue;
    KDEFFT_SWITCH_N(ilog2i(N), CALL)
#undef CALL
}
static hipError_t c2c(double2* buf, double2* out2, int64_t outer, int N, int64_t inner, int dir, int mode,
                      const double2* tw, hipStream_t s, int fs = FS_AUTO, Prune pr = Prune{0, {1, 1, 1}, {1, 1, 1}, 0}) {
    if (pr.nlive <= 0 || pr.nlive > N) pr.nlive = N;
    if (pr.na > 0) {   // the launch covers the live columns only
        outer = 1;
        for (int k = 0; k < pr.na; ++k) outer *= pr.M[k];
    }
#define CALL(NN) run_c2c<NN>(buf, out2, outer, inner, dir, mode, tw, s, fs, pr)
    KDEFFT_SWITCH_N(ilog2i(N), CALL)
#undef CALL
}

// Shape helpers: the half-spectrum is [P_0, ..., P_{d-2}, Q].
static int64_t lead_count(const kdefft_grid& g) {
    int64_t r = 1;
    for (int k = 0; k + 1 < g.d; ++k) r *= g.P[k];
    return r;
}
// the kernels decode row and column indices in 32 bits
static bool shape_ok(const kdefft_grid& g) {
    return g.d >= 1 && g.d <= 4 && lead_count(g) * (g.P[g.d - 1] / 2 + 1) < (int64_t(1) << 31);
}
static void axis_shape(const kdefft_grid& g, int axis, int64_t* outer, int64_t* inner) {
    int64_t o = 1, in = g.P[g.d - 1] / 2 + 1;
    for (int k = 0; k < axis; ++k) o *= g.P[k];
    for (int k = axis + 1; k + 1 < g.d; ++k) in *= g.P[k];
    *outer = o;
    *inner = in;
}

hipError_t fft_c2c_axis(double2* buf, const kdefft_grid& g, int axis, int dir, hipStream_t s) {
    if (!shape_ok(g)) return hipErrorInvalidValue;
    const double2* tw;
    hipError_t e = twiddles(&tw);
    if (e != hipSuccess) return e;
    int64_t outer, inner;
    axis_shape(g, axis, &outer, &inner);
    return c2c(buf, nullptr, outer, g.P[axis], inner, dir, 0, tw, s);
}

hipError_t fft_r2c_nd(const double* in, double2* out, const kdefft_grid& g, hipStream_t s) {
    if (!shape_ok(g)) return hipErrorInvalidValue;
    const double2* tw;
    hipError_t e = twiddles(&tw);
    if (e != hipSuccess) return e;
    e = r2c_last(in, out, lead_count(g), g.P[g.d - 1], tw, s);
    for (int ax = g.d - 2; ax >= 0 && e == hipSuccess; --ax) {
        int64_t outer, inner;
        axis_shape(g, ax, &outer, &inner);
        e = c2c(out, nullptr, outer, g.P[ax], inner, -1, 0, tw, s);
    }
    return e;
}

hipError_t fft_c2r_nd(double2* inout, double* out, const kdefft_grid& g, hipStream_t s) {
    if (!shape_ok(g)) return hipErrorInvalidValue;
    const double2* tw;
    hipError_t e = twiddles(&tw);
    if (e != hipSuccess) return e;
    for (int ax = 0; ax + 1 < g.d && e == hipSuccess; ++ax) {
        int64_t outer, inner;
        axis_shape(g, ax, &outer, &inner);
        e = c2c(inout, nullptr, outer, g.P[ax], inner, 1, 0, tw, s);
    }
    if (e != hipSuccess) return e;
    return c2r_last(inout, out, lead_count(g), g.P[g.d - 1], tw, s);
}

hipError_t fft_prepare_nd(const int64_t* src, int slots, int64_t* counts, double2* spec, double2* wmix,
                          const kdefft_grid& g, hipStream_t s, int fs) {
    if (fs < 0 || fs >= FFT_SCHEDULES || !shape_ok(g)) return hipErrorInvalidValue;
    const double2* tw;
    hipError_t e = twiddles(&tw);
    if (e != hipSuccess) return e;
    CountSrc cs{src, g.d, {1, 1, 1, 1}, {1, 1, 1, 1}, slots ? 1 : 0, counts, 1};
    for (int k = 0; k < g.d; ++k) {
        cs.M[k] = g.M[k];
        cs.P[k] = g.P[k];
    }
    if (slots && !counts) return hipErrorInvalidValue;
    // the R2C covers the rows inside the counts' box only (prod of the leading M)
    int64_t rows_live = 1;
    for (int k = 0; k + 1 < g.d; ++k) rows_live *= g.M[k];
    e = r2c_last(nullptr, spec, rows_live, g.P[g.d - 1], tw, s, cs, fs);
    if (e != hipSuccess) return e;
    if (g.d == 1) {
        const int64_t cnt = g.P[0] / 2 + 1;
        hipLaunchKernelGGL(k_abs2, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, spec, wmix, cnt);
        return hipGetLastError();
    }
    // forward passes over the counts' spectrum, pruned: before the pass along
    // axis a only columns with i_k < M_k (k < a) are nonzero, and only their
    // first M_a entries
    for (int ax = g.d - 2; ax >= 1 && e == hipSuccess; --ax) {
        int64_t outer, inner;
        axis_shape(g, ax, &outer, &inner);
        Prune pr{ax, {1, 1, 1}, {1, 1, 1}, g.M[ax]};
        for (int k = 0; k < ax; ++k) {
            pr.P[k] = g.P[k];
            pr.M[k] = g.M[k];
        }
        e = c2c(spec, nullptr, outer, g.P[ax], inner, -1, 0, tw, s, fs, pr);
    }
    if (e != hipSuccess) return e;
    {
        int64_t outer, inner;
        axis_shape(g, 0, &outer, &inner);
        e = c2c(spec, wmix, outer, g.P[0], inner, -1, 1, tw, s, fs, Prune{0, {1, 1, 1}, {1, 1, 1}, g.M[0]});
    }
    for (int ax = 1; ax + 1 < g.d && e == hipSuccess; ++ax) {
        int64_t outer, inner;
        axis_shape(g, ax, &outer, &inner);
        e = c2c(wmix, nullptr, outer, g.P[ax], inner, -1, 0, tw, s, fs);
    }
    return e;
}

hipError_t fft_autocorr_nd(const double2* wmix, double* alag, const kdefft_grid& g, hipStream_t s, int fs) {
    if (!shape_ok(g)) return hipErrorInvalidValue;
    if (fs < 0 || fs >= FFT_SCHEDULES) return hipErrorInvalidValue;
    const double2* tw;
    hipError_t e = twiddles(&tw);
    if (e != hipSuccess) return e;
    // inverting |C|^2 along the leading axes = the forward transform (wmix)
    // read at negated leading indices; then the last-axis inverse.  Lags with
    // |l| >= M along the last axis are zero in exact arithmetic (the counts
    // occupy [0, M)) and are stored as exact zeros.
    RowFlip fl{g.d > 1 ? 1 : 0, g.d - 1, {1, 1, 1}, g.M[g.d - 1]};
    for (int k = 0; k + 1 < g.d; ++k) fl.P[k] = g.P[k];
    return c2r_last(wmix, alag, lead_count(g), g.P[g.d - 1], tw, s, fl, fs);
}

}  // namespace kdefft
