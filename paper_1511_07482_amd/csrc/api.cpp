// C-ABI entry points of libkdefft: argument validation, grid planning,
// workspace layout, and the order of launches for each operation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"

using namespace kdefft;

namespace {

// Candidates per timed launch in kdefft_autotune.
constexpr int TUNE_B = 256;
constexpr int TUNE_PSI_OUT = 64;   // psi_4 outputs of one dataset (35 for d = 4)

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(KDEFFT_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(expr, what)                          \
    do {                                            \
        hipError_t _e = (expr);                     \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

int64_t binom(int n, int k) {
    if (k < 0 || k > n) return 0;
    int64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int check_d_r(int d, int r) {
    if (d < 1 || d > KDEFFT_MAX_D) return fail(KDEFFT_E_ARG, "d=%d outside [1,%d]", d, KDEFFT_MAX_D);
    if (r < 0 || r > KDEFFT_MAX_R) return fail(KDEFFT_E_UNSUPPORTED, "r=%d outside [0,%d]", r, KDEFFT_MAX_R);
    if (r % 2) return fail(KDEFFT_E_ODD_R, "r=%d is odd: the double sum vanishes", r);
    if (binom(d + r, r) > 84)
        return fail(KDEFFT_E_UNSUPPORTED, "d=%d, r=%d needs %lld multi-indices (limit 84)", d, r,
                    (long long)binom(d + r, r));
    return KDEFFT_OK;
}

int check_grid(const kdefft_grid* g) {
    if (!g) return fail(KDEFFT_E_ARG, "grid is NULL");
    if (g->d < 1 || g->d > KDEFFT_MAX_D) return fail(KDEFFT_E_ARG, "grid d=%d outside [1,4]", g->d);
    double total = 1.0;
    for (int k = 0; k < g->d; ++k) {
        if (g->M[k] < 2) return fail(KDEFFT_E_ARG, "M[%d]=%d < 2", k, g->M[k]);
        if (!is_pow2(g->P[k]) || g->P[k] > KDEFFT_MAX_P || g->P[k] < 2 * g->M[k] - 1 || g->P[k] < 4)
            return fail(KDEFFT_E_ARG, "P[%d]=%d must be a power of two in [max(4, 2M-1), %d]", k, g->P[k],
                        KDEFFT_MAX_P);
        if (!(g->delta[k] > 0.0) || !std::isfinite(g->delta[k]) || !std::isfinite(g->lo[k]))
            return fail(KDEFFT_E_ARG, "grid spacing/origin of axis %d not finite and positive", k);
        total *= g->P[k];
    }
    if (total > (double)(1LL << 30)) return fail(KDEFFT_E_UNSUPPORTED, "prod P = %.0f exceeds 2^30", total);
    return KDEFFT_OK;
}

int check_n(int64_t n) {
    if (n < 1) return fail(KDEFFT_E_ARG, "n=%lld < 1", (long long)n);
    if (n >= KDEFFT_MAX_N) return fail(KDEFFT_E_OVERFLOW, "n=%lld >= 2^23 could overflow an int64 bin", (long long)n);
    return KDEFFT_OK;
}

// Cholesky of a host d x d row-major matrix (row stride ld); 0 if not SPD.
bool chol_host(const double* A, int ld, int d, double* L /*[16], stride 4*/) {
    for (int i = 0; i < 16; ++i) L[i] = 0.0;
    for (int j = 0; j < d; ++j) {
        double s = A[j * ld + j];
        for (int k = 0; k < j; ++k) s -= L[j * 4 + k] * L[j * 4 + k];
        if (!(s > 0.0) || !std::isfinite(s)) return false;
        const double ljj = std::sqrt(s);
        L[j * 4 + j] = ljj;
        for (int i = j + 1; i < d; ++i) {
            double t = A[i * ld + j];
            for (int k = 0; k < j; ++k) t -= L[i * 4 + k] * L[j * 4 + k];
            L[i * 4 + j] = t / ljj;
        }
    }
    return true;
}

void chol_inv_host(const double* L, int d, double* Ainv /*stride 4*/) {
    double Li[16] = {0};
    for (int j = 0; j < d; ++j) {
        Li[j * 4 + j] = 1.0 / L[j * 4 + j];
        for (int i = j + 1; i < d; ++i) {
            double s = 0.0;
            for (int k = j; k < i; ++k) s -= L[i * 4 + k] * Li[k * 4 + j];
            Li[i * 4 + j] = s / L[i * 4 + i];
        }
    }
    for (int i = 0; i < 16; ++i) Ainv[i] = 0.0;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double s = 0.0;
            for (int k = std::max(i, j); k < d; ++k) s += Li[k * 4 + i] * Li[k * 4 + j];
            Ainv[i * 4 + j] = s;
        }
}

// Validate a symmetric positive definite d x d row-major matrix.
int check_spd(const double* A, int d, const char* name, double* L) {
    if (!A) return fail(KDEFFT_E_ARG, "%s is NULL", name);
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < i; ++j) {
            const double a = A[i * d + j], b = A[j * d + i];
            if (!(std::fabs(a - b) <= 1e-12 * (std::fabs(a) + std::fabs(b)) + 1e-300))
                return fail(KDEFFT_E_NOT_SPD, "%s is not symmetric (%g vs %g)", name, a, b);
        }
    if (!chol_host(A, d, d, L)) return fail(KDEFFT_E_NOT_SPD, "%s is not positive definite", name);
    return KDEFFT_OK;
}

const double kInvSqrt2Pi = 0.39894228040143267794;

double normal_const(const double* L, int d) {  // (2 pi)^{-d/2} / prod L_kk
    double c = 1.0;
    for (int k = 0; k < d; ++k) c *= kInvSqrt2Pi / L[k * 4 + k];
    return c;
}

// Largest eigenvalue of a symmetric d x d (row-major) matrix by cyclic Jacobi
// rotations (d <= 4; converges to rounding level in a few sweeps).
double max_eig_sym(const double* A_host, int d) {
    double a[4][4];
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) a[i][j] = 0.5 * (A_host[i * d + j] + A_host[j * d + i]);
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < d; ++i)
            for (int j = i + 1; j < d; ++j) off += a[i][j] * a[i][j];
        if (off == 0.0) break;
        for (int p = 0; p < d; ++p)
            for (int q = p + 1; q < d; ++q) {
                if (a[p][q] == 0.0) continue;
                const double th = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < d; ++k) {  // columns p, q
                    const double akp = a[k][p], akq = a[k][q];
                    a[k][p] = c * akp - sn * akq;
                    a[k][q] = sn * akp + c * akq;
                }
                for (int k = 0; k < d; ++k) {  // rows p, q
                    const double apk = a[p][k], aqk = a[q][k];
                    a[p][k] = c * apk - sn * aqk;
                    a[q][k] = sn * apk + c * aqk;
                }
            }
    }
    double m = a[0][0];
    for (int i = 1; i < d; ++i) m = std::max(m, a[i][i]);
    return m;
}

// fft-L sizes (Eq. (26)-(27)) for bandwidth S on grid g.
void fftl_sizes(const kdefft_grid& g, const double* S_host, double tau, int32_t* L, int32_t* P) {
    const double lam = max_eig_sym(S_host, g.d);
    for (int k = 0; k < g.d; ++k) {
        const double v = std::ceil(tau * std::sqrt(std::fabs(lam)) / g.delta[k]);
        const int lk = v < (double)(g.M[k] - 1) ? (int)v : g.M[k] - 1;
        L[k] = lk;
        const int64_t x = (int64_t)g.M[k] + 2 * (int64_t)lk - 1;
        int64_t p = 1;
        while (p < x) p *= 2;
        P[k] = (int32_t)p;
    }
}

struct Arena {
    char* base;
    size_t cap;
    size_t off = 0;
    bool dry;
    Arena(void* b, size_t c, bool d) : base(static_cast<char*>(b)), cap(c), dry(d) {}
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = dry ? nullptr : reinterpret_cast<T*>(base + off);
        off += count * sizeof(T);
        return p;
    }
    bool fits() const { return dry || off <= cap; }
};

struct Sizes {
    int64_t prodM = 1, prodP = 1, lead = 1, Q = 0, spec = 0;
};
Sizes sizes_of(const kdefft_grid& g) {
    Sizes s;
    for (int k = 0; k < g.d; ++k) {
        s.prodM *= g.M[k];
        s.prodP *= g.P[k];
        if (k + 1 < g.d) s.lead *= g.P[k];
    }
    s.Q = g.P[g.d - 1] / 2 + 1;
    s.spec = s.lead * s.Q;
    return s;
}

// Blocks of the bounds pass of the device-planned preparation: every block of
// the binning launch reduces their partials again, so they are kept few.
int64_t bound_blocks(int64_t n) { return std::min<int64_t>(std::max<int64_t>((n + 1023) / 1024, 1), 128); }

int nblk_dot(const kdefft_grid& g) {
    const int64_t b = (sizes_of(g).prodM + 255) / 256;
    return (int)std::min<int64_t>(std::max<int64_t>(b, 1), 1024);
}

int64_t max_nchunks(const kdefft_grid& g, int kind, int r, int64_t ncand) {
    int64_t m = 1;
    for (int v = 0; v < ROW_VARIANTS; ++v) m = std::max(m, make_geom(g, kind, r, ncand, v).nchunks);
    return m;
}

// ---------------------------------------------------------------- launch choices
// crit: the criterion the family serves (the SCV families also run LSCV,
// whose kernels are narrower, so each keeps its own choice); 0 for psi / SCV.
struct LaunchKey {
    int dev, kind, d, r, N, crit;
    bool operator<(const LaunchKey& o) const {
        return std::tie(dev, kind, d, r, N, crit) < std::tie(o.dev, o.kind, o.d, o.r, o.N, o.crit);
    }
};
std::mutex g_launch_mu;
std::map<LaunchKey, RowLaunch> g_launch;
bool g_cache_loaded = false;

std::string arch_name(int dev) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

int json_int(const std::string& line, const char* key, int dflt) {
    const std::string k = std::string("\"") + key + "\":";
    size_t p = line.find(k);
    if (p == std::string::npos) return dflt;
    p += k.size();
    while (p < line.size() && line[p] == ' ') ++p;
    return std::atoi(line.c_str() + p);
}

void fft_cache_entry(int dev, int d, const int32_t* P, int fs);

void load_cache_locked(int dev) {
    if (g_cache_loaded) return;
    g_cache_loaded = true;
    const char* path = std::getenv("KDEFFT_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    const std::string arch = arch_name(dev);
    char buf[1024];
    while (std::fgets(buf, sizeof(buf), f)) {
        std::string line(buf);
        if (line.find("\"arch\": \"" + arch + "\"") == std::string::npos) continue;
        if (json_int(line, "fft", 0) == 1) {
            const int32_t P[4] = {json_int(line, "P0", 0), json_int(line, "P1", 0), json_int(line, "P2", 0),
                                  json_int(line, "P3", 0)};
            const int fs = json_int(line, "sched", -1), d = json_int(line, "d", 0);
            if (d >= 1 && d <= 4 && fs >= 0 && fs < FFT_SCHEDULES) fft_cache_entry(dev, d, P, fs);
            continue;
        }
        LaunchKey k{dev, json_int(line, "kind", -1), json_int(line, "d", 0), json_int(line, "r", 0),
                    json_int(line, "N", 0), json_int(line, "crit", 0)};
        RowLaunch rl{json_int(line, "variant", 0), json_int(line, "grid", 0)};
        if (k.kind >= 0 && rl.variant >= 0 && rl.variant < ROW_VARIANTS) g_launch[k] = rl;
    }
    std::fclose(f);
}

RowLaunch launch_for(int kind, int d, int r, int N, int crit = 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_launch_mu);
    load_cache_locked(dev);
    auto it = g_launch.find(LaunchKey{dev, kind, d, r, N, crit});
    if (it != g_launch.end()) return it->second;
    // untuned default: the lag-domain evaluation (fewest operations, no LDS);
    // for the SCV families the compacted walk, one block per work item (it
    // builds its own parameter blocks)
    const bool mom = kind == FUN_SCV_OBJ || kind == FUN_SCV_OBJGRAD || kind == FUN_SCV_GRAD;
    return mom ? RowLaunch{5, -1} : RowLaunch{3, 0};
}

void set_launch(int kind, int d, int r, int N, RowLaunch rl, int crit = 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_launch_mu);
    g_launch[LaunchKey{dev, kind, d, r, N, crit}] = rl;
}

// FFT-stage schedule of the count transform per device and grid shape (d, P)
struct FftKey {
    int dev, d, P[4];
    bool operator<(const FftKey& o) const {
        return std::tie(dev, d, P[0], P[1], P[2], P[3]) < std::tie(o.dev, o.d, o.P[0], o.P[1], o.P[2], o.P[3]);
    }
};
std::map<FftKey, int> g_fft;

FftKey fft_key(int dev, int d, const int32_t* P) {
    FftKey k{dev, d, {0, 0, 0, 0}};
    for (int i = 0; i < d; ++i) k.P[i] = P[i];
    return k;
}

int fft_sched_for(const kdefft_grid& g) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_launch_mu);
    load_cache_locked(dev);
    auto it = g_fft.find(fft_key(dev, g.d, g.P));
    return it == g_fft.end() ? 0 : it->second;
}

void fft_cache_entry(int dev, int d, const int32_t* P, int fs) { g_fft[fft_key(dev, d, P)] = fs; }

void set_fft_sched(int d, const int32_t* P, int fs) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_launch_mu);
    if (fs < 0)
        g_fft.erase(fft_key(dev, d, P));
    else
        g_fft[fft_key(dev, d, P)] = fs;
}

void clear_launch(int kind, int d, int r, int N) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_launch_mu);
    g_launch.erase(LaunchKey{dev, kind, d, r, N, 0});
}

// ---------------------------------------------------------------- workspace plans
struct DsLayout {
    int64_t* counts;
    double2* spec;
    double2* wmix;
    double* alag;
    double* scal;
    int32_t* n_out;
    DsDev* rec;
};
DsLayout carve_dataset(Arena& a, const kdefft_grid& g) {
    const Sizes s = sizes_of(g);
    DsLayout L;
    L.counts = a.take<int64_t>(s.prodM);
    L.spec = a.take<double2>(s.spec);
    L.wmix = a.take<double2>(s.spec);
    L.alag = a.take<double>(s.prodP);
    L.scal = a.take<double>(4);
    L.n_out = a.take<int32_t>(1);
    L.rec = a.take<DsDev>(1);
    return L;
}

struct PrepScratch {
    double* prm;
    double* partial;
    int64_t* slots;     // corner slots of the binning (2^d int64 per cell)
    int32_t* counter;   // completion counter of the constant-term launch
};
PrepScratch carve_prepare(Arena& a, const kdefft_grid& g) {
    PrepScratch p;
    p.prm = a.take<double>(PRM);
    p.partial = a.take<double>(max_nchunks(g, FUN_PSI, 0, 1));
    p.slots = a.take<int64_t>(corner_slots(g.d) * sizes_of(g).prodM);
    p.counter = a.take<int32_t>(1);
    return p;
}

struct PlainScratch {
    int64_t* counts;
    int32_t* n_out;
    double* czp;
    double2* C;
    double* kreal;
    double2* K;
    double* partial;
    double* sums;
};
PlainScratch carve_plain(Arena& a, const kdefft_grid& g, bool with_counts) {
    const Sizes s = sizes_of(g);
    PlainScratch p{};
    if (with_counts) {
        p.counts = a.take<int64_t>(s.prodM);
        p.n_out = a.take<int32_t>(1);
        p.czp = a.take<double>(s.prodP);
        p.C = a.take<double2>(s.spec);
    }
    p.kreal = a.take<double>(s.prodP);
    p.K = a.take<double2>(s.spec);
    p.partial = a.take<double>(nblk_dot(g));
    p.sums = a.take<double>(16);
    return p;
}

struct BatchScratch {
    double* prm;
    double* partial;
    int32_t* counters;   // completion counters, one per candidate
    int32_t* wc;         // live segment counts per candidate (balanced plan)
    int32_t* item_off;   // first item of each candidate (balanced plan)
};

// Completion of a psi launch: fused into the row kernel for the lag-domain
// variants when a candidate has few work items (every item of a candidate
// counts on one device-scope counter, so thousands of items would queue on
// it), else (FIN_NONE) a separate final kernel.
constexpr int64_t FUSED_MAX_CHUNKS = 128;
FinishArgs fin_psi(const RowLaunch& rl, const RowGeom& geo, int ng, int32_t* counters, double* psi, double* scal) {
    FinishArgs f{};
    if (rl.variant >= 3 && geo.nchunks <= FUSED_MAX_CHUNKS) {
        f.mode = FIN_PSI;
        f.ng = ng;
        f.counters = counters;
        f.out = psi;
        f.scal = scal;
    }
    return f;
}
// Partial sums of the row kernels: sized for every family that may run in
// this workspace (the SCV families differ in grids per item and chunking).
BatchScratch carve_batch(Arena& a, const kdefft_grid& g, int kind, int r, int64_t ncand) {
    BatchScratch b;
    // the criteria add one constant-term candidate per dataset (SCV)
    if (kind != FUN_PSI) ncand += KDEFFT_MAX_BATCH_DS;
    b.prm = a.take<double>(ncand * PRM);
    int64_t need = 0;
    if (kind == FUN_PSI) {
        need = max_nchunks(g, kind, r, ncand) * ng_of(kind, g.d, r);
    } else {
        for (int k = FUN_SCV_OBJ; k <= FUN_ETA2; ++k)
            need = std::max<int64_t>(need, max_nchunks(g, k, 2, ncand) * ng_of(k, g.d, 2));
    }
    b.partial = a.take<double>(ncand * need);
    b.counters = a.take<int32_t>(ncand);
    b.wc = a.take<int32_t>(ncand);
    b.item_off = a.take<int32_t>(ncand + 1);
    return b;
}

int plan_bytes(const kdefft_grid& g, int op, int r, int64_t batch, Arena& a) {
    switch (op) {
        case KDEFFT_OP_GRID_AUTO: {
            const int64_t nb = std::min<int64_t>(std::max<int64_t>((batch + 255) / 256, 1), 1024);
            a.take<double>(nb * 8);
            return KDEFFT_OK;
        }
        case KDEFFT_OP_PSI_PLAIN: carve_plain(a, g, true); return KDEFFT_OK;
        case KDEFFT_OP_PSI_FUSED:
            carve_dataset(a, g);
            carve_prepare(a, g);
            carve_batch(a, g, FUN_PSI, r, 1);
            return KDEFFT_OK;
        case KDEFFT_OP_PREPARE: carve_prepare(a, g); return KDEFFT_OK;
        case KDEFFT_OP_PREPARE_AUTO: {
            carve_prepare(a, g);
            a.take<double>(bound_blocks(batch) * 8);
            return KDEFFT_OK;
        }
        case KDEFFT_OP_PSI_BATCH: carve_batch(a, g, FUN_PSI, r, std::max<int64_t>(batch, 1)); return KDEFFT_OK;
        case KDEFFT_OP_SCV_BATCH:
            carve_batch(a, g, FUN_SCV_OBJGRAD, 2, std::max<int64_t>(batch, 1));
            return KDEFFT_OK;
        case KDEFFT_OP_SCV_PLAIN: carve_plain(a, g, false); return KDEFFT_OK;
        case KDEFFT_OP_PSI_FFTL: {
            // the largest padded grid Eq. (27) can ask for (L_k = M_k - 1)
            kdefft_grid gm = g;
            for (int k = 0; k < g.d; ++k) {
                int p = 4;
                while (p < 3 * g.M[k] - 3) p *= 2;
                gm.P[k] = p;
            }
            carve_plain(a, gm, true);
            return KDEFFT_OK;
        }
        case KDEFFT_OP_AUTOTUNE: {
            carve_batch(a, g, FUN_SCV_OBJGRAD, 2, TUNE_B);
            const int q = g.d * (g.d + 1) / 2;
            a.take<double>(TUNE_B * q);
            a.take<double>(TUNE_B);
            a.take<double>(TUNE_B * q);
            a.take<double>(TUNE_PSI_OUT);
            // the psi_4 timings carve their own scratch from the start of the
            // workspace: at least that much
            Arena ap(nullptr, 0, true);
            carve_batch(ap, g, FUN_PSI, 4, 1);
            if (ap.off > a.off) a.off = ap.off;
            return KDEFFT_OK;
        }
        default: return fail(KDEFFT_E_ARG, "unknown op %d", op);
    }
}

hipStream_t S(void* stream) { return static_cast<hipStream_t>(stream); }

// Bin X into counts (zeroed first) and build the circular real count array.
int bin_and_fill(const double* X, int64_t n, const kdefft_grid& g, int64_t* counts, int32_t* n_out, double* czp,
                 hipStream_t s, const double* gdev = nullptr) {
    const Sizes sz = sizes_of(g);
    HIPCHK(launch_zero(counts, sz.prodM * sizeof(int64_t), s), "zero counts");
    if (n_out) HIPCHK(launch_zero(n_out, sizeof(int32_t), s), "zero n_out");
    HIPCHK(launch_linbin(X, n, g, counts, n_out, s, gdev), "linbin");
    if (czp) HIPCHK(launch_fill_czp(counts, g, czp, s), "fill czp");
    return KDEFFT_OK;
}

PsiBatchArgs psi_args(const kdefft_grid& g, int r, int n_ds, const DsDev* const* recs, const double* Gs /*d*d each*/) {
    PsiBatchArgs a{};
    a.n_ds = n_ds;
    a.d = g.d;
    a.r = r;
    a.prodP = (double)sizes_of(g).prodP;
    for (int j = 0; j < n_ds; ++j) {
        a.rec[j] = recs[j];
        int t = 0;
        for (int c = 0; c < g.d; ++c)
            for (int i = c; i < g.d; ++i) a.Gv[j][t++] = Gs[j * g.d * g.d + i * g.d + c];
    }
    return a;
}

// Prepare a dataset whose buffers are described by L (in a caller buffer or
// workspace).  partial (device, nblk per-block bound partials of X) and pad:
// the grid's origin and spacing are computed on the device from the data
// bounds (g then carries the shape only) and the binning scratch was already
// cleared by the bounds kernel; otherwise g's origin and spacing are used.
int prepare_into(const double* X, int64_t n, const kdefft_grid& g, const double* Gpilot, const DsLayout& L,
                 const PrepScratch& p, bool with_const, hipStream_t s, const double* partial = nullptr,
                 int nblk = 0, const double* pad = nullptr) {
    HeaderArgs h{};
    h.rec = L.rec;
    h.val.wmix = L.wmix;
    h.val.alag = L.alag;
    h.val.scal = L.scal;
    h.val.n = (double)n;
    for (int k = 0; k < g.d; ++k) {
        h.val.lo[k] = g.lo[k];
        h.val.delta[k] = g.delta[k];
    }
    if (Gpilot)
        for (int i = 0; i < g.d; ++i)
            for (int j = 0; j < g.d; ++j) h.val.G[i * 4 + j] = Gpilot[i * g.d + j];
    h.partial = partial;
    h.nblk = nblk;
    h.g = g;
    for (int k = 0; k < g.d; ++k) h.pad[k] = pad ? pad[k] : 0.0;
    h.n_out = L.n_out;
    h.scal = L.scal;
    h.prodP = (double)sizes_of(g).prodP;
    // the constant SCV term n^-2 sum sum phi_{2G} is evaluated by the batched SCV
    // calls themselves (one more candidate per dataset), so the header writes
    // no parameter block here
    (void)with_const;
    if (partial) {
        // grid from the bound partials and the header inside the binning launch
        // (the bounds launch cleared the counter, the scalar block and the slots)
        HIPCHK(launch_linbin_slots(X, n, g, p.slots, L.n_out, s, nullptr, true, &h), "linbin");
    } else {
        HIPCHK(launch_ds_header(h, s), "dataset header");
        HIPCHK(launch_linbin_slots(X, n, g, p.slots, L.n_out, s, nullptr, false), "linbin");
    }
    const int fs = fft_sched_for(g);
    HIPCHK(fft_prepare_nd(p.slots, 1, L.counts, L.spec, L.wmix, g, s, fs), "count transform");
    HIPCHK(fft_autocorr_nd(L.wmix, L.alag, g, s, fs), "count autocorrelation");
    return KDEFFT_OK;
}

// The batched row kernels are compiled for last-axis lengths up to 2048, 1024,
// 256, 128 (d = 1..4) and enough LDS for the family's grids.
int check_rows(int kind, int d, int r, int N) {
    // the scalar eta families exist in the lag-domain form only
    const int v = (kind == FUN_ETA1 || kind == FUN_ETA2) ? 3 : 0;
    if (rows_per_iter(kind, d, r, N, v) < 1)
        return fail(KDEFFT_E_UNSUPPORTED,
                    "no batched row kernel for d=%d, r=%d, last-axis P=%d (family %d); use the plain path", d, r, N,
                    kind);
    return KDEFFT_OK;
}

int check_ws(const Arena& a, size_t have) {
    if (!a.fits()) return fail(KDEFFT_E_WORKSPACE, "workspace of %zu bytes, need %zu", have, a.off);
    return KDEFFT_OK;
}

int check_ptr_align(const void* p, const char* name) {
    if (!p) return fail(KDEFFT_E_ARG, "%s is NULL", name);
    if (reinterpret_cast<uintptr_t>(p) % 256) return fail(KDEFFT_E_WORKSPACE, "%s is not 256-byte aligned", name);
    return KDEFFT_OK;
}

// A prepared dataset's grid may carry its shape only (origin and spacing
// computed on the device, NaN on the host): batch calls check the shape.
int check_grid_shape(const kdefft_grid* g) {
    if (!g) return fail(KDEFFT_E_ARG, "grid is NULL");
    kdefft_grid t = *g;
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(t.delta[k]) || !std::isfinite(t.lo[k])) {
            t.lo[k] = 0.0;
            t.delta[k] = 1.0;
        }
    return check_grid(&t);
}

int check_batch_ds(const kdefft_dataset* ds, int n_ds, int max_ds) {
    if (!ds) return fail(KDEFFT_E_ARG, "dataset array is NULL");
    if (n_ds < 1 || n_ds > max_ds) return fail(KDEFFT_E_ARG, "n_ds=%d outside [1,%d]", n_ds, max_ds);
    int rc = check_grid_shape(&ds[0].grid);
    if (rc) return rc;
    for (int j = 0; j < n_ds; ++j) {
        if (!ds[j].rec || !ds[j].wmix || !ds[j].alag || !ds[j].scal)
            return fail(KDEFFT_E_ARG, "dataset %d is not prepared", j);
        rc = check_grid_shape(&ds[j].grid);
        if (rc) return rc;
        if (ds[j].grid.d != ds[0].grid.d) return fail(KDEFFT_E_ARG, "datasets differ in d");
        for (int k = 0; k < ds[0].grid.d; ++k)
            if (ds[j].grid.M[k] != ds[0].grid.M[k] || ds[j].grid.P[k] != ds[0].grid.P[k])
                return fail(KDEFFT_E_ARG, "datasets in one batch must share M and P (dataset %d)", j);
        rc = check_n(ds[j].n);
        if (rc) return rc;
    }
    return KDEFFT_OK;
}


// Row-kernel timing: while armed, every row-kernel launch is bracketed by a
// pair of HIP events on its own stream, so the kernel's duration can be read
// afterwards without synchronizing in between.
struct RowTimer {
    std::mutex mu;
    bool armed = false;
    int cap = 0;
    int used = 0;
    std::vector<hipEvent_t> ev;  // 2 per record, created once and reused
    std::vector<int32_t> tag;
};
RowTimer g_timer;

hipError_t timed_rows(int kind, int d, int r, const RowGeom& geo, const double* prm, int64_t ncand,
                      double* partial, const RowLaunch& rl, hipStream_t s) {
    std::unique_lock<std::mutex> lk(g_timer.mu);
    if (!g_timer.armed || g_timer.used >= g_timer.cap) {
        lk.unlock();
        return launch_rows(kind, d, r, geo, prm, ncand, partial, rl, s);
    }
    const int k = g_timer.used++;
    g_timer.tag[k] = 16 * kind + r;
    hipError_t e = hipEventRecord(g_timer.ev[2 * k], s);
    if (e == hipSuccess) e = launch_rows(kind, d, r, geo, prm, ncand, partial, rl, s);
    if (e == hipSuccess) e = hipEventRecord(g_timer.ev[2 * k + 1], s);
    return e;
}

}  // namespace

// ==================================================================== internal helpers for other units
namespace kdefft {

int set_error(int code, const char* msg) { return fail(code, "%s", msg); }

int scv_batch_ws_need(const kdefft_dataset* ds, int n_ds, const int64_t* off, size_t* need) {
    int rc = check_batch_ds(ds, n_ds, KDEFFT_MAX_BATCH_DS);
    if (rc) return rc;
    if (!off || !need) return fail(KDEFFT_E_ARG, "NULL h_offsets or size output");
    if (off[0] != 0) return fail(KDEFFT_E_ARG, "h_offsets[0] must be 0");
    for (int j = 0; j < n_ds; ++j)
        if (off[j + 1] < off[j]) return fail(KDEFFT_E_ARG, "h_offsets must be non-decreasing");
    const int64_t B = off[n_ds];
    if (B < 1) return fail(KDEFFT_E_ARG, "no candidate bandwidths");
    if (B > (1LL << 24)) return fail(KDEFFT_E_ARG, "too many candidates in one call");
    kdefft_grid g = ds[0].grid;   // the shape decides the layout; origin and spacing may be NaN
    for (int k = 0; k < 4; ++k) {
        g.lo[k] = 0.0;
        g.delta[k] = 1.0;
    }
    Arena a(nullptr, 0, true);
    carve_batch(a, g, FUN_SCV_OBJGRAD, 2, B);
    *need = a.off + 256;
    return KDEFFT_OK;
}

}  // namespace kdefft

// ==================================================================== exports
extern "C" {

const char* kdefft_strerror(int code) {
    switch (code) {
        case KDEFFT_OK: return "ok";
        case KDEFFT_E_ARG: return "invalid argument";
        case KDEFFT_E_NOT_SPD: return "bandwidth matrix not symmetric positive definite";
        case KDEFFT_E_ODD_R: return "odd derivative order";
        case KDEFFT_E_OUT_OF_GRID: return "data outside the grid";
        case KDEFFT_E_OVERFLOW: return "sample too large for int64 fixed-point bins";
        case KDEFFT_E_WORKSPACE: return "workspace too small or misaligned";
        case KDEFFT_E_HIP: return "HIP runtime error";
        case KDEFFT_E_UNSUPPORTED: return "configuration outside the compiled limits";
        default: return "unknown error";
    }
}

const char* kdefft_last_error_detail(void) { return g_err.c_str(); }

int kdefft_version(void) { return 10000; }

int kdefft_unique_count(int d, int r) {
    if (d < 1 || d > KDEFFT_MAX_D) return fail(KDEFFT_E_ARG, "d=%d outside [1,4]", d);
    if (r < 0 || r > KDEFFT_MAX_R) return fail(KDEFFT_E_ARG, "r=%d outside [0,8]", r);
    return (int)binom(d + r - 1, r);
}

int kdefft_unique_index(int d, int r, int32_t* tuples_host) {
    const int cnt = kdefft_unique_count(d, r);
    if (cnt < 0) return cnt;
    if (r == 0) return KDEFFT_OK;
    if (!tuples_host) return fail(KDEFFT_E_ARG, "tuples_host is NULL");
    std::vector<int> idx(r, 0);
    int e = 0;
    while (true) {
        for (int m = 0; m < r; ++m) tuples_host[e * r + m] = idx[m];
        ++e;
        int m = r - 1;
        while (m >= 0 && idx[m] == d - 1) --m;
        if (m < 0) break;
        idx[m] += 1;
        for (int q = m + 1; q < r; ++q) idx[q] = idx[m];
    }
    return e == cnt ? KDEFFT_OK : fail(KDEFFT_E_ARG, "internal enumeration mismatch");
}

int kdefft_grid_plan(int d, const int32_t* M_host, const int32_t* P_host, const double* lo_host,
                     const double* hi_host, kdefft_grid* out) {
    if (!M_host || !lo_host || !hi_host || !out) return fail(KDEFFT_E_ARG, "NULL argument to kdefft_grid_plan");
    if (d < 1 || d > KDEFFT_MAX_D) return fail(KDEFFT_E_ARG, "d=%d outside [1,4]", d);
    kdefft_grid g;
    std::memset(&g, 0, sizeof(g));
    g.d = d;
    for (int k = 0; k < d; ++k) {
        g.M[k] = M_host[k];
        if (P_host) {
            g.P[k] = P_host[k];
        } else {  // smallest power of two >= 2M - 1 (circular layout without wrap-around)
            int p = 4;
            while (p < 2 * M_host[k] - 1 && p < (1 << 30)) p <<= 1;
            g.P[k] = p;
        }
        g.lo[k] = lo_host[k];
        if (!(hi_host[k] > lo_host[k])) return fail(KDEFFT_E_ARG, "hi[%d] <= lo[%d]", k, k);
        volatile double span = hi_host[k] - lo_host[k];  // one rounding, then one division
        g.delta[k] = span / (double)(M_host[k] - 1);
    }
    const int rc = check_grid(&g);
    if (rc) return rc;
    *out = g;
    return KDEFFT_OK;
}

int kdefft_ws_bytes(const kdefft_grid* g, int op, int r, int64_t batch, size_t* out) {
    if (!out) return fail(KDEFFT_E_ARG, "out is NULL");
    int rc = check_grid(g);
    if (rc) return rc;
    if (op == KDEFFT_OP_PSI_PLAIN || op == KDEFFT_OP_PSI_FUSED || op == KDEFFT_OP_PSI_BATCH || op == KDEFFT_OP_PSI_FFTL) {
        rc = check_d_r(g->d, r);
        if (rc) return rc;
    }
    Arena a(nullptr, 0, true);
    rc = plan_bytes(*g, op, r, batch, a);
    if (rc) return rc;
    *out = a.off + 256;
    return KDEFFT_OK;
}

int kdefft_grid_auto(const double* X, int64_t n, int d, const double* G_host, const int32_t* M_host,
                     double pad_sd, kdefft_grid* out, void* ws, size_t ws_bytes, void* stream) {
    if (!X || !G_host || !M_host || !out) return fail(KDEFFT_E_ARG, "NULL argument to kdefft_grid_auto");
    int rc = check_n(n);
    if (rc) return rc;
    if (d < 1 || d > KDEFFT_MAX_D) return fail(KDEFFT_E_ARG, "d=%d outside [1,4]", d);
    if (!(pad_sd >= 0.0) || !std::isfinite(pad_sd)) return fail(KDEFFT_E_ARG, "pad_sd must be finite and >= 0");
    double Lg[16];
    rc = check_spd(G_host, d, "G", Lg);
    if (rc) return rc;
    kdefft_grid probe;
    std::memset(&probe, 0, sizeof(probe));
    probe.d = d;
    for (int k = 0; k < d; ++k) { probe.M[k] = 2; probe.P[k] = 4; probe.delta[k] = 1.0; }
    Arena a(ws, ws_bytes, false);
    const int64_t nb = std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 1024);
    double* partial = a.take<double>(nb * 8);
    double* dout = a.take<double>(8);
    if (!ws) return fail(KDEFFT_E_ARG, "workspace is NULL");
    rc = check_ws(a, ws_bytes);
    if (rc) return rc;
    hipStream_t s = S(stream);
    HIPCHK(launch_bounds(X, n, d, partial, (int)nb, dout, s), "bounds");
    // 8 doubles of pinned host memory per thread, allocated once, so the
    // readback is a direct DMA rather than a staged pageable copy
    static thread_local double* pinned = nullptr;
    if (!pinned) HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&pinned), 8 * sizeof(double), hipHostMallocDefault),
                        "pinned readback buffer");
    HIPCHK(hipMemcpyAsync(pinned, dout, 8 * sizeof(double), hipMemcpyDeviceToHost, s), "bounds readback");
    HIPCHK(hipStreamSynchronize(s), "bounds sync");
    double host[8];
    for (int k = 0; k < 8; ++k) host[k] = pinned[k];
    double lo[4], hi[4];
    for (int k = 0; k < d; ++k) {
        const double sd = std::sqrt(G_host[k * d + k]);
        volatile double pad = pad_sd * sd;
        lo[k] = host[k] - pad;
        hi[k] = host[4 + k] + pad;
        if (!std::isfinite(lo[k]) || !std::isfinite(hi[k])) return fail(KDEFFT_E_ARG, "data not finite");
        if (!(hi[k] > lo[k])) hi[k] = lo[k] + 1.0;  // degenerate axis: unit span
    }
    return kdefft_grid_plan(d, M_host, nullptr, lo, hi, out);
}

int kdefft_linbin(const double* X, int64_t n, const kdefft_grid* g, int64_t* counts, int32_t* n_out_dev,
                  void* stream) {
    int rc = check_grid(g);
    if (rc) return rc;
    rc = check_n(n);
    if (rc) return rc;
    if (!X || !counts) return fail(KDEFFT_E_ARG, "NULL X or counts");
    return bin_and_fill(X, n, *g, counts, n_out_dev, nullptr, S(stream));
}

int kdefft_check_binning(const int32_t* n_out_dev, int32_t* n_out_host, void* stream) {
    if (!n_out_dev) return fail(KDEFFT_E_ARG, "n_out_dev is NULL");
    int32_t v = 0;
    HIPCHK(hipMemcpyAsync(&v, n_out_dev, sizeof(v), hipMemcpyDeviceToHost, S(stream)), "n_out readback");
    HIPCHK(hipStreamSynchronize(S(stream)), "n_out sync");
    if (n_out_host) *n_out_host = v;
    if (v) return fail(KDEFFT_E_OUT_OF_GRID, "%d points outside the grid were skipped", v);
    return KDEFFT_OK;
}

int kdefft_psi(const double* X, int64_t n, const kdefft_grid* g, const double* G_host, int r, double* psi,
               int mode, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_grid(g);
    if (rc) return rc;
    rc = check_d_r(g->d, r);
    if (rc) return rc;
    rc = check_n(n);
    if (rc) return rc;
    if (!X || !psi) return fail(KDEFFT_E_ARG, "NULL X or psi");
    if (mode != KDEFFT_PSI_PLAIN && mode != KDEFFT_PSI_FUSED) return fail(KDEFFT_E_ARG, "mode=%d", mode);
    double L[16];
    rc = check_spd(G_host, g->d, "G", L);
    if (rc) return rc;
    if (!ws) return fail(KDEFFT_E_ARG, "workspace is NULL");
    const int d = g->d;
    const Sizes sz = sizes_of(*g);
    const double scale = 1.0 / ((double)n * (double)n * (double)sz.prodP);
    const int nu = (int)binom(d + r - 1, r);
    hipStream_t s = S(stream);
    Arena a(ws, ws_bytes, false);
    if (mode == KDEFFT_PSI_PLAIN) {
        const PlainScratch p = carve_plain(a, *g, true);
        rc = check_ws(a, ws_bytes);
        if (rc) return rc;
        ParamBlock prm{};
        chol_inv_host(L, d, prm.v + S_P1);
        prm.v[S_C] = normal_const(L, d);
        rc = bin_and_fill(X, n, *g, p.counts, p.n_out, p.czp, s);
        if (rc) return rc;
        HIPCHK(fft_r2c_nd(p.czp, p.C, *g, s), "R2C counts");
        const int nb = nblk_dot(*g);
        for (int u = 0; u < nu; ++u) {
            HIPCHK(launch_kgrid_psi(p.kreal, *g, r, prm, u, s), "kernel grid");
            HIPCHK(fft_r2c_nd(p.kreal, p.K, *g, s), "R2C kernel");
            HIPCHK(launch_cmul(p.K, p.C, sz.spec, s), "spectrum product");
            HIPCHK(fft_c2r_nd(p.K, p.kreal, *g, s), "C2R");
            HIPCHK(launch_dot_counts(p.counts, p.kreal, *g, p.partial, nb, s), "count contraction");
            HIPCHK(launch_sum_scale(p.partial, nb, scale, psi + u, s), "final sum");
        }
        return KDEFFT_OK;
    }
    rc = check_rows(FUN_PSI, d, r, g->P[d - 1]);
    if (!rc) rc = check_rows(FUN_PSI, d, 0, g->P[d - 1]);
    if (rc) return rc;
    const DsLayout L2 = carve_dataset(a, *g);
    const PrepScratch pp = carve_prepare(a, *g);
    const BatchScratch b = carve_batch(a, *g, FUN_PSI, r, 1);
    rc = check_ws(a, ws_bytes);
    if (rc) return rc;
    rc = prepare_into(X, n, *g, G_host, L2, pp, false, s);
    if (rc) return rc;
    const DsDev* recs[1] = {L2.rec};
    PsiBatchArgs args = psi_args(*g, r, 1, recs, G_host);
    const RowLaunch rl = launch_for(FUN_PSI, d, r, g->P[d - 1]);
    const RowGeom geo = make_geom(*g, FUN_PSI, r, 1, rl.variant);
    args.fin = fin_psi(rl, geo, nu, b.counters, psi, nullptr);
    HIPCHK(launch_psi_setup(args, b.prm, s), "psi setup");
    HIPCHK(timed_rows(FUN_PSI, d, r, geo, b.prm, 1, b.partial, rl, s), "psi rows");
    if (args.fin.mode == FIN_NONE)
        HIPCHK(launch_psi_final(b.partial, geo, nu, b.prm, 1, psi, nullptr, s), "psi final");
    return KDEFFT_OK;
}

int kdefft_fftl_plan(const kdefft_grid* g, const double* S_host, double tau, int32_t* L_host, int32_t* P_host) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!L_host || !P_host) return fail(KDEFFT_E_ARG, "NULL output");
    if (!(tau > 0.0) || !std::isfinite(tau)) return fail(KDEFFT_E_ARG, "tau must be positive and finite");
    double Ls[16];
    rc = check_spd(S_host, g->d, "S", Ls);
    if (rc) return rc;
    fftl_sizes(*g, S_host, tau, L_host, P_host);
    return KDEFFT_OK;
}

int kdefft_psi_fftl(const double* X, int64_t n, const kdefft_grid* g, const double* G_host, int r, double tau,
                    double* psi, int32_t* L_host, int32_t* P_host, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_grid(g);
    if (rc) return rc;
    rc = check_d_r(g->d, r);
    if (rc) return rc;
    rc = check_n(n);
    if (rc) return rc;
    if (!X || !psi) return fail(KDEFFT_E_ARG, "NULL X or psi");
    if (!(tau > 0.0) || !std::isfinite(tau)) return fail(KDEFFT_E_ARG, "tau must be positive and finite");
    double L[16];
    rc = check_spd(G_host, g->d, "G", L);
    if (rc) return rc;
    if (!ws) return fail(KDEFFT_E_ARG, "workspace is NULL");
    const int d = g->d;
    int32_t Lk[4] = {0, 0, 0, 0}, Pk[4] = {0, 0, 0, 0};
    fftl_sizes(*g, G_host, tau, Lk, Pk);
    if (L_host)
        for (int k = 0; k < d; ++k) L_host[k] = Lk[k];
    if (P_host)
        for (int k = 0; k < d; ++k) P_host[k] = Pk[k];
    // g2: the data grid padded per Eq. (27); gk: the same lengths with the
    // kernel support cut to |l_k| <= L_k (lags beyond are zero-filled)
    kdefft_grid g2 = *g, gk = *g;
    double total = 1.0;
    for (int k = 0; k < d; ++k) {
        if (Pk[k] > KDEFFT_MAX_P) return fail(KDEFFT_E_UNSUPPORTED, "Eq. (27) gives P[%d]=%d > %d", k, Pk[k], KDEFFT_MAX_P);
        g2.P[k] = gk.P[k] = Pk[k];
        gk.M[k] = Lk[k] + 1;
        total *= Pk[k];
    }
    if (total > (double)(1LL << 30)) return fail(KDEFFT_E_UNSUPPORTED, "prod P = %.0f exceeds 2^30", total);
    const Sizes sz = sizes_of(g2);
    const double scale = 1.0 / ((double)n * (double)n * (double)sz.prodP);
    const int nu = (int)binom(d + r - 1, r);
    hipStream_t s = S(stream);
    Arena a(ws, ws_bytes, false);
    const PlainScratch p = carve_plain(a, g2, true);
    rc = check_ws(a, ws_bytes);
    if (rc) return rc;
    ParamBlock prm{};
    chol_inv_host(L, d, prm.v + S_P1);
    prm.v[S_C] = normal_const(L, d);
    rc = bin_and_fill(X, n, g2, p.counts, p.n_out, p.czp, s);
    if (rc) return rc;
    HIPCHK(fft_r2c_nd(p.czp, p.C, g2, s), "R2C counts");
    const int nb = nblk_dot(g2);
    for (int u = 0; u < nu; ++u) {
        HIPCHK(launch_kgrid_psi(p.kreal, gk, r, prm, u, s), "truncated kernel grid");
        HIPCHK(fft_r2c_nd(p.kreal, p.K, g2, s), "R2C kernel");
        HIPCHK(launch_cmul(p.K, p.C, sz.spec, s), "spectrum product");
        HIPCHK(fft_c2r_nd(p.K, p.kreal, g2, s), "C2R");
        HIPCHK(launch_dot_counts(p.counts, p.kreal, g2, p.partial, nb, s), "count contraction");
        HIPCHK(launch_sum_scale(p.partial, nb, scale, psi + u, s), "final sum");
    }
    return KDEFFT_OK;
}

int kdefft_dataset_bytes(const kdefft_grid* g, size_t* out) {
    if (!out) return fail(KDEFFT_E_ARG, "out is NULL");
    const int rc = check_grid(g);
    if (rc) return rc;
    Arena a(nullptr, 0, true);
    carve_dataset(a, *g);
    *out = a.off;
    return KDEFFT_OK;
}

int kdefft_dataset_prepare(const double* X, int64_t n, const kdefft_grid* g, const double* Gpilot_host,
                           void* ds_mem, size_t ds_bytes, kdefft_dataset* out, void* ws, size_t ws_bytes,
                           void* stream) {
    int rc = check_grid(g);
    if (rc) return rc;
    rc = check_n(n);
    if (rc) return rc;
    if (!X || !out) return fail(KDEFFT_E_ARG, "NULL X or out");
    double L[16];
    rc = check_spd(Gpilot_host, g->d, "Gpilot", L);
    if (rc) return rc;
    rc = check_rows(FUN_PSI, g->d, 0, g->P[g->d - 1]);
    if (rc) return rc;
    rc = check_ptr_align(ds_mem, "ds_mem");
    if (rc) return rc;
    if (!ws) return fail(KDEFFT_E_ARG, "workspace is NULL");
    Arena da(ds_mem, ds_bytes, false);
    const DsLayout dl = carve_dataset(da, *g);
    if (!da.fits()) return fail(KDEFFT_E_WORKSPACE, "dataset buffer of %zu bytes, need %zu", ds_bytes, da.off);
    Arena a(ws, ws_bytes, false);
    const PrepScratch p = carve_prepare(a, *g);
    rc = check_ws(a, ws_bytes);
    if (rc) return rc;
    rc = prepare_into(X, n, *g, Gpilot_host, dl, p, true, S(stream));
    if (rc) return rc;
    kdefft_dataset o;
    std::memset(&o, 0, sizeof(o));
    o.grid = *g;
    o.n = n;
    for (int i = 0; i < g->d * g->d; ++i) o.G[i] = Gpilot_host[i];
    o.counts = dl.counts;
    o.spec = reinterpret_cast<double*>(dl.spec);
    o.wmix = reinterpret_cast<double*>(dl.wmix);
    o.alag = dl.alag;
    o.scal = dl.scal;
    o.n_out = dl.n_out;
    o.rec = dl.rec;
    *out = o;
    return KDEFFT_OK;
}

int kdefft_dataset_prepare_auto(const double* X, int64_t n, int d, const int32_t* M_host, double pad_sd,
                                const double* Gpilot_host, void* ds_mem, size_t ds_bytes, kdefft_dataset* out,
                                void* ws, size_t ws_bytes, void* stream) {
    if (!X || !M_host || !Gpilot_host || !out) return fail(KDEFFT_E_ARG, "NULL argument");
    int rc = check_n(n);
    if (rc) return rc;
    if (d < 1 || d > KDEFFT_MAX_D) return fail(KDEFFT_E_ARG, "d=%d outside [1,4]", d);
    if (!(pad_sd >= 0.0) || !std::isfinite(pad_sd)) return fail(KDEFFT_E_ARG, "pad_sd must be finite and >= 0");
    double L[16];
    rc = check_spd(Gpilot_host, d, "Gpilot", L);
    if (rc) return rc;
    // the grid's shape (M, P) from the planner; origin and spacing follow on the device
    double lo0[4] = {0, 0, 0, 0}, hi0[4] = {1, 1, 1, 1};
    kdefft_grid g;
    rc = kdefft_grid_plan(d, M_host, nullptr, lo0, hi0, &g);
    if (rc) return rc;
    const double nan = std::numeric_limits<double>::quiet_NaN();
    for (int k = 0; k < 4; ++k) g.lo[k] = g.delta[k] = nan;
    rc = check_rows(FUN_PSI, d, 0, g.P[d - 1]);
    if (rc) return rc;
    rc = check_ptr_align(ds_mem, "ds_mem");
    if (rc) return rc;
    if (!ws) return fail(KDEFFT_E_ARG, "workspace is NULL");
    Arena da(ds_mem, ds_bytes, false);
    const DsLayout dl = carve_dataset(da, g);
    if (!da.fits()) return fail(KDEFFT_E_WORKSPACE, "dataset buffer of %zu bytes, need %zu", ds_bytes, da.off);
    Arena a(ws, ws_bytes, false);
    const PrepScratch p = carve_prepare(a, g);
    const int64_t nb = bound_blocks(n);
    double* partial = a.take<double>(nb * 8);
    rc = check_ws(a, ws_bytes);
    if (rc) return rc;
    hipStream_t s = S(stream);
    double pad[4] = {0, 0, 0, 0};
    for (int k = 0; k < d; ++k) {
        const double sd = std::sqrt(Gpilot_host[k * d + k]);
        volatile double pk = pad_sd * sd;   // the same product as kdefft_grid_auto
        pad[k] = pk;
    }
    HIPCHK(launch_bounds_partial(X, n, d, partial, (int)nb, s, p.slots,
                                 (size_t)(corner_slots(g.d) * sizes_of(g).prodM) * sizeof(int64_t), dl.n_out, dl.scal),
           "bounds");
    rc = prepare_into(X, n, g, Gpilot_host, dl, p, true, s, partial, (int)nb, pad);
    if (rc) return rc;
    kdefft_dataset o;
    std::memset(&o, 0, sizeof(o));
    o.grid = g;
    o.n = n;
    for (int i = 0; i < d * d; ++i) o.G[i] = Gpilot_host[i];
    o.counts = dl.counts;
    o.spec = reinterpret_cast<double*>(dl.spec);
    o.wmix = reinterpret_cast<double*>(dl.wmix);
    o.alag = dl.alag;
    o.scal = dl.scal;
    o.n_out = dl.n_out;
    o.rec = dl.rec;
    *out = o;
    return KDEFFT_OK;
}

int kdefft_dataset_transform(const kdefft_dataset* ds, void* stream) {
    const int rc = check_batch_ds(ds, 1, 1);
    if (rc) return rc;
    const kdefft_grid& g = ds->grid;
    hipStream_t s = S(stream);
    const int fs = fft_sched_for(g);
    HIPCHK(fft_prepare_nd(ds->counts, 0, nullptr, reinterpret_cast<double2*>(ds->spec),
                          reinterpret_cast<double2*>(ds->wmix), g, s, fs),
           "count transform");
    HIPCHK(fft_autocorr_nd(reinterpret_cast<const double2*>(ds->wmix), ds->alag, g, s, fs), "count autocorrelation");
    return KDEFFT_OK;
}

int kdefft_dataset_grid(const kdefft_dataset* ds, kdefft_grid* out, void* stream) {
    if (!ds || !out || !ds->rec) return fail(KDEFFT_E_ARG, "NULL or unprepared dataset");
    int rc = check_grid_shape(&ds->grid);
    if (rc) return rc;
    static thread_local double* pinned = nullptr;
    if (!pinned) HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&pinned), 8 * sizeof(double), hipHostMallocDefault),
                        "pinned readback buffer");
    hipStream_t s = S(stream);
    const DsDev* rec = static_cast<const DsDev*>(ds->rec);
    HIPCHK(hipMemcpyAsync(pinned, &rec->lo[0], 8 * sizeof(double), hipMemcpyDeviceToHost, s), "grid readback");
    HIPCHK(hipStreamSynchronize(s), "grid sync");
    kdefft_grid g = ds->grid;
    for (int k = 0; k < g.d; ++k) {
        g.lo[k] = pinned[k];
        g.delta[k] = pinned[4 + k];
    }
    rc = check_grid(&g);
    if (rc) return fail(KDEFFT_E_ARG, "the data of this dataset are not finite (grid origin or spacing invalid)");
    *out = g;
    return KDEFFT_OK;
}

static int psi_batch_common(const kdefft_dataset* ds, int n_ds, const double* G_host, int r, double* psi, void* ws,
                            size_t ws_bytes, void* stream, const RowLaunch* force);

int kdefft_psi_batch(const kdefft_dataset* ds, int n_ds, const double* G_host, int r, double* psi, void* ws,
                     size_t ws_bytes, void* stream) {
    return psi_batch_common(ds, n_ds, G_host, r, psi, ws, ws_bytes, stream, nullptr);
}

static int psi_batch_common(const kdefft_dataset* ds, int n_ds, const double* G_host, int r, double* psi, void* ws,
                            size_t ws_bytes, void* stream, const RowLaunch* force) {
    int rc = check_batch_ds(ds, n_ds, KDEFFT_MAX_PSI_DS);
    if (rc) return rc;
    const kdefft_grid& g = ds[0].grid;
    rc = check_d_r(g.d, r);
    if (rc) return rc;
    rc = check_rows(FUN_PSI, g.d, r, g.P[g.d - 1]);
    if (rc) return rc;
    if (!G_host || !psi) return fail(KDEFFT_E_ARG, "NULL G_host or psi");
    const int d = g.d, dd = d * d;
    std::vector<double> Gs(n_ds * dd);
    for (int j = 0; j < n_ds; ++j) {
        double L[16];
        rc = check_spd(G_host + 16 * j, d, "G", L);
        if (rc) return rc;
        for (int i = 0; i < dd; ++i) Gs[j * dd + i] = G_host[16 * j + i];
    }
    if (!ws) return fail(KDEFFT_E_ARG, "workspace is NULL");
    Arena a(ws, ws_bytes, false);
    const BatchScratch b = carve_batch(a, g, FUN_PSI, r, n_ds);
    rc = check_ws(a, ws_bytes);
    if (rc) return rc;
    std::vector<const DsDev*> recs(n_ds);
    for (int j = 0; j < n_ds; ++j) recs[j] = static_cast<const DsDev*>(ds[j].rec);
    PsiBatchArgs args = psi_args(g, r, n_ds, recs.data(), Gs.data());
    hipStream_t s = S(stream);
    const RowLaunch rl = force ? *force : launch_for(FUN_PSI, d, r, g.P[d - 1]);
    const int nu = (int)binom(d + r - 1, r);
    const RowGeom geo = make_geom(g, FUN_PSI, r, n_ds, rl.variant);
    args.fin = fin_psi(rl, geo, nu, b.counters, psi, nullptr);
    HIPCHK(launch_psi_setup(args, b.prm, s), "psi setup");
    HIPCHK(timed_rows(FUN_PSI, d, r, geo, b.prm, n_ds, b.partial, rl, s), "psi rows");
    if (args.fin.mode == FIN_NONE)
        HIPCHK(launch_psi_final(b.partial, geo, nu, b.prm, n_ds, psi, nullptr, s), "psi final");
    return KDEFFT_OK;
}

// Row-kernel family of a criterion: the two-Gaussian SCV families (with the
// Hessian grids for gradients) serve SCV and LSCV at r = 0; LSCV_r for r > 0 and
// Q_r use the scalar eta_r families.  The dispatch order passed to the row
// kernels is 2 for the SCV families and r for the eta families (which pick the
// kernel compiled for r's order class).
// The balanced plan of the compacted moment walk (variants 5, 6): for
// candidates with a few thousand rows each and at most MAX_PLAN candidates, on
// the resident grid (its items are numbered on the device).
static bool balanced_ok(const RowGeom& geo, int kind, const RowLaunch& rl, int64_t nc) {
    const bool mom = kind == FUN_SCV_OBJ || kind == FUN_SCV_OBJGRAD || kind == FUN_SCV_GRAD;
    return mom && rl.variant >= 5 && rl.grid_blocks == 0 && nc <= 1024 && geo.nrows <= 4096;
}

static int crit_kind(int crit, int r, bool want_grad, bool adjoint) {
    if (crit == KDEFFT_CRIT_QR) return FUN_ETA1;
    if (r > 0) return FUN_ETA2;
    return adjoint ? FUN_SCV_GRAD : (want_grad ? FUN_SCV_OBJGRAD : FUN_SCV_OBJ);
}

static int crit_common(const kdefft_dataset* ds, int n_ds, const int64_t* off, const double* vechL, int crit,
                       int r, int kind, const double* grad_out, double* obj, double* grad, int32_t* status,
                       void* ws, size_t ws_bytes, void* stream, const RowLaunch* force,
                       int64_t* walk_runs = nullptr) {
    int rc = check_batch_ds(ds, n_ds, KDEFFT_MAX_BATCH_DS);
    if (rc) return rc;
    if (crit < KDEFFT_CRIT_SCV || crit > KDEFFT_CRIT_QR) return fail(KDEFFT_E_ARG, "crit=%d", crit);
    if (r < 0 || r > 8) return fail(KDEFFT_E_ARG, "r=%d outside [0, 8]", r);
    if (crit == KDEFFT_CRIT_SCV && r != 0) return fail(KDEFFT_E_UNSUPPORTED, "SCV is defined for r = 0 only");
    if (!off || !vechL) return fail(KDEFFT_E_ARG, "NULL h_offsets or vechL");
    if (off[0] != 0) return fail(KDEFFT_E_ARG, "h_offsets[0] must be 0");
    for (int j = 0; j < n_ds; ++j)
        if (off[j + 1] < off[j]) return fail(KDEFFT_E_ARG, "h_offsets must be non-decreasing");
    const int64_t B = off[n_ds];
    if (B < 1) return fail(KDEFFT_E_ARG, "no candidate bandwidths");
    if (B > (1LL << 24)) return fail(KDEFFT_E_ARG, "too many candidates in one call");
    const kdefft_grid& g = ds[0].grid;
    if (crit == KDEFFT_CRIT_LSCV_EXACT)
        for (int j = 0; j < n_ds; ++j)
            if (ds[j].n < 2) return fail(KDEFFT_E_ARG, "the leave-one-out form needs n >= 2 (dataset %d)", j);
    const int kr = (kind == FUN_ETA1 || kind == FUN_ETA2) ? r : 2;
    rc = check_rows(kind, g.d, kr, g.P[g.d - 1]);
    if (rc) return rc;
    ScvBatchArgs a{};
    a.n_ds = n_ds;
    a.d = g.d;
    a.crit = crit;
    a.r = r;
    a.prodP = (double)sizes_of(g).prodP;
    for (int j = 0; j < n_ds; ++j) a.rec[j] = static_cast<const DsDev*>(ds[j].rec);
    for (int j = 0; j <= n_ds; ++j) a.off[j] = off[j];
    if (!ws) return fail(KDEFFT_E_ARG, "workspace is NULL");
    Arena ar(ws, ws_bytes, false);
    const BatchScratch b = carve_batch(ar, g, FUN_SCV_OBJGRAD, 2, B);
    rc = check_ws(ar, ws_bytes);
    if (rc) return rc;
    hipStream_t s = S(stream);
    const int ckey = crit == KDEFFT_CRIT_LSCV_EXACT ? KDEFFT_CRIT_LSCV : crit;
    const RowLaunch rl = force ? *force : launch_for(kind, g.d, kr, g.P[g.d - 1], ckey);
    // SCV objectives: each dataset's constant phi_{2G} term is evaluated in the
    // same launch, as one more candidate per dataset after the real ones
    const int npseudo = (crit == KDEFFT_CRIT_SCV && kind != FUN_SCV_GRAD) ? n_ds : 0;
    const int64_t nc = B + npseudo;
    RowGeom geo = make_geom(g, kind, kr, nc, rl.variant);
    if (balanced_ok(geo, kind, rl, nc)) {
        geo.nplan = (int)nc;
        geo.wc = b.wc;
        geo.item_off = b.item_off;
    }
    // the criteria complete in their own kernel: fused into the row kernel the
    // assembly lengthens the dominant launch by about what the separate
    // launch costs in a replayed graph
    if (walk_runs) {
        // the live runs of every candidate (the compacted walk's work), summed
        HIPCHK(launch_scv_setup(vechL, a, B, npseudo, b.prm, status, geo, b.wc, s, true), "criterion setup");
        std::vector<int32_t> wc((size_t)nc);
        HIPCHK(hipMemcpyAsync(wc.data(), b.wc, wc.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s), "readback");
        HIPCHK(hipStreamSynchronize(s), "sync");
        int64_t t = 0;
        for (int32_t v : wc) t += v;
        *walk_runs = t;
        return KDEFFT_OK;
    }
    // the compacted lag walk (variant 5) with one block per work item computes
    // its parameter blocks itself (the balanced plan needs the set-up kernel's
    // counts; a resident grid takes several items per block)
    const bool mom = kind == FUN_SCV_OBJ || kind == FUN_SCV_OBJGRAD || kind == FUN_SCV_GRAD;
    if (mom && rl.variant == 5 && rl.grid_blocks == -1 && geo.nplan == 0) {
        geo.setup.on = 1;
        geo.setup.npseudo = npseudo;
        geo.setup.ncand = B;
        geo.setup.vechL = vechL;
        geo.setup.status = status;
        geo.setup.prm_out = b.prm;
        geo.setup.a = a;
    } else {
        HIPCHK(launch_scv_setup(vechL, a, B, npseudo, b.prm, status, geo, geo.nplan > 0 ? b.wc : nullptr, s),
               "criterion setup");
    }
    HIPCHK(timed_rows(kind, g.d, kr, geo, b.prm, nc, b.partial, rl, s), "criterion rows");
    HIPCHK(launch_scv_final(kind, b.partial, geo, b.prm, B, npseudo, grad_out, obj, grad, s), "criterion final");
    return KDEFFT_OK;
}

static int scv_common(const kdefft_dataset* ds, int n_ds, const int64_t* off, const double* vechL, int kind,
                      const double* grad_out, double* obj, double* grad, int32_t* status, void* ws,
                      size_t ws_bytes, void* stream, const RowLaunch* force) {
    return crit_common(ds, n_ds, off, vechL, KDEFFT_CRIT_SCV, 0, kind, grad_out, obj, grad, status, ws, ws_bytes,
                       stream, force);
}

int kdefft_scv_batch(const kdefft_dataset* ds, int n_ds, const int64_t* h_offsets_host, const double* vechL,
                     double* obj, double* grad, int32_t* status, void* ws, size_t ws_bytes, void* stream) {
    if (!obj) return fail(KDEFFT_E_ARG, "obj is NULL");
    return scv_common(ds, n_ds, h_offsets_host, vechL, grad ? FUN_SCV_OBJGRAD : FUN_SCV_OBJ, nullptr, obj, grad,
                      status, ws, ws_bytes, stream, nullptr);
}

int kdefft_scv_adjoint(const kdefft_dataset* ds, int n_ds, const int64_t* h_offsets_host, const double* vechL,
                       const double* grad_out, double* grad_vechL, void* ws, size_t ws_bytes, void* stream) {
    if (!grad_out || !grad_vechL) return fail(KDEFFT_E_ARG, "NULL grad_out or grad_vechL");
    return scv_common(ds, n_ds, h_offsets_host, vechL, FUN_SCV_GRAD, grad_out, nullptr, grad_vechL, nullptr, ws,
                      ws_bytes, stream, nullptr);
}

int kdefft_crit_batch(const kdefft_dataset* ds, int n_ds, const int64_t* h_offsets_host, const double* vechL,
                      int crit, int r, double* obj, double* grad, int32_t* status, void* ws, size_t ws_bytes,
                      void* stream) {
    if (!obj) return fail(KDEFFT_E_ARG, "obj is NULL");
    if (grad && (r != 0 || crit == KDEFFT_CRIT_QR))
        return fail(KDEFFT_E_UNSUPPORTED, "gradients exist for r = 0 SCV / LSCV criteria only");
    return crit_common(ds, n_ds, h_offsets_host, vechL, crit, r, crit_kind(crit, r, grad != nullptr, false),
                       nullptr, obj, grad, status, ws, ws_bytes, stream, nullptr);
}

int kdefft_scv_walk_runs(const kdefft_dataset* ds, int n_ds, const int64_t* h_offsets_host, const double* vechL,
                         int64_t* runs_host, void* ws, size_t ws_bytes, void* stream) {
    if (!runs_host) return fail(KDEFFT_E_ARG, "runs_host is NULL");
    const int rc = check_batch_ds(ds, n_ds, KDEFFT_MAX_BATCH_DS);
    if (rc) return rc;
    const RowLaunch compact{5, 0};
    return crit_common(ds, n_ds, h_offsets_host, vechL, KDEFFT_CRIT_SCV, 0, FUN_SCV_OBJGRAD, nullptr, nullptr,
                       nullptr, nullptr, ws, ws_bytes, stream, &compact, runs_host);
}

int kdefft_crit_adjoint(const kdefft_dataset* ds, int n_ds, const int64_t* h_offsets_host, const double* vechL,
                        int crit, const double* grad_out, double* grad_vechL, void* ws, size_t ws_bytes,
                        void* stream) {
    if (!grad_out || !grad_vechL) return fail(KDEFFT_E_ARG, "NULL grad_out or grad_vechL");
    if (crit == KDEFFT_CRIT_QR) return fail(KDEFFT_E_UNSUPPORTED, "no adjoint for Q_r");
    return crit_common(ds, n_ds, h_offsets_host, vechL, crit, 0, FUN_SCV_GRAD, grad_out, nullptr, grad_vechL,
                       nullptr, ws, ws_bytes, stream, nullptr);
}

int kdefft_pi_batch(int d, int n_ds, const int64_t* n_host, const double* psi4, const int64_t* h_offsets_host,
                    const double* vechL, double* obj, double* grad, int32_t* status, void* stream) {
    if (d < 1 || d > 4) return fail(KDEFFT_E_ARG, "d=%d outside [1, 4]", d);
    if (n_ds < 1 || n_ds > KDEFFT_MAX_BATCH_DS) return fail(KDEFFT_E_ARG, "n_ds=%d", n_ds);
    if (!n_host || !psi4 || !h_offsets_host || !vechL) return fail(KDEFFT_E_ARG, "NULL argument");
    if (!obj && !grad) return fail(KDEFFT_E_ARG, "neither obj nor grad requested");
    if (h_offsets_host[0] != 0) return fail(KDEFFT_E_ARG, "h_offsets[0] must be 0");
    PiArgs a{};
    a.n_ds = n_ds;
    a.d = d;
    for (int j = 0; j < n_ds; ++j) {
        if (h_offsets_host[j + 1] < h_offsets_host[j]) return fail(KDEFFT_E_ARG, "h_offsets must be non-decreasing");
        if (n_host[j] < 1) return fail(KDEFFT_E_ARG, "n of dataset %d is %lld", j, (long long)n_host[j]);
        a.n[j] = (double)n_host[j];
        a.off[j] = h_offsets_host[j];
    }
    a.off[n_ds] = h_offsets_host[n_ds];
    const int64_t B = h_offsets_host[n_ds];
    if (B < 1) return fail(KDEFFT_E_ARG, "no candidate bandwidths");
    if (B > (1LL << 24)) return fail(KDEFFT_E_ARG, "too many candidates in one call");
    HIPCHK(launch_pi(a, psi4, vechL, B, obj, grad, status, S(stream)), "pi");
    return KDEFFT_OK;
}

// ---------------------------------------------------------------- minimiser

namespace {

struct MinScratch {
    double* st;
    int32_t* ist;
    double* ft;
    double* gt;
    int32_t* stt;
    double* xt;
};

MinScratch carve_min(Arena& a, int q, int64_t B) {
    MinScratch m;
    m.st = a.take<double>((size_t)B * min_state_doubles(q));
    m.ist = a.take<int32_t>((size_t)B * min_state_ints());
    m.ft = a.take<double>((size_t)B);
    m.gt = a.take<double>((size_t)B * q);
    m.stt = a.take<int32_t>((size_t)B);
    m.xt = a.take<double>((size_t)B * q);
    return m;
}

// workspace of the minimiser: its state, then the criterion's workspace (g =
// the datasets' grid, whose shape alone sizes it; NULL for PI)
int min_ws_need(const kdefft_grid* g, int q, int64_t B, size_t* out) {
    Arena a(nullptr, 0, true);
    (void)carve_min(a, q, B);
    size_t crit = 0;
    if (g) {
        Arena c(nullptr, 0, true);
        const int rc = plan_bytes(*g, KDEFFT_OP_SCV_BATCH, 0, B, c);
        if (rc) return rc;
        crit = c.off + 256;
    }
    *out = ((a.off + 255) & ~size_t(255)) + crit + 256;
    return KDEFFT_OK;
}

}  // namespace

int kdefft_minimize_ws_bytes(const kdefft_grid* g, int d, int64_t B, size_t* out) {
    if (!out) return fail(KDEFFT_E_ARG, "out is NULL");
    if (B < 1 || B > (1LL << 24)) return fail(KDEFFT_E_ARG, "B=%lld", (long long)B);
    if (g) {
        const int rc = check_grid(g);
        if (rc) return rc;
        d = g->d;
    }
    if (d < 1 || d > KDEFFT_MAX_D) return fail(KDEFFT_E_ARG, "d=%d outside [1,4]", d);
    return min_ws_need(g, d * (d + 1) / 2, B, out);
}

int kdefft_minimize(const kdefft_dataset* ds, int n_ds, const int64_t* off, int crit, int d, const int64_t* n_host,
                    const double* psi4, const double* vechL0, int evals, double tol, double* vechL_out,
                    double* obj_out, int32_t* info, void* ws, size_t ws_bytes, void* stream) {
    if (!off || !vechL0 || !vechL_out) return fail(KDEFFT_E_ARG, "NULL h_offsets, vechL0 or vechL_out");
    if (evals < 1 || evals > 100000) return fail(KDEFFT_E_ARG, "evals=%d outside [1, 100000]", evals);
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(KDEFFT_E_ARG, "tol must be finite and > 0");
    if (n_ds < 1 || n_ds > KDEFFT_MAX_BATCH_DS) return fail(KDEFFT_E_ARG, "n_ds=%d", n_ds);
    if (off[0] != 0) return fail(KDEFFT_E_ARG, "h_offsets[0] must be 0");
    for (int j = 0; j < n_ds; ++j)
        if (off[j + 1] < off[j]) return fail(KDEFFT_E_ARG, "h_offsets must be non-decreasing");
    const int64_t B = off[n_ds];
    if (B < 1 || B > (1LL << 24)) return fail(KDEFFT_E_ARG, "B=%lld", (long long)B);
    const bool pi = crit == KDEFFT_CRIT_PI;
    if (!pi && crit != KDEFFT_CRIT_SCV && crit != KDEFFT_CRIT_LSCV && crit != KDEFFT_CRIT_LSCV_EXACT)
        return fail(KDEFFT_E_ARG, "crit=%d has no gradient to minimise with", crit);
    const kdefft_grid* g = nullptr;
    if (pi) {
        if (!n_host || !psi4) return fail(KDEFFT_E_ARG, "the PI criterion needs n_host and psi4");
        if (d < 1 || d > KDEFFT_MAX_D) return fail(KDEFFT_E_ARG, "d=%d outside [1,4]", d);
    } else {
        const int rc = check_batch_ds(ds, n_ds, KDEFFT_MAX_BATCH_DS);
        if (rc) return rc;
        g = &ds[0].grid;
        d = g->d;
    }
    const int q = d * (d + 1) / 2;
    size_t need = 0;
    int rc = min_ws_need(g, q, B, &need);
    if (rc) return rc;
    if (!ws) return fail(KDEFFT_E_ARG, "workspace is NULL");
    if (ws_bytes < need) return fail(KDEFFT_E_WORKSPACE, "workspace %zu bytes < %zu", ws_bytes, need);
    Arena a(ws, ws_bytes, false);
    const MinScratch m = carve_min(a, q, B);
    char* crit_ws = static_cast<char*>(ws) + ((a.off + 255) & ~size_t(255));
    const size_t crit_bytes = ws_bytes - (size_t)(crit_ws - static_cast<char*>(ws));
    hipStream_t s = S(stream);
    HIPCHK(launch_min_init(B, q, vechL0, m.xt, m.ist, s), "minimiser init");
    for (int e = 0; e < evals; ++e) {
        if (pi) {
            rc = kdefft_pi_batch(d, n_ds, n_host, psi4, off, m.xt, m.ft, m.gt, m.stt, stream);
        } else {
            rc = crit_common(ds, n_ds, off, m.xt, crit, 0, FUN_SCV_OBJGRAD, nullptr, m.ft, m.gt, m.stt, crit_ws,
                             crit_bytes, stream, nullptr);
        }
        if (rc) return rc;
        HIPCHK(launch_min_step(B, q, tol, m.st, m.ist, m.ft, m.gt, m.stt, m.xt, s), "minimiser step");
    }
    HIPCHK(launch_min_final(B, q, m.st, m.ist, vechL_out, obj_out, info, s), "minimiser final");
    return KDEFFT_OK;
}

int kdefft_expand_full(int d, int r, const double* unique_host, double* full_host) {
    if (d < 1 || d > 4 || r < 0 || r > 8) return fail(KDEFFT_E_ARG, "d=%d r=%d", d, r);
    if (!unique_host || !full_host) return fail(KDEFFT_E_ARG, "NULL argument");
    // rank of every sorted tuple, in lexicographic order
    std::map<std::vector<int>, int> pos;
    std::vector<int> t(r, 0);
    int cnt = 0;
    while (true) {
        pos[t] = cnt++;
        int m = r - 1;
        while (m >= 0 && t[m] == d - 1) --m;
        if (m < 0) break;
        t[m] += 1;
        for (int k = m + 1; k < r; ++k) t[k] = t[m];
    }
    int64_t total = 1;
    for (int k = 0; k < r; ++k) total *= d;
    std::vector<int> idx(r);
    for (int64_t f = 0; f < total; ++f) {
        int64_t x = f;
        for (int k = r - 1; k >= 0; --k) {  // first index slowest
            idx[k] = (int)(x % d);
            x /= d;
        }
        std::vector<int> srt(idx);
        std::sort(srt.begin(), srt.end());
        full_host[f] = unique_host[pos[srt]];
    }
    return KDEFFT_OK;
}

int kdefft_scv_plain(const kdefft_dataset* ds, const double* H_host, double* out, void* ws, size_t ws_bytes,
                     void* stream) {
    if (!ds || !out) return fail(KDEFFT_E_ARG, "NULL dataset or out");
    int rc = check_batch_ds(ds, 1, 1);
    if (rc) return rc;
    if (!ds->counts || !ds->spec) return fail(KDEFFT_E_ARG, "dataset is not prepared");
    // the literal steps need the grid spacing on the host
    kdefft_grid g = ds->grid;
    if (!std::isfinite(g.delta[0])) {
        rc = kdefft_dataset_grid(ds, &g, stream);
        if (rc) return rc;
    }
    const int d = g.d, q = d * (d + 1) / 2;
    double LH[16];
    rc = check_spd(H_host, d, "H", LH);
    if (rc) return rc;
    double S1[16] = {0}, S2[16] = {0}, S3[16] = {0};
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            const double h = H_host[i * d + j], gp = ds->G[i * d + j];
            S1[i * 4 + j] = 2.0 * h + 2.0 * gp;
            S2[i * 4 + j] = h + 2.0 * gp;
            S3[i * 4 + j] = 2.0 * gp;
        }
    double L1[16], L2[16], L3[16];
    if (!chol_host(S1, 4, d, L1) || !chol_host(S2, 4, d, L2) || !chol_host(S3, 4, d, L3))
        return fail(KDEFFT_E_NOT_SPD, "2H+2G, H+2G or 2G not positive definite");
    ParamBlock kp{};
    chol_inv_host(L1, d, kp.v + S_P1);
    chol_inv_host(L2, d, kp.v + S_P2);
    chol_inv_host(L3, d, kp.v + S_L);
    kp.v[S_C1] = normal_const(L1, d);
    kp.v[S_C2] = normal_const(L2, d);
    kp.v[S_CONST] = normal_const(L3, d);
    ParamBlock fin{};
    chol_inv_host(LH, d, fin.v);
    for (int i = 0; i < 16; ++i) fin.v[16 + i] = LH[i];
    double c4 = 1.0;
    for (int k = 0; k < d; ++k) c4 *= 0.28209479177387814347 / LH[k * 4 + k];  // (4 pi)^{-1/2} / L_kk
    fin.v[32] = c4 / (double)ds->n;
    if (!ws) return fail(KDEFFT_E_ARG, "workspace is NULL");
    Arena a(ws, ws_bytes, false);
    const PlainScratch p = carve_plain(a, g, false);
    rc = check_ws(a, ws_bytes);
    if (rc) return rc;
    const Sizes sz = sizes_of(g);
    const double scale = 1.0 / ((double)ds->n * (double)ds->n * (double)sz.prodP);
    const int nb = nblk_dot(g);
    hipStream_t s = S(stream);
    const double2* C = reinterpret_cast<const double2*>(ds->spec);
    for (int e = 0; e <= q; ++e) {
        HIPCHK(launch_kgrid_scv(p.kreal, g, kp, e, s), "kernel grid");
        HIPCHK(fft_r2c_nd(p.kreal, p.K, g, s), "R2C kernel");
        HIPCHK(launch_cmul(p.K, C, sz.spec, s), "spectrum product");
        HIPCHK(fft_c2r_nd(p.K, p.kreal, g, s), "C2R");
        HIPCHK(launch_dot_counts(ds->counts, p.kreal, g, p.partial, nb, s), "count contraction");
        HIPCHK(launch_sum_scale(p.partial, nb, scale, p.sums + e, s), "final sum");
    }
    HIPCHK(launch_scv_plain_final(p.sums, fin, d, out, s), "scv assembly");
    return KDEFFT_OK;
}

int kdefft_lag_layout(int N, int moments, int* run_len, int* runs_per_seg, int* rows_per_pass) {
    if (!run_len || !runs_per_seg || !rows_per_pass) return fail(KDEFFT_E_ARG, "NULL output");
    if (moments != 0 && moments != 1) return fail(KDEFFT_E_ARG, "moments=%d", moments);
    if (!lag_layout(N, moments, run_len, runs_per_seg, rows_per_pass))
        return fail(KDEFFT_E_ARG, "N=%d is not a power of two in [4, 2048]", N);
    return KDEFFT_OK;
}

int kdefft_set_row_launch(int kind, int d, int r, int N, int variant, int grid_blocks) {
    if (kind < 0 || kind > FUN_ETA2) return fail(KDEFFT_E_ARG, "kind=%d", kind);
    if (variant == -1) {
        clear_launch(kind, d, r, N);
        return KDEFFT_OK;
    }
    if (variant < 0 || variant >= ROW_VARIANTS) return fail(KDEFFT_E_ARG, "variant=%d", variant);
    if (grid_blocks < -1) return fail(KDEFFT_E_ARG, "grid_blocks=%d", grid_blocks);
    if (rows_per_iter(kind, d, r, N, variant) < 1)
        return fail(KDEFFT_E_UNSUPPORTED, "no compiled row kernel for kind=%d d=%d r=%d N=%d", kind, d, r, N);
    set_launch(kind, d, r, N, RowLaunch{variant, grid_blocks});
    return KDEFFT_OK;
}

static int check_fft_shape(int d, const int32_t* P) {
    if (d < 1 || d > KDEFFT_MAX_D) return fail(KDEFFT_E_ARG, "d=%d outside [1,4]", d);
    if (!P) return fail(KDEFFT_E_ARG, "P_host is NULL");
    for (int k = 0; k < d; ++k)
        if (P[k] < 4 || P[k] > KDEFFT_MAX_P || (P[k] & (P[k] - 1)))
            return fail(KDEFFT_E_ARG, "P[%d]=%d is not a power of two in [4, %d]", k, P[k], KDEFFT_MAX_P);
    return KDEFFT_OK;
}

int kdefft_set_fft_schedule(int d, const int32_t* P_host, int sched) {
    const int rc = check_fft_shape(d, P_host);
    if (rc) return rc;
    if (sched < -1 || sched >= FFT_SCHEDULES) return fail(KDEFFT_E_ARG, "sched=%d", sched);
    set_fft_sched(d, P_host, sched);
    return KDEFFT_OK;
}

int kdefft_get_fft_schedule(int d, const int32_t* P_host, int* sched) {
    const int rc = check_fft_shape(d, P_host);
    if (rc) return rc;
    if (!sched) return fail(KDEFFT_E_ARG, "NULL output");
    kdefft_grid g;
    std::memset(&g, 0, sizeof(g));
    g.d = d;
    for (int k = 0; k < d; ++k) g.P[k] = P_host[k];
    *sched = fft_sched_for(g);
    return KDEFFT_OK;
}

int kdefft_get_row_launch(int kind, int d, int r, int N, int* variant, int* grid_blocks) {
    if (kind < 0 || kind > FUN_ETA2) return fail(KDEFFT_E_ARG, "kind=%d", kind);
    if (!variant || !grid_blocks) return fail(KDEFFT_E_ARG, "NULL output");
    const RowLaunch rl = launch_for(kind, d, r, N);
    *variant = rl.variant;
    *grid_blocks = rl.grid_blocks;
    return KDEFFT_OK;
}

extern "C++" {
namespace {

// Timing of one launch choice: one untimed call, then the mean of 5 between
// two events on the stream.
template <class Fn>
int time_choice(hipStream_t s, hipEvent_t e0, hipEvent_t e1, Fn&& fn, float* ms) {
    int rc = fn();
    if (rc) return rc;
    HIPCHK(hipEventRecord(e0, s), "event");
    for (int rep = 0; rep < 5; ++rep) {
        rc = fn();
        if (rc) return rc;
    }
    HIPCHK(hipEventRecord(e1, s), "event");
    HIPCHK(hipEventSynchronize(e1), "event sync");
    HIPCHK(hipEventElapsedTime(ms, e0, e1), "elapsed");
    *ms /= 5.f;
    return KDEFFT_OK;
}

// The fastest of a family's launch choices; the default keeps its place unless
// another is more than 3% faster, so that timing noise does not flip the
// choice from run to run.
struct Pick {
    RowLaunch best{0, 0};
    float best_ms = 1e30f, dflt_ms = -1.f;
    void add(RowLaunch rl, float ms, RowLaunch dflt) {
        if (ms < best_ms) {
            best_ms = ms;
            best = rl;
        }
        if (rl.variant == dflt.variant && rl.grid_blocks == dflt.grid_blocks) dflt_ms = ms;
    }
    void settle(RowLaunch dflt) {
        if (dflt_ms > 0.f && best_ms > 0.97f * dflt_ms) {
            best = dflt;
            best_ms = dflt_ms;
        }
    }
};

void append_line(std::string& lines, const char* fmt, ...) {
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    lines += buf;
}

}  // namespace
}  // extern "C++"

int kdefft_autotune(const kdefft_dataset* ds, void* ws, size_t ws_bytes, const char* cache_path, void* stream) {
    int rc = check_batch_ds(ds, 1, 1);
    if (rc) return rc;
    const kdefft_grid& g = ds->grid;
    const int d = g.d, q = d * (d + 1) / 2, N = g.P[d - 1];
    if (!ws) return fail(KDEFFT_E_ARG, "workspace is NULL");
    Arena a(ws, ws_bytes, false);
    carve_batch(a, g, FUN_SCV_OBJGRAD, 2, TUNE_B);
    double* vech = a.take<double>(TUNE_B * q);
    double* obj = a.take<double>(TUNE_B);
    double* grad = a.take<double>(TUNE_B * q);
    double* psi_out = a.take<double>(TUNE_PSI_OUT);
    rc = check_ws(a, ws_bytes);
    if (rc) return rc;
    // TUNE_B candidates H_b = s_b * Gpilot with s_b spread over [0.5, 8]
    double LG[16];
    rc = check_spd(ds->G, d, "Gpilot", LG);
    if (rc) return rc;
    std::vector<double> hv(TUNE_B * q);
    for (int b = 0; b < TUNE_B; ++b) {
        const double sc = std::sqrt(0.5 * std::pow(16.0, b / double(TUNE_B - 1)));
        int t = 0;
        for (int j = 0; j < d; ++j)
            for (int i = j; i < d; ++i) hv[b * q + t++] = sc * LG[i * 4 + j];
    }
    hipStream_t s = S(stream);
    HIPCHK(hipMemcpyAsync(vech, hv.data(), hv.size() * sizeof(double), hipMemcpyHostToDevice, s), "tuner upload");
    int64_t off[2] = {0, TUNE_B};
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0), "event");
    HIPCHK(hipEventCreate(&e1), "event");
    std::string lines, cache;
    const std::string arch = [] {
        int dev = 0;
        (void)hipGetDevice(&dev);
        return arch_name(dev);
    }();
    const int grids[2] = {0, -1};

    // 1. FFT stage: the dataset's count transform and autocorrelation under
    // every schedule (the dataset is left holding the chosen schedule's result)
    int fbest = 0;
    {
        float fbest_ms = 1e30f, f0_ms = -1.f;
        const kdefft_dataset* dsp = ds;
        for (int fs = 0; fs < FFT_SCHEDULES && !rc; ++fs) {
            float ms = 0.f;
            rc = time_choice(s, e0, e1, [&]() -> int {
                HIPCHK(fft_prepare_nd(dsp->counts, 0, nullptr, reinterpret_cast<double2*>(dsp->spec),
                                      reinterpret_cast<double2*>(dsp->wmix), g, s, fs), "count transform");
                HIPCHK(fft_autocorr_nd(reinterpret_cast<const double2*>(dsp->wmix), dsp->alag, g, s, fs),
                       "count autocorrelation");
                return KDEFFT_OK;
            }, &ms);
            if (rc) break;
            append_line(lines, "fft schedule %d: %.1f us\n", fs, ms * 1000.0);
            if (ms < fbest_ms) {
                fbest_ms = ms;
                fbest = fs;
            }
            if (fs == 0) f0_ms = ms;
        }
        if (!rc) {
            if (f0_ms > 0.f && fbest_ms > 0.97f * f0_ms) {
                fbest = 0;
                fbest_ms = f0_ms;
            }
            set_fft_sched(d, g.P, fbest);
            rc = fft_prepare_nd(ds->counts, 0, nullptr, reinterpret_cast<double2*>(ds->spec),
                                reinterpret_cast<double2*>(ds->wmix), g, s, fbest) == hipSuccess &&
                         fft_autocorr_nd(reinterpret_cast<const double2*>(ds->wmix), ds->alag, g, s, fbest) ==
                             hipSuccess
                     ? KDEFFT_OK
                     : fail(KDEFFT_E_HIP, "count transform");
            append_line(lines, "fft best: schedule %d\n", fbest);
            append_line(cache,
                        "{\"arch\": \"%s\", \"fft\": 1, \"d\": %d, \"P0\": %d, \"P1\": %d, \"P2\": %d, \"P3\": %d, "
                        "\"sched\": %d, \"us\": %.2f}\n",
                        arch.c_str(), d, g.P[0], d > 1 ? g.P[1] : 0, d > 2 ? g.P[2] : 0, d > 3 ? g.P[3] : 0, fbest,
                        fbest_ms * 1000.0);
        }
    }

    // 2. SCV families (objective + gradient timed), then the same kernels
    // serving LSCV (narrower Gaussians, their own choice)
    const int crits[2] = {KDEFFT_CRIT_SCV, KDEFFT_CRIT_LSCV};
    const RowLaunch dflt_mom{5, -1};
    for (int ci = 0; ci < 2 && !rc; ++ci) {
        const int crit = crits[ci];
        Pick pk;
        for (int v = 0; v < ROW_VARIANTS && !rc; ++v) {
            if (rows_per_iter(FUN_SCV_OBJGRAD, d, 2, N, v) < 1) continue;
            for (int gi = 0; gi < 2 && !rc; ++gi) {
                const RowLaunch rl{v, grids[gi]};
                float ms = 0.f;
                rc = time_choice(s, e0, e1, [&] {
                    return crit_common(ds, 1, off, vech, crit, 0, FUN_SCV_OBJGRAD, nullptr, obj, grad, nullptr, ws,
                                       ws_bytes, stream, &rl);
                }, &ms);
                if (rc) break;
                append_line(lines, crit == KDEFFT_CRIT_SCV ? "variant %d grid %d: %.1f us\n"
                                                           : "lscv variant %d grid %d: %.1f us\n",
                            v, rl.grid_blocks, ms * 1000.0);
                pk.add(rl, ms, dflt_mom);
            }
        }
        if (rc) break;
        pk.settle(dflt_mom);
        append_line(lines, crit == KDEFFT_CRIT_SCV ? "best: variant %d grid %d\n" : "lscv best: variant %d grid %d\n",
                    pk.best.variant, pk.best.grid_blocks);
        for (int kind = FUN_SCV_OBJ; kind <= FUN_SCV_GRAD; ++kind) {
            if (rows_per_iter(kind, d, 2, N, pk.best.variant) < 1) continue;
            set_launch(kind, d, 2, N, pk.best, crit == KDEFFT_CRIT_SCV ? 0 : KDEFFT_CRIT_LSCV);
            append_line(cache,
                        "{\"arch\": \"%s\", \"kind\": %d, \"crit\": %d, \"d\": %d, \"r\": 2, \"N\": %d, "
                        "\"variant\": %d, \"grid\": %d, \"us\": %.2f}\n",
                        arch.c_str(), kind, crit == KDEFFT_CRIT_SCV ? 0 : KDEFFT_CRIT_LSCV, d, N, pk.best.variant,
                        pk.best.grid_blocks, pk.best_ms * 1000.0);
        }
    }

    // 3. LSCV_4 (the scalar eta family, lag domain only): grid size
    if (!rc && rows_per_iter(FUN_ETA2, d, 4, N, 3) >= 1) {
        Pick pk;
        const RowLaunch dflt{3, 0};
        for (int gi = 0; gi < 2 && !rc; ++gi) {
            const RowLaunch rl{3, grids[gi]};
            float ms = 0.f;
            rc = time_choice(s, e0, e1, [&] {
                return crit_common(ds, 1, off, vech, KDEFFT_CRIT_LSCV, 4, FUN_ETA2, nullptr, obj, nullptr, nullptr, ws,
                                   ws_bytes, stream, &rl);
            }, &ms);
            if (rc) break;
            append_line(lines, "lscv4 grid %d: %.1f us\n", rl.grid_blocks, ms * 1000.0);
            pk.add(rl, ms, dflt);
        }
        if (!rc) {
            pk.settle(dflt);
            set_launch(FUN_ETA2, d, 4, N, pk.best, KDEFFT_CRIT_LSCV);
            append_line(lines, "lscv4 best: grid %d\n", pk.best.grid_blocks);
            append_line(cache,
                        "{\"arch\": \"%s\", \"kind\": %d, \"crit\": %d, \"d\": %d, \"r\": 4, \"N\": %d, "
                        "\"variant\": 3, \"grid\": %d, \"us\": %.2f}\n",
                        arch.c_str(), FUN_ETA2, KDEFFT_CRIT_LSCV, d, N, pk.best.grid_blocks, pk.best_ms * 1000.0);
        }
    }

    // 4. psi_4 at the dataset's pilot (its workspace may overlap the candidates)
    if (!rc && rows_per_iter(FUN_PSI, d, 4, N, 3) >= 1) {
        double G16[16];
        for (int i = 0; i < 16; ++i) G16[i] = 0.0;
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) G16[i * d + j] = ds->G[i * d + j];
        Pick pk;
        const RowLaunch dflt{3, 0};
        for (int v = 0; v <= 3 && !rc; ++v) {
            if (rows_per_iter(FUN_PSI, d, 4, N, v) < 1) continue;
            for (int gi = 0; gi < 2 && !rc; ++gi) {
                const RowLaunch rl{v, grids[gi]};
                float ms = 0.f;
                rc = time_choice(s, e0, e1, [&] {
                    return psi_batch_common(ds, 1, G16, 4, psi_out, ws, ws_bytes, stream, &rl);
                }, &ms);
                if (rc) break;
                append_line(lines, "psi4 variant %d grid %d: %.1f us\n", v, rl.grid_blocks, ms * 1000.0);
                pk.add(rl, ms, dflt);
            }
        }
        if (!rc) {
            pk.settle(dflt);
            set_launch(FUN_PSI, d, 4, N, pk.best);
            append_line(lines, "psi4 best: variant %d grid %d\n", pk.best.variant, pk.best.grid_blocks);
            append_line(cache,
                        "{\"arch\": \"%s\", \"kind\": %d, \"d\": %d, \"r\": 4, \"N\": %d, \"variant\": %d, "
                        "\"grid\": %d, \"us\": %.2f}\n",
                        arch.c_str(), FUN_PSI, d, N, pk.best.variant, pk.best.grid_blocks, pk.best_ms * 1000.0);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (cache_path && *cache_path) {
        FILE* f = std::fopen(cache_path, "a");
        if (f) {
            std::fputs(cache.c_str(), f);
            std::fclose(f);
        }
    }
    g_err = lines;
    return KDEFFT_OK;
}

}  // extern "C"

int kdefft_timing_start(int max_launches) {
    if (max_launches < 1 || max_launches > KDEFFT_MAX_TIMED)
        return fail(KDEFFT_E_ARG, "max_launches %d outside [1, %d]", max_launches, KDEFFT_MAX_TIMED);
    std::lock_guard<std::mutex> lk(g_timer.mu);
    while ((int)g_timer.ev.size() < 2 * max_launches) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e), "timing event");
        g_timer.ev.push_back(e);
    }
    g_timer.tag.assign(max_launches, 0);
    g_timer.cap = max_launches;
    g_timer.used = 0;
    g_timer.armed = true;
    return KDEFFT_OK;
}

int kdefft_timing_stop(float* ms_out, int32_t* tag_out, int cap, int* count_out) {
    if (!count_out || cap < 0 || (cap > 0 && (!ms_out || !tag_out)))
        return fail(KDEFFT_E_ARG, "bad output arrays");
    std::lock_guard<std::mutex> lk(g_timer.mu);
    const int used = g_timer.armed ? g_timer.used : 0;
    g_timer.armed = false;
    const int cnt = std::min(used, cap);
    for (int k = 0; k < cnt; ++k) {
        HIPCHK(hipEventSynchronize(g_timer.ev[2 * k + 1]), "timing sync");
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, g_timer.ev[2 * k], g_timer.ev[2 * k + 1]), "timing elapsed");
        ms_out[k] = ms;
        tag_out[k] = g_timer.tag[k];
    }
    *count_out = cnt;
    return KDEFFT_OK;
}
