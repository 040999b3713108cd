// Internal interface between the C-ABI layer (api.cpp) and the HIP kernels.
// Nothing here is exported.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/kdefft.h"

namespace kdefft {

constexpr int PRM = 96;     // doubles per candidate parameter block
constexpr int NT_DEF = 256;  // threads per block of the simple kernels

// Parameter block layout (float64 slots) shared by setup, row and finalize kernels.
// Matrices use row stride 4.
//   psi:  [0,16) P = G^{-1}   [16] c = (-1)^r (2pi)^{-d/2}|G|^{-1/2}
//   scv:  [0,16) P1 = (2H+2G)^{-1}  [16,32) P2 = (H+2G)^{-1}  [32] c1  [33] c2
//   both: [38] alag pointer bits  [39] wmix pointer bits  [40,44) delta  [44] n  [45] 1/(n^2 prod P)
//         [46] constant term  [47] singular flag  [48,64) L (scv) / P3 (plain scv)
//   criteria: [34] first (closed-form) term  [35] r of eta_r  [36] sign (-1)^r
//         [37] SCV: the candidate index whose objective sum is the dataset's constant phi_{2G} term
//   lag walk of Gaussian k (k = 0, 1) at [64 + 8k, 72 + 8k): dz[0..3] = delta_last P_k[i][last],
//         [4] hpl = delta_last^2 P_k[last][last] / 2, [5] sig = exp(-2 hpl), [6] log(1e-290 / c_k)
enum Slot { S_P1 = 0, S_C = 16, S_P2 = 16, S_C1 = 32, S_C2 = 33, S_FIRST = 34, S_R = 35, S_SIGN = 36, S_PSEUDO = 37,
            S_ALAG = 38,
            S_WMIX = 39, S_DELTA = 40, S_N = 44, S_SCALE = 45, S_CONST = 46, S_SING = 47, S_L = 48,
            // fused completion (FinishArgs): mode, grids, counter and output pointers
            S_FIN_MODE = 80, S_FIN_NG = 81, S_FIN_CNT = 82, S_FIN_OUT = 83, S_FIN_SCAL = 84 };

// How a psi lag launch completes (written into every candidate's parameter
// block by the setup kernels): FIN_NONE = a separate final kernel assembles
// the results; FIN_PSI = the block that finishes a candidate's last work item
// writes its psi entries.  counters: one int per candidate, cleared by the
// setup kernel.
enum FinMode { FIN_NONE = 0, FIN_PSI = 1 };
struct FinishArgs {
    int mode;
    int ng;
    int32_t* counters;
    double* out;    // psi [n_ds, ng]
    double* scal;   // psi[0, 0] also stored here (constant SCV term)
};

// Per-dataset record kept in the dataset's own device buffer (written by a
// kernel at prepare time); batched calls pass pointers to these records.
struct DsDev {
    const double2* wmix;
    const double* alag;
    const double* scal;
    double n;
    double lo[4];      // grid origin and spacing (lo, delta contiguous: the
    double delta[4];   // binning kernel reads them from here on the device path)
    double G[16];   // pilot, row stride 4
};

// Kernel-argument views of a batch (no host-to-device copies per call).
struct ScvBatchArgs {
    int n_ds;
    int d;
    int crit;   // KDEFFT_CRIT_*
    int r;      // order of eta_r (0 for SCV)
    double prodP;
    const DsDev* rec[KDEFFT_MAX_BATCH_DS];
    int64_t off[KDEFFT_MAX_BATCH_DS + 1];
};
struct PsiBatchArgs {
    int n_ds;
    int d;
    int r;
    double prodP;
    const DsDev* rec[KDEFFT_MAX_PSI_DS];
    double Gv[KDEFFT_MAX_PSI_DS][10];   // vech (columns of the lower triangle)
    FinishArgs fin;
};
struct PiArgs {
    int n_ds;
    int d;
    double n[KDEFFT_MAX_BATCH_DS];
    int64_t off[KDEFFT_MAX_BATCH_DS + 1];
};
// One parameter block passed by value.
struct ParamBlock {
    double v[64];
};

// Parameter set-up done by the lag kernel itself (the SCV families on the lag
// launches): each work item's block computes its candidate's parameter block
// in LDS from vechL and the dataset records, and the block of the candidate's
// first item also stores it to prm_out (for the final kernel) and its status.
struct ScvSetup {
    int on;
    int npseudo;
    int64_t ncand;
    const double* vechL;
    int32_t* status;
    double* prm_out;
    ScvBatchArgs a;
};

// Geometry of the row decomposition of the lag grid used by the batched kernels.
struct RowGeom {
    int d;
    int M[4];
    int P[4];
    int64_t nrows;     // rows of the half lag set with nonzero kernel values
    int64_t chunk;     // rows per work item
    int64_t nchunks;   // work items per candidate (balanced plan: an upper bound of items / candidates)
    int Q;             // P[d-1]/2 + 1
    // Balanced plan of the compacted moment walk (nplan > 0): the nplan
    // candidates' live segment counts wc (from the set-up kernel) set how many
    // items each gets; the launch writes the first item of each candidate to
    // item_off [nplan + 1] for the final kernel.
    int nplan;
    const int32_t* wc;
    int32_t* item_off;
    ScvSetup setup;    // setup.on: the SCV lag kernel computes its parameter blocks
};

// Kinds of kernel families generated on the lag grid.
// FUN_SCV_* serve every criterion with two Gaussians and a Hessian gradient
// (SCV, LSCV); FUN_ETA1 / FUN_ETA2 are the scalar eta_r families (Q_r, LSCV_r).
enum FunKind { FUN_PSI = 0, FUN_SCV_OBJ = 1, FUN_SCV_OBJGRAD = 2, FUN_SCV_GRAD = 3, FUN_ETA1 = 4, FUN_ETA2 = 5 };

int ng_of(int kind, int d, int r);   // number of kernel grids of a family

// -------------------------------------------------------------- launchers
// All return hipSuccess or the first HIP error; they only enqueue work.
hipError_t twiddles(const double2** out);  // per-device table e^{-2 pi i m/4096} + N-point subsets

// Data bounds: per-block partials (nblk blocks; 8 doubles each) then their
// reduction into out (min[4], max[4]).
hipError_t launch_bounds(const double* X, int64_t n, int d, double* partial, int nblk,
                         double* out, hipStream_t s);
// The per-block partials only, clearing zero_bytes (a multiple of 16, 16-byte
// aligned) at zero_ptr on the way.
hipError_t launch_bounds_partial(const double* X, int64_t n, int d, double* partial, int nblk, hipStream_t s,
                                 void* zero_ptr, size_t zero_bytes, int32_t* n_out = nullptr, double* scal = nullptr);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
// gdev: if not NULL, 8 device doubles (lo[4], delta[4]) that replace g's
hipError_t launch_linbin(const double* X, int64_t n, const kdefft_grid& g, int64_t* counts,
                         int32_t* n_out, hipStream_t s, const double* gdev = nullptr);
// Binning into corner slots over the last min(d, 3) axes: a record of
// S = 2^min(d, 3) int64 per cell of the count grid (slots: S * prod M int64,
// cleared here unless slots_zeroed).  A point adds its 2^d corner weights to
// 2^(d-3) records for d = 4 (one per node of axis 0: the cell of the lowest
// corner moved along axis 0 for the upper one), to one record otherwise,
// slot s of a record taking the corner's nodes along the slotted axes (bit j
// of s: upper along axis d-1-j).  A point's increments thus fall in
// 2^max(d-3, 0) contiguous records (one cache line each) instead of 2^(d-1)
// pairs of grid cells.  The count transform's first pass (fft_prepare_nd with
// slots) gathers each count exactly from S nearby slots:
// count(i) = sum over s of slot s of record i - e(s).
__host__ __device__ constexpr int slot_axes(int d) { return d < 3 ? d : 3; }
__host__ __device__ constexpr int corner_slots(int d) { return 1 << slot_axes(d); }
struct HeaderArgs;
// hdr (may be NULL): with hdr->partial set, the binning launch also computes
// the grid from the bound partials and writes the dataset header (block 0).
hipError_t launch_linbin_slots(const double* X, int64_t n, const kdefft_grid& g, int64_t* slots, int32_t* n_out,
                               hipStream_t s, const double* gdev, bool slots_zeroed, const HeaderArgs* hdr = nullptr);

// One small launch at the start of a dataset's preparation: the record (with
// the grid origin and spacing from the data bounds when `partial` is set --
// lo = min - pad, hi = max + pad, hi = lo + 1 for a degenerate axis,
// delta = (hi - lo)/(M - 1), the same IEEE steps as the host planner), the
// out-of-grid counter and scalar block cleared, and the parameter block of
// the constant SCV term (psi_0 at 2G) when prm is set.
struct HeaderArgs {
    DsDev* rec;
    DsDev val;
    const double* partial;   // per-block bound partials of the data (or NULL: keep val's grid)
    int nblk;
    kdefft_grid g;
    double pad[4];
    int32_t* n_out;
    double* scal;
    double* prm;
    double Gv2[10];   // vech of 2G (columns of the lower triangle)
    double prodP;
    FinishArgs fin;   // completion of the constant-term launch
};
hipError_t launch_ds_header(const HeaderArgs& h, hipStream_t s);
hipError_t launch_fill_czp(const int64_t* counts, const kdefft_grid& g, double* czp, hipStream_t s);


// Multi-dimensional transforms over the circular-layout arrays.
hipError_t fft_r2c_nd(const double* in, double2* out, const kdefft_grid& g, hipStream_t s);
hipError_t fft_c2r_nd(double2* inout, double* out, const kdefft_grid& g, hipStream_t s);
// FFT-stage schedules of the count transform (launch shapes and radix order
// of its passes; fft.hip FS_*): fs in [0, FFT_SCHEDULES), 0 the default.
constexpr int FFT_SCHEDULES = 6;
// Count spectrum of a prepared dataset: spec = R2C(czp); wmix = |spec|^2
// transformed forward along the leading axes.  The first pass reads the int64
// counts directly: src is the count grid itself (slots = 0) or the corner
// slots of the binning (slots = 1), from which it gathers the counts exactly
// and also writes them to counts.
hipError_t fft_prepare_nd(const int64_t* src, int slots, int64_t* counts, double2* spec, double2* wmix,
                          const kdefft_grid& g, hipStream_t s, int fs);
// alag = inverse transform of |C|^2 = prod P times the count autocorrelation,
// computed from the mixed spectrum (rows at negated leading indices).
hipError_t fft_autocorr_nd(const double2* wmix, double* alag, const kdefft_grid& g, hipStream_t s, int fs);

// Paper-literal path, one grid per launch.
hipError_t launch_kgrid_psi(double* out, const kdefft_grid& g, int r, const ParamBlock& prm,
                            int entry, hipStream_t s);
hipError_t launch_kgrid_scv(double* out, const kdefft_grid& g, const ParamBlock& prm, int entry,
                            hipStream_t s);
hipError_t launch_cmul(double2* K, const double2* C, int64_t count, hipStream_t s);
hipError_t launch_dot_counts(const int64_t* counts, const double* sreal, const kdefft_grid& g,
                             double* partial, int nblk, hipStream_t s);
hipError_t launch_sum_scale(const double* partial, int nblk, double scale, double* out,
                            hipStream_t s);
hipError_t launch_scv_plain_final(const double* sums, const ParamBlock& fin, int d, double* out,
                                  hipStream_t s);

// Batched row kernels.
struct RowLaunch {
    int variant;        // compiled launch variant (rows per iteration, radix schedule)
    int grid_blocks;    // persistent grid size; 0 = occupancy x CUs, -1 = one block per item
};
hipError_t launch_rows(int kind, int d, int r, const RowGeom& geo, const double* prm, int64_t ncand,
                       double* partial, const RowLaunch& rl, hipStream_t s);
int rows_per_iter(int kind, int d, int r, int N, int variant);
// compiled lag-kernel layout for last-axis length N (0 = unsupported N)
int lag_layout(int N, int moments, int* run_len, int* runs_per_seg, int* rows_per_pass);
// 0-2: spectral (per-candidate FFT); 3, 4: lag domain (4: scaled walk of rising
// runs); 5, 6: as 3, 4 with only the live runs of each row dealt to the threads
constexpr int ROW_VARIANTS = 7;
// ncand real candidates, then npseudo constant-term candidates (SCV: one per
// dataset); wc (may be NULL): live segment counts for the balanced plan.
hipError_t launch_scv_setup(const double* vechL, const ScvBatchArgs& a, int64_t ncand, int npseudo, double* prm,
                            int32_t* status, const RowGeom& geo, int32_t* wc, hipStream_t s, bool count_runs = false);
hipError_t launch_psi_setup(const PsiBatchArgs& a, double* prm, hipStream_t s);
hipError_t launch_scv_final(int kind, const double* partial, const RowGeom& geo,
                            const double* prm, int64_t ncand, int npseudo, const double* grad_out,
                            double* obj, double* grad, hipStream_t s);
hipError_t launch_psi_final(const double* partial, const RowGeom& geo, int ng,
                            const double* prm, int64_t ncand, double* psi, double* scal_out,
                            hipStream_t s);

// batched quasi-Newton minimiser (minimize.hip): per-candidate state of
// min_state_doubles(q) doubles and min_state_ints() int32
int min_state_doubles(int q);
int min_state_ints();
hipError_t launch_min_init(int64_t B, int q, const double* x0, double* xt, int32_t* ist, hipStream_t s);
hipError_t launch_min_step(int64_t B, int q, double tol, double* st, int32_t* ist, const double* ft,
                           const double* gt, const int32_t* stt, double* xt, hipStream_t s);
hipError_t launch_min_final(int64_t B, int q, const double* st, const int32_t* ist, double* x_out, double* f_out,
                            int32_t* info, hipStream_t s);
hipError_t launch_pi(const PiArgs& a, const double* psi4, const double* vechL, int64_t ncand, double* obj,
                     double* grad, int32_t* status, hipStream_t s);

RowGeom make_geom(const kdefft_grid& g, int kind, int r, int64_t ncand, int variant);

// Host helpers of the C-ABI layer shared with other units: record an error
// (returned code, message for kdefft_last_error_detail), and the workspace
// bytes kdefft_scv_batch needs for a batch (validates the datasets and offsets).
int set_error(int code, const char* msg);
int scv_batch_ws_need(const kdefft_dataset* ds, int n_ds, const int64_t* off, size_t* need);

}  // namespace kdefft
