/*
 * kdefft — FFT-based integrated density-derivative functionals psi_r and the
 * smoothed cross-validation (SCV) bandwidth objective, for full (unconstrained)
 * d x d bandwidth matrices, on AMD Instinct MI355X (gfx950).
 *
 * Method: Gramacki & Gramacki, "FFT-based fast bandwidth selector for
 * multivariate kernel density estimation".  The quantity computed is
 *
 *     psi_r(G) = n^-2 sum_i sum_j D^{(x)r} phi_G(X_i - X_j)          (Eq. (13))
 *
 * by the paper's four steps (Sec. 4): linear binning onto an M_1 x ... x M_d
 * grid (Eq. (14)), the kernel on the full symmetric lag grid (Eq. (17)-(18)),
 * a zero-padded FFT convolution (Eq. (19)-(23)) and the count-weighted sum
 * (Eq. (24)).  Sec. 5 extends the route to derivative functionals of any even
 * order r and to the double sums of the PI and SCV selectors.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Return value   int: KDEFFT_OK (0) or a negative KDEFFT_E_* code.  On error a
 *                human-readable reason is available from
 *                kdefft_last_error_detail() (per calling thread).  Argument
 *                errors are detected on the host before anything is launched.
 * Pointers       Arrays are DEVICE pointers unless the name ends in _host.
 * Ownership      The caller owns all memory.  The library never allocates
 *                device memory: functions that need scratch space take a
 *                workspace (ws, ws_bytes) whose size is obtained first from
 *                kdefft_ws_bytes(); a too-small workspace is KDEFFT_E_WORKSPACE.
 * Streams        `stream` is a hipStream_t passed as void* (NULL = the default
 *                stream).  All device work is enqueued on it and the call
 *                returns without waiting, except kdefft_grid_auto() (reads the
 *                data bounds back) and kdefft_autotune().
 * Layouts        X: row-major [n, d] float64.  G, H: d x d row-major float64.
 *                Grid counts: row-major [M_0, ..., M_{d-1}], last axis fastest.
 *                vechL: [B, q], q = d(d+1)/2, lower Cholesky factor L of
 *                H = L L^T with the columns of the lower triangle stacked:
 *                (L11, L21, ..., Ld1, L22, ..., Ldd).
 *                psi: the C(d+r-1, r) unique entries of D^{(x)r} (Sec. 5) in
 *                canonical order: index tuples i_1 <= ... <= i_r, sorted
 *                lexicographically (d=2, r=4: 1111,1112,1122,1222,2222).
 * Limits         1 <= d <= 4; r even, 0 <= r <= 8, and the number of
 *                multi-indices of order <= r, C(d+r, r), at most 84 (so d=3
 *                allows r <= 6 and d=4 allows r <= 4); 2 <= M_k; P_k a power of
 *                two with 2 M_k - 1 <= P_k <= 4096; 1 <= n < 2^23 per dataset.
 * Determinism    Counts are bit-exact (integer atomics).  Every floating-point
 *                reduction has a fixed order, so repeated calls with the same
 *                inputs and launch configuration give identical bits.
 */
#ifndef KDEFFT_H
#define KDEFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KDEFFT_OK 0
#define KDEFFT_E_ARG (-1)          /* invalid argument (null pointer, bad size, bad layout) */
#define KDEFFT_E_NOT_SPD (-2)      /* a bandwidth matrix is not symmetric positive definite */
#define KDEFFT_E_ODD_R (-3)        /* derivative order r is odd (the functional is 0) */
#define KDEFFT_E_OUT_OF_GRID (-4)  /* data outside the grid (reported by kdefft_check_binning) */
#define KDEFFT_E_OVERFLOW (-5)     /* n >= 2^23: an int64 bin could overflow */
#define KDEFFT_E_WORKSPACE (-6)    /* workspace or dataset buffer too small / misaligned */
#define KDEFFT_E_HIP (-7)          /* a HIP runtime call failed */
#define KDEFFT_E_UNSUPPORTED (-8)  /* (d, r, P) outside the compiled limits */

#define KDEFFT_MAX_D 4
#define KDEFFT_MAX_R 8
#define KDEFFT_MAX_P 4096
#define KDEFFT_MAX_N (((int64_t)1) << 23)
#define KDEFFT_QBITS 40            /* binning quantum 2^-40 of a unit point mass */

/* Grid descriptor (Sec. 4, Eq. (15)-(16)): node j of axis k is lo[k] + j*delta[k],
 * j = 0..M[k]-1.  P[k] is the length of the zero-padded circular transform. */
typedef struct kdefft_grid {
    int32_t d;
    int32_t M[4];
    int32_t P[4];
    double lo[4];
    double delta[4];
} kdefft_grid;

/* A binned, transformed dataset, filled by kdefft_dataset_prepare().  The
 * device arrays live inside one caller buffer (see kdefft_dataset_bytes):
 *   counts  int64 [prod M]                  grid counts, 2^-40 quanta
 *   spec    complex [prod_{k<d-1} P_k][Q]   C = R2C(counts), Q = P_{d-1}/2+1,
 *                                           interleaved (re, im) float64
 *   wmix    complex [prod_{k<d-1} P_k][Q]   |C|^2 transformed forward along
 *                                           axes 0..d-2 (mixed-domain spectrum)
 *   alag    float64 [P_0, ..., P_{d-1}]     prod P times the autocorrelation of the
 *                                           counts, A_l = sum_i c_i c_{i+l}, lag l at
 *                                           index l mod P (inverse transform of |C|^2);
 *                                           exact zeros where the last-axis lag has
 *                                           |l_{d-1}| > M_{d-1} - 1 (zero exactly)
 *   scal    float64 [4]                     scal[0] = n^-2 sum sum phi_{2G} (binned), the
 *                                           constant SCV term, written by every batched
 *                                           SCV objective call on the dataset (0 after
 *                                           preparation)
 *   n_out   int32 [1]                       number of points outside the grid
 *   rec     opaque device record (pointers, n, spacing, pilot) read by the
 *           batched kernels, so batch calls need no host-to-device copies */
typedef struct kdefft_dataset {
    kdefft_grid grid;
    int64_t n;
    double G[16];            /* pilot bandwidth, row-major d x d (host copy) */
    int64_t* counts;
    double* spec;
    double* wmix;
    double* alag;
    double* scal;
    int32_t* n_out;
    void* rec;
} kdefft_dataset;

/* Datasets per batched call: kdefft_scv_batch / kdefft_scv_adjoint accept up
 * to KDEFFT_MAX_BATCH_DS datasets per call, kdefft_psi_batch up to
 * KDEFFT_MAX_PSI_DS (their record pointers travel as kernel arguments). */
#define KDEFFT_MAX_BATCH_DS 64
#define KDEFFT_MAX_PSI_DS 32

/* Operation selectors for kdefft_ws_bytes(). */
#define KDEFFT_OP_GRID_AUTO 1   /* kdefft_grid_auto: batch = n (points) */
#define KDEFFT_OP_PSI_PLAIN 2   /* kdefft_psi(mode = PLAIN) */
#define KDEFFT_OP_PSI_FUSED 3   /* kdefft_psi(mode = FUSED) */
#define KDEFFT_OP_PREPARE 4     /* kdefft_dataset_prepare */
#define KDEFFT_OP_PSI_BATCH 5   /* kdefft_psi_batch: batch = number of datasets */
#define KDEFFT_OP_SCV_BATCH 6   /* kdefft_scv_batch / kdefft_scv_adjoint: batch = total H */
#define KDEFFT_OP_SCV_PLAIN 7   /* kdefft_scv_plain */
#define KDEFFT_OP_AUTOTUNE 8    /* kdefft_autotune */
#define KDEFFT_OP_PSI_FFTL 9    /* kdefft_psi_fftl (sized for the largest Eq. (27) padding) */
#define KDEFFT_OP_PREPARE_AUTO 10 /* kdefft_dataset_prepare_auto: batch = n (points) */

/* psi modes */
#define KDEFFT_PSI_PLAIN 0  /* the paper's steps literally: per entry, kernel grid ->
                               R2C -> multiply by C -> C2R -> scale 1/prod P ->
                               contract with the counts (Eq. (22)-(24)) */
#define KDEFFT_PSI_FUSED 1  /* Parseval form: one fused launch for all entries */

/* Human-readable name of an error code (static string). */
const char* kdefft_strerror(int code);

/* Detail of the last error raised on the calling thread ("" if none). */
const char* kdefft_last_error_detail(void);

/* Library version, major*10000 + minor*100 + patch. */
int kdefft_version(void);

/* Number of unique entries C(d+r-1, r) of D^{(x)r} (Sec. 5), or a negative code. */
int kdefft_unique_count(int d, int r);

/* The unique index tuples in canonical order, 0-based: tuples_host[k*r + m] is
 * the m-th index of entry k; tuples_host must hold kdefft_unique_count(d,r)*r
 * int32 (nothing is written for r = 0). Host only. */
int kdefft_unique_index(int d, int r, int32_t* tuples_host);

/* Grid from explicit bounds (Sec. 4, Eq. (16)): delta_k = (hi_k - lo_k)/(M_k - 1),
 * one float64 subtraction and one division.  P_host may be NULL (then P_k is the
 * smallest power of two >= max(4, 2 M_k - 1); P_k = 2 M_k when M_k is a power
 * of two) or give the padded lengths.  Host only. */
int kdefft_grid_plan(int d, const int32_t* M_host, const int32_t* P_host,
                     const double* lo_host, const double* hi_host, kdefft_grid* out);

/* Grid spanning the data padded by pad_sd kernel standard deviations:
 * lo_k = min_i X_ik - pad_sd*sqrt(G_kk), hi_k = max_i X_ik + pad_sd*sqrt(G_kk)
 * (the paper leaves the span open; Sec. 4 only asks that it contain the data).
 * Reads the bounds back, so it synchronizes `stream`.  Workspace:
 * KDEFFT_OP_GRID_AUTO with batch = n. */
int kdefft_grid_auto(const double* X, int64_t n, int d, const double* G_host,
                     const int32_t* M_host, double pad_sd, kdefft_grid* out,
                     void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for operation `op` on grid g with derivative order r and
 * batch size `batch` (meaning per op above); written to *out. Host only. */
int kdefft_ws_bytes(const kdefft_grid* g, int op, int r, int64_t batch, size_t* out);

/* Step 1 of Sec. 4: linear binning of X [n,d] onto g into int64 counts
 * [prod M] (zeroed first), fixed-point quanta of 2^-40 per unit mass; the
 * corner with the largest quantum absorbs the rounding so each point adds
 * exactly 2^40.  Points with (X_ik - lo_k)/delta_k outside [0, M_k - 1] are
 * skipped and counted into *n_out_dev (device int32, may be NULL). */
int kdefft_linbin(const double* X, int64_t n, const kdefft_grid* g,
                  int64_t* counts, int32_t* n_out_dev, void* stream);

/* psi_r(G) (Eq. (13)) of X on grid g by the binned FFT route (Eq. (14)-(24)).
 * psi: device float64 [kdefft_unique_count(d, r)].  mode: KDEFFT_PSI_PLAIN or
 * KDEFFT_PSI_FUSED.  Workspace: KDEFFT_OP_PSI_PLAIN / KDEFFT_OP_PSI_FUSED.
 * Out-of-grid points are dropped (see kdefft_check_binning on the workspace). */
int kdefft_psi(const double* X, int64_t n, const kdefft_grid* g, const double* G_host,
               int r, double* psi, int mode, void* ws, size_t ws_bytes, void* stream);

/* fft-L sizes (Sec. 4, Eq. (26)-(27)) for bandwidth matrix S_host (d x d
 * row-major, SPD) on grid g: L_k = min(M_k - 1, ceil(tau sqrt(lambda)/delta_k))
 * with lambda the largest eigenvalue of S (Jacobi rotations on the host), and
 * P_k the smallest power of two >= M_k + 2 L_k - 1.  The paper suggests
 * tau = 3.7 for the two-dimensional normal kernel.  L_host, P_host: int32 [d].
 * Host only. */
int kdefft_fftl_plan(const kdefft_grid* g, const double* S_host, double tau, int32_t* L_host,
                     int32_t* P_host);

/* psi_r(G) by the paper's fft-L variant (Eq. (25)-(27)): the kernel support is
 * cut to |l_k| <= L_k (L from G by kdefft_fftl_plan) and the transforms use the
 * Eq. (27) lengths P_k instead of g's; otherwise the literal four steps of
 * kdefft_psi(PLAIN).  An approximation of Eq. (17): lags beyond L_k are
 * dropped.  L_host, P_host (int32 [d], may be NULL) receive the sizes used.
 * Workspace: KDEFFT_OP_PSI_FFTL.  KDEFFT_E_UNSUPPORTED if some P_k > 4096. */
int kdefft_psi_fftl(const double* X, int64_t n, const kdefft_grid* g, const double* G_host, int r,
                    double tau, double* psi, int32_t* L_host, int32_t* P_host, void* ws,
                    size_t ws_bytes, void* stream);

/* Synchronize `stream` and return KDEFFT_E_OUT_OF_GRID if the int32 counter
 * n_out_dev is non-zero (its value is stored in *n_out_host if not NULL). */
int kdefft_check_binning(const int32_t* n_out_dev, int32_t* n_out_host, void* stream);

/* Device bytes of the buffer that holds one prepared dataset on grid g. */
int kdefft_dataset_bytes(const kdefft_grid* g, size_t* out);

/* Bin X onto g and transform the counts once (C = R2C(counts), then |C|^2 and
 * its transform along the leading axes, and the lag array); the pilot
 * Gpilot_host is kept for the SCV calls (which also evaluate the constant
 * phi_{2G} term).  ds_mem: device buffer of kdefft_dataset_bytes(g)
 * bytes, 256-byte aligned; *out receives the descriptor.  Workspace:
 * KDEFFT_OP_PREPARE. */
int kdefft_dataset_prepare(const double* X, int64_t n, const kdefft_grid* g,
                           const double* Gpilot_host, void* ds_mem, size_t ds_bytes,
                           kdefft_dataset* out, void* ws, size_t ws_bytes, void* stream);

/* kdefft_grid_auto and kdefft_dataset_prepare in one call, with no host
 * round trip: the data bounds, the grid origin and spacing (the same IEEE
 * steps as kdefft_grid_auto / kdefft_grid_plan, bit for bit) and the binning
 * all stay on the device.  The grid in *out carries d, M and P; its lo and
 * delta are NaN on the host until kdefft_dataset_grid reads them back (every
 * batched call works without them; kdefft_scv_plain reads them back itself).
 * Non-finite data leave non-finite spacing: every point is then counted as out
 * of the grid (kdefft_check_binning) and kdefft_dataset_grid reports
 * KDEFFT_E_ARG.  ds_mem: kdefft_dataset_bytes of the grid's shape (any lo,
 * delta).  Workspace: KDEFFT_OP_PREPARE_AUTO with batch = n. */
int kdefft_dataset_prepare_auto(const double* X, int64_t n, int d, const int32_t* M_host, double pad_sd,
                                const double* Gpilot_host, void* ds_mem, size_t ds_bytes,
                                kdefft_dataset* out, void* ws, size_t ws_bytes, void* stream);

/* The grid of a prepared dataset with its device-side origin and spacing
 * read back into *out (synchronizes `stream`). */
int kdefft_dataset_grid(const kdefft_dataset* ds_host, kdefft_grid* out, void* stream);

/* The count transform of a prepared dataset alone (Sec. 4, Eq. (19)-(22):
 * C = R2C of the counts, |C|^2, and its inverse transform): recomputes spec,
 * wmix and alag from the dataset's counts with the current FFT schedule of its
 * grid shape (kdefft_set_fft_schedule).  Needs no workspace; returns without
 * waiting. */
int kdefft_dataset_transform(const kdefft_dataset* ds_host, void* stream);

/* psi_r at bandwidth G_host + 16*j (row-major d x d) for each of n_ds prepared
 * datasets, one launch: the binned double sum of Eq. (13) as sum_l k(l) A(l)
 * over the prepared lag array (or, for the spectral launch variants, the
 * Parseval form against the prepared spectra; Sec. 5).
 * psi: device float64 [n_ds, kdefft_unique_count(d, r)].  All datasets must
 * share d and the grid lengths P. Workspace: KDEFFT_OP_PSI_BATCH, batch = n_ds. */
int kdefft_psi_batch(const kdefft_dataset* ds_host, int n_ds, const double* G_host,
                     int r, double* psi, void* ws, size_t ws_bytes, void* stream);

/* SCV objective for B = h_offsets_host[n_ds] candidate bandwidths, candidate b
 * belonging to dataset j when h_offsets_host[j] <= b < h_offsets_host[j+1]:
 *   SCV(H) = n^-1 (4 pi)^{-d/2} |H|^{-1/2}
 *          + n^-2 sum sum [phi_{2H+2G} - 2 phi_{H+2G} + phi_{2G}](X_i - X_j)
 * with the double sum binned and evaluated against the dataset's prepared
 * transforms (lag array or spectra, by launch variant; the SCV selector
 * of Sec. 3 and Sec. 5, V-statistic form).  vechL [B, q] parametrises H = L L^T.
 * obj: device [B].  grad: device [B, q] or NULL; if given it receives
 * d SCV / d vechL.  status: device int32 [B] or NULL; 0 = ok, 1 = H singular
 * (a zero diagonal entry of L; obj and grad are NaN for that entry).  One
 * persistent launch covers all datasets and candidates.  All datasets must
 * share d and P.  Workspace: KDEFFT_OP_SCV_BATCH with batch = B. */
int kdefft_scv_batch(const kdefft_dataset* ds_host, int n_ds, const int64_t* h_offsets_host,
                     const double* vechL, double* obj, double* grad, int32_t* status,
                     void* ws, size_t ws_bytes, void* stream);

/* Adjoint of kdefft_scv_batch's objective: grad_vechL[b, :] = grad_out[b] *
 * d SCV(H_b) / d vechL_b, recomputing the Hessian kernel grids (never stored).
 * grad_out: device [B]; grad_vechL: device [B, q].  Same workspace as
 * kdefft_scv_batch. */
int kdefft_scv_adjoint(const kdefft_dataset* ds_host, int n_ds, const int64_t* h_offsets_host,
                       const double* vechL, const double* grad_out, double* grad_vechL,
                       void* ws, size_t ws_bytes, void* stream);

/* Criteria built on the same batched lag-domain evaluation (crit):
 *   KDEFFT_CRIT_SCV         the SCV objective above (r must be 0);
 *   KDEFFT_CRIT_LSCV        LSCV_r of Eq. (36) (n - 1 replaced by n):
 *       (-1)^r { n^-2 sum sum [eta_r(.; 2H) - 2 eta_r(.; H)] + 2 n^-1 eta_r(0; H) },
 *       for r = 0 the paper's LSCV of Eq. (10)-(11);
 *   KDEFFT_CRIT_LSCV_EXACT  LSCV_r of Eq. (35), the leave-one-out weights:
 *       (-1)^r { n^-2 sum sum [eta_r(.; 2H) - 2n/(n-1) eta_r(.; H)] + 2 (n-1)^-1 eta_r(0; H) };
 *   KDEFFT_CRIT_QR          the V-statistic Q_r(S) of Eq. (32) with S = L L^T
 *       the candidate matrix itself: n^-2 sum sum eta_r(X_i - X_j; S).
 * eta_r(x; S) = (vec^T I)^{(x)r} D^{(x)2r} phi_S(x) (Eq. (31)); the paper prints
 * K_H(0) for the diagonal correction at every r, read here as eta_r(0; H), its
 * r = 0 value.  Binned sums as in the SCV path (the binned self-pairs make the
 * diagonal correction approximate, as in the paper). */
#define KDEFFT_CRIT_SCV 0
#define KDEFFT_CRIT_LSCV 1
#define KDEFFT_CRIT_LSCV_EXACT 2
#define KDEFFT_CRIT_QR 3

/* Batched criterion for B = h_offsets_host[n_ds] candidates (dataset grouping
 * and vechL as in kdefft_scv_batch), r in [0, 8] (0 for SCV).  obj: device
 * [B].  grad: device [B, q] = d crit / d vechL, or NULL; a gradient exists for
 * r = 0 and the SCV / LSCV criteria only (else KDEFFT_E_UNSUPPORTED).  status
 * as in kdefft_scv_batch.  Workspace: KDEFFT_OP_SCV_BATCH with batch = B. */
int kdefft_crit_batch(const kdefft_dataset* ds_host, int n_ds, const int64_t* h_offsets_host,
                      const double* vechL, int crit, int r, double* obj, double* grad,
                      int32_t* status, void* ws, size_t ws_bytes, void* stream);

/* Work of the compacted lag walk (row-kernel variants 5 and 6) for the SCV
 * objective + gradient of these candidates (Sec. 4, Eq. (17)-(18) in the lag
 * domain): the number of runs of kdefft_lag_layout(P_{d-1}, 1) positions that
 * hold a lag whose Gaussians reach 1e-30 of their peak -- the runs the walk
 * visits -- summed over all candidates and each dataset's constant term.
 * *runs_host receives the sum.  Arguments and workspace as in
 * kdefft_scv_batch.  Synchronizes `stream` (a measurement helper). */
int kdefft_scv_walk_runs(const kdefft_dataset* ds_host, int n_ds, const int64_t* h_offsets_host,
                         const double* vechL, int64_t* runs_host, void* ws, size_t ws_bytes, void* stream);

/* Adjoint of kdefft_crit_batch for r = 0 and crit SCV / LSCV / LSCV_EXACT:
 * grad_vechL[b, :] = grad_out[b] * d crit(H_b) / d vechL_b.  Same workspace. */
int kdefft_crit_adjoint(const kdefft_dataset* ds_host, int n_ds, const int64_t* h_offsets_host,
                        const double* vechL, int crit, const double* grad_out, double* grad_vechL,
                        void* ws, size_t ws_bytes, void* stream);

/* Plug-in criterion (Sec. 5 names the PI selector; normal-kernel AMISE with
 * the estimated fourth-derivative functional):
 *   PI(H) = n^-1 (4 pi)^{-d/2} |H|^{-1/2} + 1/4 (vec H (x) vec H)^T psi_4,
 * psi_4 the d^4 Kronecker-ordered vector filled from the unique entries.
 * psi4: device [n_ds, kdefft_unique_count(d, 4)] (e.g. from kdefft_psi_batch at
 * the pilot bandwidths); n_host[j] the sample size of dataset j; candidates
 * grouped by h_offsets_host as in kdefft_scv_batch.  obj: device [B]; grad:
 * device [B, q] = d PI / d vechL or NULL; status: device int32 [B] or NULL
 * (1 = singular H, NaN results).  No workspace; one launch. */
int kdefft_pi_batch(int d, int n_ds, const int64_t* n_host, const double* psi4,
                    const int64_t* h_offsets_host, const double* vechL, double* obj, double* grad,
                    int32_t* status, void* stream);

/* Gradient-based minimisation of a selector criterion over vech(L), H = L L^T
 * (Sec. 5 names the PI and SCV selectors; Sec. 6 minimises them numerically
 * without derivatives).  Each of the B = h_offsets_host[n_ds] starting points
 * vechL0 [B, q] is its own problem: quasi-Newton steps (BFGS update of an
 * inverse-Hessian approximation, started from the identity scaled by the
 * first step's curvature) with a backtracking Armijo line search (sufficient
 * decrease 1e-4; rejected steps shortened to the minimiser of the quadratic
 * through the two values and the slope, within [0.1, 0.5] of the step; a new
 * direction's first step moves no entry by more than 1/4 of max |vechL|).
 * Every evaluation is one batched criterion + gradient launch at all B trial
 * points followed by one small update launch; `evals` evaluations are enqueued
 * on `stream` without host synchronisation (the sequence can be captured in a
 * graph).  A candidate stops when max|grad| * max|vechL| <= tol * |crit|
 * (converged); as stalled (no decrease left in float64) after 60 shortenings
 * of one step or two accepted steps in a row that lower crit by no more than
 * 4 roundings; or when the evaluations run out.  The inverse-Hessian update is
 * skipped when s.y <= 1e-10 |s| |y| (s the step, y the gradient change).
 *   crit KDEFFT_CRIT_SCV, KDEFFT_CRIT_LSCV, KDEFFT_CRIT_LSCV_EXACT: ds_host,
 *       n_ds and h_offsets_host as in kdefft_crit_batch (r = 0); n_host, psi4
 *       and d unused;
 *   crit KDEFFT_CRIT_PI: the plug-in criterion of kdefft_pi_batch; d, n_host
 *       and psi4 as there, ds_host unused (NULL), n_ds and h_offsets_host group
 *       the candidates.
 * vechL_out: device [B, q], the final points; obj_out: device [B] or NULL,
 * their criterion values; info: device int32 [B, 2] or NULL: outcome
 * (KDEFFT_MIN_*) and the number of accepted steps.  evals in [1, 100000],
 * tol > 0.  Workspace: kdefft_minimize_ws_bytes. */
#define KDEFFT_CRIT_PI 4
#define KDEFFT_MIN_CONVERGED 0
#define KDEFFT_MIN_RUNNING 1    /* evaluations ran out first */
#define KDEFFT_MIN_STALLED 2
#define KDEFFT_MIN_BAD_START 3  /* the criterion is not finite at the start (singular H) */
int kdefft_minimize(const kdefft_dataset* ds_host, int n_ds, const int64_t* h_offsets_host, int crit,
                    int d, const int64_t* n_host, const double* psi4, const double* vechL0, int evals,
                    double tol, double* vechL_out, double* obj_out, int32_t* info, void* ws,
                    size_t ws_bytes, void* stream);

/* Workspace bytes of kdefft_minimize for B candidates: g is the datasets'
 * grid (SCV / LSCV), or NULL for KDEFFT_CRIT_PI with dimension d. */
int kdefft_minimize_ws_bytes(const kdefft_grid* g, int d, int64_t B, size_t* out);

/* Fill the d^r Kronecker-ordered vector (first index slowest) from the unique
 * entries (sorted index tuples in lexicographic order; Sec. 5): full_host
 * [d^r] from unique_host [kdefft_unique_count(d, r)].  Host only. */
int kdefft_expand_full(int d, int r, const double* unique_host, double* full_host);

/* One candidate H at a time by the paper's literal steps: for the objective
 * grid and each of the q Hessian grids, kernel grid -> R2C -> multiply by the
 * prepared count spectrum -> C2R -> scale -> contract with the counts, each a
 * separate launch.  out: device [1 + q] = (SCV(H), d SCV / d vechL).
 * H_host: d x d row-major.  Workspace: KDEFFT_OP_SCV_PLAIN. */
int kdefft_scv_plain(const kdefft_dataset* ds_host, const double* H_host, double* out,
                     void* ws, size_t ws_bytes, void* stream);

/* Pin the launch of the batched row kernels for one kernel family (kind: 0 psi,
 * 1 SCV objective, 2 SCV objective+gradient, 3 SCV gradient, 4 Q_r, 5 LSCV_r
 * for r > 0), dimension d, order r (2 for the SCV families) and last-axis
 * length N for the rest of the process, for the psi / SCV / Q_r calls (LSCV
 * keeps its own choice): variant in [0, 7): 0, 1, 2 run the per-candidate
 * last-axis FFTs in LDS (0: one radix-8 butterfly per lane per stage, radix-8
 * first; 1: twice the rows per wavefront; 2: radix-4 first); grid_blocks =
 * persistent grid size, 0 = resident blocks per CU x CUs, -1 = one block per
 * work item.  Variants 3 and 4 evaluate each candidate in the lag domain
 * instead: sum_l k(l) A(l) against the prepared count autocorrelation
 * (identical sums, no per-candidate transform); for the SCV families, runs of
 * lags that start below 1e-290 and rise are evaluated lag by lag (3) or
 * walked with values scaled by e^600 (4); the psi and eta families treat 3 and
 * 4 alike and have no spectral variants for eta.  Variants 5 and 6 are 3 and 4
 * with the work compacted: each row's lags whose Gaussians all stay below
 * 1e-30 of their peak are bounded analytically and skipped, and only the
 * remaining runs are dealt to the threads (the dropped terms are far below
 * float64 rounding of the result; the psi and eta families treat 5 and 6 as
 * 3); variant 5 with one block per work item (the untuned default of the SCV
 * families) deals each candidate's rows round-robin over its items and also
 * builds the candidates' parameter blocks inside the launch.
 * The untuned default of the other families is variant 3, grid 0.
 * variant = -1 drops the pinned (or tuned) choice of that key, so the untuned
 * default applies again.  Used by kdefft_autotune and by tests that cover
 * every variant.  Host only. */
int kdefft_set_row_launch(int kind, int d, int r, int N, int variant, int grid_blocks);

/* The launch the batched calls of that key (kind, d, r, N as in
 * kdefft_set_row_launch) use now on the current device: pinned, tuned or the
 * untuned default.  Lets a caller restore a choice after pinning another.
 * Host only. */
int kdefft_get_row_launch(int kind, int d, int r, int N, int* variant, int* grid_blocks);

/* Layout of the compiled lag-domain kernels (variants 3 and 4) for a last-axis
 * length N (a power of two in [4, 2048]): *run_len = lags per run (one
 * exponential recurrence start per run, or per segment for the moment
 * families), *runs_per_seg = consecutive runs one thread walks carrying the
 * recurrence (moment families; 1 otherwise), *rows_per_pass = rows one
 * 256-thread block covers per pass.  moments = 1 for the SCV / LSCV families
 * (moment form), 0 for the psi_r and eta_r families with at most 12 outputs
 * per lag.  Lets a caller's work model use the constants the kernels were
 * compiled with.  Host only; KDEFFT_E_ARG for other N or NULL outputs. */
int kdefft_lag_layout(int N, int moments, int* run_len, int* runs_per_seg, int* rows_per_pass);

/* Measurement hook for the batched row kernels (the dominant launches of
 * kdefft_psi, kdefft_psi_batch, kdefft_scv_batch, kdefft_scv_adjoint and
 * kdefft_autotune).  kdefft_timing_start arms it for up to max_launches
 * launches, max_launches in [1, KDEFFT_MAX_TIMED]: each of the next row-kernel
 * launches, on any stream, is bracketed by a pair of HIP events recorded on
 * that launch's stream (events are created once and reused; no device memory
 * is allocated).  kdefft_timing_stop disarms, waits for the recorded events
 * and writes, for the first min(recorded, cap) launches in launch order, the
 * kernel's duration in milliseconds to ms_out[k] and a tag 16 * family + r to
 * tag_out[k] (family: 0 psi_r, 1 SCV objective, 2 objective + gradient,
 * 3 adjoint gradient); *count_out receives that number.  Stopping when not
 * armed reports 0 launches.  One timer per process; calls from several threads
 * are serialized. */
#define KDEFFT_MAX_TIMED 4096
int kdefft_timing_start(int max_launches);
int kdefft_timing_stop(float* ms_out, int32_t* tag_out, int cap, int* count_out);

/* FFT-stage schedule of the count transform (Sec. 4, Eq. (19)-(23): the
 * R2C, leading-axis and C2R passes of dataset preparation) for grids of shape
 * (d, P_host[0..d-1]) on the current device, for the rest of the process:
 *   0 (default) 256-thread blocks of ~2048 values, or, when that shape would
 *     give fewer than 512 blocks, 256-thread blocks of a few pencils (half of
 *     what one wavefront takes, at least one: more blocks, more lanes per
 *     pencil for the loads); radix-8 Stockham stages first (radix 4 or 2 for
 *     the remainder), radix-4 stages for 64-point passes;
 *   1 the same shapes with radix-4 stages (one radix-8 or 2 when log2 P is odd);
 *   2 256-thread blocks of ~2048 values for every pass (strided passes on
 *     16-column tiles, or whole [P][Q] slabs for Q = 17, 33);
 *   3 one-wavefront blocks for every pass that has them;
 *   4 strided passes on half-width tiles (twice the blocks);
 *   5 the small problems' 256-thread shape of schedule 0 for every pass.
 * All schedules compute the same transform (they differ in rounding order
 * only).  sched = -1 drops the pinned or tuned choice.  Host only. */
#define KDEFFT_FFT_SCHEDULES 6
int kdefft_set_fft_schedule(int d, const int32_t* P_host, int sched);
int kdefft_get_fft_schedule(int d, const int32_t* P_host, int* sched);

/* Time the compiled launch choices for this dataset's grid shape on the
 * current device, keep the fastest of each for the rest of the process, and
 * append the choices to cache_path (one JSON object per line; NULL = no file;
 * the file named by the environment variable KDEFFT_TUNE_CACHE is read back at
 * the first batched call of a process):
 *   the count transform's FFT schedule (kdefft_set_fft_schedule), re-running
 *     the dataset's transform, which is left computed by the chosen schedule;
 *   the SCV families and the same kernels serving LSCV (row-kernel variant and
 *     persistent grid size, as kdefft_set_row_launch), timed on 256 candidates
 *     H = s G (s spread over [0.5, 8], G the dataset's matrix);
 *   LSCV_4 (the scalar eta family: grid size) on the same candidates;
 *   psi_4 at the dataset's pilot (variants 0-3, grid size).
 * Each default (FFT schedule 0; variant 5 with one block per work item for
 * SCV / LSCV; variant 3 grid 0 otherwise) is kept unless another choice is
 * more than 3% faster.
 * kdefft_last_error_detail() returns the timings afterwards.  Workspace:
 * KDEFFT_OP_AUTOTUNE.  Synchronizes `stream`. */
int kdefft_autotune(const kdefft_dataset* ds_host, void* ws, size_t ws_bytes,
                    const char* cache_path, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the batched
 * SCV objective (+ gradient) of kdefft_scv_batch with the same arguments,
 * kernels and results, but no workspace argument.  Its workspace is a fixed
 * device array of KDEFFT_NOALLOC_BYTES bytes inside the library; each GPU the
 * library runs on holds one for the rest of the process.  The call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine); a batch whose
 * workspace (kdefft_ws_bytes, KDEFFT_OP_SCV_BATCH) exceeds the array is
 * rejected with KDEFFT_E_WORKSPACE before anything is launched.  Every call on
 * one GPU shares that GPU's array, which keeps the last call's contents
 * (nothing in it needs to start at zero): calls that overlap on one GPU --
 * on different streams, or from several threads -- race and must be
 * serialized by the caller. */
#define KDEFFT_NOALLOC_BYTES (16u << 20)
int kdefft_scv_batch_noalloc(const kdefft_dataset* ds_host, int n_ds, const int64_t* h_offsets_host,
                             const double* vechL, double* obj, double* grad, int32_t* status, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* KDEFFT_H */
