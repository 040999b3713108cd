// Host-side exercise of the C-ABI under AddressSanitizer and
// UndefinedBehaviorSanitizer: every path here returns before anything is
// launched (planning, sizing, tables, argument validation), so it runs without
// a GPU.  Exits 0 after printing "ok"; any sanitizer report aborts it.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "kdefft.h"

static int fails = 0;
#define EXPECT(cond)                                                   \
    do {                                                               \
        if (!(cond)) {                                                 \
            std::fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, #cond); \
            ++fails;                                                   \
        }                                                              \
    } while (0)

static kdefft_grid plan(int d, int M, double span) {
    int32_t Mv[4] = {M, M, M, M};
    double lo[4] = {-1, -2, -3, -4}, hi[4];
    for (int k = 0; k < 4; ++k) hi[k] = lo[k] + span;
    kdefft_grid g;
    std::memset(&g, 0, sizeof(g));
    EXPECT(kdefft_grid_plan(d, Mv, nullptr, lo, hi, &g) == KDEFFT_OK);
    return g;
}

int main() {
    EXPECT(kdefft_version() >= 10000);
    for (int c = 0; c >= -9; --c) EXPECT(kdefft_strerror(c) != nullptr);
    EXPECT(kdefft_last_error_detail() != nullptr);

    // multi-index tables and the Kronecker expansion, every (d, r)
    for (int d = 1; d <= 4; ++d)
        for (int r = 0; r <= 8; ++r) {
            const int nu = kdefft_unique_count(d, r);
            EXPECT(nu >= 1);
            std::vector<int32_t> t((size_t)nu * (r > 0 ? r : 1));
            EXPECT(kdefft_unique_index(d, r, t.data()) == KDEFFT_OK);
            std::vector<double> u(nu, 1.0);
            size_t full = 1;
            for (int k = 0; k < r; ++k) full *= d;
            std::vector<double> f(full);
            EXPECT(kdefft_expand_full(d, r, u.data(), f.data()) == KDEFFT_OK);
            for (double v : f) EXPECT(v == 1.0);
        }
    EXPECT(kdefft_unique_count(5, 2) < 0);
    EXPECT(kdefft_expand_full(2, 9, nullptr, nullptr) == KDEFFT_E_ARG);

    // planning and sizing for every operation on grids of every dimension
    for (int d = 1; d <= 4; ++d)
        for (int M : {2, 3, 17, 32}) {
            const kdefft_grid g = plan(d, M, 3.5);
            size_t b = 0;
            for (int op = 1; op <= 10; ++op) {
                const int r = (op == 2 || op == 3 || op == 5 || op == 9) ? 4 : 0;
                const int rc = kdefft_ws_bytes(&g, op, r, 7, &b);
                EXPECT(rc == KDEFFT_OK || rc == KDEFFT_E_UNSUPPORTED);
            }
            EXPECT(kdefft_ws_bytes(&g, 99, 0, 1, &b) == KDEFFT_E_ARG);
            EXPECT(kdefft_dataset_bytes(&g, &b) == KDEFFT_OK && b > 0);
            EXPECT(kdefft_minimize_ws_bytes(&g, 0, 9, &b) == KDEFFT_OK && b > 0);
            double S[16] = {0};
            for (int k = 0; k < d; ++k) S[k * d + k] = 0.2;
            int32_t L[4];
            int32_t P[4];
            const int rc = kdefft_fftl_plan(&g, S, 1e-6, L, P);
            EXPECT(rc == KDEFFT_OK || rc == KDEFFT_E_UNSUPPORTED);
        }
    {
        int32_t M[2] = {1, 8};
        double lo[2] = {0, 0}, hi[2] = {1, 1};
        kdefft_grid g;
        EXPECT(kdefft_grid_plan(2, M, nullptr, lo, hi, &g) == KDEFFT_E_ARG);
        EXPECT(kdefft_grid_plan(5, M, nullptr, lo, hi, &g) == KDEFFT_E_ARG);
        hi[0] = NAN;
        M[0] = 8;
        EXPECT(kdefft_grid_plan(2, M, nullptr, lo, hi, &g) == KDEFFT_E_ARG);
    }

    // launch tables
    for (int kind = 0; kind <= 5; ++kind) {
        int v = -9, gb = -9;
        EXPECT(kdefft_get_row_launch(kind, 2, kind == 0 ? 4 : 2, 256, &v, &gb) == KDEFFT_OK);
        EXPECT(v >= 0 && v < 7);
    }
    EXPECT(kdefft_set_row_launch(2, 2, 2, 256, 5, -1) == KDEFFT_OK);
    EXPECT(kdefft_set_row_launch(2, 2, 2, 256, -1, 0) == KDEFFT_OK);
    EXPECT(kdefft_set_row_launch(2, 2, 2, 256, 7, 0) == KDEFFT_E_ARG);
    EXPECT(kdefft_set_row_launch(9, 2, 2, 256, 0, 0) == KDEFFT_E_ARG);
    {
        int32_t P[3] = {64, 64, 32};
        int s = -1;
        for (int k = 0; k < KDEFFT_FFT_SCHEDULES; ++k) {
            EXPECT(kdefft_set_fft_schedule(3, P, k) == KDEFFT_OK);
            EXPECT(kdefft_get_fft_schedule(3, P, &s) == KDEFFT_OK && s == k);
        }
        EXPECT(kdefft_set_fft_schedule(3, P, -1) == KDEFFT_OK);
        P[1] = 48;
        EXPECT(kdefft_set_fft_schedule(3, P, 0) == KDEFFT_E_ARG);
    }
    int nl = 0, rl = 0, sg = 0, rp = 0;
    EXPECT(kdefft_lag_layout(512, 1, &rl, &sg, &rp) == KDEFFT_OK && rl > 0);
    (void)nl;

    // argument validation of compute entries (fake device pointers are never touched)
    {
        const kdefft_grid g = plan(2, 16, 2.0);
        kdefft_dataset ds;
        std::memset(&ds, 0, sizeof(ds));
        ds.grid = g;
        ds.n = 100;
        ds.G[0] = ds.G[3] = 0.1;
        void* fake = reinterpret_cast<void*>(0x100000);
        ds.counts = static_cast<int64_t*>(fake);
        ds.spec = ds.wmix = ds.alag = ds.scal = static_cast<double*>(fake);
        ds.n_out = static_cast<int32_t*>(fake);
        ds.rec = fake;
        const int64_t off[2] = {0, 4};
        const int64_t bad[2] = {1, 4};
        double* fd = static_cast<double*>(fake);
        EXPECT(kdefft_scv_batch(&ds, 1, off, fd, nullptr, nullptr, nullptr, fake, 1 << 30, nullptr) ==
               KDEFFT_E_ARG);
        EXPECT(kdefft_scv_batch(&ds, 1, bad, fd, fd, nullptr, nullptr, fake, 1 << 30, nullptr) == KDEFFT_E_ARG);
        EXPECT(kdefft_scv_batch(&ds, 1, off, fd, fd, nullptr, nullptr, fake, 64, nullptr) == KDEFFT_E_WORKSPACE);
        EXPECT(kdefft_crit_batch(&ds, 1, off, fd, 7, 0, fd, nullptr, nullptr, fake, 1 << 30, nullptr) ==
               KDEFFT_E_ARG);
        EXPECT(kdefft_crit_batch(&ds, 1, off, fd, KDEFFT_CRIT_QR, 0, fd, fd, nullptr, fake, 1 << 30, nullptr) ==
               KDEFFT_E_UNSUPPORTED);
        double G16[16] = {0.1, 0, 0, 0.1};
        EXPECT(kdefft_psi_batch(&ds, 1, G16, 3, fd, fake, 1 << 30, nullptr) == KDEFFT_E_ODD_R);
        const int64_t nn[1] = {100};
        EXPECT(kdefft_pi_batch(5, 1, nn, fd, off, fd, fd, nullptr, nullptr, nullptr) == KDEFFT_E_ARG);
        EXPECT(kdefft_minimize(&ds, 1, off, KDEFFT_CRIT_SCV, 2, nn, fd, fd, 0, 1e-9, fd, nullptr, nullptr, fake,
                               1 << 30, nullptr) == KDEFFT_E_ARG);
        EXPECT(kdefft_minimize(&ds, 1, off, KDEFFT_CRIT_SCV, 2, nn, fd, fd, 10, 1e-9, fd, nullptr, nullptr, fake,
                               64, nullptr) == KDEFFT_E_WORKSPACE);
        EXPECT(kdefft_minimize(nullptr, 1, off, KDEFFT_CRIT_PI, 2, nn, nullptr, fd, 10, 1e-9, fd, nullptr,
                               nullptr, fake, 1 << 30, nullptr) == KDEFFT_E_ARG);
        EXPECT(kdefft_scv_batch_noalloc(&ds, 1, bad, fd, fd, nullptr, nullptr, nullptr) == KDEFFT_E_ARG);
        EXPECT(kdefft_timing_start(0) == KDEFFT_E_ARG);
    }
    if (fails) {
        std::fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
