// Scalar eta_r families (Q_r, LSCV_r) for d = 4: lag-domain kernel only (variants 3 and 4
// coincide for them; see rows_impl.h).
#include "eta_fun.h"
#include "rows_dispatch.h"

namespace kdefft {

template <class Fun>
static hipError_t lag_4(int N, const double* prm, RowGeom geo, int64_t nitems, double* partial, int gb, hipStream_t s) {
    switch (N) {
        case 4: return run_lag_t<4, 4, Fun>(prm, geo, nitems, partial, gb, s, 3);
        case 8: return run_lag_t<4, 8, Fun>(prm, geo, nitems, partial, gb, s, 3);
        case 16: return run_lag_t<4, 16, Fun>(prm, geo, nitems, partial, gb, s, 3);
        case 32: return run_lag_t<4, 32, Fun>(prm, geo, nitems, partial, gb, s, 3);
        case 64: return run_lag_t<4, 64, Fun>(prm, geo, nitems, partial, gb, s, 3);
        case 128: return run_lag_t<4, 128, Fun>(prm, geo, nitems, partial, gb, s, 3);
        default: return hipErrorInvalidValue;
    }
}

// One kernel per order r, so a lag costs the work of its own order.
template <int NGS>
static hipError_t eta_4(int r, int N, const double* prm, RowGeom geo, int64_t nitems, double* partial, int gb,
                         hipStream_t s) {
    switch (r) {
        case 0: return lag_4<EtaFun<4, NGS, 0>>(N, prm, geo, nitems, partial, gb, s);
        case 1: return lag_4<EtaFun<4, NGS, 1>>(N, prm, geo, nitems, partial, gb, s);
        case 2: return lag_4<EtaFun<4, NGS, 2>>(N, prm, geo, nitems, partial, gb, s);
        case 3: return lag_4<EtaFun<4, NGS, 3>>(N, prm, geo, nitems, partial, gb, s);
        case 4: return lag_4<EtaFun<4, NGS, 4>>(N, prm, geo, nitems, partial, gb, s);
        case 5: return lag_4<EtaFun<4, NGS, 5>>(N, prm, geo, nitems, partial, gb, s);
        case 6: return lag_4<EtaFun<4, NGS, 6>>(N, prm, geo, nitems, partial, gb, s);
        case 7: return lag_4<EtaFun<4, NGS, 7>>(N, prm, geo, nitems, partial, gb, s);
        default: return lag_4<EtaFun<4, NGS, ETA_RMAX>>(N, prm, geo, nitems, partial, gb, s);
    }
}

hipError_t launch_rows_eta_d4(int kind, int r, int N, int var, const double* prm, RowGeom geo, int64_t nitems,
                               double* partial, int gb, hipStream_t s) {
    if (var != 3 && var != 4) return hipErrorInvalidValue;
    if (r < 0 || r > ETA_RMAX) return hipErrorInvalidValue;
    switch (kind) {
        case FUN_ETA1: return eta_4<1>(r, N, prm, geo, nitems, partial, gb, s);
        case FUN_ETA2: return eta_4<2>(r, N, prm, geo, nitems, partial, gb, s);
        default: return hipErrorInvalidValue;
    }
}

int rows_iter_eta_d4(int kind, int N, int var) {
    if ((var != 3 && var != 4) || (kind != FUN_ETA1 && kind != FUN_ETA2)) return 0;
    switch (N) {
        case 4: return lag_rows_per_pass<4>();
        case 8: return lag_rows_per_pass<8>();
        case 16: return lag_rows_per_pass<16>();
        case 32: return lag_rows_per_pass<32>();
        case 64: return lag_rows_per_pass<64>();
        case 128: return lag_rows_per_pass<128>();
        default: return 0;
    }
}

}  // namespace kdefft
