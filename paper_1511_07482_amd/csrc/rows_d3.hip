// Batched row kernels for d = 3 (see rows_impl.h).
#include "rows_dispatch.h"

namespace kdefft {

template <class Fun>
static hipError_t ndisp_3(int N, int var, const double* prm, RowGeom geo, int64_t nitems, double* partial, int gb, const double2* tw, hipStream_t s) {
    switch (N) {
        case 4: return rows_var<3, 4, Fun>(var, prm, geo, nitems, partial, gb, tw, s);
        case 8: return rows_var<3, 8, Fun>(var, prm, geo, nitems, partial, gb, tw, s);
        case 16: return rows_var<3, 16, Fun>(var, prm, geo, nitems, partial, gb, tw, s);
        case 32: return rows_var<3, 32, Fun>(var, prm, geo, nitems, partial, gb, tw, s);
        case 64: return rows_var<3, 64, Fun>(var, prm, geo, nitems, partial, gb, tw, s);
        case 128: return rows_var<3, 128, Fun>(var, prm, geo, nitems, partial, gb, tw, s);
        case 256: return rows_var<3, 256, Fun>(var, prm, geo, nitems, partial, gb, tw, s);
        default: return hipErrorInvalidValue;
    }
}

template <class Fun>
static int nrows_3(int N, int var) {
    switch (N) {
        case 4: return rows_fits<4, Fun>() ? rows_per_iter_t<3, 4, Fun>(var) : 0;
        case 8: return rows_fits<8, Fun>() ? rows_per_iter_t<3, 8, Fun>(var) : 0;
        case 16: return rows_fits<16, Fun>() ? rows_per_iter_t<3, 16, Fun>(var) : 0;
        case 32: return rows_fits<32, Fun>() ? rows_per_iter_t<3, 32, Fun>(var) : 0;
        case 64: return rows_fits<64, Fun>() ? rows_per_iter_t<3, 64, Fun>(var) : 0;
        case 128: return rows_fits<128, Fun>() ? rows_per_iter_t<3, 128, Fun>(var) : 0;
        case 256: return rows_fits<256, Fun>() ? rows_per_iter_t<3, 256, Fun>(var) : 0;
        default: return 0;
    }
}

hipError_t launch_rows_d3(int kind, int r, int N, int var, const double* prm, RowGeom geo, int64_t nitems,
                           double* partial, int gb, const double2* tw, hipStream_t s) {
    switch (kind) {
        case FUN_PSI:
            switch (r) {
                case 0: return ndisp_3<PsiFun<3, 0>>(N, var, prm, geo, nitems, partial, gb, tw, s);
                case 2: return ndisp_3<PsiFun<3, 2>>(N, var, prm, geo, nitems, partial, gb, tw, s);
                case 4: return ndisp_3<PsiFun<3, 4>>(N, var, prm, geo, nitems, partial, gb, tw, s);
                case 6: return ndisp_3<PsiFun<3, 6>>(N, var, prm, geo, nitems, partial, gb, tw, s);
                default: return hipErrorInvalidValue;
            }
        case FUN_SCV_OBJ: return ndisp_3<ScvFun<3, 0>>(N, var, prm, geo, nitems, partial, gb, tw, s);
        case FUN_SCV_OBJGRAD: return ndisp_3<ScvFun<3, 1>>(N, var, prm, geo, nitems, partial, gb, tw, s);
        case FUN_SCV_GRAD: return ndisp_3<ScvFun<3, 2>>(N, var, prm, geo, nitems, partial, gb, tw, s);
        default: return hipErrorInvalidValue;
    }
}

int rows_iter_d3(int kind, int r, int N, int var) {
    switch (kind) {
        case FUN_PSI:
            switch (r) {
                case 0: return nrows_3<PsiFun<3, 0>>(N, var);
                case 2: return nrows_3<PsiFun<3, 2>>(N, var);
                case 4: return nrows_3<PsiFun<3, 4>>(N, var);
                case 6: return nrows_3<PsiFun<3, 6>>(N, var);
                default: return 0;
            }
        case FUN_SCV_OBJ: return nrows_3<ScvFun<3, 0>>(N, var);
        case FUN_SCV_OBJGRAD: return nrows_3<ScvFun<3, 1>>(N, var);
        case FUN_SCV_GRAD: return nrows_3<ScvFun<3, 2>>(N, var);
        default: return 0;
    }
}

}  // namespace kdefft
