// FP64 weights kernel instance: K = 84 (m = 6, n = 56), one stencil per
// two-wavefront block.  Plain weights: LU blocked by panels of four columns
// with the trailing updates on the matrix cores (weights_mf.h).  With the
// factors saved for the adjoint: the column-split kernel (weights_cs.h),
// which keeps L in registers for the save.
#include "weights_cs.h"
#include "weights_mf.h"

#ifndef RBFFD_K84_MFMA
#define RBFFD_K84_MFMA 1
#endif

namespace rbffd {
int weights_fp64_k84(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr, int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev, int64_t n_rows, int n, int m, double *w, int32_t *status, const wk::SaveView &sv, int32_t ok_code, hipStream_t stream) {
    if (RBFFD_K84_MFMA && !sv.lu)
        return wk::launch_mf<84, 56, 6, 2, 2>(x, y, n_nodes, nbr, k_stride, rows, n_rows_dev, n_rows, w, status, sv, ok_code, stream);
    return wk::launch_cs<84, 56, 6>(x, y, n_nodes, nbr, k_stride, rows, n_rows_dev, n_rows, n, m, w, status, sv, ok_code, stream);
}
}  // namespace rbffd
