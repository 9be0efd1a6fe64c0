// FP64 weights kernel instance: KP = 96 rows padded, 128 lanes per stencil.
#include "weights_kernel.h"

#ifndef RBFFD_OCC_P96
#define RBFFD_OCC_P96 0
#endif

namespace rbffd {
int weights_fp64_p96(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr, int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev, int64_t n_rows, int n, int m, double *w, int32_t *status, const wk::SaveView &sv, int32_t ok_code, hipStream_t stream) {
    return wk::launch_fp64<96, 128, 0, 0, RBFFD_OCC_P96>(x, y, n_nodes, nbr, k_stride, rows, n_rows_dev, n_rows, n, m, w, status, sv, ok_code, stream);
}
}  // namespace rbffd
