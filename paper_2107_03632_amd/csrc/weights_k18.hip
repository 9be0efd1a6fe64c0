// FP64 weights kernel instance: K = 18 (m = 2, n = 12), 8 lanes x 3 rows per stencil, 8 stencils per wave.
#include "weights_ms.h"

#ifndef RBFFD_SEG_K18
#define RBFFD_SEG_K18 8
#endif
#ifndef RBFFD_SL_K18
#define RBFFD_SL_K18 3
#endif
#ifndef RBFFD_OCC_K18
#define RBFFD_OCC_K18 3
#endif

namespace rbffd {
int weights_fp64_k18(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr, int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev, int64_t n_rows, int n, int m, double *w, int32_t *status, const wk::SaveView &sv, int32_t ok_code, hipStream_t stream) {
    return wk::launch_ms<18, RBFFD_SEG_K18, RBFFD_SL_K18, 12, 2, RBFFD_OCC_K18>(x, y, n_nodes, nbr, k_stride, rows, n_rows_dev, n_rows, n, m, w, status, sv, ok_code, stream);
}
}  // namespace rbffd
