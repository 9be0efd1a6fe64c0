// FP64 weights kernel instance: systems padded to 32 rows, 16 lanes x 2 rows per stencil.
#include "weights_ms.h"

#ifndef RBFFD_SEG_P32
#define RBFFD_SEG_P32 16
#endif
#ifndef RBFFD_SL_P32
#define RBFFD_SL_P32 2
#endif
#ifndef RBFFD_OCC_P32
#define RBFFD_OCC_P32 0
#endif

namespace rbffd {
int weights_fp64_p32(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr, int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev, int64_t n_rows, int n, int m, double *w, int32_t *status, const wk::SaveView &sv, int32_t ok_code, hipStream_t stream) {
    return wk::launch_ms<32, RBFFD_SEG_P32, RBFFD_SL_P32, 0, 0, RBFFD_OCC_P32>(x, y, n_nodes, nbr, k_stride, rows, n_rows_dev, n_rows, n, m, w, status, sv, ok_code, stream);
}
}  // namespace rbffd
