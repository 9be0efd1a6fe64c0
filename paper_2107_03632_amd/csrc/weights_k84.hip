// FP64 weights kernel instance: K = 84 (m = 6, n = 56), one stencil per
// two-wavefront block, columns split between the wavefronts.
#include "weights_cs.h"

namespace rbffd {
int weights_fp64_k84(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr, int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev, int64_t n_rows, int n, int m, double *w, int32_t *status, const wk::SaveView &sv, int32_t ok_code, hipStream_t stream) {
    return wk::launch_cs<84, 56, 6>(x, y, n_nodes, nbr, k_stride, rows, n_rows_dev, n_rows, n, m, w, status, sv, ok_code, stream);
}
}  // namespace rbffd
