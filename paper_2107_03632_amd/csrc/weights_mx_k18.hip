// Mixed-precision weights kernel instance: K = 18 (m = 2, n = 12), 4 lanes x 5 rows, 16 stencils per wave.
#include "weights_mx.h"

#ifndef RBFFD_OCC_MX_K18
#define RBFFD_OCC_MX_K18 0
#endif

namespace rbffd {
using MxL_k18 = wk::MixedLaunch<18, 4, 5, 12, 2, RBFFD_OCC_MX_K18>;
size_t weights_mx_k18_scratch(int64_t n_rows) { return MxL_k18::scratch_bytes(n_rows); }
int weights_mx_k18(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                    int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev,
                    int64_t n_rows, double *w, int32_t *status, int32_t *iters, double *scratch,
                    int32_t *fb_count, int32_t *fb_list, hipStream_t stream) {
    return MxL_k18::run(x, y, n_nodes, nbr, k_stride, rows, n_rows_dev, n_rows, w, status,
                          iters, scratch, fb_count, fb_list, stream);
}
}  // namespace rbffd
