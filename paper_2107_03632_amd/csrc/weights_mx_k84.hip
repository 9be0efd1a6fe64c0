// Mixed-precision weights kernel instance: K = 84 (m = 6, n = 56), 64 lanes x 2 rows, 1 stencil per wave.
#include "weights_gj.h"
#include "weights_mx.h"

#ifndef RBFFD_OCC_MX_K84
#define RBFFD_OCC_MX_K84 2
#endif

namespace rbffd {
#ifndef RBFFD_MX_GJ_K84
#define RBFFD_MX_GJ_K84 1
#endif
#ifndef RBFFD_GJ_UNR_K84
#define RBFFD_GJ_UNR_K84 1
#endif
#if RBFFD_MX_GJ_K84
using MxL_k84 = wk::GjLaunch<84, 56, 6, false, RBFFD_OCC_MX_K84, RBFFD_GJ_UNR_K84>;
#else
using MxL_k84 = wk::MixedLaunch<84, 64, 2, 56, 6, RBFFD_OCC_MX_K84>;
#endif
size_t weights_mx_k84_scratch(int64_t n_rows) { return MxL_k84::scratch_bytes(n_rows); }
int weights_mx_k84(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                    int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev,
                    int64_t n_rows, double *w, int32_t *status, int32_t *iters, double *scratch,
                    int32_t *fb_count, int32_t *fb_list, hipStream_t stream) {
    return MxL_k84::run(x, y, n_nodes, nbr, k_stride, rows, n_rows_dev, n_rows, w, status,
                          iters, scratch, fb_count, fb_list, stream);
}
}  // namespace rbffd
