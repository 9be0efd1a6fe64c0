// Mixed-precision weights kernel instance: K = 45 (m = 4, n = 30), 16 lanes x 3 rows, 4 stencils per wave.
#include "weights_gj.h"
#include "weights_mx.h"

#ifndef RBFFD_OCC_MX_K45
#define RBFFD_OCC_MX_K45 4
#endif

namespace rbffd {
#ifndef RBFFD_MX_GJ_K45
#define RBFFD_MX_GJ_K45 1
#endif
#ifndef RBFFD_GJ_UNR_K45
#define RBFFD_GJ_UNR_K45 4
#endif
#if RBFFD_MX_GJ_K45
using MxL_k45 = wk::GjLaunch<45, 30, 4, true, RBFFD_OCC_MX_K45, RBFFD_GJ_UNR_K45>;
#else
using MxL_k45 = wk::MixedLaunch<45, 16, 3, 30, 4, RBFFD_OCC_MX_K45>;
#endif
size_t weights_mx_k45_scratch(int64_t n_rows) { return MxL_k45::scratch_bytes(n_rows); }
int weights_mx_k45(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                    int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev,
                    int64_t n_rows, double *w, int32_t *status, int32_t *iters, double *scratch,
                    int32_t *fb_count, int32_t *fb_list, hipStream_t stream) {
    return MxL_k45::run(x, y, n_nodes, nbr, k_stride, rows, n_rows_dev, n_rows, w, status,
                          iters, scratch, fb_count, fb_list, stream);
}
}  // namespace rbffd
