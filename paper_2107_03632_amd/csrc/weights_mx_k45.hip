// Mixed-precision weights kernel instance: K = 45 (m = 4, n = 30), one
// stencil per wavefront: FP32 Gauss-Jordan inverse on the matrix cores, the
// FP64 A block kept in registers for the residual (weights_gj.h).
// Compile-time overrides: RBFFD_OCC_MX_K45 (wavefronts per SIMD the
// register allocation aims at; 6 measured fastest: 11.3 ms on the 1M-node
// square against 12.3 ms at 4), RBFFD_GJ_UNR_K45 (4: panel loop unrolled;
// 1: rolled within each tile column), RBFFD_GJ_RCP_K45 (1: hardware
// reciprocal of the FP32 pivots; 0: IEEE division).
#include "weights_gj.h"

#ifndef RBFFD_OCC_MX_K45
#define RBFFD_OCC_MX_K45 6
#endif
#ifndef RBFFD_GJ_UNR_K45
#define RBFFD_GJ_UNR_K45 4
#endif
#ifndef RBFFD_GJ_RCP_K45
#define RBFFD_GJ_RCP_K45 1
#endif

namespace rbffd {
using MxL_k45 =
    wk::GjLaunch<45, 30, 4, true, RBFFD_OCC_MX_K45, RBFFD_GJ_UNR_K45, RBFFD_GJ_RCP_K45>;
size_t weights_mx_k45_scratch(int64_t n_rows) { return MxL_k45::scratch_bytes(n_rows); }
int weights_mx_k45(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                   int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev,
                   int64_t n_rows, double *w, int32_t *status, int32_t *iters, double *scratch,
                   int32_t *fb_count, int32_t *fb_list, hipStream_t stream) {
    return MxL_k45::run(x, y, n_nodes, nbr, k_stride, rows, n_rows_dev, n_rows, w, status,
                        iters, scratch, fb_count, fb_list, stream);
}
}  // namespace rbffd
