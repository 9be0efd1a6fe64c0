// Mixed-precision weights kernel instance: K = 84 (m = 6, n = 56), one
// stencil per wavefront: FP32 Gauss-Jordan inverse on the matrix cores, the
// FP64 residual's entries formed anew at each correction (weights_gj.h).
// Compile-time overrides: RBFFD_OCC_MX_K84 (2 wavefronts per SIMD: the FP32
// tiles alone take 144 VGPRs), RBFFD_GJ_UNR_K84 (1: panel loop rolled
// within each tile column, 2% faster than unrolled here), RBFFD_GJ_RCP_K84
// (0: IEEE division of the FP32 pivots; 1: the hardware reciprocal, within
// an ulp, is 1% faster here but changes the correction count of about a
// third of the stencils against the IEEE-division form).
#include "weights_gj.h"

#ifndef RBFFD_OCC_MX_K84
#define RBFFD_OCC_MX_K84 2
#endif
#ifndef RBFFD_GJ_UNR_K84
#define RBFFD_GJ_UNR_K84 1
#endif
#ifndef RBFFD_GJ_RCP_K84
#define RBFFD_GJ_RCP_K84 0
#endif

namespace rbffd {
using MxL_k84 =
    wk::GjLaunch<84, 56, 6, false, RBFFD_OCC_MX_K84, RBFFD_GJ_UNR_K84, RBFFD_GJ_RCP_K84>;
size_t weights_mx_k84_scratch(int64_t n_rows) { return MxL_k84::scratch_bytes(n_rows); }
int weights_mx_k84(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                   int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev,
                   int64_t n_rows, double *w, int32_t *status, int32_t *iters, double *scratch,
                   int32_t *fb_count, int32_t *fb_list, hipStream_t stream) {
    return MxL_k84::run(x, y, n_nodes, nbr, k_stride, rows, n_rows_dev, n_rows, w, status,
                        iters, scratch, fb_count, fb_list, stream);
}
}  // namespace rbffd
