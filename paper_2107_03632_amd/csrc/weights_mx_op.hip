// Mixed-precision derivative weights (d/dx, d/dy): the Laplacian's
// mixed-precision kernels with the operator's right-hand side and scale;
// m = 2 here (the LU kernel with FP64 row scratch), m = 4 and 6 in
// weights_mx_op_k45.hip / weights_mx_op_k84.hip (Gauss-Jordan).
#include "weights_mx.h"

#ifndef RBFFD_OCC_MX_K18
#define RBFFD_OCC_MX_K18 0
#endif

namespace rbffd {
int weights_mx_op_k45(int op, const double *x, const double *y, int64_t n_nodes,
                      const int32_t *nbr, int32_t k_stride, double *w, int32_t *status,
                      int32_t *iters, int32_t *fb_count, int32_t *fb_list, hipStream_t stream);
int weights_mx_op_k84(int op, const double *x, const double *y, int64_t n_nodes,
                      const int32_t *nbr, int32_t k_stride, double *w, int32_t *status,
                      int32_t *iters, int32_t *fb_count, int32_t *fb_list, hipStream_t stream);

namespace {
template <int OP>
using MxOp18 = wk::MixedLaunch<18, 4, 5, 12, 2, RBFFD_OCC_MX_K18, OP>;
}  // namespace

size_t weights_mx_op_scratch(int m, int64_t n_rows) {
    return m == 2 ? MxOp18<RBFFD_OP_DX>::scratch_bytes(n_rows) : 0;
}

// every node of the standard support of order m; scratch: the K = 18
// kernel's FP64 rows (weights_mx_op_scratch bytes)
int weights_mx_op(int m, int op, const double *x, const double *y, int64_t n_nodes,
                  const int32_t *nbr, int32_t k_stride, double *w, int32_t *status,
                  int32_t *iters, double *scratch, int32_t *fb_count, int32_t *fb_list,
                  hipStream_t stream) {
    if (m == 4)
        return weights_mx_op_k45(op, x, y, n_nodes, nbr, k_stride, w, status, iters, fb_count,
                                 fb_list, stream);
    if (m == 6)
        return weights_mx_op_k84(op, x, y, n_nodes, nbr, k_stride, w, status, iters, fb_count,
                                 fb_list, stream);
    if (op == RBFFD_OP_DX)
        return MxOp18<RBFFD_OP_DX>::run(x, y, n_nodes, nbr, k_stride, nullptr, nullptr, n_nodes, w,
                                        status, iters, scratch, fb_count, fb_list, stream);
    return MxOp18<RBFFD_OP_DY>::run(x, y, n_nodes, nbr, k_stride, nullptr, nullptr, n_nodes, w,
                                    status, iters, scratch, fb_count, fb_list, stream);
}
}  // namespace rbffd
