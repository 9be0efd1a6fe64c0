// First-derivative weights on supports with 64 < K <= 96 (the two-wavefront
// kernel of weights_kernel.h with the operator's right-hand side and scale).
#include "weights_kernel.h"

namespace rbffd {
int weights_op_p96(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                   int32_t k_stride, int64_t n_rows, int n, int m, int op, double *w,
                   int32_t *status, hipStream_t stream) {
    const wk::SaveView none;
    if (op == RBFFD_OP_DX)
        return wk::launch_fp64<96, 128, 0, 0, 0, RBFFD_OP_DX>(x, y, n_nodes, nbr, k_stride,
                                                              nullptr, nullptr, n_rows, n, m, w,
                                                              status, none, RBFFD_OK, stream);
    return wk::launch_fp64<96, 128, 0, 0, 0, RBFFD_OP_DY>(x, y, n_nodes, nbr, k_stride, nullptr,
                                                          nullptr, n_rows, n, m, w, status, none,
                                                          RBFFD_OK, stream);
}
}  // namespace rbffd
