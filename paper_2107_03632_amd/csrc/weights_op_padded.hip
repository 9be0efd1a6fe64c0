// First-derivative weights (d/dx, d/dy) of eq. (1) on supports other than
// the three standard ones: the padded Laplacian instances with the
// operator's right-hand side and scale (K <= 32 and K <= 64: the multi-slot
// kernel of weights_ms.h; K <= 96: the two-wavefront kernel of
// weights_kernel.h, in weights_op_p96.hip).
#include "weights_ms.h"

namespace rbffd {

int weights_op_p96(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                   int32_t k_stride, int64_t n_rows, int n, int m, int op, double *w,
                   int32_t *status, hipStream_t stream);

namespace {

template <int OP>
int op_padded(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
              int32_t k_stride, int64_t n_rows, int n, int m, double *w, int32_t *status,
              hipStream_t stream) {
    const wk::SaveView none;
    const int K = n + n_monomials(m);
    if (K <= 32)
        return wk::launch_ms<32, 16, 2, 0, 0, 0, OP>(x, y, n_nodes, nbr, k_stride, nullptr,
                                                     nullptr, n_rows, n, m, w, status, none,
                                                     RBFFD_OK, stream);
    return wk::launch_ms<64, 32, 2, 0, 0, 0, OP>(x, y, n_nodes, nbr, k_stride, nullptr, nullptr,
                                                 n_rows, n, m, w, status, none, RBFFD_OK,
                                                 stream);
}

}  // namespace

int weights_op_padded(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                      int32_t k_stride, int64_t n_rows, int n, int m, int op, double *w,
                      int32_t *status, hipStream_t stream) {
    const int K = n + n_monomials(m);
    if (K > 96) return RBFFD_ERR_UNSUPPORTED;
    if (K > 64)
        return weights_op_p96(x, y, n_nodes, nbr, k_stride, n_rows, n, m, op, w, status, stream);
    return op == RBFFD_OP_DX
               ? op_padded<RBFFD_OP_DX>(x, y, n_nodes, nbr, k_stride, n_rows, n, m, w, status,
                                        stream)
               : op_padded<RBFFD_OP_DY>(x, y, n_nodes, nbr, k_stride, n_rows, n, m, w, status,
                                        stream);
}

}  // namespace rbffd
