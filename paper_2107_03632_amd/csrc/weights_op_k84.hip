// First-derivative weights (d/dx, d/dy) for m = 6, n = 56: the blocked LU
// of the Laplacian with the operator's right-hand side and scale.
#include "weights_mf.h"

namespace rbffd {
// rows, n_rows_dev: null (every node), or a device-counted list of at most
// n_rows node ids: one block per possible entry (per_entry) or a capped
// grid walking it.  ok_code: the status of a stencil solved here.
int weights_op_k84(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                   int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev,
                   int64_t n_rows, int op, double *w, int32_t *status, hipStream_t stream,
                   bool per_entry, int32_t ok_code) {
    const wk::SaveView none;
    if (op == RBFFD_OP_DX)
        return wk::launch_mf<84, 56, 6, 2, 2, RBFFD_OP_DX>(x, y, n_nodes, nbr, k_stride, rows,
                                                           n_rows_dev, n_rows, w, status, none,
                                                           ok_code, stream, per_entry);
    return wk::launch_mf<84, 56, 6, 2, 2, RBFFD_OP_DY>(x, y, n_nodes, nbr, k_stride, rows,
                                                       n_rows_dev, n_rows, w, status, none,
                                                       ok_code, stream, per_entry);
}
}  // namespace rbffd
