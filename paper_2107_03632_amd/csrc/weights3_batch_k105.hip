// Three-dimensional mixed-order batch, the m = 4 class (n = 70, K = 105):
// the blocked kernel of weights3_k105.h over the class's device-counted
// list.  Its own translation unit, so that it compiles beside the others.
#include "weights3_k105.h"

namespace rbffd {
int weights3_list_k105(const double *x, const double *y, const double *z, int64_t n_nodes,
                       const int32_t *nbr, int32_t k_stride, const int32_t *rows,
                       const int32_t *n_rows_dev, int64_t max_rows, double *w, int32_t *status,
                       hipStream_t stream) {
    return wk::launch_mf3_list<105, 70, 4, RBFFD_NW_MF3_K105, RBFFD_OCC_MF3_K105, 0>(
        x, y, z, n_nodes, nbr, k_stride, rows, n_rows_dev, max_rows, w, status, stream);
}
}  // namespace rbffd
