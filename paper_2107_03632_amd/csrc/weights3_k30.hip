// Three-dimensional weights, m = 2, n = 20 (K = 30): the blocked LU of
// weights_mf.h (two tiles per dimension, one wavefront per stencil).
#include "weights_mf.h"

#ifndef RBFFD_OCC_MF3_K30
#define RBFFD_OCC_MF3_K30 4
#endif

namespace rbffd {
int weights3_blocked_k30(const double *x, const double *y, const double *z, int64_t n_nodes,
                         const int32_t *nbr, int32_t k_stride, int op, double *w,
                         int32_t *status, hipStream_t stream) {
    switch (op) {
#define W3_K30_CASE(OP)                                                                        \
    case OP:                                                                                   \
        return wk::launch_mf3<30, 20, 2, 1, RBFFD_OCC_MF3_K30, OP>(x, y, z, n_nodes, nbr,      \
                                                                   k_stride, w, status, stream);
        W3_K30_CASE(0)
        W3_K30_CASE(1)
        W3_K30_CASE(2)
        W3_K30_CASE(3)
#undef W3_K30_CASE
    default:
        return RBFFD_ERR_ARG;
    }
}
}  // namespace rbffd
