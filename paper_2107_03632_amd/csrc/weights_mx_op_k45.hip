// Mixed-precision derivative weights (d/dx, d/dy), m = 4: the Laplacian's
// Gauss-Jordan kernel (weights_gj.h, same tuning) with the operator's
// right-hand side and scale.
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
int weights_mx_op_k45(int op, const double *x, const double *y, int64_t n_nodes,
                      const int32_t *nbr, int32_t k_stride, double *w, int32_t *status,
                      int32_t *iters, int32_t *fb_count, int32_t *fb_list, hipStream_t stream) {
    if (op == RBFFD_OP_DX)
        return wk::GjLaunch<45, 30, 4, true, RBFFD_OCC_MX_K45, RBFFD_GJ_UNR_K45, RBFFD_GJ_RCP_K45, RBFFD_OP_DX>::run(
            x, y, n_nodes, nbr, k_stride, nullptr, nullptr, n_nodes, w, status, iters, nullptr,
            fb_count, fb_list, stream);
    return wk::GjLaunch<45, 30, 4, true, RBFFD_OCC_MX_K45, RBFFD_GJ_UNR_K45, RBFFD_GJ_RCP_K45, RBFFD_OP_DY>::run(
        x, y, n_nodes, nbr, k_stride, nullptr, nullptr, n_nodes, w, status, iters, nullptr,
        fb_count, fb_list, stream);
}
}  // namespace rbffd
