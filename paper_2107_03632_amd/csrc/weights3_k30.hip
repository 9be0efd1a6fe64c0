// Three-dimensional weights, m = 2, n = 20 (K = 30): the blocked LU with two
// tiles per dimension.  RBFFD_W3_K30_PAIRS = 1 (the default): two stencils
// per wavefront (weights_mf2.h); 0: one stencil per wavefront
// (weights_mf.h).
#include "weights_mf2.h"

#ifndef RBFFD_W3_K30_PAIRS
#define RBFFD_W3_K30_PAIRS 1
#endif
#ifndef RBFFD_OCC_MF3_K30
#define RBFFD_OCC_MF3_K30 4
#endif
#ifndef RBFFD_OCC_MF2_K30
#define RBFFD_OCC_MF2_K30 4
#endif

namespace rbffd {
namespace {

template <int OP>
int launch_k30(const double *x, const double *y, const double *z, int64_t n_nodes,
               const int32_t *nbr, int32_t k_stride, double *w, int32_t *status,
               hipStream_t stream) {
    if (!RBFFD_W3_K30_PAIRS)
        return wk::launch_mf3<30, 20, 2, 1, RBFFD_OCC_MF3_K30, OP>(x, y, z, n_nodes, nbr,
                                                                  k_stride, w, status, stream);
    if (n_nodes <= 0) return RBFFD_SUCCESS;
    const int64_t blocks = ceil_div(n_nodes, 2);
    if (blocks > 0x7fffffff) return RBFFD_ERR_UNSUPPORTED;
    hipLaunchKernelGGL((wk::weights_mf2_kernel<30, 20, 2, OP, 3, 1, RBFFD_OCC_MF2_K30>),
                       dim3((unsigned)blocks), dim3(kWave), 0, stream, x, y, z, n_nodes, nbr,
                       k_stride, nullptr, n_nodes, w, status, RBFFD_OK);
    return last_launch_rc();
}

}  // namespace

int weights3_blocked_k30(const double *x, const double *y, const double *z, int64_t n_nodes,
                         const int32_t *nbr, int32_t k_stride, int op, double *w,
                         int32_t *status, hipStream_t stream) {
    switch (op) {
    case 0: return launch_k30<0>(x, y, z, n_nodes, nbr, k_stride, w, status, stream);
    case 1: return launch_k30<1>(x, y, z, n_nodes, nbr, k_stride, w, status, stream);
    case 2: return launch_k30<2>(x, y, z, n_nodes, nbr, k_stride, w, status, stream);
    case 3: return launch_k30<3>(x, y, z, n_nodes, nbr, k_stride, w, status, stream);
    default: return RBFFD_ERR_ARG;
    }
}
}  // namespace rbffd
