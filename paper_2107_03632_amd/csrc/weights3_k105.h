// Three-dimensional weights, m = 4, n = 70 (K = 105, the 35 monomials of
// degree <= 4): the blocked LU of weights_mf.h, seven tiles per dimension
// shared by RBFFD_NW_MF3_K105 wavefronts per stencil (a run-time wavefront
// index; four: tile columns {w, w + 4}, 168 VGPRs) at RBFFD_OCC_MF3_K105
// wavefronts per SIMD; 59 KB of LDS per block, two blocks per CU.  Seven
// wavefronts (one tile column each) measured the same, 201.6 ms against
// 200.7 ms on the 1M-node cube.  One operator per translation unit
// (weights3_k105_op*.hip): the instances compile in parallel.
#pragma once
#include "weights_mf.h"

#ifndef RBFFD_NW_MF3_K105
#define RBFFD_NW_MF3_K105 4
#endif
#ifndef RBFFD_OCC_MF3_K105
#define RBFFD_OCC_MF3_K105 2
#endif

#define RBFFD_W3_K105_INSTANCE(OP)                                                             \
    namespace rbffd {                                                                          \
    int weights3_blocked_k105_op##OP(const double *x, const double *y, const double *z,        \
                                     int64_t n_nodes, const int32_t *nbr, int32_t k_stride,    \
                                     double *w, int32_t *status, hipStream_t stream) {         \
        return wk::launch_mf3<105, 70, 4, RBFFD_NW_MF3_K105, RBFFD_OCC_MF3_K105, OP>(          \
            x, y, z, n_nodes, nbr, k_stride, w, status, stream);                               \
    }                                                                                          \
    }

// Other supports of m = 4 (35 <= n <= 76): the same kernel at KP = 111 (seven
// tiles, rhs in column 111) with a run-time n and identity padding up to 111.
#define RBFFD_W3_M4_ANY_INSTANCE(OP)                                                           \
    namespace rbffd {                                                                          \
    int weights3_blocked_m4_any_op##OP(const double *x, const double *y, const double *z,      \
                                       int64_t n_nodes, const int32_t *nbr, int32_t k_stride,  \
                                       int n, double *w, int32_t *status, hipStream_t stream) { \
        return wk::launch_mf3<111, 0, 4, RBFFD_NW_MF3_K105, RBFFD_OCC_MF3_K105, OP>(           \
            x, y, z, n_nodes, nbr, k_stride, w, status, stream, n);                            \
    }                                                                                          \
    }
