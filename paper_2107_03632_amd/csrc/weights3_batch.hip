// Three-dimensional Laplacian weights for nodes of mixed order (eq. (1) with
// d = 3; m in {2, 4} per node on the supports n = 20 and n = 70): the nodes
// are bucketed by order on the device, then each class runs its
// single-order blocked kernel over its list, the K = 105 class first.  The
// weights and statuses are those of rbffd_weights3 at each node's order.
#include "weights_mf2.h"

#ifndef RBFFD_OCC_MF2_K30
#define RBFFD_OCC_MF2_K30 4
#endif

namespace rbffd {
int weights3_list_k105(const double *x, const double *y, const double *z, int64_t n_nodes,
                       const int32_t *nbr, int32_t k_stride, const int32_t *rows,
                       const int32_t *n_rows_dev, int64_t max_rows, double *w, int32_t *status,
                       hipStream_t stream);

namespace {

constexpr int kBucketThreads = 256;

// Node i goes to list 0 (m = 2) or 1 (m = 4); any other order gets NaN
// weights and RBFFD_BAD_ORDER.  Block-local counts first, then one atomic
// per block and list.
__global__ __launch_bounds__(kBucketThreads) void bucket3_by_order(
    const int8_t *__restrict__ order, int64_t n_nodes, int32_t k_stride,
    int32_t *__restrict__ counts, int32_t *__restrict__ lists, double *__restrict__ w,
    int32_t *__restrict__ status) {
    __shared__ int32_t s_cnt[2];
    __shared__ int32_t s_base[2];
    if (threadIdx.x < 2) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kBucketThreads + threadIdx.x;
    int b = -1;
    int local = 0;
    if (i < n_nodes) {
        const int m = order[i];
        if (m == 2 || m == 4) {
            b = m / 2 - 1;
            local = atomicAdd(&s_cnt[b], 1);
        } else {
            for (int q = 0; q < k_stride; ++q) w[i * (int64_t)k_stride + q] = __builtin_nan("");
            if (status) status[i] = RBFFD_BAD_ORDER;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2) s_base[threadIdx.x] = atomicAdd(&counts[threadIdx.x], s_cnt[threadIdx.x]);
    __syncthreads();
    if (b >= 0) lists[(int64_t)b * n_nodes + s_base[b] + local] = (int32_t)i;
}

struct Batch3Ws {
    int32_t *counts;  // [2]
    int32_t *lists;   // [2][n_nodes]
    size_t bytes;
};

Batch3Ws carve_batch3(void *base, int64_t n_nodes) {
    Carver c(base);
    Batch3Ws b;
    b.counts = c.take<int32_t>(64);
    b.lists = c.take<int32_t>((size_t)2 * n_nodes);
    b.bytes = c.bytes();
    return b;
}

}  // namespace
}  // namespace rbffd

using namespace rbffd;

extern "C" int rbffd_weights3_batch_workspace_size(int64_t n_nodes, size_t *bytes) {
    if (!bytes || n_nodes < 1 || n_nodes >= INT32_MAX) return RBFFD_ERR_ARG;
    *bytes = carve_batch3(nullptr, n_nodes).bytes;
    return RBFFD_SUCCESS;
}

extern "C" int rbffd_weights3_batch(const double *x, const double *y, const double *z,
                                    int64_t n_nodes, const int32_t *nbr, int32_t k_stride,
                                    const int8_t *order, double *w, int32_t *status,
                                    void *workspace, size_t workspace_bytes, void *stream) {
    if (!x || !y || !z || !nbr || !order || !w || n_nodes < 1 || n_nodes >= INT32_MAX ||
        k_stride < 70)
        return RBFFD_ERR_ARG;
    Batch3Ws b = carve_batch3(nullptr, n_nodes);
    if (!workspace || workspace_bytes < b.bytes) return RBFFD_ERR_WORKSPACE;
    b = carve_batch3(workspace, n_nodes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = fill_i32(b.counts, 0, 64, s);
    if (rc) return rc;
    hipLaunchKernelGGL(bucket3_by_order, dim3((unsigned)ceil_div(n_nodes, kBucketThreads)),
                       dim3(kBucketThreads), 0, s, order, n_nodes, k_stride, b.counts, b.lists,
                       w, status);
    if ((rc = last_launch_rc())) return rc;
    // m = 4 (K = 105) first: the longer stencils start before the short ones
    rc = weights3_list_k105(x, y, z, n_nodes, nbr, k_stride, b.lists + n_nodes, b.counts + 1,
                            n_nodes, w, status, s);
    if (rc) return rc;
    // m = 2 (K = 30): two possible list entries per wavefront
    const int64_t blocks = ceil_div(n_nodes, 2);
    hipLaunchKernelGGL((wk::weights_mf2_list_kernel<30, 20, 2, 0, 3, 1, RBFFD_OCC_MF2_K30>),
                       dim3((unsigned)blocks), dim3(kWave), 0, s, x, y, z, n_nodes, nbr, k_stride,
                       b.lists, b.counts, w, status, RBFFD_OK);
    return last_launch_rc();
}
