// CSR form of the discrete Laplacian (eq. (1) rows, Dirichlet identity rows
// of section IV) and the operator product y = W u - f (eq. (3)).

#include "common.h"

namespace rbffd {
namespace {

constexpr int kThreads = 256;

struct OrderTable {
    int32_t n[3];  // support size for m = 2, 4, 6
};

__device__ __forceinline__ int row_support(const int8_t *order, int n_uniform, OrderTable t,
                                           int64_t i) {
    if (!order) return n_uniform;
    const int m = order[i];
    return (m == 2 || m == 4 || m == 6) ? t.n[m / 2 - 1] : 0;
}

__global__ __launch_bounds__(kThreads) void csr_row_len(int64_t n_nodes, const int8_t *order,
                                                        int n_uniform, OrderTable tab,
                                                        const uint8_t *is_boundary,
                                                        int64_t *row_ptr) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i > n_nodes) return;
    if (i == n_nodes) {
        row_ptr[i] = 0;
        return;
    }
    row_ptr[i] = (is_boundary && is_boundary[i]) ? 1 : row_support(order, n_uniform, tab, i);
}

// One thread per (row, slot): the slot's rank among the row's entries ordered
// by (column, slot) is its offset inside the row.
__global__ __launch_bounds__(kThreads) void csr_fill(int64_t n_nodes, const int32_t *nbr,
                                                     int32_t k_stride, int32_t kmax,
                                                     const int8_t *order, int n_uniform,
                                                     OrderTable tab, const double *w,
                                                     const uint8_t *is_boundary,
                                                     const int64_t *row_ptr, int32_t *col,
                                                     double *val) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t i = e / kmax;
    const int k = (int)(e - i * kmax);
    if (i >= n_nodes) return;
    const int64_t at = row_ptr[i];
    if (is_boundary && is_boundary[i]) {
        if (k == 0) {
            col[at] = (int32_t)i;
            val[at] = 1.0;
        }
        return;
    }
    const int n = row_support(order, n_uniform, tab, i);
    if (k >= n) return;
    const int32_t *c = nbr + i * (int64_t)k_stride;
    const int32_t ck = c[k];
    int rank = 0;
    for (int l = 0; l < n; ++l) {
        const int32_t cl = c[l];
        rank += (cl < ck || (cl == ck && l < k)) ? 1 : 0;
    }
    col[at + rank] = ck;
    val[at + rank] = w[i * (int64_t)k_stride + k];
}

__global__ __launch_bounds__(kThreads) void spmv_rows(int64_t n_rows,
                                                      const int64_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col,
                                                      const double *__restrict__ val,
                                                      const double *__restrict__ u,
                                                      const double *__restrict__ f,
                                                      double *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n_rows) return;
    double acc = 0.0;
    const int64_t e1 = row_ptr[i + 1];
    for (int64_t e = row_ptr[i]; e < e1; ++e) {
        const int32_t c = col[e];
        // the operator is square: a column outside [0, n_rows) poisons the row
        acc = ((int64_t)c >= 0 && (int64_t)c < n_rows) ? fma(val[e], u[c], acc)
                                                        : __builtin_nan("");
    }
    y[i] = f ? acc - f[i] : acc;
}

}  // namespace
}  // namespace rbffd

using namespace rbffd;

extern "C" int rbffd_assemble_csr_workspace_size(int64_t n_nodes, size_t *bytes) {
    if (!bytes || n_nodes < 1) return RBFFD_ERR_ARG;
    *bytes = scan_workspace_bytes(n_nodes + 1);
    return RBFFD_SUCCESS;
}

extern "C" int rbffd_assemble_csr(int64_t n_nodes, const int32_t *nbr, int32_t k_stride,
                                  const int8_t *order, int32_t n, const int32_t *n_for_order,
                                  const double *w, const uint8_t *is_boundary, int64_t *row_ptr,
                                  int32_t *col, double *val, int64_t capacity, void *workspace,
                                  size_t workspace_bytes, void *stream) {
    if (n_nodes < 1 || n_nodes >= INT32_MAX || !nbr || !w || !row_ptr || !col || !val ||
        k_stride < 1)
        return RBFFD_ERR_ARG;
    OrderTable tab = {{0, 0, 0}};
    int kmax = 0;
    if (order) {
        if (!n_for_order) return RBFFD_ERR_ARG;
        for (int q = 0; q < 3; ++q) {
            tab.n[q] = n_for_order[q];
            if (n_for_order[q] < 1 || n_for_order[q] > k_stride) return RBFFD_ERR_ARG;
            kmax = n_for_order[q] > kmax ? n_for_order[q] : kmax;
        }
    } else {
        if (n < 1 || n > k_stride) return RBFFD_ERR_ARG;
        kmax = n;
    }
    if (capacity < n_nodes * (int64_t)kmax) return RBFFD_ERR_ARG;
    if (!workspace || workspace_bytes < scan_workspace_bytes(n_nodes + 1))
        return RBFFD_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(csr_row_len, dim3((unsigned)ceil_div(n_nodes + 1, kThreads)),
                       dim3(kThreads), 0, s, n_nodes, order, n, tab, is_boundary, row_ptr);
    int rc = exclusive_scan_i64(row_ptr, row_ptr, n_nodes + 1, workspace, s);
    if (rc) return rc;
    const int64_t slots = n_nodes * (int64_t)kmax;
    hipLaunchKernelGGL(csr_fill, dim3((unsigned)ceil_div(slots, kThreads)), dim3(kThreads), 0, s,
                       n_nodes, nbr, k_stride, (int32_t)kmax, order, n, tab, w, is_boundary,
                       (const int64_t *)row_ptr, col, val);
    return last_launch_rc();
}

extern "C" int rbffd_spmv(int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
                          const double *val, const double *u, const double *f, double *y,
                          void *stream) {
    if (n_rows < 0 || !row_ptr || !col || !val || !u || !y) return RBFFD_ERR_ARG;
    if (n_rows == 0) return RBFFD_SUCCESS;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(spmv_rows, dim3((unsigned)ceil_div(n_rows, kThreads)), dim3(kThreads), 0,
                       s, n_rows, row_ptr, col, val, u, f, y);
    return last_launch_rc();
}
