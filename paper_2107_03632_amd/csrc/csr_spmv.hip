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

// csr_fill with the block's rows (their first kmax support entries) staged
// in LDS first: the rank loop then reads LDS, where the threads of one row
// read one address at a time.  For kmax <= kFillMaxK.
constexpr int kFillMaxK = 128;

__global__ __launch_bounds__(kThreads) void csr_fill_staged(
    int64_t n_nodes, const int32_t *nbr, int32_t k_stride, int32_t kmax, const int8_t *order,
    int n_uniform, OrderTable tab, const double *w, const uint8_t *is_boundary,
    const int64_t *row_ptr, int32_t *col, double *val) {
    // rows overlapping one block: at most kThreads / kmax + 2
    __shared__ int32_t s_nbr[kThreads + 2 * kFillMaxK];
    const int64_t e0 = (int64_t)blockIdx.x * kThreads;
    const int64_t i_first = e0 / kmax;
    const int64_t i_end = (e0 + kThreads - 1) / kmax;
    const int64_t i_last = i_end < n_nodes - 1 ? i_end : n_nodes - 1;
    const int staged = (int)(i_last - i_first + 1) * kmax;
    for (int q = threadIdx.x; q < staged; q += kThreads) {
        const int rr = q / kmax;
        s_nbr[q] = nbr[(i_first + rr) * (int64_t)k_stride + (q - rr * kmax)];
    }
    __syncthreads();
    const int64_t e = e0 + threadIdx.x;
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
    const int32_t *c = s_nbr + (i - i_first) * kmax;
    const int32_t ck = c[k];
    int rank = 0;
    for (int l = 0; l < n; ++l) {
        const int32_t cl = c[l];
        rank += (cl < ck || (cl == ck && l < k)) ? 1 : 0;
    }
    col[at + rank] = ck;
    val[at + rank] = w[i * (int64_t)k_stride + k];
}

// One thread per row, one wavefront per block of 64 rows.  The block's
// nonzeros are a contiguous range of col / val: they are staged through LDS
// in chunks, with consecutive lanes loading consecutive entries and the
// gathered u of each entry (all lanes' gathers in flight at once), and each
// thread then sums its own row from LDS in CSR order (the same operands in
// the same order as a plain sequential loop, so the sums are the same
// doubles; an entry whose column lies outside [0, n_rows) stages NaN, which
// poisons its row as before).
constexpr int kSpRows = 64;
constexpr int kSpChunk = 1024;  // entries per staging pass (16 KB of LDS)

__global__ __launch_bounds__(kSpRows) void spmv_rows(int64_t n_rows,
                                                     const int64_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col,
                                                     const double *__restrict__ val,
                                                     const double *__restrict__ u,
                                                     const double *__restrict__ f,
                                                     double *__restrict__ y) {
    __shared__ double s_val[kSpChunk];
    __shared__ double s_u[kSpChunk];
    const int t = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * kSpRows;
    const int64_t i = r0 + t;
    const int64_t rl = r0 + kSpRows < n_rows ? r0 + kSpRows : n_rows;  // past the last row
    const int64_t b0 = row_ptr[r0], b1 = row_ptr[rl];
    int64_t e = i < n_rows ? row_ptr[i] : b1;
    const int64_t e1 = i < n_rows ? row_ptr[i + 1] : b1;
    double acc = 0.0;
    for (int64_t c0 = b0; c0 < b1; c0 += kSpChunk) {
        const int64_t c1 = c0 + kSpChunk < b1 ? c0 + kSpChunk : b1;
        for (int64_t q = c0 + t; q < c1; q += kSpRows) {
            const int32_t c = col[q];
            s_val[q - c0] = val[q];
            // the operator is square: a column outside [0, n_rows) poisons the row
            s_u[q - c0] = ((int64_t)c >= 0 && (int64_t)c < n_rows) ? u[c] : __builtin_nan("");
        }
        __syncthreads();
        // this row's entries in the chunk (e >= c0 here: rows are ascending)
        for (; e < e1 && e < c1; ++e) acc = fma(s_val[e - c0], s_u[e - c0], acc);
        __syncthreads();
    }
    if (i < n_rows) y[i] = f ? acc - f[i] : acc;
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
    if (kmax <= kFillMaxK)
        hipLaunchKernelGGL(csr_fill_staged, dim3((unsigned)ceil_div(slots, kThreads)),
                           dim3(kThreads), 0, s, n_nodes, nbr, k_stride, (int32_t)kmax, order, n,
                           tab, w, is_boundary, (const int64_t *)row_ptr, col, val);
    else
        hipLaunchKernelGGL(csr_fill, dim3((unsigned)ceil_div(slots, kThreads)), dim3(kThreads),
                           0, s, n_nodes, nbr, k_stride, (int32_t)kmax, order, n, tab, w,
                           is_boundary, (const int64_t *)row_ptr, col, val);
    return last_launch_rc();
}

extern "C" int rbffd_spmv(int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
                          const double *val, const double *u, const double *f, double *y,
                          void *stream) {
    if (n_rows < 0 || !row_ptr || !col || !val || !u || !y) return RBFFD_ERR_ARG;
    if (n_rows == 0) return RBFFD_SUCCESS;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(spmv_rows, dim3((unsigned)ceil_div(n_rows, kSpRows)), dim3(kSpRows), 0,
                       s, n_rows, row_ptr, col, val, u, f, y);
    return last_launch_rc();
}
