// First-derivative weights (d/dx, d/dy) of eq. (1) for the standard supports
// of m = 2 and 4, and the C entry point rbffd_weights_op.  The kernels are
// the Laplacian's (one row per lane for K = 18, the blocked LU for K = 45
// and 84) with the operator's right-hand side and scale; K = 84 lives in
// weights_op_k84.hip, the other supports (K <= 96) in weights_op_padded.hip.
#include "weights_ms.h"
#include "weights_mf.h"

namespace rbffd {

int weights_fp64_class(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                       int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev,
                       int64_t n_rows, int n, int m, double *w, int32_t *status,
                       double *sv_lu, double *sv_z, double *sv_s, uint8_t *sv_perm,
                       int32_t sv_kmax, int32_t ok_code, hipStream_t stream);
int weights_op_k84(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                   int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev,
                   int64_t n_rows, int op, double *w, int32_t *status, hipStream_t stream,
                   bool per_entry, int32_t ok_code);
int weights_mx_op(int m, int op, const double *x, const double *y, int64_t n_nodes,
                  const int32_t *nbr, int32_t k_stride, double *w, int32_t *status,
                  int32_t *iters, double *scratch, int32_t *fb_count, int32_t *fb_list,
                  hipStream_t stream);
size_t weights_mx_op_scratch(int m, int64_t n_rows);
int bucket_orders(const int8_t *order, int64_t n_nodes, int32_t k_stride, int32_t *counts,
                  int32_t *lists, double *w, int32_t *status, hipStream_t s);
int weights_op_padded(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                      int32_t k_stride, int64_t n_rows, int n, int m, int op, double *w,
                      int32_t *status, hipStream_t stream);

namespace {

// rows, n_rows_dev: null (every node), or a device-counted list of at most
// n_rows node ids: one block per possible entry (per_entry) or a capped
// grid walking it.  ok_code: the status of a stencil solved here.
template <int OP>
int op_small(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
             int32_t k_stride, int64_t n_rows, int m, double *w, int32_t *status,
             hipStream_t stream, const int32_t *rows = nullptr,
             const int32_t *n_rows_dev = nullptr, bool per_entry = true,
             int32_t ok_code = RBFFD_OK) {
    const wk::SaveView none;
    if (m == 2)
        return wk::launch_ms<18, 8, 3, 12, 2, 3, OP>(x, y, n_nodes, nbr, k_stride, rows,
                                                     n_rows_dev, n_rows, 12, 2, w, status, none,
                                                     ok_code, stream, per_entry);
    return wk::launch_mf<45, 30, 4, 1, 4, OP>(x, y, n_nodes, nbr, k_stride, rows, n_rows_dev,
                                              n_rows, w, status, none, ok_code, stream,
                                              per_entry);
}

// The FP64 derivative weights of one standard class over a device list.
int op_fp64_list(int m, int op, const double *x, const double *y, int64_t n_nodes,
                 const int32_t *nbr, int32_t k_stride, const int32_t *rows,
                 const int32_t *n_rows_dev, int64_t max_rows, double *w, int32_t *status,
                 bool per_entry, int32_t ok_code, hipStream_t s) {
    if (m == 6)
        return weights_op_k84(x, y, n_nodes, nbr, k_stride, rows, n_rows_dev, max_rows, op, w,
                              status, s, per_entry, ok_code);
    return op == RBFFD_OP_DX ? op_small<RBFFD_OP_DX>(x, y, n_nodes, nbr, k_stride, max_rows, m,
                                                     w, status, s, rows, n_rows_dev, per_entry,
                                                     ok_code)
                             : op_small<RBFFD_OP_DY>(x, y, n_nodes, nbr, k_stride, max_rows, m,
                                                     w, status, s, rows, n_rows_dev, per_entry,
                                                     ok_code);
}

struct OpMixedWs {
    int32_t *fb_count;  // [1]
    int32_t *fb_list;   // [n_nodes]
    double *scratch;
    size_t bytes;
};

OpMixedWs carve_op_mixed(void *base, int64_t n_nodes, int m) {
    Carver c(base);
    OpMixedWs o;
    o.fb_count = c.take<int32_t>(64);
    o.fb_list = c.take<int32_t>((size_t)n_nodes);
    o.scratch = c.take<double>(weights_mx_op_scratch(m, n_nodes) / sizeof(double) + 1);
    o.bytes = c.bytes();
    return o;
}

struct OpBatchWs {
    int32_t *counts;  // [3]
    int32_t *lists;   // [3][n_nodes]
    size_t bytes;
};

OpBatchWs carve_op_batch(void *base, int64_t n_nodes) {
    Carver c(base);
    OpBatchWs b;
    b.counts = c.take<int32_t>(64);
    b.lists = c.take<int32_t>((size_t)3 * n_nodes);
    b.bytes = c.bytes();
    return b;
}

}  // namespace
}  // namespace rbffd

using namespace rbffd;

extern "C" int rbffd_weights_op(const double *x, const double *y, int64_t n_nodes,
                                const int32_t *nbr, int32_t k_stride, int32_t m, int32_t n,
                                int32_t op, double *w, int32_t *status, void *stream) {
    if (!x || !y || !nbr || !w || n_nodes < 1 || n_nodes >= INT32_MAX || k_stride < 1 ||
        n > k_stride || (m != 2 && m != 4 && m != 6) || n < n_monomials(m) ||
        op < RBFFD_OP_LAPLACIAN || op > RBFFD_OP_DY)
        return RBFFD_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (op == RBFFD_OP_LAPLACIAN)
        return weights_fp64_class(x, y, n_nodes, nbr, k_stride, nullptr, nullptr, n_nodes, n, m,
                                  w, status, nullptr, nullptr, nullptr, nullptr, 0, RBFFD_OK, s);
    const bool standard = (m == 2 && n == 12) || (m == 4 && n == 30) || (m == 6 && n == 56);
    if (!standard)
        return weights_op_padded(x, y, n_nodes, nbr, k_stride, n_nodes, n, m, op, w, status, s);
    if (m == 6)
        return weights_op_k84(x, y, n_nodes, nbr, k_stride, nullptr, nullptr, n_nodes, op, w,
                              status, s, false, RBFFD_OK);
    return op == RBFFD_OP_DX ? op_small<RBFFD_OP_DX>(x, y, n_nodes, nbr, k_stride, n_nodes, m, w,
                                                     status, s)
                             : op_small<RBFFD_OP_DY>(x, y, n_nodes, nbr, k_stride, n_nodes, m, w,
                                                     status, s);
}

extern "C" int rbffd_weights_op_batch_workspace_size(int64_t n_nodes, size_t *bytes) {
    if (!bytes || n_nodes < 1 || n_nodes >= INT32_MAX) return RBFFD_ERR_ARG;
    *bytes = carve_op_batch(nullptr, n_nodes).bytes;
    return RBFFD_SUCCESS;
}

extern "C" int rbffd_weights_op_batch(const double *x, const double *y, int64_t n_nodes,
                                      const int32_t *nbr, int32_t k_stride, const int8_t *order,
                                      int32_t op, double *w, int32_t *status, void *workspace,
                                      size_t workspace_bytes, void *stream) {
    if (!x || !y || !nbr || !order || !w || n_nodes < 1 || n_nodes >= INT32_MAX ||
        k_stride < 56 || (op != RBFFD_OP_DX && op != RBFFD_OP_DY))
        return RBFFD_ERR_ARG;
    OpBatchWs b = carve_op_batch(nullptr, n_nodes);
    if (!workspace || workspace_bytes < b.bytes) return RBFFD_ERR_WORKSPACE;
    b = carve_op_batch(workspace, n_nodes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = fill_i32(b.counts, 0, 64, s);
    if (rc) return rc;
    if ((rc = bucket_orders(order, n_nodes, k_stride, b.counts, b.lists, w, status, s))) return rc;
    // the largest systems first, one block per possible list entry
    for (int q = 2; q >= 0; --q) {
        rc = op_fp64_list(2 * q + 2, op, x, y, n_nodes, nbr, k_stride,
                          b.lists + (int64_t)q * n_nodes, b.counts + q, n_nodes, w, status, true,
                          RBFFD_OK, s);
        if (rc) return rc;
    }
    return RBFFD_SUCCESS;
}

extern "C" int rbffd_weights_op_mixed_workspace_size(int64_t n_nodes, int32_t m, size_t *bytes) {
    if (!bytes || n_nodes < 1 || n_nodes >= INT32_MAX || (m != 2 && m != 4 && m != 6))
        return RBFFD_ERR_ARG;
    *bytes = carve_op_mixed(nullptr, n_nodes, m).bytes;
    return RBFFD_SUCCESS;
}

extern "C" int rbffd_weights_op_mixed(const double *x, const double *y, int64_t n_nodes,
                                      const int32_t *nbr, int32_t k_stride, int32_t m, int32_t n,
                                      int32_t op, double *w, int32_t *status,
                                      int32_t *refine_steps, void *workspace,
                                      size_t workspace_bytes, void *stream) {
    if (!x || !y || !nbr || !w || n_nodes < 1 || n_nodes >= INT32_MAX || k_stride < 1 ||
        n > k_stride || (m != 2 && m != 4 && m != 6) || n < n_monomials(m) ||
        (op != RBFFD_OP_DX && op != RBFFD_OP_DY))
        return RBFFD_ERR_ARG;
    const bool standard = (m == 2 && n == 12) || (m == 4 && n == 30) || (m == 6 && n == 56);
    if (!standard) return RBFFD_ERR_UNSUPPORTED;
    OpMixedWs o = carve_op_mixed(nullptr, n_nodes, m);
    if (!workspace || workspace_bytes < o.bytes) return RBFFD_ERR_WORKSPACE;
    o = carve_op_mixed(workspace, n_nodes, m);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = fill_i32(o.fb_count, 0, 1, s);
    if (rc) return rc;
    // FP32 factorisation + FP64 refinement; the stencils it cannot refine go
    // to the fallback list, which the FP64 kernel then solves
    rc = weights_mx_op(m, op, x, y, n_nodes, nbr, k_stride, w, status, refine_steps, o.scratch,
                       o.fb_count, o.fb_list, s);
    if (rc) return rc;
    return op_fp64_list(m, op, x, y, n_nodes, nbr, k_stride, o.fb_list, o.fb_count, n_nodes, w,
                        status, false, RBFFD_FELL_BACK_FP64, s);
}
