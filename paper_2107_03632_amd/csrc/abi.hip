// C ABI: argument checking, workspace carving and the per-order bucketing of
// rbffd_weights.  Kernels live in the other sources of this directory.

#include "common.h"

namespace rbffd {

int weights_fp64_class(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                       int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev,
                       int64_t n_rows, int n, int m, double *w, int32_t *status,
                       double *sv_lu, double *sv_z, double *sv_s, uint8_t *sv_perm,
                       int32_t sv_kmax, int32_t ok_code, hipStream_t stream);

int weights_fp64_batch(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                       int32_t k_stride, const int32_t *lists, const int32_t *counts,
                       int32_t *queue, double *w, int32_t *status, double *sv_lu, double *sv_z,
                       double *sv_s, uint8_t *sv_perm, int32_t sv_kmax, hipStream_t stream);

#define RBFFD_MX_DECL(name)                                                                    \
    size_t weights_mx_##name##_scratch(int64_t n_rows);                                         \
    int weights_mx_##name(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr, \
                          int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev,      \
                          int64_t n_rows, double *w, int32_t *status, int32_t *iters,            \
                          double *scratch, int32_t *fb_count, int32_t *fb_list,                  \
                          hipStream_t stream);
RBFFD_MX_DECL(k18)
RBFFD_MX_DECL(k45)
RBFFD_MX_DECL(k84)
#undef RBFFD_MX_DECL

namespace {

constexpr int kThreads = 256;

// mixed-precision instances exist for the standard supports only
int mixed_class(int m, int n) {
    if (m == 2 && n == 12) return 0;
    if (m == 4 && n == 30) return 1;
    if (m == 6 && n == 56) return 2;
    return -1;
}

size_t mixed_scratch(int cls, int64_t n_rows) {
    return cls == 0 ? weights_mx_k18_scratch(n_rows)
                    : cls == 1 ? weights_mx_k45_scratch(n_rows) : weights_mx_k84_scratch(n_rows);
}

int mixed_run(int cls, const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
              int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev, int64_t n_rows,
              double *w, int32_t *status, int32_t *iters, double *scratch, int32_t *fb_count,
              int32_t *fb_list, hipStream_t s) {
    if (cls == 0)
        return weights_mx_k18(x, y, n_nodes, nbr, k_stride, rows, n_rows_dev, n_rows, w, status,
                              iters, scratch, fb_count, fb_list, s);
    if (cls == 1)
        return weights_mx_k45(x, y, n_nodes, nbr, k_stride, rows, n_rows_dev, n_rows, w, status,
                              iters, scratch, fb_count, fb_list, s);
    return weights_mx_k84(x, y, n_nodes, nbr, k_stride, rows, n_rows_dev, n_rows, w, status,
                          iters, scratch, fb_count, fb_list, s);
}

// Bucket the nodes by order: node i goes to list b = m/2 - 1.  Nodes with an
// order outside {2,4,6} get NaN weights and status RBFFD_BAD_ORDER here.
__global__ __launch_bounds__(kThreads) void bucket_by_order(
    const int8_t *__restrict__ order, int64_t n_nodes, int32_t k_stride,
    int32_t *__restrict__ counts, int32_t *__restrict__ lists, double *__restrict__ w,
    int32_t *__restrict__ status) {
    __shared__ int32_t s_cnt[3];
    __shared__ int32_t s_base[3];
    if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    int b = -1;
    int local = 0;
    if (i < n_nodes) {
        const int m = order[i];
        if (m == 2 || m == 4 || m == 6) {
            b = m / 2 - 1;
            local = atomicAdd(&s_cnt[b], 1);
        } else {
            for (int q = 0; q < k_stride; ++q) w[i * (int64_t)k_stride + q] = __builtin_nan("");
            if (status) status[i] = RBFFD_BAD_ORDER;
        }
    }
    __syncthreads();
    if (threadIdx.x < 3) s_base[threadIdx.x] = atomicAdd(&counts[threadIdx.x], s_cnt[threadIdx.x]);
    __syncthreads();
    if (b >= 0) lists[(int64_t)b * n_nodes + s_base[b] + local] = (int32_t)i;
}

struct SaveLayout {
    double *lu, *z, *s;
    uint8_t *perm;
    size_t bytes;
};

SaveLayout carve_save(void *base, int64_t n_nodes, int32_t kmax) {
    Carver c(base);
    SaveLayout L;
    L.lu = c.take<double>((size_t)n_nodes * kmax * kmax);
    L.z = c.take<double>((size_t)n_nodes * kmax);
    L.s = c.take<double>((size_t)n_nodes);
    L.perm = c.take<uint8_t>((size_t)n_nodes * kmax);
    L.bytes = c.bytes();
    return L;
}

struct OrderWs {
    int32_t *counts;
    int32_t *queue;  // work queue of the persistent batch launch
    int32_t *lists;
    int32_t *fb_count;  // mixed precision: stencils sent to the FP64 path
    int32_t *fb_list;
    double *scratch;
    size_t bytes;
};

// order lists when has_order; the mixed-precision scratch and fallback list
// when mixed (scratch sized for the largest standard class)
OrderWs carve_order(void *base, int64_t n_nodes, bool has_order, bool mixed) {
    Carver c(base);
    OrderWs o = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0};
    o.counts = c.take<int32_t>(64);
    o.queue = c.take<int32_t>(64);
    if (has_order) o.lists = c.take<int32_t>((size_t)3 * n_nodes);
    if (mixed) {
        o.fb_count = c.take<int32_t>(64);
        o.fb_list = c.take<int32_t>((size_t)n_nodes);
        size_t sb = 0;
        for (int q = 0; q < 3; ++q) sb = mixed_scratch(q, n_nodes) > sb ? mixed_scratch(q, n_nodes) : sb;
        o.scratch = c.take<double>(sb / sizeof(double) + 1);
    }
    o.bytes = c.bytes();
    return o;
}

bool valid_m(int m) { return m == 2 || m == 4 || m == 6; }

}  // namespace

// The bucketing above for the operator batch: counts [3] must be zero.
int bucket_orders(const int8_t *order, int64_t n_nodes, int32_t k_stride, int32_t *counts,
                  int32_t *lists, double *w, int32_t *status, hipStream_t s) {
    hipLaunchKernelGGL(bucket_by_order, dim3((unsigned)ceil_div(n_nodes, kThreads)),
                       dim3(kThreads), 0, s, order, n_nodes, k_stride, counts, lists, w, status);
    return last_launch_rc();
}
}  // namespace rbffd

using namespace rbffd;

extern "C" const char *rbffd_error_string(int code) {
    switch (code) {
    case RBFFD_SUCCESS: return "success / RBFFD_OK";
    case RBFFD_ERR_ARG: return "invalid argument";
    case RBFFD_ERR_WORKSPACE: return "workspace missing or too small";
    case RBFFD_ERR_UNSUPPORTED: return "unsupported configuration";
    case RBFFD_ERR_TOO_LARGE: return "input exceeds the fixed scratch of a no-allocation call";
    case RBFFD_SINGULAR: return "stencil: zero pivot (singular system)";
    case RBFFD_FELL_BACK_FP64: return "stencil: mixed precision fell back to FP64";
    case RBFFD_NONFINITE: return "stencil: non-finite coordinate, pivot or solution";
    case RBFFD_BAD_INDEX: return "stencil: support index out of range";
    case RBFFD_DUPLICATE: return "stencil: coincident support nodes";
    case RBFFD_BAD_ORDER: return "stencil: order not in {2,4,6}";
    default: break;
    }
    if (code <= RBFFD_ERR_HIP) return "HIP runtime error (RBFFD_ERR_HIP - hipError_t)";
    return "unknown code";
}

extern "C" int rbffd_version(void) { return 100; }

extern "C" int rbffd_weights_workspace_size(int64_t n_nodes, int32_t has_order, int32_t precision,
                                            size_t *bytes) {
    if (!bytes || n_nodes < 1 || (precision != RBFFD_FP64 && precision != RBFFD_MIXED))
        return RBFFD_ERR_ARG;
    *bytes = carve_order(nullptr, n_nodes, has_order != 0, precision == RBFFD_MIXED).bytes;
    return RBFFD_SUCCESS;
}

extern "C" int rbffd_weights_save_size(int64_t n_nodes, int32_t kmax, size_t *bytes) {
    if (!bytes || n_nodes < 1 || kmax < 1 || kmax > 96) return RBFFD_ERR_ARG;
    *bytes = carve_save(nullptr, n_nodes, kmax).bytes;
    return RBFFD_SUCCESS;
}

extern "C" int rbffd_weights(const double *x, const double *y, int64_t n_nodes,
                             const int32_t *nbr, int32_t k_stride, const int8_t *order, int32_t m,
                             int32_t n, const int32_t *n_for_order, int32_t precision, double *w,
                             int32_t *status, int32_t *refine_steps, void *save, size_t save_bytes,
                             void *workspace, size_t workspace_bytes, void *stream) {
    if (!x || !y || !nbr || !w || n_nodes < 1 || n_nodes >= INT32_MAX || k_stride < 1)
        return RBFFD_ERR_ARG;
    if (precision != RBFFD_FP64 && precision != RBFFD_MIXED) return RBFFD_ERR_ARG;
    const bool mixed = precision == RBFFD_MIXED;
    int ms[3], ns[3], nclass;
    if (order) {
        if (!n_for_order) return RBFFD_ERR_ARG;
        nclass = 3;
        for (int q = 0; q < 3; ++q) {
            ms[q] = 2 * q + 2;
            ns[q] = n_for_order[q];
        }
    } else {
        nclass = 1;
        ms[0] = m;
        ns[0] = n;
    }
    int kmax = 0;
    for (int q = 0; q < nclass; ++q) {
        if (!valid_m(ms[q]) || ns[q] < n_monomials(ms[q]) || ns[q] > k_stride)
            return RBFFD_ERR_ARG;
        const int K = ns[q] + n_monomials(ms[q]);
        if (K > 96) return RBFFD_ERR_UNSUPPORTED;
        kmax = K > kmax ? K : kmax;
    }
    if (mixed) {
        if (save) return RBFFD_ERR_ARG;  // the adjoint uses FP64 factors
        for (int q = 0; q < nclass; ++q)
            if (mixed_class(ms[q], ns[q]) < 0) return RBFFD_ERR_UNSUPPORTED;
    }
    SaveLayout sv = {nullptr, nullptr, nullptr, nullptr, 0};
    if (save) {
        sv = carve_save(nullptr, n_nodes, kmax);
        if (save_bytes < sv.bytes) return RBFFD_ERR_WORKSPACE;
        sv = carve_save(save, n_nodes, kmax);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!order && !mixed)
        return weights_fp64_class(x, y, n_nodes, nbr, k_stride, nullptr, nullptr, n_nodes, n, m, w,
                                  status, sv.lu, sv.z, sv.s, sv.perm, kmax, RBFFD_OK, s);
    OrderWs ow = carve_order(nullptr, n_nodes, order != nullptr, mixed);
    if (!workspace || workspace_bytes < ow.bytes) return RBFFD_ERR_WORKSPACE;
    ow = carve_order(workspace, n_nodes, order != nullptr, mixed);
    int rc;
    if (order) {
        if ((rc = fill_i32(ow.counts, 0, 64, s))) return rc;
        hipLaunchKernelGGL(bucket_by_order, dim3((unsigned)ceil_div(n_nodes, kThreads)),
                           dim3(kThreads), 0, s, order, n_nodes, k_stride, ow.counts, ow.lists, w,
                           status);
        if ((rc = last_launch_rc())) return rc;
    }
    // the standard mixed-order batch: one persistent launch over all classes
    if (order && !mixed && mixed_class(ms[0], ns[0]) == 0 && mixed_class(ms[1], ns[1]) == 1 &&
        mixed_class(ms[2], ns[2]) == 2)
        return weights_fp64_batch(x, y, n_nodes, nbr, k_stride, ow.lists, ow.counts, ow.queue, w,
                                  status, sv.lu, sv.z, sv.s, sv.perm, kmax, s);
    // otherwise one launch per class, largest systems first
    for (int q = nclass - 1; q >= 0; --q) {
        const int32_t *rows = order ? ow.lists + (int64_t)q * n_nodes : nullptr;
        const int32_t *cnt = order ? ow.counts + q : nullptr;
        if (!mixed) {
            rc = weights_fp64_class(x, y, n_nodes, nbr, k_stride, rows, cnt, n_nodes, ns[q], ms[q],
                                    w, status, sv.lu, sv.z, sv.s, sv.perm, kmax, RBFFD_OK, s);
            if (rc) return rc;
            continue;
        }
        // mixed: FP32 factorisation + FP64 refinement, then the FP64 kernel on
        // the stencils it could not refine
        if ((rc = fill_i32(ow.fb_count, 0, 1, s))) return rc;
        rc = mixed_run(mixed_class(ms[q], ns[q]), x, y, n_nodes, nbr, k_stride, rows, cnt, n_nodes,
                       w, status, refine_steps, ow.scratch, ow.fb_count, ow.fb_list, s);
        if (rc) return rc;
        rc = weights_fp64_class(x, y, n_nodes, nbr, k_stride, ow.fb_list, ow.fb_count, n_nodes,
                                ns[q], ms[q], w, status, nullptr, nullptr, nullptr, nullptr, 0,
                                RBFFD_FELL_BACK_FP64, s);
        if (rc) return rc;
    }
    return RBFFD_SUCCESS;
}
