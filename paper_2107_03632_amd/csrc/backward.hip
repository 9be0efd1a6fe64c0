// Adjoint of the stencil weights: dL/d(x, y) of every node from G = dL/dw.
//
// For stencil i with unit-scale solution z = (w_hat, lambda) of M z = rhs
// (forward factors PM = LU saved by rbffd_weights), mu = M^{-1} [G_i / s^2; 0]
// (M is symmetric, so the saved factors solve with M^T as well), and for
// every support node k that is not node i itself
//   dL/du_k = 9 mu_k u_k/|u_k|
//           - sum_l 3 |u_k - u_l| (u_k - u_l) (mu_k w_l + mu_l w_k)
//           - sum_j grad p_j(u_k) (mu_k lambda_j + w_k mu_{n+j}),
// contributing dL/du_k / s to node idx_k and its negative to node i (the
// scale s is held fixed: w does not depend on it).
//
// Kernels:
//   1. adjoint_stencil (K <= 64): one wavefront per stencil; lane p reads
//      row p of the saved factors (pivot order) straight from memory, the
//      right-hand side and solution stay in registers, and the two
//      triangular solves walk the columns, each column's value reaching the
//      lanes by readlane (adjoint_stencil_blk for K > 64: two wavefronts,
//      the factors staged in LDS, the vector in LDS);
//      then each support lane evaluates its dL/du_k.  Per-slot
//      contributions go to contrib[i][k]; the stencil's own term (minus the
//      sum over its slots, reduced in a fixed order) to self[i].
//   2. reverse adjacency of the supports (counting sort, then each node's
//      list sorted by flat slot index) and a gather that sums, for every
//      node, its self term and the contributions of the slots naming it, in
//      that fixed order.  No floating-point atomics: results are
//      reproducible run to run.

#include "common.h"

namespace rbffd {
namespace {

constexpr int kThreads = 256;

struct BwdTable {
    int32_t n[3];
};

__device__ __forceinline__ void order_of(const int8_t *order, int m_u, int n_u, BwdTable t,
                                         int64_t i, int &m, int &n) {
    if (!order) {
        m = m_u;
        n = n_u;
        return;
    }
    m = order[i];
    // selects, not an index: a runtime index would put the table in scratch
    n = m == 2 ? t.n[0] : (m == 4 ? t.n[1] : (m == 6 ? t.n[2] : 0));
}

// graded monomial order: j -> (a, b)
__device__ __forceinline__ void mono_ab(int j, int &a, int &b) {
    int d = 0;
    while ((d + 1) * (d + 2) / 2 <= j) ++d;
    b = j - d * (d + 1) / 2;
    a = d - b;
}

__device__ __forceinline__ double rep_pow(double u, int e) {
    double p = 1.0;
    for (int t = 0; t < e; ++t) p = p * u;
    return p;
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Dynamic LDS: mu[K], z[K], ux[K], uy[K].  One wavefront (64 threads) per
// block, K <= 64: lane p takes position p, reads its saved row of the
// factors straight from memory (each element once) and keeps its entry of
// the right-hand side and of the solution in a register.
__global__ __launch_bounds__(64) void adjoint_stencil(
    const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
    const int32_t *__restrict__ nbr, int32_t k_stride, const int8_t *__restrict__ order,
    int32_t m_u, int32_t n_u, BwdTable tab, const double *__restrict__ G,
    const double *__restrict__ sv_lu, const double *__restrict__ sv_z,
    const double *__restrict__ sv_s, const uint8_t *__restrict__ sv_perm, int32_t kmax,
    const int32_t *__restrict__ status, double *__restrict__ contrib, double *__restrict__ self) {
    extern __shared__ double lds[];
    const int64_t i = blockIdx.x;
    const int tid = threadIdx.x;
    int m, n;
    order_of(order, m_u, n_u, tab, i, m, n);
    const int NM = (m + 1) * (m + 2) / 2;
    const int K = n + NM;
    const bool ok = n > 0 && (!status || status[i] == RBFFD_OK);
    double *cst = contrib + i * (int64_t)k_stride * 2;
    if (!ok) {  // failed stencil: contributes nothing
        for (int k = tid; k < k_stride; k += blockDim.x) {
            cst[2 * k] = 0.0;
            cst[2 * k + 1] = 0.0;
        }
        if (tid == 0) {
            self[2 * i] = 0.0;
            self[2 * i + 1] = 0.0;
        }
        return;
    }
    double *mu = lds;
    double *zs = mu + K;
    double *ux = zs + K;
    double *uy = ux + K;
    __shared__ double red[2][64];

    const double s = sv_s[i];
    const double s2 = s * s;
    // lane p: row p of PM = LU is the saved row perm[p]
    const double *src = sv_lu + i * (int64_t)kmax * kmax;
    const int p = tid;
    const int rp = p < K ? sv_perm[i * (int64_t)kmax + p] : 0;
    const double *rowp = src + (int64_t)rp * K;
    const double xi = x[i], yi = y[i];
    double vr = 0.0;   // (P b)_p, then the solves' entry p
    double upp = 1.0;  // U_pp
    if (p < K) {
        zs[p] = sv_z[i * (int64_t)kmax + p];
        // (P b)[p] = b[perm[p]], b = [G_i / s^2 ; 0]
        vr = (rp < n) ? G[i * (int64_t)k_stride + rp] / s2 : 0.0;
        upp = rowp[p];
        if (p < n) {
            const int32_t j = nbr[i * (int64_t)k_stride + p];
            ux[p] = (x[j] - xi) / s;
            uy[p] = (y[j] - yi) / s;
        }
    }
    __syncthreads();
    // forward substitution with unit L, column by column: v_p -= L_pc v_c
    for (int c = 0; c < K; ++c) {
        const double vc = readlane_f64(vr, c);
        if (p > c && p < K) vr = fma(-rowp[c], vc, vr);
    }
    // back substitution: mu_c = v_c * (1 / U_cc), then eliminate column c
    for (int c = K - 1; c >= 0; --c) {
        const double mc = readlane_f64(vr, c) * (1.0 / readlane_f64(upp, c));
        if (tid == 0) mu[c] = mc;
        if (p < c) vr = fma(-rowp[c], mc, vr);
    }
    __syncthreads();

    // dL/du_k for the support slots
    double sx = 0.0, sy = 0.0;
    for (int k = tid; k < k_stride; k += blockDim.x) {
        double gx = 0.0, gy = 0.0;
        if (k < n && nbr[i * (int64_t)k_stride + k] != (int32_t)i) {
            const double uxk = ux[k], uyk = uy[k], mk = mu[k], wk = zs[k];
            const double rk = sqrt(uxk * uxk + uyk * uyk);
            if (rk > 0.0) {
                gx += 9.0 * mk * uxk / rk;
                gy += 9.0 * mk * uyk / rk;
            }
            for (int l = 0; l < n; ++l) {
                const double ex = uxk - ux[l];
                const double ey = uyk - uy[l];
                const double r = sqrt(ex * ex + ey * ey);
                const double c = 3.0 * r * (mk * zs[l] + mu[l] * wk);
                gx -= c * ex;
                gy -= c * ey;
            }
            for (int j = 0; j < NM; ++j) {
                int a, b;
                mono_ab(j, a, b);
                double dpx = 0.0, dpy = 0.0;
                if (a > 0) dpx = (double)a * rep_pow(uxk, a - 1) * rep_pow(uyk, b);
                if (b > 0) dpy = (double)b * rep_pow(uxk, a) * rep_pow(uyk, b - 1);
                const double c = mk * zs[n + j] + wk * mu[n + j];
                gx -= dpx * c;
                gy -= dpy * c;
            }
            gx /= s;
            gy /= s;
        }
        cst[2 * k] = gx;
        cst[2 * k + 1] = gy;
        sx += gx;
        sy += gy;
    }
    // self term: minus the sum over the slots, reduced in a fixed order
    red[0][tid] = sx;
    red[1][tid] = sy;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (tid < o) {
            red[0][tid] += red[0][tid + o];
            red[1][tid] += red[1][tid + o];
        }
        __syncthreads();
    }
    if (tid == 0) {
        self[2 * i] = -red[0][0];
        self[2 * i + 1] = -red[1][0];
    }
}

// The same for K > 64 with 128 threads (two wavefronts, so that a system of
// K = 84 whose 59 KB of LDS allow two blocks per CU still has four
// wavefronts there): the solves run through v[] in LDS with a block barrier
// per column.  Same operations in the same order, so the same bits.
// Dynamic LDS: A[K][K] (saved factors), then v[K], mu[K], z[K], ux[K], uy[K].
__global__ __launch_bounds__(128) void adjoint_stencil_blk(
    const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
    const int32_t *__restrict__ nbr, int32_t k_stride, const int8_t *__restrict__ order,
    int32_t m_u, int32_t n_u, BwdTable tab, const double *__restrict__ G,
    const double *__restrict__ sv_lu, const double *__restrict__ sv_z,
    const double *__restrict__ sv_s, const uint8_t *__restrict__ sv_perm, int32_t kmax,
    const int32_t *__restrict__ status, double *__restrict__ contrib, double *__restrict__ self) {
    extern __shared__ double lds[];
    const int64_t i = blockIdx.x;
    const int tid = threadIdx.x;
    int m, n;
    order_of(order, m_u, n_u, tab, i, m, n);
    const int NM = (m + 1) * (m + 2) / 2;
    const int K = n + NM;
    const bool ok = n > 0 && (!status || status[i] == RBFFD_OK);
    double *cst = contrib + i * (int64_t)k_stride * 2;
    if (!ok) {  // failed stencil: contributes nothing
        for (int k = tid; k < k_stride; k += blockDim.x) {
            cst[2 * k] = 0.0;
            cst[2 * k + 1] = 0.0;
        }
        if (tid == 0) {
            self[2 * i] = 0.0;
            self[2 * i + 1] = 0.0;
        }
        return;
    }
    double *A = lds;
    double *v = A + K * K;
    double *mu = v + K;
    double *zs = mu + K;
    double *ux = zs + K;
    double *uy = ux + K;
    __shared__ double red[2][128];

    const double s = sv_s[i];
    const double s2 = s * s;
    // the factors in pivot order: the saved row perm[p] is row p of PM = LU
    // (the row index of each position through LDS, then one flat copy)
    const double *src = sv_lu + i * (int64_t)kmax * kmax;
    __shared__ int32_t s_perm[128];
    for (int p = tid; p < K; p += blockDim.x) s_perm[p] = sv_perm[i * (int64_t)kmax + p];
    __syncthreads();
    for (int e = tid; e < K * K; e += blockDim.x) {
        const int p = e / K, q = e - p * K;
        A[e] = src[(int64_t)s_perm[p] * K + q];
    }
    const double xi = x[i], yi = y[i];
    for (int p = tid; p < K; p += blockDim.x) {
        zs[p] = sv_z[i * (int64_t)kmax + p];
        // (P b)[p] = b[perm[p]], b = [G_i / s^2 ; 0]
        const int r = sv_perm[i * (int64_t)kmax + p];
        v[p] = (r < n) ? G[i * (int64_t)k_stride + r] / s2 : 0.0;
        if (p < n) {
            const int32_t j = nbr[i * (int64_t)k_stride + p];
            ux[p] = (x[j] - xi) / s;
            uy[p] = (y[j] - yi) / s;
        }
    }
    __syncthreads();
    // forward substitution with unit L, column by column
    for (int c = 0; c < K; ++c) {
        const double vc = v[c];
        for (int p = c + 1 + tid; p < K; p += blockDim.x) v[p] = fma(-A[p * K + c], vc, v[p]);
        __syncthreads();
    }
    // back substitution: mu_c = v_c * (1 / U_cc), then eliminate column c
    for (int c = K - 1; c >= 0; --c) {
        if (tid == 0) mu[c] = v[c] * (1.0 / A[c * K + c]);
        __syncthreads();
        const double mc = mu[c];
        for (int p = tid; p < c; p += blockDim.x) v[p] = fma(-A[p * K + c], mc, v[p]);
        __syncthreads();
    }

    // dL/du_k for the support slots
    double sx = 0.0, sy = 0.0;
    for (int k = tid; k < k_stride; k += blockDim.x) {
        double gx = 0.0, gy = 0.0;
        if (k < n && nbr[i * (int64_t)k_stride + k] != (int32_t)i) {
            const double uxk = ux[k], uyk = uy[k], mk = mu[k], wk = zs[k];
            const double rk = sqrt(uxk * uxk + uyk * uyk);
            if (rk > 0.0) {
                gx += 9.0 * mk * uxk / rk;
                gy += 9.0 * mk * uyk / rk;
            }
            for (int l = 0; l < n; ++l) {
                const double ex = uxk - ux[l];
                const double ey = uyk - uy[l];
                const double r = sqrt(ex * ex + ey * ey);
                const double c = 3.0 * r * (mk * zs[l] + mu[l] * wk);
                gx -= c * ex;
                gy -= c * ey;
            }
            for (int j = 0; j < NM; ++j) {
                int a, b;
                mono_ab(j, a, b);
                double dpx = 0.0, dpy = 0.0;
                if (a > 0) dpx = (double)a * rep_pow(uxk, a - 1) * rep_pow(uyk, b);
                if (b > 0) dpy = (double)b * rep_pow(uxk, a) * rep_pow(uyk, b - 1);
                const double c = mk * zs[n + j] + wk * mu[n + j];
                gx -= dpx * c;
                gy -= dpy * c;
            }
            gx /= s;
            gy /= s;
        }
        cst[2 * k] = gx;
        cst[2 * k + 1] = gy;
        sx += gx;
        sy += gy;
    }
    // self term: minus the sum over the slots, reduced in a fixed order
    red[0][tid] = sx;
    red[1][tid] = sy;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (tid < o) {
            red[0][tid] += red[0][tid + o];
            red[1][tid] += red[1][tid + o];
        }
        __syncthreads();
    }
    if (tid == 0) {
        self[2 * i] = -red[0][0];
        self[2 * i + 1] = -red[1][0];
    }
}

__global__ __launch_bounds__(kThreads) void rev_count(int64_t n_nodes, const int32_t *nbr,
                                                      int32_t k_stride, const int8_t *order,
                                                      int32_t m_u, int32_t n_u, BwdTable tab,
                                                      int32_t *cnt) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t i = e / k_stride;
    const int k = (int)(e - i * k_stride);
    if (i >= n_nodes) return;
    int m, n;
    order_of(order, m_u, n_u, tab, i, m, n);
    if (k >= n) return;
    const int32_t j = nbr[e];
    if (j >= 0 && (int64_t)j < n_nodes && j != (int32_t)i) atomicAdd(&cnt[j], 1);
}

__global__ __launch_bounds__(kThreads) void rev_fill(int64_t n_nodes, const int32_t *nbr,
                                                     int32_t k_stride, const int8_t *order,
                                                     int32_t m_u, int32_t n_u, BwdTable tab,
                                                     const int32_t *off, int32_t *fill,
                                                     int64_t *rev) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t i = e / k_stride;
    const int k = (int)(e - i * k_stride);
    if (i >= n_nodes) return;
    int m, n;
    order_of(order, m_u, n_u, tab, i, m, n);
    if (k >= n) return;
    const int32_t j = nbr[e];
    if (j >= 0 && (int64_t)j < n_nodes && j != (int32_t)i)
        rev[off[j] + atomicAdd(&fill[j], 1)] = e;
}

// per node: sort its slot list (fixed order), then sum self + contributions
__global__ __launch_bounds__(kThreads) void rev_gather(int64_t n_nodes, const int32_t *off,
                                                       int64_t *rev, const double *contrib,
                                                       const double *self, double *gx,
                                                       double *gy) {
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j >= n_nodes) return;
    const int64_t b = off[j], e1 = off[j + 1];
    for (int64_t p = b + 1; p < e1; ++p) {
        const int64_t v = rev[p];
        int64_t q = p - 1;
        while (q >= b && rev[q] > v) {
            rev[q + 1] = rev[q];
            --q;
        }
        rev[q + 1] = v;
    }
    double ax = self[2 * j], ay = self[2 * j + 1];
    for (int64_t p = b; p < e1; ++p) {
        const int64_t e = rev[p];
        ax += contrib[2 * e];
        ay += contrib[2 * e + 1];
    }
    gx[j] = ax;
    gy[j] = ay;
}

struct BwdWs {
    double *contrib, *self;
    int32_t *cnt, *fill;
    int64_t *rev;
    void *scan;
    size_t bytes;
};

BwdWs carve_bwd(void *base, int64_t n_nodes, int32_t k_stride) {
    Carver c(base);
    BwdWs w;
    w.contrib = c.take<double>((size_t)n_nodes * k_stride * 2);
    w.self = c.take<double>((size_t)n_nodes * 2);
    w.cnt = c.take<int32_t>(n_nodes + 1);
    w.fill = c.take<int32_t>(n_nodes + 1);
    w.rev = c.take<int64_t>((size_t)n_nodes * k_stride);
    w.scan = c.take<char>(scan_workspace_bytes(n_nodes + 1));
    w.bytes = c.bytes();
    return w;
}

struct SaveLayoutB {
    const double *lu, *z, *s;
    const uint8_t *perm;
    size_t bytes;
};

SaveLayoutB carve_save_b(const void *base, int64_t n_nodes, int32_t kmax) {
    Carver c(const_cast<void *>(base));
    SaveLayoutB L;
    L.lu = c.take<double>((size_t)n_nodes * kmax * kmax);
    L.z = c.take<double>((size_t)n_nodes * kmax);
    L.s = c.take<double>((size_t)n_nodes);
    L.perm = c.take<uint8_t>((size_t)n_nodes * kmax);
    L.bytes = c.bytes();
    return L;
}

}  // namespace
}  // namespace rbffd

using namespace rbffd;

extern "C" int rbffd_weights_backward_workspace_size(int64_t n_nodes, int32_t k_stride,
                                                     size_t *bytes) {
    if (!bytes || n_nodes < 1 || k_stride < 1) return RBFFD_ERR_ARG;
    *bytes = carve_bwd(nullptr, n_nodes, k_stride).bytes;
    return RBFFD_SUCCESS;
}

extern "C" int rbffd_weights_backward(const double *x, const double *y, int64_t n_nodes,
                                      const int32_t *nbr, int32_t k_stride, const int8_t *order,
                                      int32_t m, int32_t n, const int32_t *n_for_order,
                                      const double *grad_w, const void *save, size_t save_bytes,
                                      const int32_t *status, double *grad_x, double *grad_y,
                                      void *workspace, size_t workspace_bytes, void *stream) {
    if (!x || !y || !nbr || !grad_w || !save || !grad_x || !grad_y || n_nodes < 1 ||
        n_nodes >= INT32_MAX || k_stride < 1)
        return RBFFD_ERR_ARG;
    BwdTable tab = {{0, 0, 0}};
    int kmax = 0;
    if (order) {
        if (!n_for_order) return RBFFD_ERR_ARG;
        for (int q = 0; q < 3; ++q) {
            const int mm = 2 * q + 2;
            tab.n[q] = n_for_order[q];
            if (n_for_order[q] < n_monomials(mm) || n_for_order[q] > k_stride) return RBFFD_ERR_ARG;
            kmax = n_for_order[q] + n_monomials(mm) > kmax ? n_for_order[q] + n_monomials(mm) : kmax;
        }
    } else {
        if ((m != 2 && m != 4 && m != 6) || n < n_monomials(m) || n > k_stride) return RBFFD_ERR_ARG;
        kmax = n + n_monomials(m);
    }
    if (kmax > 96) return RBFFD_ERR_UNSUPPORTED;
    SaveLayoutB sv = carve_save_b(nullptr, n_nodes, kmax);
    if (save_bytes < sv.bytes) return RBFFD_ERR_WORKSPACE;
    sv = carve_save_b(save, n_nodes, kmax);
    BwdWs w = carve_bwd(nullptr, n_nodes, k_stride);
    if (!workspace || workspace_bytes < w.bytes) return RBFFD_ERR_WORKSPACE;
    w = carve_bwd(workspace, n_nodes, k_stride);
    hipStream_t s = static_cast<hipStream_t>(stream);

    const size_t lds = ((size_t)kmax * kmax + 5 * (size_t)kmax) * sizeof(double);
    if (lds > 65536) {  // systems above K = 88 need more than the default 64 KiB
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&adjoint_stencil_blk),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return hip_rc(e);
    }
    if (kmax <= 64)
        hipLaunchKernelGGL(adjoint_stencil, dim3((unsigned)n_nodes), dim3(64),
                           4 * (size_t)kmax * sizeof(double), s, x, y,
                           n_nodes, nbr, k_stride, order, m, n, tab, grad_w, sv.lu, sv.z, sv.s,
                           sv.perm, (int32_t)kmax, status, w.contrib, w.self);
    else
        hipLaunchKernelGGL(adjoint_stencil_blk, dim3((unsigned)n_nodes), dim3(128), lds, s, x,
                           y, n_nodes, nbr, k_stride, order, m, n, tab, grad_w, sv.lu, sv.z,
                           sv.s, sv.perm, (int32_t)kmax, status, w.contrib, w.self);
    int rc = last_launch_rc();
    if (rc) return rc;
    if ((rc = fill_i32(w.cnt, 0, n_nodes + 1, s))) return rc;
    if ((rc = fill_i32(w.fill, 0, n_nodes + 1, s))) return rc;
    const int64_t slots = n_nodes * (int64_t)k_stride;
    const unsigned sb = (unsigned)ceil_div(slots, kThreads);
    hipLaunchKernelGGL(rev_count, dim3(sb), dim3(kThreads), 0, s, n_nodes, nbr, k_stride, order, m,
                       n, tab, w.cnt);
    if ((rc = exclusive_scan_i32(w.cnt, w.cnt, n_nodes + 1, w.scan, s))) return rc;
    hipLaunchKernelGGL(rev_fill, dim3(sb), dim3(kThreads), 0, s, n_nodes, nbr, k_stride, order, m,
                       n, tab, (const int32_t *)w.cnt, w.fill, w.rev);
    hipLaunchKernelGGL(rev_gather, dim3((unsigned)ceil_div(n_nodes, kThreads)), dim3(kThreads), 0,
                       s, n_nodes, (const int32_t *)w.cnt, w.rev, (const double *)w.contrib,
                       (const double *)w.self, grad_x, grad_y);
    return last_launch_rc();
}
