// Implicit solve of the assembled operator W u = b (the Dirichlet Poisson
// system of eq. (2) with the boundary rows of section IV): BiCGSTAB
// (H. A. van der Vorst, SIAM J. Sci. Stat. Comput. 13 (1992)), without a
// preconditioner, on device-resident vectors.
//
// One iteration is five launches on the caller's stream:
//   K1  v = W p,                 partials of (r0, v)
//   K2  alpha = rho / (r0, v),   s = r - alpha v
//   K3  t = W s,                 partials of (t, s), (t, t)
//   K4  omega = (t, s) / (t, t), x += alpha p + omega s, r = s - omega t,
//                                partials of (r0, r), (r, r)
//   K5  convergence test on (r, r); rho' = (r0, r),
//       beta = (rho' / rho)(alpha / omega), p = r + beta (p - omega v)
// Dot products are reduced in two deterministic passes: each block writes
// one partial sum (fixed grid, fixed order inside the block), and every
// block of the next launch sums all partials in the same fixed order, so
// all blocks hold the same scalar and repeated solves give the same bits.
// The scalars live in device memory; a flag set by K2 (breakdown) or K5
// (converged, non-finite) makes every later launch return at once, and the
// host reads the flag only every few iterations.
//
// The SpMV gives each CSR row 16 lanes (coalesced reads of col / val), sums
// the lanes' fma chains with a fixed xor-shuffle tree, and turns a row with a
// column outside [0, n) into NaN.

#include <algorithm>

#include "common.h"

namespace rbffd {
namespace {

constexpr int kT = 256;          // threads per block
constexpr int kMaxBlocks = 1024;  // grid of every solver launch
constexpr int kRowLanes = 16;     // lanes per CSR row
constexpr int kCheckEvery = 8;    // iterations between host reads of the flag

enum : int32_t { kRunning = 0, kConverged = 1, kBreakdown = 2, kNonFinite = 3 };

struct SolveState {
    double rho[2];  // (r0, r) of the current direction, by iteration parity
    double alpha, omega, bb, rr, tol2;
    int32_t flag, iters;
};

// Sum of v over the block (kT threads), in a fixed order; every thread
// receives the result.
__device__ __forceinline__ double block_sum(double v, double *sh) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    const int wv = threadIdx.x / kWave;
    __syncthreads();  // sh may still be read by a previous call
    if ((threadIdx.x & (kWave - 1)) == 0) sh[wv] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < kT / kWave; ++k) t += sh[k];
    return t;
}

// Sum of the first n entries of part[] with stride `stride` (the same value,
// the same bits, in every block).
__device__ __forceinline__ double sum_partials(const double *part, int n, int stride, double *sh) {
    double a = 0.0;
    for (int j = threadIdx.x; j < n; j += kT) a += part[j * stride];
    return block_sum(a, sh);
}

// Row r of W times u (times D^-1 u when dinv is given), in lane 0 of the
// row's 16 lanes.
__device__ __forceinline__ double row_dot(int64_t r, int64_t n, const int64_t *__restrict__ row_ptr,
                                          const int32_t *__restrict__ col,
                                          const double *__restrict__ val,
                                          const double *__restrict__ u,
                                          const double *__restrict__ dinv, int l16) {
    double acc = 0.0;
    bool bad = false;
    const int64_t e1 = row_ptr[r + 1];
    for (int64_t e = row_ptr[r] + l16; e < e1; e += kRowLanes) {
        const int32_t c = col[e];
        const bool ok = (int64_t)c >= 0 && (int64_t)c < n;
        bad = bad || !ok;
        const int64_t cc = ok ? c : 0;
        acc = fma(val[e], dinv ? u[cc] * dinv[cc] : u[cc], acc);
    }
#pragma unroll
    for (int o = kRowLanes / 2; o > 0; o >>= 1) {
        acc += __shfl_xor(acc, o, kRowLanes);
        bad = (__shfl_xor(bad ? 1 : 0, o, kRowLanes) != 0) || bad;
    }
    return bad ? __builtin_nan("") : acc;
}

// out = W in, or sub - W in when sub is given (rows grid-stride, 16 lanes
// per row), with the block partial sums of (out, w0) - of (out, out) when w0
// is null - in partial[b * np], and with `two` also (out, out) in
// partial[b * np + 1].  out never aliases an input.
__global__ __launch_bounds__(kT) void k_spmv_dot(int64_t n, const int64_t *__restrict__ row_ptr,
                                                const int32_t *__restrict__ col,
                                                const double *__restrict__ val,
                                                const double *__restrict__ in,
                                                const double *__restrict__ sub,
                                                double *__restrict__ out,
                                                const double *__restrict__ w0, bool two,
                                                double *__restrict__ partial, int np,
                                                const SolveState *__restrict__ st,
                                                const double *__restrict__ dinv) {
    __shared__ double sh[kT / kWave];
    if (st && st->flag != kRunning) return;
    const int l16 = threadIdx.x & (kRowLanes - 1);
    double d0 = 0.0, d1 = 0.0;
    const int64_t stride = (int64_t)gridDim.x * (kT / kRowLanes);
    for (int64_t r = (int64_t)blockIdx.x * (kT / kRowLanes) + threadIdx.x / kRowLanes; r < n;
         r += stride) {
        const double y0 = row_dot(r, n, row_ptr, col, val, in, dinv, l16);
        const double y = sub ? sub[r] - y0 : y0;
        if (l16 == 0) {
            out[r] = y;
            d0 = fma(y, w0 ? w0[r] : y, d0);
            d1 = fma(y, y, d1);
        }
    }
    const double s0 = block_sum(d0, sh);
    const double s1 = two ? block_sum(d1, sh) : 0.0;
    if (threadIdx.x == 0) {
        partial[blockIdx.x * np] = s0;
        if (two) partial[blockIdx.x * np + 1] = s1;
    }
}

// Start: r0 = p = r = b - W x (already in r), (r, r) summed; block 0 sets up
// the state ((b, b) is already there).
__global__ __launch_bounds__(kT) void k_start(int64_t n, double *__restrict__ r,
                                             double *__restrict__ r0, double *__restrict__ p,
                                             const double *__restrict__ part, int nb,
                                             double tol2, SolveState *__restrict__ st) {
    __shared__ double sh[kT / kWave];
    const double rr = sum_partials(part, nb, 1, sh);  // (r, r)
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
        r0[i] = r[i];
        p[i] = r[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rho[0] = rr;
        st->rr = rr;
        st->tol2 = tol2;
        st->alpha = 0.0;
        st->omega = 0.0;
        st->iters = 0;
        st->flag = !isfinite(rr) ? kNonFinite : (rr <= tol2 * st->bb ? kConverged : kRunning);
    }
}

// (b, b) by block partials, then the norm into the state (one block).
__global__ __launch_bounds__(kT) void k_norm_b(int64_t n, const double *__restrict__ b,
                                              double *__restrict__ part) {
    __shared__ double sh[kT / kWave];
    double a = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
        a = fma(b[i], b[i], a);
    const double s = block_sum(a, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kT) void k_set_bb(const double *__restrict__ part, int nb,
                                              SolveState *__restrict__ st) {
    __shared__ double sh[kT / kWave];
    const double bb = sum_partials(part, nb, 1, sh);
    if (threadIdx.x == 0) st->bb = bb;
}

// K2: alpha, s = r - alpha v.
__global__ __launch_bounds__(kT) void k_s(int64_t n, const double *__restrict__ r,
                                         const double *__restrict__ v, double *__restrict__ s,
                                         const double *__restrict__ part, int nb, int par,
                                         SolveState *__restrict__ st) {
    __shared__ double sh[kT / kWave];
    if (st->flag != kRunning) return;
    const double r0v = sum_partials(part, nb, 1, sh);
    const double alpha = st->rho[par] / r0v;
    if (r0v == 0.0 || !isfinite(alpha)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->flag = r0v == 0.0 ? kBreakdown : kNonFinite;
        return;
    }
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
        s[i] = fma(-alpha, v[i], r[i]);
    if (blockIdx.x == 0 && threadIdx.x == 0) st->alpha = alpha;
}

// K4: omega, x += alpha p + omega s (with dinv: x += D^-1 (alpha p + omega s),
// the right-preconditioned update), r = s - omega t, partials (r0, r), (r, r).
__global__ __launch_bounds__(kT) void k_xr(int64_t n, double *__restrict__ x,
                                          const double *__restrict__ p,
                                          const double *__restrict__ s,
                                          const double *__restrict__ t, double *__restrict__ r,
                                          const double *__restrict__ r0,
                                          const double *__restrict__ part_ts, int nb,
                                          double *__restrict__ part_out,
                                          SolveState *__restrict__ st,
                                          const double *__restrict__ dinv) {
    __shared__ double sh[kT / kWave];
    if (st->flag != kRunning) return;
    const double ts = sum_partials(part_ts, nb, 2, sh);
    const double tt = sum_partials(part_ts + 1, nb, 2, sh);
    // t = 0 means s = 0 (W regular): the step along p alone solves it
    const double omega = tt == 0.0 ? 0.0 : ts / tt;
    const double alpha = st->alpha;
    double d0 = 0.0, d1 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
        if (dinv)
            x[i] = fma(omega, s[i] * dinv[i], fma(alpha, p[i] * dinv[i], x[i]));
        else
            x[i] = fma(omega, s[i], fma(alpha, p[i], x[i]));
        const double ri = fma(-omega, t[i], s[i]);
        r[i] = ri;
        d0 = fma(r0[i], ri, d0);
        d1 = fma(ri, ri, d1);
    }
    const double s0 = block_sum(d0, sh);
    const double s1 = block_sum(d1, sh);
    if (threadIdx.x == 0) {
        part_out[2 * blockIdx.x] = s0;
        part_out[2 * blockIdx.x + 1] = s1;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) st->omega = omega;
}

// K5: convergence test, then beta and p = r + beta (p - omega v).
__global__ __launch_bounds__(kT) void k_p(int64_t n, double *__restrict__ p,
                                         const double *__restrict__ r,
                                         const double *__restrict__ v,
                                         const double *__restrict__ part, int nb, int par,
                                         SolveState *__restrict__ st) {
    __shared__ double sh[kT / kWave];
    if (st->flag != kRunning) return;
    const double rho1 = sum_partials(part, nb, 2, sh);
    const double rr = sum_partials(part + 1, nb, 2, sh);
    const double omega = st->omega;
    int32_t flag = kRunning;
    if (!isfinite(rr) || !isfinite(rho1)) flag = kNonFinite;
    else if (rr <= st->tol2 * st->bb) flag = kConverged;
    else if (rho1 == 0.0 || omega == 0.0) flag = kBreakdown;
    if (flag == kRunning) {
        const double beta = (rho1 / st->rho[par]) * (st->alpha / omega);
        for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * kT)
            p[i] = fma(beta, fma(-omega, v[i], p[i]), r[i]);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rho[par ^ 1] = rho1;
        st->rr = rr;
        st->iters += 1;
        st->flag = flag;
    }
}

// Jacobi scaling: dinv[i] = 1 / W_ii (1 where the row has no non-zero
// diagonal entry; the first diagonal entry of a row counts).
__global__ __launch_bounds__(kT) void k_diag(int64_t n, const int64_t *__restrict__ row_ptr,
                                            const int32_t *__restrict__ col,
                                            const double *__restrict__ val,
                                            double *__restrict__ dinv) {
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
        double d = 0.0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            if ((int64_t)col[e] == i) {
                d = val[e];
                break;
            }
        dinv[i] = (d != 0.0 && isfinite(d)) ? 1.0 / d : 1.0;
    }
}

// the outcome into a device record (iterations, info, relative residual)
__global__ void k_report(const SolveState *__restrict__ st, const double *__restrict__ fin,
                         rbffd_solve_result *__restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int32_t flag = st->flag;
    out->iters = st->iters;
    out->info = flag == kRunning ? RBFFD_SOLVE_MAX_ITER
              : flag == kConverged ? RBFFD_SOLVE_CONVERGED
              : flag == kBreakdown ? RBFFD_SOLVE_BREAKDOWN
                                   : RBFFD_SOLVE_NONFINITE;
    out->relres = st->bb > 0.0 ? sqrt(*fin / st->bb) : sqrt(*fin);
}

// the final residual norm (b - W x, b - W x) from block partials
__global__ __launch_bounds__(kT) void k_final(const double *__restrict__ part, int nb,
                                             double *__restrict__ out) {
    __shared__ double sh[kT / kWave];
    const double v = sum_partials(part, nb, 1, sh);
    if (threadIdx.x == 0) *out = v;
}

struct Ws {
    double *r, *r0, *p, *v, *s, *t, *p1, *p3, *p4, *pf, *fin, *dinv;
    SolveState *st;
    size_t bytes;
};

Ws carve_ws(void *base, int64_t n) {
    Carver c(base);
    Ws w;
    w.r = c.take<double>(n);
    w.r0 = c.take<double>(n);
    w.p = c.take<double>(n);
    w.v = c.take<double>(n);
    w.s = c.take<double>(n);
    w.t = c.take<double>(n);
    w.p1 = c.take<double>(kMaxBlocks);
    w.p3 = c.take<double>(2 * kMaxBlocks);
    w.p4 = c.take<double>(2 * kMaxBlocks);
    w.pf = c.take<double>(2 * kMaxBlocks);
    w.fin = c.take<double>(1);
    w.st = c.take<SolveState>(1);
    w.dinv = c.take<double>(n);
    w.bytes = c.bytes();
    return w;
}

}  // namespace
}  // namespace rbffd

using namespace rbffd;

extern "C" int rbffd_solve_workspace_size(int64_t n_rows, size_t *bytes) {
    if (!bytes || n_rows < 1) return RBFFD_ERR_ARG;
    *bytes = carve_ws(nullptr, n_rows).bytes;
    return RBFFD_SUCCESS;
}

namespace rbffd {
namespace {

// The whole solve on stream s.  check_every > 0: the host reads the state
// every check_every iterations and stops enqueueing once it is final, then
// fills *host_out.  check_every == 0: all max_iter iterations are enqueued
// (each launch returns at once when the solve has ended) and the outcome
// goes to the device record dev_out; nothing waits on the host.
int solve_impl(int64_t n_rows, const int64_t *row_ptr, const int32_t *col, const double *val,
               const double *b, double *x, double rtol, int32_t max_iter, bool jacobi,
               int check_every, rbffd_solve_result *host_out, rbffd_solve_result *dev_out,
               const Ws &w, hipStream_t s) {
    const int nb = (int)std::min<int64_t>(kMaxBlocks, ceil_div(n_rows, kT / kRowLanes));
    const int nv = (int)std::min<int64_t>(kMaxBlocks, ceil_div(n_rows, kT));
    const double *dv = jacobi ? w.dinv : nullptr;
    int rc;
#define LAUNCH(...)                                  \
    do {                                             \
        hipLaunchKernelGGL(__VA_ARGS__);             \
        if ((rc = last_launch_rc()) != 0) return rc; \
    } while (0)
    if (jacobi) LAUNCH(k_diag, dim3(nv), dim3(kT), 0, s, n_rows, row_ptr, col, val, w.dinv);
    // (b, b); r = b - W x with (r, r); start
    LAUNCH(k_norm_b, dim3(nv), dim3(kT), 0, s, n_rows, b, w.p1);
    LAUNCH(k_set_bb, dim3(1), dim3(kT), 0, s, w.p1, nv, w.st);
    LAUNCH(k_spmv_dot, dim3(nb), dim3(kT), 0, s, n_rows, row_ptr, col, val, x, b, w.r,
           (const double *)nullptr, false, w.p3, 1, (const SolveState *)nullptr,
           (const double *)nullptr);
    LAUNCH(k_start, dim3(nv), dim3(kT), 0, s, n_rows, w.r, w.r0, w.p, w.p3, nb, rtol * rtol,
           w.st);
    SolveState h{};
    for (int it = 0; it < max_iter; ++it) {
        const int par = it & 1;
        LAUNCH(k_spmv_dot, dim3(nb), dim3(kT), 0, s, n_rows, row_ptr, col, val, w.p,
               (const double *)nullptr, w.v, w.r0, false, w.p1, 1, w.st, dv);
        LAUNCH(k_s, dim3(nv), dim3(kT), 0, s, n_rows, w.r, w.v, w.s, w.p1, nb, par, w.st);
        LAUNCH(k_spmv_dot, dim3(nb), dim3(kT), 0, s, n_rows, row_ptr, col, val, w.s,
               (const double *)nullptr, w.t, w.s, true, w.p3, 2, w.st, dv);
        LAUNCH(k_xr, dim3(nv), dim3(kT), 0, s, n_rows, x, w.p, w.s, w.t, w.r, w.r0, w.p3, nb,
               w.p4, w.st, dv);
        LAUNCH(k_p, dim3(nv), dim3(kT), 0, s, n_rows, w.p, w.r, w.v, w.p4, nv, par, w.st);
        if (check_every > 0 && ((it + 1) % check_every == 0 || it + 1 == max_iter)) {
            if ((rc = hip_rc(hipMemcpyAsync(&h, w.st, sizeof(h), hipMemcpyDeviceToHost, s))))
                return rc;
            if ((rc = hip_rc(hipStreamSynchronize(s)))) return rc;
            if (h.flag != kRunning) break;
        }
    }
    // the true residual b - W x of the returned x
    LAUNCH(k_spmv_dot, dim3(nb), dim3(kT), 0, s, n_rows, row_ptr, col, val, x, b, w.t,
           (const double *)nullptr, false, w.pf, 1, (const SolveState *)nullptr,
           (const double *)nullptr);
    LAUNCH(k_final, dim3(1), dim3(kT), 0, s, w.pf, nb, w.fin);
    if (dev_out) {
        LAUNCH(k_report, dim3(1), dim3(kWave), 0, s, (const SolveState *)w.st,
               (const double *)w.fin, dev_out);
        return RBFFD_SUCCESS;
    }
#undef LAUNCH
    double fin = 0.0;
    if ((rc = hip_rc(hipMemcpyAsync(&h, w.st, sizeof(h), hipMemcpyDeviceToHost, s)))) return rc;
    if ((rc = hip_rc(hipMemcpyAsync(&fin, w.fin, sizeof(fin), hipMemcpyDeviceToHost, s))))
        return rc;
    if ((rc = hip_rc(hipStreamSynchronize(s)))) return rc;
    host_out->iters = h.iters;
    host_out->relres = h.bb > 0.0 ? sqrt(fin / h.bb) : sqrt(fin);
    host_out->info = h.flag == kRunning ? RBFFD_SOLVE_MAX_ITER
                   : h.flag == kConverged ? RBFFD_SOLVE_CONVERGED
                   : h.flag == kBreakdown ? RBFFD_SOLVE_BREAKDOWN
                                          : RBFFD_SOLVE_NONFINITE;
    return RBFFD_SUCCESS;
}

}  // namespace
}  // namespace rbffd

extern "C" int rbffd_solve(int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
                           const double *val, const double *b, double *x, double rtol,
                           int32_t max_iter, int32_t *iters, double *relres, int32_t *info,
                           void *workspace, size_t workspace_bytes, void *stream) {
    if (n_rows < 1 || !row_ptr || !col || !val || !b || !x || !iters || !relres || !info)
        return RBFFD_ERR_ARG;
    if (!(rtol >= 0.0) || max_iter < 0) return RBFFD_ERR_ARG;
    const Ws w = carve_ws(workspace, n_rows);
    if (!workspace || workspace_bytes < w.bytes) return RBFFD_ERR_WORKSPACE;
    rbffd_solve_result res{};
    const int rc = solve_impl(n_rows, row_ptr, col, val, b, x, rtol, max_iter, false, kCheckEvery,
                              &res, nullptr, w, static_cast<hipStream_t>(stream));
    if (rc) return rc;
    *iters = res.iters;
    *relres = res.relres;
    *info = res.info;
    return RBFFD_SUCCESS;
}

extern "C" int rbffd_solve_async(int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
                                 const double *val, const double *b, double *x, double rtol,
                                 int32_t max_iter, int32_t precond, rbffd_solve_result *result,
                                 void *workspace, size_t workspace_bytes, void *stream) {
    if (n_rows < 1 || !row_ptr || !col || !val || !b || !x || !result) return RBFFD_ERR_ARG;
    if (!(rtol >= 0.0) || max_iter < 0) return RBFFD_ERR_ARG;
    if (precond != RBFFD_PRECOND_NONE && precond != RBFFD_PRECOND_JACOBI) return RBFFD_ERR_ARG;
    const Ws w = carve_ws(workspace, n_rows);
    if (!workspace || workspace_bytes < w.bytes) return RBFFD_ERR_WORKSPACE;
    return solve_impl(n_rows, row_ptr, col, val, b, x, rtol, max_iter,
                      precond == RBFFD_PRECOND_JACOBI, 0, nullptr, result, w,
                      static_cast<hipStream_t>(stream));
}
