// The explicit pseudo-time loop of section IV, eq. (3):
//   u_2(x_i) = u_1(x_i) + dt (f(x_i) + lap u_1(x_i)),  lap u_1(x_i) = sum_k w_ik u_1(x_nbr_ik),
// for interior nodes; Dirichlet nodes keep their values.
// Once per call the first n columns of the supports and weights are copied
// to k-major order (workspace), so that every step's loads are coalesced:
// thread i reads entry k of row i at k * N + i.  One launch per step, one
// thread per node summing its row with fma in k order; the neighbours'
// values are gathered (the spatial order of the nodes keeps them in cache).
// The two value buffers swap roles each step.

#include "common.h"

namespace rbffd {
namespace {

constexpr int kTL = 256;

// k-major copies: nbrT[k * n + i] = nbr[i][k], wT likewise, k < nk
__global__ __launch_bounds__(kTL) void ell_to_kmajor(int64_t n, const int32_t *__restrict__ nbr,
                                                      int32_t k_stride, int32_t nk,
                                                      const double *__restrict__ w,
                                                      int32_t *__restrict__ nbrT,
                                                      double *__restrict__ wT) {
    const int64_t e = (int64_t)blockIdx.x * kTL + threadIdx.x;  // destination index
    if (e >= n * nk) return;
    const int64_t k = e / n, i = e - k * n;
    nbrT[e] = nbr[i * (int64_t)k_stride + k];
    wT[e] = w[i * (int64_t)k_stride + k];
}

// node i of one step: dst[i] from src
__device__ __forceinline__ void step_node(int64_t i, int64_t n, const int32_t *__restrict__ nbrT,
                                          int32_t nk, const double *__restrict__ wT,
                                          const uint8_t *__restrict__ is_boundary,
                                          const double *__restrict__ f, double dt,
                                          const double *src, double *dst) {
    const double ui = src[i];
    if (is_boundary && is_boundary[i]) {
        dst[i] = ui;
        return;
    }
    double lap = 0.0;
    bool bad = false;
    for (int k = 0; k < nk; ++k) {
        const int32_t j = nbrT[k * n + i];
        const bool ok = j >= 0 && (int64_t)j < n;
        bad = bad || !ok;
        lap = fma(wT[k * n + i], src[ok ? j : 0], lap);
    }
    const double t = f[i] + lap;
    dst[i] = bad ? __builtin_nan("") : ui + dt * t;
}

__global__ __launch_bounds__(kTL) void explicit_step(int64_t n, const int32_t *__restrict__ nbrT,
                                                      int32_t nk, const double *__restrict__ wT,
                                                      const uint8_t *__restrict__ is_boundary,
                                                      const double *__restrict__ f, double dt,
                                                      const double *__restrict__ src,
                                                      double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * kTL + threadIdx.x;
    if (i >= n) return;
    step_node(i, n, nbrT, nk, wT, is_boundary, f, dt, src, dst);
}

__global__ __launch_bounds__(kTL) void copy_f64(int64_t n, const double *__restrict__ src,
                                                 double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * kTL + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

}  // namespace
}  // namespace rbffd

using namespace rbffd;

namespace {
struct TlWs {
    int32_t *nbrT;
    double *wT;
    size_t bytes;
};
TlWs carve_tl(void *base, int64_t n_nodes, int32_t n) {
    Carver c(base);
    TlWs ws;
    ws.nbrT = c.take<int32_t>((size_t)n_nodes * n);
    ws.wT = c.take<double>((size_t)n_nodes * n);
    ws.bytes = c.bytes();
    return ws;
}
}  // namespace

extern "C" int rbffd_time_steps_workspace_size(int64_t n_nodes, int32_t n, size_t *bytes) {
    if (!bytes || n_nodes < 1 || n < 1) return RBFFD_ERR_ARG;
    *bytes = carve_tl(nullptr, n_nodes, n).bytes;
    return RBFFD_SUCCESS;
}

extern "C" int rbffd_time_steps(int64_t n_nodes, const int32_t *nbr, int32_t k_stride, int32_t n,
                                const double *w, const uint8_t *is_boundary, const double *f,
                                double dt, int64_t n_steps, double *u, double *u_work,
                                void *workspace, size_t workspace_bytes, void *stream) {
    if (n_nodes < 1 || !nbr || !w || !f || !u || !u_work || n < 1 || k_stride < n ||
        n_steps < 0 || !(dt == dt) || u == u_work || !workspace)
        return RBFFD_ERR_ARG;
    const TlWs ws = carve_tl(workspace, n_nodes, n);
    if (workspace_bytes < ws.bytes) return RBFFD_ERR_ARG;
    if (n_steps == 0) return RBFFD_SUCCESS;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t blocks = ceil_div(n_nodes, kTL);
    const int64_t tblocks = ceil_div(n_nodes * n, kTL);
    if (tblocks > 0x7fffffff) return RBFFD_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(ell_to_kmajor, dim3((unsigned)tblocks), dim3(kTL), 0, s, n_nodes, nbr,
                       k_stride, n, w, ws.nbrT, ws.wT);
    double *a = u, *b = u_work;
    for (int64_t t = 0; t < n_steps; ++t) {
        hipLaunchKernelGGL(explicit_step, dim3((unsigned)blocks), dim3(kTL), 0, s, n_nodes,
                           (const int32_t *)ws.nbrT, n, (const double *)ws.wT, is_boundary, f,
                           dt, (const double *)a, b);
        double *c = a;
        a = b;
        b = c;
    }
    if (a != u)
        hipLaunchKernelGGL(copy_f64, dim3((unsigned)blocks), dim3(kTL), 0, s, n_nodes,
                           (const double *)a, u);
    return last_launch_rc();
}
