// The explicit pseudo-time loop of section IV, eq. (3):
//   u_2(x_i) = u_1(x_i) + dt (f(x_i) + lap u_1(x_i)),  lap u_1(x_i) = sum_k w_ik u_1(x_nbr_ik),
// for interior nodes; Dirichlet nodes keep their values.  One launch per
// step, one thread per node: each thread streams its row of supports and
// weights (rows are contiguous, so a wavefront's 64 rows form one
// contiguous span) and gathers the neighbours' values, which the spatial
// order of the nodes keeps in cache.  The two buffers swap roles each step.

#include "common.h"

namespace rbffd {
namespace {

constexpr int kTL = 256;

__global__ __launch_bounds__(kTL) void explicit_step(int64_t n, const int32_t *__restrict__ nbr,
                                                      int32_t k_stride, int32_t nk,
                                                      const double *__restrict__ w,
                                                      const uint8_t *__restrict__ is_boundary,
                                                      const double *__restrict__ f, double dt,
                                                      const double *__restrict__ src,
                                                      double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * kTL + threadIdx.x;
    if (i >= n) return;
    const double ui = src[i];
    if (is_boundary && is_boundary[i]) {
        dst[i] = ui;
        return;
    }
    const int32_t *ni = nbr + i * (int64_t)k_stride;
    const double *wi = w + i * (int64_t)k_stride;
    double lap = 0.0;
    bool bad = false;
    for (int k = 0; k < nk; ++k) {
        const int32_t j = ni[k];
        const bool ok = j >= 0 && (int64_t)j < n;
        bad = bad || !ok;
        lap = fma(wi[k], src[ok ? j : 0], lap);
    }
    const double t = f[i] + lap;
    dst[i] = bad ? __builtin_nan("") : ui + dt * t;
}

__global__ __launch_bounds__(kTL) void copy_f64(int64_t n, const double *__restrict__ src,
                                                 double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * kTL + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

}  // namespace
}  // namespace rbffd

using namespace rbffd;

extern "C" int rbffd_time_steps(int64_t n_nodes, const int32_t *nbr, int32_t k_stride, int32_t n,
                                const double *w, const uint8_t *is_boundary, const double *f,
                                double dt, int64_t n_steps, double *u, double *u_work,
                                void *stream) {
    if (n_nodes < 1 || !nbr || !w || !f || !u || !u_work || n < 1 || k_stride < n ||
        n_steps < 0 || !(dt == dt) || u == u_work)
        return RBFFD_ERR_ARG;
    if (n_steps == 0) return RBFFD_SUCCESS;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t blocks = ceil_div(n_nodes, kTL);
    if (blocks > 0x7fffffff) return RBFFD_ERR_UNSUPPORTED;
    double *a = u, *b = u_work;
    for (int64_t t = 0; t < n_steps; ++t) {
        hipLaunchKernelGGL(explicit_step, dim3((unsigned)blocks), dim3(kTL), 0, s, n_nodes, nbr,
                           k_stride, n, w, is_boundary, f, dt, (const double *)a, b);
        double *c = a;
        a = b;
        b = c;
    }
    if (a != u)
        hipLaunchKernelGGL(copy_f64, dim3((unsigned)blocks), dim3(kTL), 0, s, n_nodes,
                           (const double *)a, u);
    return last_launch_rc();
}
