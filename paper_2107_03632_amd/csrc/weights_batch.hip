// Mixed-order batch of FP64 stencils.
//
// The nodes have been bucketed by order (m = 2, 4, 6 -> system sizes 18, 45,
// 84).  Three forms, chosen by the tuning table: one persistent launch
// (below), one looping launch per order (class*_kernel), or one launch per
// order of the single-order kernels with a block per list entry.  In the
// persistent launch a fixed grid of 128-thread blocks pulls tiles from an
// atomic work queue, largest systems first so the long tiles start early
// and the short ones fill the tail:
//   * an order-6 tile is gpt[2] stencils, each spread over both wavefronts
//     of the block: the blocked LU with the trailing updates on the matrix
//     cores (weights_mf.h), or, when the factors are saved for the adjoint,
//     the column-split kernel (weights_cs.h);
//   * an order-4 tile gives each wavefront gpt[1] stencils (the blocked
//     LU of weights_mf.h, one stencil per wavefront; one row per lane in the
//     launch that saves factors);
//   * an order-2 tile gives each wavefront gpt[0] groups of 8 stencils
//     (8 lanes x 3 rows per stencil).
// Tile sizes and the grid size (blocks per compute unit) are runtime
// parameters chosen by the autotuner (rbffd_batch_tuning_set).
// The arithmetic is that of the per-order kernels, so the weights are the
// same bits as the single-order path.

#include <atomic>

#include "weights_cs.h"
#include "weights_mf.h"
#include "weights_ms.h"

namespace rbffd {
namespace {

#ifndef RBFFD_BATCH_OCC
#define RBFFD_BATCH_OCC 2
#endif

constexpr int kPB = 128;
// per-wavefront layouts of the K = 18 and K = 45 bodies (segment width, rows
// per lane): the same as the single-order kernels
constexpr int kSeg18 = 8, kSl18 = 3;
constexpr int kSeg45 = 64, kSl45 = 1;
constexpr int kG18 = kWave / kSeg18;  // stencils per wavefront group, K = 18
constexpr int kG45 = kWave / kSeg45;  // K = 45
// LDS of one K = 45 blocked-LU stencil (one per wavefront), 16-byte aligned
constexpr int kMf45 = (wk::mf_lds_bytes<45, 30, 4>(1) + 15) & ~15;

template <bool SAVE>
__global__ __launch_bounds__(kPB) __attribute__((amdgpu_waves_per_eu(RBFFD_BATCH_OCC))) void weights_batch_kernel(
    const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
    const int32_t *__restrict__ nbr, int32_t k_stride, const int32_t *__restrict__ lists,
    const int32_t *__restrict__ counts, int32_t *__restrict__ queue, int32_t gpt2, int32_t gpt4,
    int32_t gpt6, double *__restrict__ w, int32_t *__restrict__ status,
    double *__restrict__ sv_lu, double *__restrict__ sv_z, double *__restrict__ sv_s,
    uint8_t *__restrict__ sv_perm, int32_t sv_kmax) {
    __shared__ int32_t s_tile;
    // one LDS buffer serves whichever body the current tile runs
    constexpr int kLds0 = SAVE || wk::cs_lds_bytes<84, 6>() > wk::mf_lds_bytes<84, 56, 6>(2)
                              ? wk::cs_lds_bytes<84, 6>()
                              : wk::mf_lds_bytes<84, 56, 6>(2);
    constexpr int kLds1 = SAVE || wk::ms_lds_bytes<45, kSeg45, 4, 2>() > 2 * kMf45
                              ? wk::ms_lds_bytes<45, kSeg45, 4, 2>()
                              : 2 * kMf45;
    constexpr int kLds2 = wk::ms_lds_bytes<18, kSeg18, 2, 2>();
    constexpr int kLds = kLds0 > kLds1 ? (kLds0 > kLds2 ? kLds0 : kLds2) : (kLds1 > kLds2 ? kLds1 : kLds2);
    __shared__ __align__(16) char lds[kLds];
    const int64_t c2 = counts[0], c4 = counts[1], c6 = counts[2];
    const int64_t T6 = ceil_div(c6, gpt6);
    const int64_t T4 = ceil_div(c4, 2 * (int64_t)gpt4 * kG45);
    const int64_t T2 = ceil_div(c2, 2 * (int64_t)gpt2 * kG18);
    const int64_t total = T6 + T4 + T2;
    const int wave = threadIdx.x >> 6;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(queue, 1);
        __syncthreads();
        const int64_t tile = s_tile;
        __syncthreads();
        if (tile >= total) break;
        if (tile < T6) {
            for (int q = 0; q < gpt6; ++q) {
                if constexpr (SAVE)
                    wk::weights_cs_body<84, 56, 6, SAVE>(
                        x, y, n_nodes, nbr, k_stride, lists + 2 * n_nodes, c6, 56, 6, w, status,
                        sv_lu, sv_z, sv_s, sv_perm, sv_kmax, RBFFD_OK, tile * gpt6 + q, lds);
                else
                    wk::weights_mf_body<84, 56, 6, 2>(x, y, n_nodes, nbr, k_stride, lists + 2 * n_nodes, c6, w,
                                        status, RBFFD_OK, tile * gpt6 + q, lds);
            }
        } else if (tile < T6 + T4) {
            const int64_t base = (tile - T6) * 2 * gpt4;
            for (int q = 0; q < gpt4; ++q) {
                if constexpr (SAVE)
                    wk::weights_ms_body<45, kSeg45, kSl45, 30, 4, 2, SAVE>(
                        x, y, n_nodes, nbr, k_stride, lists + n_nodes, c4, 30, 4, w, status,
                        sv_lu, sv_z, sv_s, sv_perm, sv_kmax, RBFFD_OK, base + 2 * q + wave, wave,
                        lds);
                else
                    wk::weights_mf_body<45, 30, 4, 1>(x, y, n_nodes, nbr, k_stride,
                                                      lists + n_nodes, c4, w, status, RBFFD_OK,
                                                      base + 2 * q + wave, lds + wave * kMf45);
            }
        } else {
            const int64_t base = (tile - T6 - T4) * 2 * gpt2;
            for (int q = 0; q < gpt2; ++q)
                wk::weights_ms_body<18, kSeg18, kSl18, 12, 2, 2, SAVE>(
                    x, y, n_nodes, nbr, k_stride, lists, c2, 12, 2, w, status, sv_lu, sv_z, sv_s,
                    sv_perm, sv_kmax, RBFFD_OK, base + 2 * q + wave, wave, lds);
        }
    }
}

// ---- one persistent launch per order ---------------------------------------
// Each class runs with the block shape, occupancy and LDS of its own
// single-order kernel; a block walks the class's list with a grid stride
// (every stencil of a class costs the same, so no work queue and nothing to
// clear).  The bodies are those of the single-order kernels: same bits.

#ifndef RBFFD_BATCH_OCC84
#define RBFFD_BATCH_OCC84 2
#endif
#ifndef RBFFD_BATCH_OCC45
#define RBFFD_BATCH_OCC45 4
#endif
#ifndef RBFFD_BATCH_OCC18
#define RBFFD_BATCH_OCC18 3
#endif

__global__ __launch_bounds__(2 * kWave) __attribute__((amdgpu_waves_per_eu(RBFFD_BATCH_OCC84)))
void class84_kernel(const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
                    const int32_t *__restrict__ nbr, int32_t k_stride,
                    const int32_t *__restrict__ list, const int32_t *__restrict__ count,
                    double *__restrict__ w, int32_t *__restrict__ status) {
    __shared__ __align__(16) char lds[wk::mf_lds_bytes<84, 56, 6>(2)];
    const int64_t c = *count;
    for (int64_t t = blockIdx.x; t < c; t += gridDim.x) {
        __syncthreads();  // the previous stencil's LDS is free
        wk::weights_mf_body<84, 56, 6, 2>(x, y, n_nodes, nbr, k_stride, list, c, w, status,
                                          RBFFD_OK, t, lds);
    }
}

__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(RBFFD_BATCH_OCC45)))
void class45_kernel(const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
                    const int32_t *__restrict__ nbr, int32_t k_stride,
                    const int32_t *__restrict__ list, const int32_t *__restrict__ count,
                    double *__restrict__ w, int32_t *__restrict__ status) {
    __shared__ __align__(16) char lds[wk::mf_lds_bytes<45, 30, 4>(1)];
    const int64_t c = *count;
    for (int64_t t = blockIdx.x; t < c; t += gridDim.x) {
        wk::lds_order();  // one wavefront: its LDS accesses stay in program order
        wk::weights_mf_body<45, 30, 4, 1>(x, y, n_nodes, nbr, k_stride, list, c, w, status,
                                          RBFFD_OK, t, lds);
    }
}

__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(RBFFD_BATCH_OCC18)))
void class18_kernel(const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
                    const int32_t *__restrict__ nbr, int32_t k_stride,
                    const int32_t *__restrict__ list, const int32_t *__restrict__ count,
                    double *__restrict__ w, int32_t *__restrict__ status) {
    __shared__ __align__(16) char lds[wk::ms_lds_bytes<18, kSeg18, 2, 1>()];
    const int64_t c = *count;
    const int64_t groups = ceil_div(c, kG18);
    for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        wk::lds_order();
        wk::weights_ms_body<18, kSeg18, kSl18, 12, 2, 1, false>(
            x, y, n_nodes, nbr, k_stride, list, c, 12, 2, w, status, nullptr, nullptr, nullptr,
            nullptr, 0, RBFFD_OK, g, 0, lds);
    }
}

// the process-wide tuning table (the library's only mutable state)
std::atomic<int32_t> g_blocks_per_cu{2};
std::atomic<int32_t> g_gpt[3] = {{1}, {1}, {1}};
std::atomic<int32_t> g_per_order{0};
std::atomic<int32_t> g_order_bpc[3] = {{12}, {16}, {4}};

}  // namespace

// Persistent launch over the three standard classes (m, n) = (2,12), (4,30),
// (6,56); lists holds 3 x n_nodes node ids, counts the 3 list lengths and
// queue one int32 that this call zeroes.
int weights_fp64_batch(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                       int32_t k_stride, const int32_t *lists, const int32_t *counts,
                       int32_t *queue, double *w, int32_t *status, double *sv_lu, double *sv_z,
                       double *sv_s, uint8_t *sv_perm, int32_t sv_kmax, hipStream_t stream) {
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_rc(e);
    if (!sv_lu && g_per_order.load() == 2) {
        // one launch per order with the single-order kernels themselves:
        // one block (K = 84, 45) or one group of 8 stencils (K = 18) per
        // possible list entry, the blocks past the list's length returning
        // at once (no loop: the looping kernels above keep more values live
        // and spill)
        const int64_t N = n_nodes;
        hipLaunchKernelGGL((wk::weights_mf_kernel<84, 56, 6, 2, 2, false, 0>), dim3((unsigned)N),
                           dim3(2 * kWave), 0, stream, x, y, n_nodes, nbr, k_stride,
                           lists + 2 * N, counts + 2, N, w, status, wk::SaveView{}, RBFFD_OK);
        hipLaunchKernelGGL((wk::weights_mf_kernel<45, 30, 4, 1, 4, false, 0>), dim3((unsigned)N),
                           dim3(kWave), 0, stream, x, y, n_nodes, nbr, k_stride, lists + N,
                           counts + 1, N, w, status, wk::SaveView{}, RBFFD_OK);
        hipLaunchKernelGGL((wk::weights_ms_kernel<18, kSeg18, kSl18, 12, 2, RBFFD_BATCH_OCC18,
                                                  false, 0>),
                           dim3((unsigned)ceil_div(N, kG18)), dim3(kWave), 0, stream, x, y,
                           n_nodes, nbr, k_stride, lists, counts, N, 12, 2, w, status, nullptr,
                           nullptr, nullptr, nullptr, 0, RBFFD_OK);
        return last_launch_rc();
    }
    if (!sv_lu && g_per_order.load()) {
        // largest systems first
        const unsigned b6 = (unsigned)(g_order_bpc[2].load() * cus);
        const unsigned b4 = (unsigned)(g_order_bpc[1].load() * cus);
        const unsigned b2 = (unsigned)(g_order_bpc[0].load() * cus);
        hipLaunchKernelGGL(class84_kernel, dim3(b6), dim3(2 * kWave), 0, stream, x, y, n_nodes,
                           nbr, k_stride, lists + 2 * n_nodes, counts + 2, w, status);
        hipLaunchKernelGGL(class45_kernel, dim3(b4), dim3(kWave), 0, stream, x, y, n_nodes, nbr,
                           k_stride, lists + n_nodes, counts + 1, w, status);
        hipLaunchKernelGGL(class18_kernel, dim3(b2), dim3(kWave), 0, stream, x, y, n_nodes, nbr,
                           k_stride, lists, counts, w, status);
        return last_launch_rc();
    }
    int rc = fill_i32(queue, 0, 1, stream);
    if (rc) return rc;
    const int64_t blocks = (int64_t)g_blocks_per_cu.load() * cus;
    if (sv_lu)
        hipLaunchKernelGGL(weights_batch_kernel<true>, dim3((unsigned)blocks), dim3(kPB), 0, stream,
                           x, y, n_nodes, nbr, k_stride, lists, counts, queue, g_gpt[0].load(),
                           g_gpt[1].load(), g_gpt[2].load(), w, status, sv_lu, sv_z, sv_s, sv_perm,
                           sv_kmax);
    else
        hipLaunchKernelGGL(weights_batch_kernel<false>, dim3((unsigned)blocks), dim3(kPB), 0,
                           stream, x, y, n_nodes, nbr, k_stride, lists, counts, queue,
                           g_gpt[0].load(), g_gpt[1].load(), g_gpt[2].load(), w, status, nullptr,
                           nullptr, nullptr, nullptr, 0);
    return last_launch_rc();
}

}  // namespace rbffd

extern "C" int rbffd_batch_tuning_set(const rbffd_batch_tuning *t) {
    if (!t) {
        rbffd::g_blocks_per_cu = 2;
        for (auto &v : rbffd::g_gpt) v = 1;
        rbffd::g_per_order = 0;
        rbffd::g_order_bpc[0] = 12;
        rbffd::g_order_bpc[1] = 16;
        rbffd::g_order_bpc[2] = 4;
        return RBFFD_SUCCESS;
    }
    if (t->blocks_per_cu < 1 || t->blocks_per_cu > 64) return RBFFD_ERR_ARG;
    for (int q = 0; q < 3; ++q)
        if (t->groups_per_tile[q] < 1 || t->groups_per_tile[q] > 64 ||
            t->order_blocks_per_cu[q] < 1 || t->order_blocks_per_cu[q] > 64)
            return RBFFD_ERR_ARG;
    if (t->per_order < 0 || t->per_order > 2) return RBFFD_ERR_ARG;
    rbffd::g_blocks_per_cu = t->blocks_per_cu;
    for (int q = 0; q < 3; ++q) rbffd::g_gpt[q] = t->groups_per_tile[q];
    rbffd::g_per_order = t->per_order;
    for (int q = 0; q < 3; ++q) rbffd::g_order_bpc[q] = t->order_blocks_per_cu[q];
    return RBFFD_SUCCESS;
}

extern "C" int rbffd_batch_tuning_get(rbffd_batch_tuning *t) {
    if (!t) return RBFFD_ERR_ARG;
    t->blocks_per_cu = rbffd::g_blocks_per_cu.load();
    for (int q = 0; q < 3; ++q) t->groups_per_tile[q] = rbffd::g_gpt[q].load();
    t->per_order = rbffd::g_per_order.load();
    for (int q = 0; q < 3; ++q) t->order_blocks_per_cu[q] = rbffd::g_order_bpc[q].load();
    return RBFFD_SUCCESS;
}
