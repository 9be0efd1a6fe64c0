// Device exclusive prefix sums (int32 / int64) and a fill kernel, used to
// build the kNN cell grid, the CSR row pointers and the adjoint's reverse
// adjacency.  Three passes: per-tile scans, a single-block scan of the tile
// totals, then the tile offsets added back.

#include "common.h"

namespace rbffd {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kTile = kScanThreads * kScanItems;

template <typename T>
__device__ __forceinline__ T block_inclusive_scan(T v, T *sh) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int o = 1; o < kScanThreads; o <<= 1) {
        T add = tid >= o ? sh[tid - o] : T(0);
        __syncthreads();
        v += add;
        sh[tid] = v;
        __syncthreads();
    }
    return v;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_tiles(const T *in, T *out, int64_t n,
                                                           T *tile_sums) {
    __shared__ T sh[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kScanItems;
    T v[kScanItems];
    T run = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        const int64_t idx = base + q;
        const T a = idx < n ? in[idx] : T(0);
        v[q] = run;
        run += a;
    }
    const T incl = block_inclusive_scan<T>(run, sh);
    const T excl = incl - run;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        const int64_t idx = base + q;
        if (idx < n) out[idx] = v[q] + excl;
    }
    if (threadIdx.x == kScanThreads - 1) tile_sums[blockIdx.x] = incl;
}

// exclusive scan of the tile totals in place, one block, chunk by chunk
template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_tile_sums(T *sums, int64_t n_tiles) {
    __shared__ T sh[kScanThreads];
    T carry = 0;
    for (int64_t base = 0; base < n_tiles; base += kTile) {
        const int64_t b0 = base + (int64_t)threadIdx.x * kScanItems;
        T v[kScanItems];
        T run = 0;
#pragma unroll
        for (int q = 0; q < kScanItems; ++q) {
            const int64_t idx = b0 + q;
            const T a = idx < n_tiles ? sums[idx] : T(0);
            v[q] = run;
            run += a;
        }
        const T incl = block_inclusive_scan<T>(run, sh);
        const T excl = incl - run;
#pragma unroll
        for (int q = 0; q < kScanItems; ++q) {
            const int64_t idx = b0 + q;
            if (idx < n_tiles) sums[idx] = v[q] + excl + carry;
        }
        const T total = sh[kScanThreads - 1];
        __syncthreads();
        carry += total;
    }
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_add(T *out, int64_t n, const T *tile_offs) {
    const T off = tile_offs[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int q = threadIdx.x; q < kTile; q += kScanThreads) {
        const int64_t idx = base + q;
        if (idx < n) out[idx] += off;
    }
}

template <typename T>
int exclusive_scan(const T *in, T *out, int64_t n, void *ws, hipStream_t s) {
    if (n <= 0) return RBFFD_SUCCESS;
    const int64_t tiles = ceil_div(n, kTile);
    T *sums = static_cast<T *>(ws);
    hipLaunchKernelGGL(scan_tiles<T>, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, in, out, n,
                       sums);
    hipLaunchKernelGGL(scan_tile_sums<T>, dim3(1), dim3(kScanThreads), 0, s, sums, tiles);
    hipLaunchKernelGGL(scan_add<T>, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, out, n,
                       (const T *)sums);
    return last_launch_rc();
}

__global__ void fill_i32_kernel(int32_t *p, int32_t v, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) p[k] = v;
}

}  // namespace

size_t scan_workspace_bytes(int64_t n) {
    return (size_t)(ceil_div(n > 0 ? n : 1, kTile) + 1) * sizeof(int64_t);
}

int exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, void *ws, hipStream_t s) {
    return exclusive_scan<int32_t>(in, out, n, ws, s);
}

int exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, void *ws, hipStream_t s) {
    return exclusive_scan<int64_t>(in, out, n, ws, s);
}

int fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return RBFFD_SUCCESS;
    const int64_t blocks = ceil_div(n, 256) < 4096 ? ceil_div(n, 256) : 4096;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
    return last_launch_rc();
}

}  // namespace rbffd
