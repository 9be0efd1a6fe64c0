// Calibration kernels for the benchmark's roofline: the rate at which this
// device retires plain (non-packed) vector FMAs, FP64 and FP32.  Not part of
// the rbffd library; only the benchmark loads it.
//
// Each thread runs 8 independent fma chains; with 4 wavefronts per block
// and many blocks per CU the VALU is never starved of independent work.

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

template <typename T>
__global__ __launch_bounds__(256) void fma_loop(T *__restrict__ sink, int64_t iters, T a, T b) {
    T acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = (T)(threadIdx.x % 7) * (T)1e-3 + (T)j;
#pragma unroll 4
    for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = fma(acc[j], a, b);
    }
    T s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += acc[j];
    sink[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace

// dtype 0: FP64, 1: FP32.  sink: device buffer of blocks * 256 elements of
// that type.  Flops per launch: blocks * 256 * iters * 8 * 2.
extern "C" int calib_fma_loop(int32_t dtype, int64_t iters, void *sink, int32_t blocks,
                              void *stream) {
    if (!sink || blocks < 1 || iters < 1 || (dtype != 0 && dtype != 1)) return -1;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (dtype == 0)
        hipLaunchKernelGGL(fma_loop<double>, dim3(blocks), dim3(256), 0, s,
                           reinterpret_cast<double *>(sink), iters, 0.9999999, 1e-7);
    else
        hipLaunchKernelGGL(fma_loop<float>, dim3(blocks), dim3(256), 0, s,
                           reinterpret_cast<float *>(sink), iters, 0.9999f, 1e-4f);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}
