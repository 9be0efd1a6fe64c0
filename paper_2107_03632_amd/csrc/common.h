// Internal helpers shared by the library's HIP sources (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rbffd.h"

namespace rbffd {

constexpr int kWave = 64;

// Workspace carving: 256-byte aligned sub-buffers of one caller allocation.
struct Carver {
    char *base;
    size_t used;
    explicit Carver(void *p) : base(static_cast<char *>(p)), used(0) {}
    template <typename T>
    T *take(size_t count) {
        used = (used + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
        used += count * sizeof(T);
        return p;
    }
    size_t bytes() const { return (used + 255) & ~size_t(255); }
};

inline int hip_rc(hipError_t e) { return e == hipSuccess ? RBFFD_SUCCESS : RBFFD_ERR_HIP - int(e); }

inline int last_launch_rc() { return hip_rc(hipGetLastError()); }

inline int n_monomials(int m) { return (m + 1) * (m + 2) / 2; }

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Exclusive prefix sum over n int32 or int64 values (device, stream-ordered).
// out may alias in.  Workspace from scan_workspace_elems().
size_t scan_workspace_bytes(int64_t n);
int exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, void *ws, hipStream_t s);
int exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, void *ws, hipStream_t s);
int fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);

}  // namespace rbffd
