// The sorted k-best list of the kNN queries (2-D and 3-D), in registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rbffd {

// Keys (d2, j) in lexicographic order; a NaN d2 precedes nothing.
__device__ __forceinline__ bool key_less(double d1, int32_t j1, double d2, int32_t j2) {
    return d1 < d2 || (d1 == d2 && j1 < j2);
}

// The k best keys, ascending, in slots KMAX - k .. KMAX - 1.  The slots below
// hold the key (-1, -1), which precedes every candidate's (d2 >= 0 or NaN),
// so nothing is ever inserted there and the current k-th key is always the
// last slot: no slot depends on k at run time.
template <int KMAX>
struct TopK {
    double d[KMAX];
    int32_t j[KMAX];

    __device__ __forceinline__ void init(int k) {
#pragma unroll
        for (int s = 0; s < KMAX; ++s) {
            const bool live = s >= KMAX - k;
            d[s] = live ? __builtin_inf() : -1.0;
            j[s] = live ? INT32_MAX : -1;
        }
    }
    __device__ __forceinline__ double wd() const { return d[KMAX - 1]; }
    __device__ __forceinline__ int32_t wj() const { return j[KMAX - 1]; }

    // insert a key known to precede the last slot; keys are unique (distinct
    // j).  The list is sorted, so the slots the key precedes form a suffix:
    // each of them takes its left neighbour, and the first takes the key.
    __device__ __forceinline__ void insert(double cd, int32_t cj) {
        bool lt[KMAX];
#pragma unroll
        for (int s = 0; s < KMAX; ++s) lt[s] = key_less(cd, cj, d[s], j[s]);
#pragma unroll
        for (int s = KMAX - 1; s > 0; --s) {
            d[s] = lt[s - 1] ? d[s - 1] : (lt[s] ? cd : d[s]);
            j[s] = lt[s - 1] ? j[s - 1] : (lt[s] ? cj : j[s]);
        }
        d[0] = lt[0] ? cd : d[0];
        j[0] = lt[0] ? cj : j[0];
    }
};

}  // namespace rbffd
