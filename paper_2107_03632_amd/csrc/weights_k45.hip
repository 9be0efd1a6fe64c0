// FP64 weights kernel instance: K = 45 (m = 4, n = 30), one stencil per
// wave: the blocked LU with MFMA trailing updates (weights_mf.h; also the
// launches that save the factors for the adjoint), or, with
// RBFFD_K45_MFMA=0, one row per lane (weights_ms.h).
#include "weights_ms.h"
#include "weights_mf.h"

#ifndef RBFFD_SEG_K45
#define RBFFD_SEG_K45 64
#endif
#ifndef RBFFD_SL_K45
#define RBFFD_SL_K45 1
#endif
#ifndef RBFFD_OCC_K45
#define RBFFD_OCC_K45 4
#endif
#ifndef RBFFD_K45_MFMA
#define RBFFD_K45_MFMA 1
#endif
#ifndef RBFFD_OCC_MF45
#define RBFFD_OCC_MF45 4
#endif

namespace rbffd {
// one wavefront's LDS within a sixteenth of the CU's 160 KB: 16 per CU
static_assert(wk::mf_lds_bytes<45, 30, 4>(1) <= 160 * 1024 / 16, "K = 45 LDS per wavefront");

int weights_fp64_k45(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr, int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev, int64_t n_rows, int n, int m, double *w, int32_t *status, const wk::SaveView &sv, int32_t ok_code, hipStream_t stream) {
    if (RBFFD_K45_MFMA)
        return wk::launch_mf<45, 30, 4, 1, RBFFD_OCC_MF45>(x, y, n_nodes, nbr, k_stride, rows, n_rows_dev, n_rows, w, status, sv, ok_code, stream);
    return wk::launch_ms<45, RBFFD_SEG_K45, RBFFD_SL_K45, 30, 4, RBFFD_OCC_K45>(x, y, n_nodes, nbr, k_stride, rows, n_rows_dev, n_rows, n, m, w, status, sv, ok_code, stream);
}
}  // namespace rbffd
