// Dispatch of the FP64 weights kernel over its compiled instances: exact
// sizes for the standard supports (m, n) = (2, 12), (4, 30), (6, 56), and
// identity-padded systems of 32, 64 or 96 rows for any other (m, n).

#include "weights_kernel.h"

namespace rbffd {

#define RBFFD_WEIGHTS_INSTANCE(name)                                                           \
    int weights_fp64_##name(const double *x, const double *y, int64_t n_nodes,                 \
                            const int32_t *nbr, int32_t k_stride, const int32_t *rows,         \
                            const int32_t *n_rows_dev, int64_t n_rows, int n, int m, double *w, \
                            int32_t *status, const wk::SaveView &sv, int32_t ok_code, hipStream_t stream);
RBFFD_WEIGHTS_INSTANCE(k18)
RBFFD_WEIGHTS_INSTANCE(k45)
RBFFD_WEIGHTS_INSTANCE(k84)
RBFFD_WEIGHTS_INSTANCE(p32)
RBFFD_WEIGHTS_INSTANCE(p64)
RBFFD_WEIGHTS_INSTANCE(p96)
#undef RBFFD_WEIGHTS_INSTANCE

// Launch the FP64 weights kernel for one (m, n) class over n_rows stencils
// (rows == nullptr: stencil t is node t; otherwise node rows[t]; when
// n_rows_dev is given the row count is read on the device, n_rows being an
// upper bound used for the grid).  Successful stencils get status ok_code.
int weights_fp64_class(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                       int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev,
                       int64_t n_rows, int n, int m, double *w, int32_t *status,
                       double *sv_lu, double *sv_z, double *sv_s, uint8_t *sv_perm,
                       int32_t sv_kmax, int32_t ok_code, hipStream_t stream) {
    wk::SaveView sv;
    sv.lu = sv_lu;
    sv.z = sv_z;
    sv.s = sv_s;
    sv.perm = sv_perm;
    sv.kmax = sv_kmax;
    const int K = n + n_monomials(m);
#define GO(name) \
    return weights_fp64_##name(x, y, n_nodes, nbr, k_stride, rows, n_rows_dev, n_rows, n, m, w, status, sv, ok_code, stream)
    if (m == 2 && n == 12) GO(k18);
    if (m == 4 && n == 30) GO(k45);
    if (m == 6 && n == 56) GO(k84);
    if (K <= 32) GO(p32);
    if (K <= 64) GO(p64);
    if (K <= 96) GO(p96);
#undef GO
    return RBFFD_ERR_UNSUPPORTED;
}

}  // namespace rbffd
