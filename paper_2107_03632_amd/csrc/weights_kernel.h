#pragma once
// RBF-FD Laplacian stencil weights, FP64, one stencil per lane group.
//
// Method (paper eq. (1), sections I, II, V): for node x_i with support
// {x_idx_k}, k < n, solve the augmented PHS r^3 + monomial system
// [A P; P^T 0] z = [9|u_k| ; lap p_j(0)] on the shifted, scaled offsets
// u_k = (x_idx_k - x_i) / s, s = max_k |x_idx_k - x_i|, and return
// w_k = z_k / s^2.
//
// Layout on the GPU (gfx950, wave64):
//   * A group of G lanes (32, 64 or 128) owns one stencil; lane r owns row r
//     of the augmented matrix [M | rhs], held in registers (a[0..KP), yv).
//     K = n + M(m) real rows; rows K..KP-1 are identity padding, which leaves
//     every operation on the real rows unchanged.
//   * Partial pivoting is logical: rows stay in their lanes and carry their
//     current position `pos`.  Column c's pivot is the active row with the
//     largest |a[c]|, ties to the lowest position -- exactly the row a
//     physical row-swapping elimination would pick.  The search is a
//     butterfly over (|a| high word, |a| low word, position) keys.
//   * The pivot row is broadcast through LDS (double-buffered by step parity,
//     so one barrier per step), and every other active lane applies
//     l = a[c] * (1/pivot), a[q] = fma(-l, u[q], a[q]) to its own row.
//   * Back substitution walks the columns from the last, one LDS broadcast of
//     z_c per step.  Each lane ends with z at its position.
// The sequence of IEEE operations equals that of the FP64 reference
// definition (same divisions, square roots, products and fused updates in the
// same order), so results agree to the last bit where the compiler keeps
// that order (no contraction: built with -ffp-contract=off).

#include "common.h"

namespace rbffd {
namespace wk {

// per-lane flags, OR-reduced over the group at the end
constexpr uint32_t F_BADIDX = 1u;
constexpr uint32_t F_NONFIN = 2u;
constexpr uint32_t F_DUP = 4u;
constexpr uint32_t F_ZBAD = 8u;
// LU failures (first failing column only)
constexpr uint32_t L_SING = 1u;
constexpr uint32_t L_NONFIN = 2u;

// graded monomial order: j -> (a, b) with p_j = x^a y^b
__host__ __device__ constexpr int mono_deg(int j) {
    int d = 0;
    while ((d + 1) * (d + 2) / 2 <= j) ++d;
    return d;
}
__host__ __device__ constexpr int mono_b(int j) { return j - mono_deg(j) * (mono_deg(j) + 1) / 2; }
__host__ __device__ constexpr int mono_a(int j) { return mono_deg(j) - mono_b(j); }

// u^a by repeated multiplication starting from 1
__device__ __forceinline__ double rep_pow(double u, int a) {
    double p = 1.0;
    for (int t = 0; t < a; ++t) p = p * u;
    return p;
}

template <int W>
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, W));
    return v;
}

template <int W>
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v |= (uint32_t)__shfl_xor((int)v, o, W);
    return v;
}

// key (hi, lo, pos): larger |value| first, then lower position
__device__ __forceinline__ bool key_better(uint32_t h1, uint32_t l1, int p1, uint32_t h2,
                                           uint32_t l2, int p2) {
    return h1 > h2 || (h1 == h2 && (l1 > l2 || (l1 == l2 && p1 < p2)));
}

template <int W>
__device__ __forceinline__ void wave_argmax(uint32_t &kh, uint32_t &kl, int &kp) {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) {
        uint32_t oh = (uint32_t)__shfl_xor((int)kh, o, W);
        uint32_t ol = (uint32_t)__shfl_xor((int)kl, o, W);
        int op = __shfl_xor(kp, o, W);
        if (key_better(oh, ol, op, kh, kl, kp)) {
            kh = oh;
            kl = ol;
            kp = op;
        }
    }
}

__host__ __device__ constexpr int block_threads(int G) { return G < kWave ? kWave : G; }

template <int KP, int G>
struct Shape {
    static constexpr int kBlock = G < kWave ? kWave : G;  // threads per block
    static constexpr int kGroups = kBlock / G;            // stencils per block
    static constexpr int kW = G < kWave ? G : kWave;      // group lanes per wave
    static constexpr int kNW = G / kW;                    // waves per group
    static_assert(KP <= G, "one row per lane");
};

template <int KP, int G, int NFIX, int MFIX>
__global__ __launch_bounds__(block_threads(G)) void weights_fp64_kernel(
    const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
    const int32_t *__restrict__ nbr, int32_t k_stride, const int32_t *__restrict__ rows,
    const int32_t *__restrict__ n_rows_dev, int64_t n_rows, int32_t n_arg, int32_t m_arg,
    double *__restrict__ w, int32_t *__restrict__ status, double *__restrict__ sv_lu,
    double *__restrict__ sv_z, double *__restrict__ sv_s, uint8_t *__restrict__ sv_perm,
    int32_t sv_kmax) {
    using S = Shape<KP, G>;
    constexpr int GPB = S::kGroups;
    constexpr int W = S::kW;
    constexpr int NW = S::kNW;
    const int n = NFIX ? NFIX : n_arg;
    const int m = MFIX ? MFIX : m_arg;
    const int K = n + (m + 1) * (m + 2) / 2;

    __shared__ double s_ux[GPB][KP];
    __shared__ double s_uy[GPB][KP];
    __shared__ double s_row[2][GPB][NW][KP + 1];
    __shared__ uint32_t s_key[2][GPB][NW][4];
    __shared__ double s_z[GPB][KP];
    __shared__ double s_red[GPB][NW];
    __shared__ uint32_t s_flg[GPB][NW];

    const int tid = threadIdx.x;
    const int g = tid / G;
    const int r = tid % G;              // row owned by this lane
    const int wv = (tid % G) / W;       // wave of the group this lane sits in
    const bool wave_leader = (tid % W) == 0;
    if (n_rows_dev) n_rows = *n_rows_dev;
    if ((int64_t)blockIdx.x * GPB >= n_rows) return;  // whole block idle: no barrier reached
    const int64_t t = (int64_t)blockIdx.x * GPB + g;
    const bool valid = t < n_rows;
    const int64_t i = valid ? (rows ? (int64_t)rows[t] : t) : 0;

    // ---- shift: offsets of the support nodes, scale s --------------------
    uint32_t flags = 0;
    double dx = 0.0, dy = 0.0, d2 = 0.0;
    const double xi = x[i], yi = y[i];
    if (valid && r < n) {
        const int32_t j = nbr[i * (int64_t)k_stride + r];
        if (j < 0 || (int64_t)j >= n_nodes) {
            flags |= F_BADIDX;
        } else {
            dx = x[j] - xi;
            dy = y[j] - yi;
            if (!isfinite(dx) || !isfinite(dy)) {
                flags |= F_NONFIN;
                dx = dy = 0.0;
            } else {
                d2 = dx * dx + dy * dy;
            }
        }
    }
    double d2max = wave_max<W>(d2);
    if constexpr (NW > 1) {
        if (wave_leader) s_red[g][wv] = d2max;
        __syncthreads();
#pragma unroll
        for (int v = 0; v < NW; ++v) d2max = fmax(d2max, s_red[g][v]);
    }
    const double s = sqrt(d2max);
    if (s == 0.0) flags |= F_DUP;

    // ---- scale -----------------------------------------------------------
    double ux = 0.0, uy = 0.0;
    if (r < n) {
        ux = dx / s;
        uy = dy / s;
        s_ux[g][r] = ux;
        s_uy[g][r] = uy;
    }
    __syncthreads();

    // ---- assemble row r of [A P; P^T 0 | rhs] ---------------------------
    double a[KP];
    double yv = 0.0;
    if (r < n) {
#pragma unroll
        for (int l = 0; l < KP; ++l) {
            if (l < n) {
                const double ex = ux - s_ux[g][l];
                const double ey = uy - s_uy[g][l];
                const double rr = ex * ex + ey * ey;
                if (l != r && rr == 0.0) flags |= F_DUP;
                a[l] = rr * sqrt(rr);
            } else if (l < K) {
                const int j = l - n;
                a[l] = rep_pow(ux, mono_a(j)) * rep_pow(uy, mono_b(j));
            } else {
                a[l] = 0.0;
            }
        }
        const double r0 = ux * ux + uy * uy;
        yv = 9.0 * sqrt(r0);
    } else if (r < K) {
        const int j = r - n;
        const int ea = mono_a(j), eb = mono_b(j);
#pragma unroll
        for (int l = 0; l < KP; ++l)
            a[l] = (l < n) ? rep_pow(s_ux[g][l], ea) * rep_pow(s_uy[g][l], eb) : 0.0;
        yv = ((ea == 2 && eb == 0) || (ea == 0 && eb == 2)) ? 2.0 : 0.0;
    } else {
#pragma unroll
        for (int l = 0; l < KP; ++l) a[l] = (l == r) ? 1.0 : 0.0;
    }

    // ---- LU with partial pivoting, right-looking, rhs carried along ------
    int pos = r;
    bool done = r >= KP;
    double myinv = 0.0;
    uint32_t luflag = 0;
#pragma unroll
    for (int c = 0; c < KP; ++c) {
        const int buf = c & 1;
        const uint64_t bits = (uint64_t)__double_as_longlong(a[c]) & 0x7fffffffffffffffull;
        uint32_t kh = done ? 0u : (uint32_t)(bits >> 32) + 1u;
        uint32_t kl = done ? 0u : (uint32_t)bits;
        int kp = done ? 0x7fffffff : pos;
        wave_argmax<W>(kh, kl, kp);
        // the wave-local winner publishes its row, the wave leader its key
        if (!done && pos == kp) {
#pragma unroll
            for (int q = c; q < KP; ++q) s_row[buf][g][wv][q] = a[q];
            s_row[buf][g][wv][KP] = yv;
        }
        if constexpr (NW > 1) {
            if (wave_leader) {
                s_key[buf][g][wv][0] = kh;
                s_key[buf][g][wv][1] = kl;
                s_key[buf][g][wv][2] = (uint32_t)kp;
            }
        }
        __syncthreads();
        int src = 0;
        if constexpr (NW > 1) {
            kh = s_key[buf][g][0][0];
            kl = s_key[buf][g][0][1];
            kp = (int)s_key[buf][g][0][2];
#pragma unroll
            for (int v = 1; v < NW; ++v) {
                const uint32_t oh = s_key[buf][g][v][0], ol = s_key[buf][g][v][1];
                const int op = (int)s_key[buf][g][v][2];
                if (key_better(oh, ol, op, kh, kl, kp)) {
                    kh = oh;
                    kl = ol;
                    kp = op;
                    src = v;
                }
            }
        }
        const double *u = s_row[buf][g][src];
        const double piv = u[c];
        const double inv = 1.0 / piv;
        if (luflag == 0) {
            if (!isfinite(piv)) luflag = L_NONFIN;
            else if (piv == 0.0) luflag = L_SING;
        }
        if (!done) {
            if (pos == kp) {
                done = true;
                myinv = inv;
                pos = c;
            } else {
                if (pos == c) pos = kp;  // the row at position c takes the pivot's place
                const double l = a[c] * inv;
                a[c] = l;
#pragma unroll
                for (int q = c + 1; q < KP; ++q) a[q] = fma(-l, u[q], a[q]);
                yv = fma(-l, u[KP], yv);
            }
        }
    }

    // ---- back substitution: z_c = y_c / U_cc, from the last column -------
    double zmine = 0.0;
#pragma unroll
    for (int c = KP - 1; c >= 0; --c) {
        if (pos == c) {
            zmine = yv * myinv;
            s_z[g][c] = zmine;
        }
        __syncthreads();
        if (pos < c) yv = fma(-a[c], s_z[g][c], yv);
    }

    // ---- status ----------------------------------------------------------
    if (pos < K && !isfinite(zmine)) flags |= F_ZBAD;
    flags = wave_or<W>(flags);
    if constexpr (NW > 1) {
        if (wave_leader) s_flg[g][wv] = flags;
        __syncthreads();
#pragma unroll
        for (int v = 0; v < NW; ++v) flags |= s_flg[g][v];
    }
    int st = RBFFD_OK;
    if (flags & F_BADIDX) st = RBFFD_BAD_INDEX;
    else if (flags & F_NONFIN) st = RBFFD_NONFINITE;
    else if (flags & F_DUP) st = RBFFD_DUPLICATE;
    else if (luflag == L_NONFIN) st = RBFFD_NONFINITE;
    else if (luflag == L_SING) st = RBFFD_SINGULAR;
    else if (flags & F_ZBAD) st = RBFFD_NONFINITE;

    if (!valid) return;
    double *wi = w + i * (int64_t)k_stride;
    if (pos < n) wi[pos] = (st == RBFFD_OK) ? zmine / (s * s) : __builtin_nan("");
    for (int q = n + r; q < k_stride; q += G) wi[q] = 0.0;
    if (r == 0 && status) status[i] = st;
    if (sv_lu && r < KP && pos < K) {
        const int64_t kk = (int64_t)sv_kmax * sv_kmax;
        double *dst = sv_lu + i * kk + (int64_t)pos * K;
#pragma unroll
        for (int q = 0; q < KP; ++q)
            if (q < K) dst[q] = a[q];
        sv_z[i * (int64_t)sv_kmax + pos] = zmine;
        sv_perm[i * (int64_t)sv_kmax + pos] = (uint8_t)r;
        if (pos == 0) sv_s[i] = s;
    }
}


struct SaveView {
    double *lu = nullptr, *z = nullptr, *s = nullptr;
    uint8_t *perm = nullptr;
    int32_t kmax = 0;
};

template <int KP, int G, int NFIX, int MFIX>
inline int launch_fp64(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev,
                int64_t n_rows, int n, int m, double *w, int32_t *status, const SaveView &sv,
                hipStream_t stream) {
    using S = Shape<KP, G>;
    if (n_rows <= 0) return RBFFD_SUCCESS;
    const int64_t blocks = ceil_div(n_rows, S::kGroups);
    if (blocks > 0x7fffffff) return RBFFD_ERR_UNSUPPORTED;
    hipLaunchKernelGGL((weights_fp64_kernel<KP, G, NFIX, MFIX>), dim3((unsigned)blocks),
                       dim3(S::kBlock), 0, stream, x, y, n_nodes, nbr, k_stride, rows,
                       n_rows_dev, n_rows, n, m, w, status, sv.lu, sv.z, sv.s, sv.perm,
                       sv.kmax);
    return last_launch_rc();
}

}  // namespace wk
}  // namespace rbffd
