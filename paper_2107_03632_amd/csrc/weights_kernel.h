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
//   * Assembly is divergence-free: every lane evaluates the r^3 entries of
//     its row; the monomials of each support node are tabulated once in LDS
//     and read back both as the P block (support rows) and as P^T
//     (polynomial rows).
//   * Partial pivoting is logical: rows stay in their lanes and carry their
//     current position `pos`.  Column c's pivot is the active row with the
//     largest |a[c]|, ties to the lowest position -- exactly the row a
//     physical row-swapping elimination picks.  The search takes the maximum
//     of the high words of |a[c]| with a DPP row_shr/row_bcast reduction and
//     a ballot; only when that maximum is not unique does it fall back to a
//     butterfly over the full (|a|, position) key.
//   * The pivot row is broadcast through LDS (double-buffered by step
//     parity).  Every row applies l = a[c] * (1/pivot),
//     a[q] = fma(-l, u[q], a[q]); rows already pivoted use l = 0, which
//     leaves their values unchanged (up to the sign of an exact zero), so the
//     update needs no divergent branch.
//   * Back substitution walks the columns from the last; z_c is read from the
//     lane holding position c with readlane (one wave) or through LDS (a group
//     spanning two waves).
// The sequence of IEEE operations equals that of the FP64 reference
// definition (same divisions, square roots, products and fused updates in the
// same order), so the values agree exactly (no contraction: built with
// -ffp-contract=off).

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

// graded monomial order in three variables (inside a degree the x exponent
// descending, then the y exponent descending): exponents (a[j], b[j], c[j])
// of p_j = x^a y^b z^c, j < MM, as a compile-time table (indexed by
// unrolled loop counters, so every lookup folds to a constant)
template <int MM>
struct Mono3Table {
    int a[MM], b[MM], c[MM];
    constexpr Mono3Table() : a(), b(), c() {
        int t = 0;
        for (int d = 0; t < MM; ++d)
            for (int ea = d; ea >= 0 && t < MM; --ea)
                for (int eb = d - ea; eb >= 0 && t < MM; --eb, ++t) {
                    a[t] = ea;
                    b[t] = eb;
                    c[t] = d - ea - eb;
                }
    }
};

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

// full-key butterfly over the W-lane segment (the rare tie path)
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

// one DPP step of an unsigned max (lanes without a source read 0)
template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint32_t umax_dpp(uint32_t v) {
    const uint32_t o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWMASK, 0xf, true);
    return v > o ? v : o;
}

// Maximum over each W-lane segment (W = 32 or 64), returned to every lane of
// the segment.  row_shr 1/2/4/8 leave each 16-lane row's maximum in its
// last lane; row_bcast:15 folds rows pairwise (lanes 31 and 63), row_bcast:31
// folds the two halves (lane 63).
template <int W>
__device__ __forceinline__ uint32_t seg_umax(uint32_t v, int lane) {
    v = umax_dpp<0x111, 0xf>(v);  // row_shr:1
    v = umax_dpp<0x112, 0xf>(v);  // row_shr:2
    v = umax_dpp<0x114, 0xf>(v);  // row_shr:4
    v = umax_dpp<0x118, 0xf>(v);  // row_shr:8
    v = umax_dpp<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    if constexpr (W == 64) {
        v = umax_dpp<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
        return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
    } else {
        const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
        const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
        return lane < 32 ? a : b;
    }
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// First set lane of a ballot inside the caller's W-lane segment, or -1.
template <int W>
__device__ __forceinline__ int seg_first(uint64_t mask, int lane) {
    if constexpr (W == 64) {
        return mask ? __ffsll((unsigned long long)mask) - 1 : -1;
    } else {
        const uint32_t lo = (uint32_t)mask, hi = (uint32_t)(mask >> 32);
        const int a = lo ? __ffs(lo) - 1 : -1;
        const int b = hi ? __ffs(hi) + 31 : -1;
        return lane < 32 ? a : b;
    }
}

// Every W-lane segment of the ballot has at most one bit set.
template <int W>
__device__ __forceinline__ bool seg_at_most_one(uint64_t mask) {
    if constexpr (W == 64) {
        return __popcll((unsigned long long)mask) <= 1;
    } else {
        return __popc((uint32_t)mask) <= 1 && __popc((uint32_t)(mask >> 32)) <= 1;
    }
}

// readlane of an int from the segment's lane L (uniform per segment)
template <int W>
__device__ __forceinline__ int seg_read_i(int v, int L0, int L1, int lane) {
    if constexpr (W == 64) {
        return __builtin_amdgcn_readlane(v, L0);
    } else {
        const int a = __builtin_amdgcn_readlane(v, L0 < 0 ? 0 : L0);
        const int b = __builtin_amdgcn_readlane(v, L1 < 0 ? 32 : L1);
        return lane < 32 ? a : b;
    }
}

template <int W>
__device__ __forceinline__ double seg_read_d(double v, int L0, int L1, int lane) {
    if constexpr (W == 64) {
        return readlane_d(v, L0);
    } else {
        const double a = readlane_d(v, L0 < 0 ? 0 : L0);
        const double b = readlane_d(v, L1 < 0 ? 32 : L1);
        return lane < 32 ? a : b;
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
    static_assert(kW == 32 || kW == 64, "segments of 32 or 64 lanes");
};

// One block (G/64 wavefronts, or one wavefront holding 64/G groups) computes
// the stencils of block-group `grp` of the row list.
// OP: 0 the Laplacian, 1 d/dx, 2 d/dy (right-hand side and power of the scale).
template <int KP, int G, int NFIX, int MFIX, int OP = 0>
__device__ __forceinline__ void weights_fp64_body(
    const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
    const int32_t *__restrict__ nbr, int32_t k_stride, const int32_t *__restrict__ rows,
    int64_t n_rows, int32_t n_arg, int32_t m_arg, double *__restrict__ w,
    int32_t *__restrict__ status, double *__restrict__ sv_lu, double *__restrict__ sv_z,
    double *__restrict__ sv_s, uint8_t *__restrict__ sv_perm, int32_t sv_kmax, int32_t ok_code,
    int64_t grp) {
    using S = Shape<KP, G>;
    constexpr int GPB = S::kGroups;
    constexpr int W = S::kW;
    constexpr int NW = S::kNW;
    constexpr int MM = MFIX ? (MFIX + 1) * (MFIX + 2) / 2 : 28;  // monomial table width
    const int n = NFIX ? NFIX : n_arg;
    const int m = MFIX ? MFIX : m_arg;
    const int NM = (m + 1) * (m + 2) / 2;
    const int K = n + NM;

    __shared__ double s_ux[GPB][KP];
    __shared__ double s_uy[GPB][KP];
    __shared__ double s_P[GPB][KP][MM];
    __shared__ double s_row[2][GPB][NW][KP + 1];
    __shared__ uint32_t s_key[2][GPB][NW][4];
    __shared__ double s_z[GPB][KP];
    __shared__ double s_red[GPB][NW];
    __shared__ uint32_t s_flg[GPB][NW];

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int g = tid / G;
    const int r = tid % G;         // row owned by this lane
    const int wv = (tid % G) / W;  // wave of the group this lane sits in
    const bool wave_leader = (tid % W) == 0;
    if (grp * GPB >= n_rows) return;  // whole block idle: no barrier reached
    const int64_t t = grp * GPB + g;
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
    if (!isfinite(s)) flags |= F_NONFIN;  // an offset's square overflowed
    if (s == 0.0) flags |= F_DUP;

    // ---- scale; monomials of each support node ---------------------------
    const bool prow = r < n;             // support (r^3) row
    const bool qrow = r >= n && r < K;   // polynomial row
    const int jr = qrow ? r - n : 0;     // its monomial index
    double ux = 0.0, uy = 0.0;
    if (prow) {
        ux = dx / s;
        uy = dy / s;
        s_ux[g][r] = ux;
        s_uy[g][r] = uy;
        double px[7], py[7];
        px[0] = 1.0;
        py[0] = 1.0;
#pragma unroll
        for (int e = 1; e < 7; ++e) {
            px[e] = px[e - 1] * ux;
            py[e] = py[e - 1] * uy;
        }
#pragma unroll
        for (int j = 0; j < MM; ++j)
            if (j < NM) s_P[g][r][j] = px[mono_a(j)] * py[mono_b(j)];
    }
    __syncthreads();

    // ---- assemble row r of [A P; P^T 0 | rhs] ---------------------------
    double a[KP];
#pragma unroll
    for (int l = 0; l < KP; ++l) {
        if (l < n) {
            const double ex = ux - s_ux[g][l];
            const double ey = uy - s_uy[g][l];
            const double rr = ex * ex + ey * ey;
            if (prow && l != r && rr == 0.0) flags |= F_DUP;
            const double phs = rr * sqrt(rr);
            const double pt = s_P[g][l][jr];
            a[l] = prow ? phs : (qrow ? pt : 0.0);
        } else if (l < K) {
            a[l] = prow ? s_P[g][r < KP ? r : 0][l - n] : 0.0;
        } else {
            a[l] = (l == r) ? 1.0 : 0.0;
        }
    }
    double yv;
    {
        const double r0 = ux * ux + uy * uy;
        const double rb = OP == 0 ? 9.0 * sqrt(r0) : -3.0 * sqrt(r0) * (OP == 1 ? ux : uy);
        const bool one = OP == 0 ? (jr == 3 || jr == 5) : jr == OP;
        yv = prow ? rb : ((qrow && one) ? (OP == 0 ? 2.0 : 1.0) : 0.0);
    }

    // materialise the flags here: otherwise the duplicate checks sink to the
    // end of the kernel and keep every squared distance alive through the LU
    asm volatile("" : "+v"(flags));

    // ---- LU with partial pivoting, right-looking, rhs carried along ------
    int pos = r;
    bool done = r >= KP;
    double myinv = 0.0;
    uint32_t luflag = 0;
#pragma unroll
    for (int c = 0; c < KP; ++c) {
        const int buf = c & 1;
        const uint64_t bits = (uint64_t)__double_as_longlong(a[c]) & 0x7fffffffffffffffull;
        const uint32_t kh = done ? 0u : (uint32_t)(bits >> 32) + 1u;
        // winner lane of this wave's segment (uniform per segment), -1 if none
        int win;
        {
            const uint32_t mh = seg_umax<W>(kh, lane);
            const uint64_t cand = __ballot(!done && kh == mh);
            if (__builtin_expect(seg_at_most_one<W>(cand), 1)) {
                win = seg_first<W>(cand, lane);
            } else {
                uint32_t h2 = kh, l2 = done ? 0u : (uint32_t)bits;
                int p2 = done ? 0x7fffffff : pos;
                wave_argmax<W>(h2, l2, p2);
                win = seg_first<W>(__ballot(!done && pos == p2), lane);
            }
        }
        // segment winners as scalars (for readlane)
        int w0, w1;
        if constexpr (W == 64) {
            w0 = __builtin_amdgcn_readfirstlane(win);
            w1 = w0;
        } else {
            w0 = __builtin_amdgcn_readlane(win, 0);
            w1 = __builtin_amdgcn_readlane(win, 32);
        }
        const bool local_piv = (lane == win);
        if (local_piv) {
#pragma unroll
            for (int q = c; q < KP; ++q) s_row[buf][g][wv][q] = a[q];
            s_row[buf][g][wv][KP] = yv;
        }
        int kp = seg_read_i<W>(pos, w0, w1, lane);
        int src = 0;
        if constexpr (NW > 1) {
            if (wave_leader) {
                const bool any = w0 >= 0;
                s_key[buf][g][wv][0] = any ? (uint32_t)__builtin_amdgcn_readlane((int)kh, w0) : 0u;
                s_key[buf][g][wv][1] =
                    any ? (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)bits, w0) : 0u;
                s_key[buf][g][wv][2] = any ? (uint32_t)kp : 0x7fffffffu;
            }
        }
        __syncthreads();
        if constexpr (NW > 1) {
            uint32_t bh = s_key[buf][g][0][0], bl = s_key[buf][g][0][1];
            int bp = (int)s_key[buf][g][0][2];
#pragma unroll
            for (int v = 1; v < NW; ++v) {
                const uint32_t oh = s_key[buf][g][v][0], ol = s_key[buf][g][v][1];
                const int op = (int)s_key[buf][g][v][2];
                if (key_better(oh, ol, op, bh, bl, bp)) {
                    bh = oh;
                    bl = ol;
                    bp = op;
                    src = v;
                }
            }
            kp = bp;
        }
        const bool is_piv = local_piv && (wv == src);
        const double *u = s_row[buf][g][src];
        const double piv = u[c];
        const double inv = 1.0 / piv;
        if (luflag == 0) {
            if (!isfinite(piv)) luflag = L_NONFIN;
            else if (piv == 0.0) luflag = L_SING;
        }
        const bool upd = !done && !is_piv;
        const double l = upd ? a[c] * inv : 0.0;
        a[c] = upd ? l : a[c];
#pragma unroll
        for (int q = c + 1; q < KP; ++q) a[q] = fma(-l, u[q], a[q]);
        yv = fma(-l, u[KP], yv);
        // the row at position c takes the pivot's old place
        pos = is_piv ? c : ((!done && pos == c) ? kp : pos);
        myinv = is_piv ? inv : myinv;
        done = done || is_piv;
    }

    // ---- back substitution: z_c = y_c / U_cc, from the last column -------
    double zmine = 0.0;
#pragma unroll
    for (int c = KP - 1; c >= 0; --c) {
        const double zc = yv * myinv;
        double z;
        if constexpr (NW == 1) {
            const int L = seg_first<W>(__ballot(pos == c), lane);
            int L0, L1;
            if constexpr (W == 64) {
                L0 = __builtin_amdgcn_readfirstlane(L);
                L1 = L0;
            } else {
                L0 = __builtin_amdgcn_readlane(L, 0);
                L1 = __builtin_amdgcn_readlane(L, 32);
            }
            z = seg_read_d<W>(zc, L0, L1, lane);
        } else {
            if (pos == c) s_z[g][c] = zc;
            __syncthreads();
            z = s_z[g][c];
        }
        zmine = (pos == c) ? zc : zmine;
        yv = (pos < c) ? fma(-a[c], z, yv) : yv;
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
    const bool good = st == RBFFD_OK;
    const double s2 = OP == 0 ? s * s : s;  // the operator's power of the scale
    if (pos < n) wi[pos] = good ? zmine / s2 : __builtin_nan("");
    for (int q = n + r; q < k_stride; q += G) wi[q] = 0.0;
    if (r == 0 && status) status[i] = good ? ok_code : st;
    if (sv_lu) {
        // row r of the factors at row r; the position of each row in perm
        const int64_t kk = (int64_t)sv_kmax * sv_kmax;
        if (r < K) {
            double *dst = sv_lu + i * kk + (int64_t)r * K;
#pragma unroll
            for (int q = 0; q < KP; ++q)
                if (q < K) dst[q] = a[q];
        }
        if (r < KP && pos < K) {
            sv_z[i * (int64_t)sv_kmax + pos] = zmine;
            sv_perm[i * (int64_t)sv_kmax + pos] = (uint8_t)r;
            if (pos == 0) sv_s[i] = s;
        }
    }
}

// OCC: minimum waves per SIMD the register allocation must allow (0: the
// compiler's choice).
template <int KP, int G, int NFIX, int MFIX, int OCC, int OP = 0>
__global__ __launch_bounds__(block_threads(G))
__attribute__((amdgpu_waves_per_eu(OCC > 0 ? OCC : 1))) void weights_fp64_kernel(
    const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
    const int32_t *__restrict__ nbr, int32_t k_stride, const int32_t *__restrict__ rows,
    const int32_t *__restrict__ n_rows_dev, int64_t n_rows, int32_t n_arg, int32_t m_arg,
    double *__restrict__ w, int32_t *__restrict__ status, double *__restrict__ sv_lu,
    double *__restrict__ sv_z, double *__restrict__ sv_s, uint8_t *__restrict__ sv_perm,
    int32_t sv_kmax, int32_t ok_code) {
    if (n_rows_dev) n_rows = *n_rows_dev;
    weights_fp64_body<KP, G, NFIX, MFIX, OP>(x, y, n_nodes, nbr, k_stride, rows, n_rows, n_arg,
                                             m_arg, w, status, sv_lu, sv_z, sv_s, sv_perm,
                                             sv_kmax, ok_code, (int64_t)blockIdx.x);
}

struct SaveView {
    double *lu = nullptr, *z = nullptr, *s = nullptr;
    uint8_t *perm = nullptr;
    int32_t kmax = 0;
};

template <int KP, int G, int NFIX, int MFIX, int OCC = 0, int OP = 0>
inline int launch_fp64(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                       int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev,
                       int64_t n_rows, int n, int m, double *w, int32_t *status,
                       const SaveView &sv, int32_t ok_code, hipStream_t stream) {
    using S = Shape<KP, G>;
    if (n_rows <= 0) return RBFFD_SUCCESS;
    if (sv.lu && OP != 0) return RBFFD_ERR_UNSUPPORTED;  // factors: the Laplacian only
    const int64_t blocks = ceil_div(n_rows, S::kGroups);
    if (blocks > 0x7fffffff) return RBFFD_ERR_UNSUPPORTED;
    hipLaunchKernelGGL((weights_fp64_kernel<KP, G, NFIX, MFIX, OCC, OP>), dim3((unsigned)blocks),
                       dim3(S::kBlock), 0, stream, x, y, n_nodes, nbr, k_stride, rows,
                       n_rows_dev, n_rows, n, m, w, status, sv.lu, sv.z, sv.s, sv.perm,
                       sv.kmax, ok_code);
    return last_launch_rc();
}

}  // namespace wk
}  // namespace rbffd
