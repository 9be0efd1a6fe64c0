// Laplacian stencil weights of eq. (1) for nodes in three dimensions: the
// polyharmonic spline r^3 (lap r^3 = 12 r in 3-D) augmented with the ten
// monomials of degree <= 2 in (x, y, z), on the node's n nearest neighbours
// (10 <= n <= 54, so K = n + 10 <= 64), shifted to the node and scaled to a
// unit stencil.  m = 2, n = 20 and every m = 4 support (35 <= n <= 76) run
// the blocked LU of weights_mf.h / weights_mf2.h instead (weights3_k30.hip,
// weights3_k105_op*.hip for n = 70, weights3_m4any_op*.hip).
//
// One wavefront per stencil, one row of [A P; P^T 0 | rhs] per lane, in
// registers.  Rows never move: each lane tracks the position its row holds
// in the partially pivoted order.  Per column: the pivot is the not yet
// pivoted row with the largest |a| (ties to the lowest position), its
// entries are broadcast with readlane, the multipliers a * (1 / pivot)
// replace the column and every other live row takes fma(-l, u, a), the
// right-hand side carried along.  Back substitution runs from the last
// position to the first, multiplying by the pivot's reciprocal and
// broadcasting each solved unknown.  The operations and their order are
// those of a partial-pivoting LU followed by the two triangular solves, so
// the weights are the same doubles as a sequential evaluation of that
// definition.

#include "common.h"
#include "weights_ms.h"

namespace rbffd {
namespace {

constexpr int kMono3 = 10;   // monomials of degree <= 2 in three variables
constexpr int kWaves3 = 4;   // stencils (wavefronts) per block

enum : uint32_t { G_BADIDX = 1u, G_NONFIN = 2u, G_DUP = 4u, G_ZBAD = 8u };
enum : uint32_t { G_LU_SING = 1u, G_LU_NONFIN = 2u };

__device__ __forceinline__ double bcast_d(double v, int lane) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// reductions over one stencil's SEG lanes (each lane receives the result)
template <int SEG>
__device__ __forceinline__ uint32_t seg_max_u32(uint32_t v) {
    return wk::seg_all<SEG, wk::OpMax>(v, 0);
}

template <int SEG>
__device__ __forceinline__ uint32_t seg_or_u32(uint32_t v) {
    return wk::seg_all<SEG, wk::OpOr>(v, 0);
}

// v of lane w0 to the lanes of stencil 0, of lane w1 to those of stencil 1
template <int SEG>
__device__ __forceinline__ double bcast_seg(double v, int w0, int w1, int h) {
    const double v0 = bcast_d(v, w0);
    if constexpr (SEG == kWave) return v0;
    const double v1 = bcast_d(v, w1);
    return h ? v1 : v0;
}

// the ten monomials at (u, v, t): 1, x, y, z, x^2, xy, xz, y^2, yz, z^2
__device__ __forceinline__ double mono3(int j, double u, double v, double t) {
    switch (j) {
    case 0: return 1.0;
    case 1: return u;
    case 2: return v;
    case 3: return t;
    case 4: return u * u;
    case 5: return u * v;
    case 6: return u * t;
    case 7: return v * v;
    case 8: return v * t;
    default: return t * t;
    }
}

// SEG lanes per stencil: 64 (one stencil per wavefront, KP = 32 or 64) or
// 32 (two stencils per wavefront, KP = 32: the pivot searches, reciprocals
// and bookkeeping of one instruction then serve two stencils).
// Occupancy target: 5 wavefronts per SIMD (at most 96 VGPRs) with 32 rows,
// 3 with 64.
// OP: 0 the Laplacian, 1 d/dx, 2 d/dy, 3 d/dz (right-hand side and the
// power of the scale).
template <int KP, int SEG, int OP>
__global__ __launch_bounds__(kWave * kWaves3)
__attribute__((amdgpu_waves_per_eu(KP == 32 ? 5 : 3))) void weights3_kernel(
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
    int64_t n_nodes, const int32_t *__restrict__ nbr, int32_t k_stride, int n, int64_t n_rows,
    double *__restrict__ w, int32_t *__restrict__ status) {
    static_assert((SEG == kWave && (KP == 32 || KP == 64)) || (SEG == 32 && KP == 32),
                  "rows per stencil");
    constexpr int SPW = kWave / SEG;                            // stencils per wavefront
    constexpr uint64_t kLo = SEG == kWave ? ~0ull : 0xffffffffull;  // stencil 0's lanes
    // per stencil: the scaled offsets and monomials of the assembly
    constexpr int kAsm = 3 * KP + KP * (kMono3 + 1);
    __shared__ double s_buf[kWaves3 * SPW][kAsm];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    const int h = SEG == kWave ? 0 : lane / SEG;  // this lane's stencil in the wavefront
    const int r = lane & (SEG - 1);               // its row
    double(*s_u)[KP] = reinterpret_cast<double(*)[KP]>(&s_buf[wv * SPW + h][0]);
    double(*s_p)[kMono3 + 1] =
        reinterpret_cast<double(*)[kMono3 + 1]>(&s_buf[wv * SPW + h][3 * KP]);
    const int64_t i0 = ((int64_t)blockIdx.x * kWaves3 + wv) * SPW;
    if (i0 >= n_rows) return;  // whole wavefronts only; no block barrier below
    // a stencil past the end repeats the last one and writes nothing
    const bool live = i0 + h < n_rows;
    const int64_t i = live ? i0 + h : n_rows - 1;
    const int K = n + kMono3;

    // ---- shift and scale -------------------------------------------------
    uint32_t flags = 0;
    double dx = 0.0, dy = 0.0, dz = 0.0, d2 = 0.0;
    const double xi = x[i], yi = y[i], zi = z[i];
    if (r < n) {
        const int32_t j = nbr[i * (int64_t)k_stride + r];
        if (j < 0 || (int64_t)j >= n_nodes) {
            flags |= G_BADIDX;
        } else {
            const double ex = x[j] - xi, ey = y[j] - yi, ez = z[j] - zi;
            if (!isfinite(ex) || !isfinite(ey) || !isfinite(ez)) {
                flags |= G_NONFIN;
            } else {
                dx = ex;
                dy = ey;
                dz = ez;
                d2 = (ex * ex + ey * ey) + ez * ez;
            }
        }
    }
    // d2 >= 0 (or +inf), so its bit pattern orders like its value
    const uint64_t d2b = (uint64_t)__double_as_longlong(d2);
    const uint32_t mh = seg_max_u32<SEG>((uint32_t)(d2b >> 32));
    const uint32_t ml = seg_max_u32<SEG>((uint32_t)(d2b >> 32) == mh ? (uint32_t)d2b : 0u);
    const double sc = sqrt(__longlong_as_double((long long)(((uint64_t)mh << 32) | ml)));
    if (!isfinite(sc)) flags |= G_NONFIN;
    if (sc == 0.0) flags |= G_DUP;
    const double ux = dx / sc, uy = dy / sc, uz = dz / sc;
    if (r < KP) {
        s_u[0][r] = r < n ? ux : 0.0;
        s_u[1][r] = r < n ? uy : 0.0;
        s_u[2][r] = r < n ? uz : 0.0;
#pragma unroll
        for (int j = 0; j < kMono3; ++j) s_p[r][j] = r < n ? mono3(j, ux, uy, uz) : 0.0;
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_wave_barrier();  // one wavefront: its LDS accesses are in order
    __atomic_signal_fence(__ATOMIC_SEQ_CST);

    // ---- this lane's row ---------------------------------------------------
    const bool prow = r < n;
    const bool qrow = r >= n && r < K;
    const int jr = qrow ? r - n : 0;
    double a[KP];
    double b = 0.0;
#pragma unroll
    for (int q = 0; q < KP; ++q) {
        double v = 0.0;
        if (q < n) {
            if (prow) {
                const double ex = ux - s_u[0][q];
                const double ey = uy - s_u[1][q];
                const double ez = uz - s_u[2][q];
                const double rr = (ex * ex + ey * ey) + ez * ez;
                if (q != r && rr == 0.0) flags |= G_DUP;
                v = rr * sqrt(rr);
            } else if (qrow) {
                v = s_p[q][jr];
            }
        } else if (q < K) {
            v = prow ? s_p[r][q - n] : 0.0;
        } else if (q == r) {
            v = 1.0;  // identity padding up to KP
        }
        a[q] = v;
        // one column at a time: hoisting every column's loads would hold
        // 3 KP offsets in registers at once
        __builtin_amdgcn_sched_barrier(0);
    }
    if (prow) {
        const double r0 = (ux * ux + uy * uy) + uz * uz;
        // lap r^3 = 12 r; d/dx r^3 of node k at the centre = -3 r u_kx
        b = OP == 0 ? 12.0 * sqrt(r0)
                    : -3.0 * sqrt(r0) * (OP == 1 ? ux : (OP == 2 ? uy : uz));
    } else if (qrow) {
        // lap of x^2, y^2, z^2 (j = 4, 7, 9); d/dx x, d/dy y, d/dz z (j = OP)
        b = OP == 0 ? ((jr == 4 || jr == 7 || jr == 9) ? 2.0 : 0.0) : (jr == OP ? 1.0 : 0.0);
    }

    // ---- LU with partial pivoting, right-hand side carried along ----------
    // Rows K .. KP-1 are identity padding: they take no multiplier in the
    // first K columns (their entries there are 0, and a lower position wins
    // ties), and the real rows are all pivoted by then, so the padding
    // columns change nothing of the real solution.  Lanes past KP sit out.
    int pos = r;                // position of this lane's row
    bool done = r >= KP;        // pivoted already (or outside the system)
    double my_inv = 0.0, my_piv = 1.0;
#pragma unroll
    for (int c = 0; c < KP; ++c) {
        const uint64_t bits = (uint64_t)__double_as_longlong(a[c]) & 0x7fffffffffffffffull;
        const uint32_t kh = done ? 0u : (uint32_t)(bits >> 32) + 1u;
        const uint32_t hmax = seg_max_u32<SEG>(kh);
        uint64_t cand = __ballot(!done && kh == hmax);
        bool multi = ((cand & kLo) & ((cand & kLo) - 1ull)) != 0ull;
        if constexpr (SEG != kWave) multi = multi || ((cand >> 32) & ((cand >> 32) - 1ull)) != 0ull;
        if (multi) {
            // equal high words: the low words, then the lowest position
            const bool in = (cand >> lane) & 1ull;
            const uint32_t kl = in ? (uint32_t)bits : 0u;
            const uint32_t lmax = seg_max_u32<SEG>(kl);
            const bool in2 = in && kl == lmax;
            const uint32_t pk = in2 ? (uint32_t)(KP - pos) : 0u;
            const uint32_t pmax = seg_max_u32<SEG>(pk);
            cand = __ballot(in2 && pk == pmax);
        }
        // the pivot lane of each stencil
        const int win0 = __builtin_amdgcn_readfirstlane(__ffsll((unsigned long long)(cand & kLo)) - 1);
        const int win1 = SEG == kWave ? win0
                                      : __builtin_amdgcn_readfirstlane(
                                            32 + __ffsll((unsigned long long)(cand >> 32)) - 1);
        const int win = h ? win1 : win0;
        const int kp0 = __builtin_amdgcn_readlane(pos, win0);
        const int kp = SEG == kWave ? kp0 : (h ? __builtin_amdgcn_readlane(pos, win1) : kp0);
        const double piv = bcast_seg<SEG>(a[c], win0, win1, h);
        const double inv = 1.0 / piv;
        const bool isp = lane == win;
        my_inv = isp ? inv : my_inv;
        my_piv = isp ? piv : my_piv;
        pos = isp ? c : ((!done && pos == c) ? kp : pos);
        done = done || isp;
        // in place, as above: deferred, every column's pivot and mask would
        // stay live to the end
        int dn = done ? 1 : 0;
        asm volatile("" : "+v"(my_inv), "+v"(my_piv), "+v"(pos), "+v"(dn));
        done = dn != 0;
        const double l = done ? 0.0 : a[c] * inv;
        a[c] = done ? a[c] : l;
        asm volatile("" : "+v"(a[c]));
#pragma unroll
        for (int q = c + 1; q < KP; ++q) {
            const double u = bcast_seg<SEG>(a[q], win0, win1, h);
            const double nv = fma(-l, u, a[q]);
            a[q] = done ? a[q] : nv;
            // the select happens here: deferred to the entry's next use, it
            // would keep both values and every column's mask alive
            asm volatile("" : "+v"(a[q]));
        }
        const double ub = bcast_seg<SEG>(b, win0, win1, h);
        const double nb = fma(-l, ub, b);
        b = done ? b : nb;
        asm volatile("" : "+v"(b));
    }

    // ---- back substitution: z_c = y_c / U_cc, from the last position -------
    double zf = 0.0;
#pragma unroll
    for (int c = KP - 1; c >= 0; --c) {
        const uint64_t at = __ballot(pos == c);
        const int wl0 = __builtin_amdgcn_readfirstlane(__ffsll((unsigned long long)(at & kLo)) - 1);
        const int wl1 = SEG == kWave ? wl0
                                     : __builtin_amdgcn_readfirstlane(
                                           32 + __ffsll((unsigned long long)(at >> 32)) - 1);
        const double zc = bcast_seg<SEG>(b * my_inv, wl0, wl1, h);
        if (lane == (h ? wl1 : wl0)) zf = zc;
        if (pos < c) b = fma(-a[c], zc, b);
    }

    // ---- status and output ------------------------------------------------
    uint32_t lukey = 0;
    if (pos < K) {
        const uint32_t f = !isfinite(my_piv) ? G_LU_NONFIN : (my_piv == 0.0 ? G_LU_SING : 0u);
        if (f) lukey = ((uint32_t)(KP - pos) << 2) | f;
        if (!isfinite(zf)) flags |= G_ZBAD;
    }
    const uint32_t luflag = seg_max_u32<SEG>(lukey) & 3u;
    const uint32_t fl = seg_or_u32<SEG>(flags);
    int st = RBFFD_OK;
    if (fl & G_BADIDX) st = RBFFD_BAD_INDEX;
    else if (fl & G_NONFIN) st = RBFFD_NONFINITE;
    else if (fl & G_DUP) st = RBFFD_DUPLICATE;
    else if (luflag == G_LU_NONFIN) st = RBFFD_NONFINITE;
    else if (luflag == G_LU_SING) st = RBFFD_SINGULAR;
    else if (fl & G_ZBAD) st = RBFFD_NONFINITE;
    if (!live) return;
    const bool good = st == RBFFD_OK;
    double *wi = w + i * (int64_t)k_stride;
    const double s2 = OP == 0 ? sc * sc : sc;  // the operator's power of the scale
    if (pos < n) wi[pos] = good ? zf / s2 : __builtin_nan("");
    for (int q = n + r; q < k_stride; q += SEG) wi[q] = 0.0;
    if (r == 0 && status) status[i] = st;
}

template <int OP>
int launch3(const double *x, const double *y, const double *z, int64_t n_nodes,
            const int32_t *nbr, int32_t k_stride, int32_t n, double *w, int32_t *status,
            hipStream_t s) {
    if (n + kMono3 <= 32)  // two stencils per wavefront
        hipLaunchKernelGGL((weights3_kernel<32, 32, OP>),
                           dim3((unsigned)ceil_div(n_nodes, 2 * kWaves3)), dim3(kWave * kWaves3),
                           0, s, x, y, z, n_nodes, nbr, k_stride, (int)n, n_nodes, w, status);
    else
        hipLaunchKernelGGL((weights3_kernel<64, kWave, OP>),
                           dim3((unsigned)ceil_div(n_nodes, kWaves3)), dim3(kWave * kWaves3), 0,
                           s, x, y, z, n_nodes, nbr, k_stride, (int)n, n_nodes, w, status);
    return last_launch_rc();
}

}  // namespace

// the blocked LU of the matrix cores: K = 30 (m = 2, n = 20) and K = 105
// (m = 4, n = 70), one translation unit per operator at K = 105
int weights3_blocked_k30(const double *x, const double *y, const double *z, int64_t n_nodes,
                         const int32_t *nbr, int32_t k_stride, int op, double *w,
                         int32_t *status, hipStream_t stream);
#define RBFFD_W3_K105_DECL(OP)                                                                 \
    int weights3_blocked_k105_op##OP(const double *x, const double *y, const double *z,        \
                                     int64_t n_nodes, const int32_t *nbr, int32_t k_stride,    \
                                     double *w, int32_t *status, hipStream_t stream);
RBFFD_W3_K105_DECL(0)
RBFFD_W3_K105_DECL(1)
RBFFD_W3_K105_DECL(2)
RBFFD_W3_K105_DECL(3)
#undef RBFFD_W3_K105_DECL
// m = 4 on the other supports (35 <= n <= 76): identity padding to K = 111
#define RBFFD_W3_M4_ANY_DECL(OP)                                                               \
    int weights3_blocked_m4_any_op##OP(const double *x, const double *y, const double *z,      \
                                       int64_t n_nodes, const int32_t *nbr, int32_t k_stride,  \
                                       int n, double *w, int32_t *status, hipStream_t stream);
RBFFD_W3_M4_ANY_DECL(0)
RBFFD_W3_M4_ANY_DECL(1)
RBFFD_W3_M4_ANY_DECL(2)
RBFFD_W3_M4_ANY_DECL(3)
#undef RBFFD_W3_M4_ANY_DECL

}  // namespace rbffd

#ifndef RBFFD_W3_K30_BLOCKED
#define RBFFD_W3_K30_BLOCKED 1
#endif

using namespace rbffd;

extern "C" int rbffd_weights3_op(const double *x, const double *y, const double *z,
                                 int64_t n_nodes, const int32_t *nbr, int32_t k_stride,
                                 int32_t m, int32_t n, int32_t op, double *w, int32_t *status,
                                 void *stream) {
    if (!x || !y || !z || !nbr || !w || n_nodes < 1 || n_nodes >= INT32_MAX || k_stride < 1 ||
        n > k_stride || (m != 2 && m != 4) || n < (m == 2 ? kMono3 : 35) || op < 0 || op > 3)
        return RBFFD_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (m == 4 && n != 70) {
        if (n > 76) return RBFFD_ERR_UNSUPPORTED;
        switch (op) {
        case 0: return weights3_blocked_m4_any_op0(x, y, z, n_nodes, nbr, k_stride, n, w, status, s);
        case 1: return weights3_blocked_m4_any_op1(x, y, z, n_nodes, nbr, k_stride, n, w, status, s);
        case 2: return weights3_blocked_m4_any_op2(x, y, z, n_nodes, nbr, k_stride, n, w, status, s);
        default:
            return weights3_blocked_m4_any_op3(x, y, z, n_nodes, nbr, k_stride, n, w, status, s);
        }
    }
    if (m == 4) {
        switch (op) {
        case 0: return weights3_blocked_k105_op0(x, y, z, n_nodes, nbr, k_stride, w, status, s);
        case 1: return weights3_blocked_k105_op1(x, y, z, n_nodes, nbr, k_stride, w, status, s);
        case 2: return weights3_blocked_k105_op2(x, y, z, n_nodes, nbr, k_stride, w, status, s);
        default: return weights3_blocked_k105_op3(x, y, z, n_nodes, nbr, k_stride, w, status, s);
        }
    }
    if (RBFFD_W3_K30_BLOCKED && n == 20)
        return weights3_blocked_k30(x, y, z, n_nodes, nbr, k_stride, op, w, status, s);
    if (n + kMono3 > 64) return RBFFD_ERR_UNSUPPORTED;
    switch (op) {
    case 0: return launch3<0>(x, y, z, n_nodes, nbr, k_stride, n, w, status, s);
    case 1: return launch3<1>(x, y, z, n_nodes, nbr, k_stride, n, w, status, s);
    case 2: return launch3<2>(x, y, z, n_nodes, nbr, k_stride, n, w, status, s);
    default: return launch3<3>(x, y, z, n_nodes, nbr, k_stride, n, w, status, s);
    }
}

extern "C" int rbffd_weights3(const double *x, const double *y, const double *z,
                              int64_t n_nodes, const int32_t *nbr, int32_t k_stride, int32_t m,
                              int32_t n, double *w, int32_t *status, void *stream) {
    return rbffd_weights3_op(x, y, z, n_nodes, nbr, k_stride, m, n, 0, w, status, stream);
}
