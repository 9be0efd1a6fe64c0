#pragma once
// RBF-FD Laplacian stencil weights, FP64, for large systems (K = 84): one
// stencil per two-wavefront block, the columns split between the wavefronts.
//
// Same arithmetic as weights_ms.h (the sequence of IEEE operations of the
// reference definition), laid out for a system whose rows do not fit one
// wavefront's registers:
//   * both wavefronts hold every row (lane l: rows l and l + 64); wavefront v
//     holds the columns q with q % 2 == v (interleaved, so both have the
//     same amount of trailing work at every step); the right-hand side is
//     column KP and belongs to wavefront KP % 2;
//   * column c is searched by its owner wavefront (exact (|a|, position) key,
//     VALU all-reduce and ballot, as in weights_ms.h); the owner forms the
//     multipliers of all rows and publishes them, with the pivot's lane, slot
//     and position, through LDS; one block barrier per column;
//   * each wavefront then updates its own columns with the pivot row's
//     entries read from the winning lane by readlane (scalar operands);
//   * the rows of U are written to a packed triangle in LDS as they are
//     pivoted; wavefront 0 runs the back substitution from there.

#include "weights_ms.h"

namespace rbffd {
namespace wk {

// The part of one stencil that wavefront WV (its column parity) runs.
template <int KP, int NFIX, int MFIX, bool SAVE, int WV>
__device__ __forceinline__ void weights_cs_wave(
    const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
    const int32_t *__restrict__ nbr, int32_t k_stride, int64_t i, int32_t n_arg, int32_t m_arg,
    double *__restrict__ w, int32_t *__restrict__ status, double *__restrict__ sv_lu,
    double *__restrict__ sv_z, double *__restrict__ sv_s, uint8_t *__restrict__ sv_perm,
    int32_t sv_kmax, int32_t ok_code, double *sU, double (*s_lm)[2][kWave],
    int32_t (*s_pv)[4], uint32_t *s_fl) {
    constexpr int SEG = kWave, SL = 2, KC = (KP + 1) / 2;
    constexpr int wv = WV;
    static_assert(SEG * SL >= KP, "two rows per lane must cover the system");
    constexpr int MM = MFIX ? (MFIX + 1) * (MFIX + 2) / 2 : 28;
    constexpr int RHS_OWNER = KP % 2;
    using L = MsLds<KP, MM>;
    const int n = NFIX ? NFIX : n_arg;
    const int m = MFIX ? MFIX : m_arg;
    const int NM = (m + 1) * (m + 2) / 2;
    const int K = n + NM;

    double *s_ux = sU;
    double *s_uy = sU + KP;
    double(*s_P)[MM] = reinterpret_cast<double(*)[MM]>(sU + 2 * KP);

    const int lane = threadIdx.x & (kWave - 1);

    // ---- shift (both wavefronts: every row) --------------------------------
    uint32_t flags = 0;
    double dx[SL], dy[SL];
    double d2m = 0.0;
    const double xi = x[i], yi = y[i];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int r = lane + SEG * s;
        dx[s] = 0.0;
        dy[s] = 0.0;
        if (r < n) {
            const int32_t j = nbr[i * (int64_t)k_stride + r];
            if (j < 0 || (int64_t)j >= n_nodes) {
                flags |= F_BADIDX;
            } else {
                const double ddx = x[j] - xi, ddy = y[j] - yi;
                if (!isfinite(ddx) || !isfinite(ddy)) {
                    flags |= F_NONFIN;
                } else {
                    dx[s] = ddx;
                    dy[s] = ddy;
                    const double d2 = ddx * ddx + ddy * ddy;
                    d2m = fmax(d2m, d2);
                }
            }
        }
    }
    const double sc = sqrt(seg_all_max_d<SEG>(d2m, lane));
    if (!isfinite(sc)) flags |= F_NONFIN;  // an offset's square overflowed
    if (sc == 0.0) flags |= F_DUP;

    // ---- scale; monomial table (written by wavefront 0) --------------------
    double ux[SL], uy[SL];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int r = lane + SEG * s;
        ux[s] = 0.0;
        uy[s] = 0.0;
        if (r < n) {
            ux[s] = dx[s] / sc;
            uy[s] = dy[s] / sc;
            if (wv == 0) {
                s_ux[r] = ux[s];
                s_uy[r] = uy[s];
                double px[7], py[7];
                px[0] = 1.0;
                py[0] = 1.0;
#pragma unroll
                for (int e = 1; e < 7; ++e) {
                    px[e] = px[e - 1] * ux[s];
                    py[e] = py[e - 1] * uy[s];
                }
#pragma unroll
                for (int j = 0; j < MM; ++j)
                    if (j < NM) s_P[r][j] = px[mono_a(j)] * py[mono_b(j)];
            }
        }
    }
    __syncthreads();

    // ---- assemble this wavefront's columns of every row --------------------
    double a[SL][KC];
    double yv[SL];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int r = lane + SEG * s;
        const bool prow = r < n;
        const bool qrow = r >= n && r < K;
        const int jr = qrow ? r - n : 0;
#pragma unroll
        for (int jj = 0; jj < KC; ++jj) {
            const int l = 2 * jj + wv;
            double v = 0.0;
            if (l < KP) {
                if (l < n) {
                    double phs = 0.0;
                    if (!NFIX || SEG * s < NFIX) {
                        const double ex = ux[s] - s_ux[l];
                        const double ey = uy[s] - s_uy[l];
                        const double rr = ex * ex + ey * ey;
                        if (prow && l != r && rr == 0.0) flags |= F_DUP;
                        asm volatile("" : "+v"(flags));
                        phs = rr * sqrt(rr);
                    }
                    const double pt = s_P[l][jr];
                    v = prow ? phs : (qrow ? pt : 0.0);
                } else if (l < K) {
                    v = prow ? s_P[r < KP ? r : 0][l - n] : 0.0;
                } else {
                    v = (l == r) ? 1.0 : 0.0;
                }
            }
            a[s][jj] = v;
            if ((jj & 1) == 1) __builtin_amdgcn_sched_barrier(0);
        }
        const double r0 = ux[s] * ux[s] + uy[s] * uy[s];
        const double rb = 9.0 * sqrt(r0);
        yv[s] = prow ? rb : ((qrow && (jr == 3 || jr == 5)) ? 2.0 : 0.0);
    }
    asm volatile("" : "+v"(flags));
    __syncthreads();  // the assembly tables' space becomes the rows of U

    // ---- LU with partial pivoting, columns split between the wavefronts ----
    int pos[SL];
    bool done[SL];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        pos[s] = lane + SEG * s;
        done[s] = pos[s] >= KP;
    }
#pragma unroll
    for (int c = 0; c < KP; ++c) {
        const int buf = c & 1;
        const int jc = c / 2;       // local index of column c in its owner
        const bool own = (c & 1) == wv;
        int win, bs, kp;
        double lm[SL];
        if (own) {
            // pivot search over both slots: exact key (|a| bits, position)
            uint64_t bb = 0;
            int bp = 0x7fffffff, bsl = 0;
            double bv = 0.0;
            bool ba = false;
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                const uint64_t bits =
                    (uint64_t)__double_as_longlong(a[s][jc]) & 0x7fffffffffffffffull;
                const bool take = !done[s] && (!ba || bits > bb || (bits == bb && pos[s] < bp));
                bb = take ? bits : bb;
                bp = take ? pos[s] : bp;
                bsl = take ? s : bsl;
                bv = take ? a[s][jc] : bv;
                ba = ba || !done[s];
            }
            const uint32_t kh = ba ? (uint32_t)(bb >> 32) + 1u : 0u;
            const uint32_t mh = seg_all<SEG, OpMax>(kh, lane);
            uint64_t chunk = __ballot(ba && kh == mh);
            if (__builtin_expect((chunk & (chunk - 1ull)) != 0ull, 0)) {
                uint32_t h2 = kh, l2 = ba ? (uint32_t)bb : 0u;
                int p2 = ba ? bp : 0x7fffffff;
                seg_argmax_full<SEG>(h2, l2, p2);
                chunk = __ballot(ba && bp == p2);
            }
            win = __builtin_amdgcn_readfirstlane(__ffsll((unsigned long long)chunk) - 1);
            bs = __builtin_amdgcn_readlane(bsl, win);
            kp = __builtin_amdgcn_readlane(bp, win);
            const double piv = readlane_d(bv, win);
            const double inv = 1.0 / piv;
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                const bool upd = !done[s] && !(lane == win && bs == s);
                lm[s] = upd ? a[s][jc] * inv : 0.0;
                if constexpr (SAVE) a[s][jc] = upd ? lm[s] : a[s][jc];
                s_lm[buf][s][lane] = lm[s];
            }
            if (lane == 0) {
                s_pv[buf][0] = win;
                s_pv[buf][1] = bs;
                s_pv[buf][2] = kp;
            }
        }
        __syncthreads();
        if (!own) {
            win = __builtin_amdgcn_readfirstlane(s_pv[buf][0]);
            bs = __builtin_amdgcn_readfirstlane(s_pv[buf][1]);
            kp = __builtin_amdgcn_readfirstlane(s_pv[buf][2]);
#pragma unroll
            for (int s = 0; s < SL; ++s) lm[s] = s_lm[buf][s][lane];
        }
        // the pivot row's entries in this wavefront's columns: to the rows of
        // U in LDS (winning lane only), then to every lane by readlane
        double *u = sU + L::ubase(c);
        if (lane == win) {
#pragma unroll
            for (int jj = 0; jj < KC; ++jj) {
                const int q = 2 * jj + wv;
                if (q >= c && q < KP) u[2 * q] = bs == 0 ? a[0][jj] : a[1][jj];
            }
            if (wv == RHS_OWNER) u[2 * KP] = bs == 0 ? yv[0] : yv[1];
        }
        // The winner's slot is wave-uniform; a select (not a branch on it)
        // keeps one copy of the update.  Columns go in chunks of CH with a
        // scheduling barrier between them, which bounds how many readlane
        // results (scalar registers) are held at once.
        {
            constexpr int CH = 6;
            const bool b1 = bs != 0;
#pragma unroll
            for (int j0 = 0; j0 < KC; j0 += CH) {
#pragma unroll
                for (int jj = j0; jj < j0 + CH && jj < KC; ++jj) {
                    const int q = 2 * jj + wv;
                    if (q > c && q < KP) {
                        const double uq = readlane_d(b1 ? a[1][jj] : a[0][jj], win);
#pragma unroll
                        for (int s = 0; s < SL; ++s) a[s][jj] = fma(-lm[s], uq, a[s][jj]);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            if (wv == RHS_OWNER) {
                const double uq = readlane_d(b1 ? yv[1] : yv[0], win);
#pragma unroll
                for (int s = 0; s < SL; ++s) yv[s] = fma(-lm[s], uq, yv[s]);
            }
        }
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const bool isp = lane == win && bs == s;
            pos[s] = isp ? c : ((!done[s] && pos[s] == c) ? kp : pos[s]);
            done[s] = done[s] || isp;
            int dn = done[s] ? 1 : 0;
            asm volatile("" : "+v"(pos[s]), "+v"(dn));
            done[s] = dn != 0;
        }
    }
    // wavefront 1's flags to wavefront 0
    uint32_t fl = seg_all<SEG, OpOr>(flags, lane);
    if (wv == 1 && lane == 0) *s_fl = fl;
    __syncthreads();  // the rows of U and the flags are visible

    if constexpr (SAVE) {
        // this wavefront's columns of every row, at the row's own index; the
        // position of each row in perm
        const int64_t kk = (int64_t)sv_kmax * sv_kmax;
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const int r = lane + SEG * s;
            if (r < K) {
                double *dst = sv_lu + i * kk + (int64_t)r * K;
#pragma unroll
                for (int jj = 0; jj < KC; ++jj) {
                    const int q = 2 * jj + wv;
                    if (q < K) dst[q] = a[s][jj];
                }
            }
            if (wv == 0 && pos[s] < K) sv_perm[i * (int64_t)sv_kmax + pos[s]] = (uint8_t)r;
        }
    }
    if (wv != 0) return;
    fl |= *s_fl;

    // ---- back substitution over the rows of U in LDS (wavefront 0) ---------
    int ub[SL];
    double yb[SL], mb[SL], zm[SL];
    double ur[1][1];
    uint32_t lukey = 0;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int r0 = lane + SEG * s;
        const int r = r0 < KP ? r0 : KP - 1;
        ub[s] = L::ubase(r);
        yb[s] = sU[ub[s] + 2 * KP];
        const double d = sU[ub[s] + 2 * r];
        mb[s] = 1.0 / d;
        zm[s] = 0.0;
        const uint32_t f = !isfinite(d) ? L_NONFIN : (d == 0.0 ? L_SING : 0u);
        const uint32_t key = ((uint32_t)(KP - r0) << 2) | f;
        if (r0 < KP && f && key > lukey) lukey = key;
    }
    const uint32_t luflag = seg_all<SEG, OpMax>(lukey, lane) & 3u;
    bc_step<KP, SEG, SL, KP - 1, false>(sU, ub, ur[0], yb, mb, zm, lane, false);

    // ---- status and outputs -----------------------------------------------
#pragma unroll
    for (int s = 0; s < SL; ++s)
        if (lane + SEG * s < K && !isfinite(zm[s])) fl |= F_ZBAD;
    fl = seg_all<SEG, OpOr>(fl, lane);
    int st = RBFFD_OK;
    if (fl & F_BADIDX) st = RBFFD_BAD_INDEX;
    else if (fl & F_NONFIN) st = RBFFD_NONFINITE;
    else if (fl & F_DUP) st = RBFFD_DUPLICATE;
    else if (luflag == L_NONFIN) st = RBFFD_NONFINITE;
    else if (luflag == L_SING) st = RBFFD_SINGULAR;
    else if (fl & F_ZBAD) st = RBFFD_NONFINITE;

    double *wi = w + i * (int64_t)k_stride;
    const double s2 = sc * sc;
    const bool good = st == RBFFD_OK;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int r = lane + SEG * s;
        if (r < n) wi[r] = good ? zm[s] / s2 : __builtin_nan("");
    }
    for (int q = n + lane; q < k_stride; q += SEG) wi[q] = 0.0;
    if (lane == 0 && status) status[i] = good ? ok_code : st;
    if constexpr (SAVE) {
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const int r = lane + SEG * s;
            if (r < K) sv_z[i * (int64_t)sv_kmax + r] = zm[s];
        }
        if (lane == 0) sv_s[i] = sc;
    }
}

// LDS bytes of weights_cs_body: the U triangle / assembly tables, the
// multipliers [2][2][64], the pivot record [2][4] and one flag word.
template <int KP, int MFIX>
__host__ __device__ constexpr int cs_lds_bytes() {
    constexpr int MM = MFIX ? (MFIX + 1) * (MFIX + 2) / 2 : 28;
    return (int)sizeof(double) * (MsLds<KP, MM>::SZ + 2 * 2 * kWave) + 4 * 8 + 16;
}

// One block (two wavefronts) computes stencil `t` of the row list.
template <int KP, int NFIX, int MFIX, bool SAVE>
__device__ __forceinline__ void weights_cs_body(
    const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
    const int32_t *__restrict__ nbr, int32_t k_stride, const int32_t *__restrict__ rows,
    int64_t n_rows, int32_t n_arg, int32_t m_arg, double *__restrict__ w,
    int32_t *__restrict__ status, double *__restrict__ sv_lu, double *__restrict__ sv_z,
    double *__restrict__ sv_s, uint8_t *__restrict__ sv_perm, int32_t sv_kmax, int32_t ok_code,
    int64_t t, char *lds) {
    constexpr int MM = MFIX ? (MFIX + 1) * (MFIX + 2) / 2 : 28;
    constexpr int SZ = MsLds<KP, MM>::SZ;
    double *sU = reinterpret_cast<double *>(lds);
    auto s_lm = reinterpret_cast<double(*)[2][kWave]>(lds + sizeof(double) * SZ);
    auto s_pv = reinterpret_cast<int32_t(*)[4]>(lds + sizeof(double) * (SZ + 2 * 2 * kWave));
    uint32_t *s_fl_p = reinterpret_cast<uint32_t *>(lds + sizeof(double) * (SZ + 2 * 2 * kWave) + 32);
    if (t >= n_rows) return;  // whole block idle
    const int64_t i = rows ? (int64_t)rows[t] : t;
    if ((threadIdx.x >> 6) & 1)
        weights_cs_wave<KP, NFIX, MFIX, SAVE, 1>(x, y, n_nodes, nbr, k_stride, i, n_arg, m_arg, w,
                                                 status, sv_lu, sv_z, sv_s, sv_perm, sv_kmax,
                                                 ok_code, sU, s_lm, s_pv, s_fl_p);
    else
        weights_cs_wave<KP, NFIX, MFIX, SAVE, 0>(x, y, n_nodes, nbr, k_stride, i, n_arg, m_arg, w,
                                                 status, sv_lu, sv_z, sv_s, sv_perm, sv_kmax,
                                                 ok_code, sU, s_lm, s_pv, s_fl_p);
}

template <int KP, int NFIX, int MFIX, bool SAVE>
__global__ __launch_bounds__(2 * kWave)
__attribute__((amdgpu_waves_per_eu(2))) void weights_cs_kernel(
    const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
    const int32_t *__restrict__ nbr, int32_t k_stride, const int32_t *__restrict__ rows,
    const int32_t *__restrict__ n_rows_dev, int64_t n_rows, int32_t n_arg, int32_t m_arg,
    double *__restrict__ w, int32_t *__restrict__ status, double *__restrict__ sv_lu,
    double *__restrict__ sv_z, double *__restrict__ sv_s, uint8_t *__restrict__ sv_perm,
    int32_t sv_kmax, int32_t ok_code) {
    __shared__ __align__(16) char lds[cs_lds_bytes<KP, MFIX>()];
    if (n_rows_dev) n_rows = *n_rows_dev;
    weights_cs_body<KP, NFIX, MFIX, SAVE>(x, y, n_nodes, nbr, k_stride, rows, n_rows, n_arg,
                                          m_arg, w, status, sv_lu, sv_z, sv_s, sv_perm,
                                          sv_kmax, ok_code, (int64_t)blockIdx.x, lds);
}

template <int KP, int NFIX, int MFIX>
inline int launch_cs(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                     int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev,
                     int64_t n_rows, int n, int m, double *w, int32_t *status,
                     const SaveView &sv, int32_t ok_code, hipStream_t stream) {
    if (n_rows <= 0) return RBFFD_SUCCESS;
    if (n_rows > 0x7fffffff) return RBFFD_ERR_UNSUPPORTED;
    if (sv.lu)
        hipLaunchKernelGGL((weights_cs_kernel<KP, NFIX, MFIX, true>), dim3((unsigned)n_rows),
                           dim3(2 * kWave), 0, stream, x, y, n_nodes, nbr, k_stride, rows,
                           n_rows_dev, n_rows, n, m, w, status, sv.lu, sv.z, sv.s, sv.perm,
                           sv.kmax, ok_code);
    else
        hipLaunchKernelGGL((weights_cs_kernel<KP, NFIX, MFIX, false>), dim3((unsigned)n_rows),
                           dim3(2 * kWave), 0, stream, x, y, n_nodes, nbr, k_stride, rows,
                           n_rows_dev, n_rows, n, m, w, status, nullptr, nullptr, nullptr,
                           nullptr, 0, ok_code);
    return last_launch_rc();
}

}  // namespace wk
}  // namespace rbffd
