#pragma once
// Two stencils per wavefront for the blocked LU of weights_mf.h, for systems
// whose padded size is 32 or 48 (K + 1 <= 48: 2 x 2 or 3 x 3 tiles of
// 16 x 16).
//
// The panel's column steps work in row layout.  Here the two halves of the
// wavefront carry two stencils: lane l holds rows (l & 31) + 32 s (s < SL)
// of stencil l >> 5.  The pivot search (a 32-lane reduction), the
// reciprocal, the multipliers and the row bookkeeping of a column then serve
// both stencils with one instruction stream, and so does the back
// substitution.  The tiles, the panel transposes and the trailing MFMA
// updates stay per stencil: a matrix-core instruction takes the whole
// wavefront.
//
// The arithmetic of each stencil is that of weights_mf.h (same shift,
// scale, assembly, pivot rule, multipliers, fused updates in the same order,
// back substitution), so the weights are the same bits.

#include "weights_mf.h"

namespace rbffd {
namespace wk {

// LDS per stencil: the U triangle / assembly tables, then the panel in row
// layout [NP][5] (the pivot rows of a panel's end, [NT][4][16], overlay it,
// read out first); the pivot record of the panel [4][2] int32 per stencil
// follows both stencils' doubles.
template <int KP, int MM, int DIM>
struct Mf2Lds {
    using L = MsLds<KP, MM>;
    static constexpr int NT = (KP + 1 + 15) / 16;
    static constexpr int NP = 16 * NT;
    static constexpr int ASZ3 = DIM == 3 ? (KP * (MM + 3) + 1) & ~1 : 0;
    static constexpr int SZ = L::SZ > ASZ3 ? L::SZ : ASZ3;
    static constexpr int PAN = SZ;                               // [NP][5]
    static constexpr int PER = SZ + (NP * 5 > NT * 64 ? NP * 5 : NT * 64);
    static constexpr int DBL = 2 * PER;
    static constexpr int BYTES = 8 * DBL + 4 * 2 * 8;
};

template <int KP, int NFIX, int MFIX, int DIM>
__host__ __device__ constexpr int mf2_lds_bytes() {
    constexpr int MM = DIM == 2 ? (MFIX + 1) * (MFIX + 2) / 2
                                : (MFIX + 1) * (MFIX + 2) * (MFIX + 3) / 6;
    return Mf2Lds<KP, MM, DIM>::BYTES;
}

// v of lane w0 to the lanes of half 0, of lane w1 to those of half 1
__device__ __forceinline__ double bcast2_d(double v, int w0, int w1, int h) {
    const double v0 = readlane_d(v, w0);
    const double v1 = readlane_d(v, w1);
    return h ? v1 : v0;
}
__device__ __forceinline__ int bcast2_i(int v, int w0, int w1, int h) {
    const int v0 = __builtin_amdgcn_readlane(v, w0);
    const int v1 = __builtin_amdgcn_readlane(v, w1);
    return h ? v1 : v0;
}

// Stencils i0 and i0 + 1 of the row list (the second may be past n_rows:
// it then repeats the first and writes nothing).
template <int KP, int NFIX, int MFIX, int OP, int DIM>
__device__ __forceinline__ void weights_mf2_wave(
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
    int64_t n_nodes, const int32_t *__restrict__ nbr, int32_t k_stride,
    const int32_t *__restrict__ rows, int64_t i0, int64_t n_rows, double *__restrict__ w,
    int32_t *__restrict__ status, int32_t ok_code, char *lds) {
    static_assert(DIM == 2 || DIM == 3, "two or three dimensions");
    static_assert(OP >= 0 && OP <= DIM, "operator");
    constexpr int MM = DIM == 2 ? (MFIX + 1) * (MFIX + 2) / 2
                                : (MFIX + 1) * (MFIX + 2) * (MFIX + 3) / 6;
    constexpr int n = NFIX, K = NFIX + MM;
    static_assert(K == KP, "no identity padding in the blocked kernel");
    using L = MsLds<KP, MM>;
    using B = Mf2Lds<KP, MM, DIM>;
    constexpr int NT = B::NT, NP = B::NP;
    static_assert(NT == 2 || NT == 3, "two or three tiles per dimension");
    constexpr int SL = (NP + 31) / 32;  // rows per lane in row layout

    const int lane = threadIdx.x & (kWave - 1);
    const int h = lane >> 5;      // this lane's stencil in the row layout
    const int r = lane & 31;      // its row
    const int g = lane >> 4, jl = lane & 15;  // tile layout (each stencil in turn)
    const bool live = i0 + h < n_rows;
    const int64_t t = live ? i0 + h : i0;
    const int64_t i = rows ? (int64_t)rows[t] : t;

    double *sbase = reinterpret_cast<double *>(lds);
    // stencil hh's regions
    auto sU_of = [&](int hh) { return sbase + hh * B::PER; };
    int32_t *s_rec = reinterpret_cast<int32_t *>(lds + 8 * B::DBL);  // [2][4][2]
    double *sU = sU_of(h);  // this lane's stencil

    // ---- shift and scale (rows r + 32 s of stencil h) ---------------------
    uint32_t flags = 0;
    double dx[SL], dy[SL], dz[SL];
    double d2m = 0.0;
    const double xi = x[i], yi = y[i];
    const double zi = DIM == 3 ? z[i] : 0.0;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int rs = r + 32 * s;
        dx[s] = 0.0;
        dy[s] = 0.0;
        dz[s] = 0.0;
        if (rs < n) {
            const int32_t j = nbr[i * (int64_t)k_stride + rs];
            if (j < 0 || (int64_t)j >= n_nodes) {
                flags |= F_BADIDX;
            } else {
                const double ddx = x[j] - xi, ddy = y[j] - yi;
                const double ddz = DIM == 3 ? z[j] - zi : 0.0;
                if (!isfinite(ddx) || !isfinite(ddy) || (DIM == 3 && !isfinite(ddz))) {
                    flags |= F_NONFIN;
                } else {
                    dx[s] = ddx;
                    dy[s] = ddy;
                    dz[s] = ddz;
                    const double d2 = DIM == 3 ? (ddx * ddx + ddy * ddy) + ddz * ddz
                                               : ddx * ddx + ddy * ddy;
                    d2m = fmax(d2m, d2);
                }
            }
        }
    }
    const double sc = sqrt(seg_all_max_d<32>(d2m, lane));
    if (!isfinite(sc)) flags |= F_NONFIN;  // an offset's square overflowed
    if (sc == 0.0) flags |= F_DUP;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int rs = r + 32 * s;
        double *s_ux = sU, *s_uy = sU + KP, *s_uz = sU + 2 * KP;
        double(*s_P)[MM] = reinterpret_cast<double(*)[MM]>(sU + DIM * KP);
        if (rs < n) {
            const double ux = dx[s] / sc, uy = dy[s] / sc;
            s_ux[rs] = ux;
            s_uy[rs] = uy;
            if constexpr (DIM == 2) {
                double px[7], py[7];
                px[0] = 1.0;
                py[0] = 1.0;
#pragma unroll
                for (int e = 1; e < 7; ++e) {
                    px[e] = px[e - 1] * ux;
                    py[e] = py[e - 1] * uy;
                }
#pragma unroll
                for (int j = 0; j < MM; ++j) s_P[rs][j] = px[mono_a(j)] * py[mono_b(j)];
            } else {
                const double uz = dz[s] / sc;
                s_uz[rs] = uz;
                double px[MFIX + 1], py[MFIX + 1], pt[MFIX + 1];
                px[0] = 1.0;
                py[0] = 1.0;
                pt[0] = 1.0;
#pragma unroll
                for (int e = 1; e <= MFIX; ++e) {
                    px[e] = px[e - 1] * ux;
                    py[e] = py[e - 1] * uy;
                    pt[e] = pt[e - 1] * uz;
                }
                constexpr Mono3Table<MM> e3{};
#pragma unroll
                for (int j = 0; j < MM; ++j)
                    s_P[rs][j] = (px[e3.a[j]] * py[e3.b[j]]) * pt[e3.c[j]];
            }
        }
    }
    lds_order();

    // ---- assembly of both stencils' tiles (transposed, as in weights_mf.h) -
    // the duplicate flags of stencil hh are found by every lane: kept apart
    mf_v4d T[2][NT][NT];
    uint32_t dupf[2] = {0u, 0u};
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
        const double *s_ux = sU_of(hh), *s_uy = sU_of(hh) + KP, *s_uz = sU_of(hh) + 2 * KP;
        const double(*s_P)[MM] = reinterpret_cast<const double(*)[MM]>(sU_of(hh) + DIM * KP);
#pragma unroll
        for (int I = 0; I < NT; ++I) {
            const int R = 16 * I + jl;
            const bool prow = R < n;
            const bool qrow = R >= n && R < K;
            const int jr = qrow ? R - n : 0;
            const double uxr = (16 * I < n && prow) ? s_ux[R] : 0.0;
            const double uyr = (16 * I < n && prow) ? s_uy[R] : 0.0;
            const double uzr = (DIM == 3 && 16 * I < n && prow) ? s_uz[R] : 0.0;
#pragma unroll
            for (int J = 0; J < NT; ++J) {
#pragma unroll
                for (int rr4 = 0; rr4 < 4; ++rr4) {
                    const int C = 16 * J + g + 4 * rr4;
                    double v = 0.0;
                    if (16 * J < n && C < n) {
                        double phs = 0.0;
                        if (16 * I < n) {
                            const double ex = uxr - s_ux[C];
                            const double ey = uyr - s_uy[C];
                            double rr;
                            if constexpr (DIM == 2) {
                                rr = ex * ex + ey * ey;
                            } else {
                                const double ez = uzr - s_uz[C];
                                rr = (ex * ex + ey * ey) + ez * ez;
                            }
                            if (prow && C != R && rr == 0.0) dupf[hh] |= F_DUP;
                            asm volatile("" : "+v"(dupf[hh]));
                            phs = rr * sqrt(rr);
                        }
                        const double pt = s_P[C][jr];
                        v = prow ? phs : (qrow ? pt : 0.0);
                    } else if (16 * J + 15 >= n && 16 * J < K && C >= n && C < K) {
                        v = prow ? s_P[prow ? R : 0][C - n] : 0.0;
                    } else if (16 * J + 15 >= KP && 16 * J <= KP && C == KP) {
                        double rb, rq;
                        if constexpr (DIM == 2) {
                            const double r0 = uxr * uxr + uyr * uyr;
                            rb = OP == 0 ? 9.0 * sqrt(r0)
                                         : -3.0 * sqrt(r0) * (OP == 1 ? uxr : uyr);
                            rq = OP == 0 ? ((jr == 3 || jr == 5) ? 2.0 : 0.0)
                                         : (jr == OP ? 1.0 : 0.0);
                        } else {
                            const double r0 = (uxr * uxr + uyr * uyr) + uzr * uzr;
                            rb = OP == 0 ? 12.0 * sqrt(r0)
                                         : -3.0 * sqrt(r0) *
                                               (OP == 1 ? uxr : (OP == 2 ? uyr : uzr));
                            rq = OP == 0 ? ((jr == 4 || jr == 7 || jr == 9) ? 2.0 : 0.0)
                                         : (jr == OP ? 1.0 : 0.0);
                        }
                        v = prow ? rb : (qrow ? rq : 0.0);
                    }
                    T[hh][I][J][rr4] = v;
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    // stencil hh's duplicate flag, from every lane, to the lanes of half hh
    {
        const uint32_t d0 = seg_all<kWave, OpOr>(dupf[0], lane);
        const uint32_t d1 = seg_all<kWave, OpOr>(dupf[1], lane);
        flags |= h ? d1 : d0;
    }
    lds_order();  // the assembly tables' space becomes the rows of U

    // ---- LU, panels of four columns ----------------------------------------
    int pos[SL];
    bool done[SL];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        pos[s] = r + 32 * s;
        done[s] = pos[s] >= KP;
    }
#pragma unroll
    for (int c0 = 0; c0 < KP; c0 += 4) {
        const int J0 = c0 >> 4;             // tile column of the panel
        const int rc = (c0 & 15) >> 2;      // its register
        const int nk = KP - c0 < 4 ? KP - c0 : 4;
        // the panel to row layout through LDS, each stencil's own buffer
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            double(*s_pan)[5] = reinterpret_cast<double(*)[5]>(sU_of(hh) + B::PAN);
#pragma unroll
            for (int I = 0; I < NT; ++I) s_pan[16 * I + jl][g] = T[hh][I][J0][rc];
        }
        lds_order();
        double(*s_panh)[5] = reinterpret_cast<double(*)[5]>(sU + B::PAN);
        double pc[SL][4];
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const int rs = r + 32 * s;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) pc[s][jj] = rs < NP ? s_panh[rs < NP ? rs : 0][jj] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k >= nk) break;
            const int c = c0 + k;
            // pivot search over the lane's slots, then per half: exact key
            // (|a| bits, position); bb, bp and bv are read only where ba holds
            uint64_t bb = 0;
            int bp = 0, bsl = 0;
            double bv = 0.0;
            bool ba = false;
            if constexpr (SL == 1) {
                bb = (uint64_t)__double_as_longlong(pc[0][k]) & 0x7fffffffffffffffull;
                bp = pos[0];
                bv = pc[0][k];
                ba = !done[0];
            } else {
#pragma unroll
                for (int s = 0; s < SL; ++s) {
                    const uint64_t bits =
                        (uint64_t)__double_as_longlong(pc[s][k]) & 0x7fffffffffffffffull;
                    const bool take =
                        !done[s] && (!ba || bits > bb || (bits == bb && pos[s] < bp));
                    bb = take ? bits : bb;
                    bp = take ? pos[s] : bp;
                    bsl = take ? s : bsl;
                    bv = take ? pc[s][k] : bv;
                    ba = ba || !done[s];
                }
            }
            const uint32_t kh = ba ? (uint32_t)(bb >> 32) + 1u : 0u;
            const uint32_t mh = seg_all<32, OpMax>(kh, lane);
            // (each half keeps a row in the search, so its mh >= 1 and only
            // rows still in the search can equal it)
            uint64_t chunk = __ballot(kh == mh);
            uint32_t c0m = (uint32_t)chunk, c1m = (uint32_t)(chunk >> 32);
            if (__builtin_expect(((c0m & (c0m - 1u)) | (c1m & (c1m - 1u))) != 0u, 0)) {
                uint32_t h2 = kh, l2 = ba ? (uint32_t)bb : 0u;
                int p2 = ba ? bp : 0x7fffffff;
                seg_argmax_full<32>(h2, l2, p2);
                chunk = __ballot(ba && bp == p2);
                c0m = (uint32_t)chunk;
                c1m = (uint32_t)(chunk >> 32);
            }
            const int w0 = __builtin_amdgcn_readfirstlane(__ffs((int)c0m) - 1);
            const int w1 = __builtin_amdgcn_readfirstlane(__ffs((int)c1m) - 1 + 32);
            const int win = h ? w1 : w0;
            const int bs = bcast2_i(bsl, w0, w1, h);  // the winner's slot
            const int kp = bcast2_i(bp, w0, w1, h);
            const double piv = bcast2_d(bv, w0, w1, h);
            const double inv = recip_div(piv);
            // row c of U, panel columns c .. c0 + 3 (up to the rhs)
            if (lane == win) {
#pragma unroll
                for (int jj = k; jj < 4; ++jj) {
                    double v = pc[0][jj];
#pragma unroll
                    for (int s = 1; s < SL; ++s) v = bs == s ? pc[s][jj] : v;
                    if (c0 + jj <= KP) sU[L::ubase(c) + 2 * (c0 + jj)] = v;
                }
            }
            double uq[4];
#pragma unroll
            for (int jj = k + 1; jj < 4; ++jj) {
                double v = pc[0][jj];
#pragma unroll
                for (int s = 1; s < SL; ++s) v = bs == s ? pc[s][jj] : v;
                uq[jj] = c0 + jj <= KP ? bcast2_d(v, w0, w1, h) : 0.0;
            }
            // multipliers, in place (zero for pivoted rows and the pivot)
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                const bool isp = lane == win && bs == s;
                const bool upd = !done[s] && !isp;
                const double lmv = upd ? pc[s][k] * inv : 0.0;
                pc[s][k] = lmv;
#pragma unroll
                for (int jj = k + 1; jj < 4; ++jj)
                    if (c0 + jj <= KP) pc[s][jj] = fma(-lmv, uq[jj], pc[s][jj]);
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
            if (r == 0) {
                s_rec[(h * 4 + k) * 2 + 0] = (win - 32 * h) + 32 * bs;  // the pivot's row
                s_rec[(h * 4 + k) * 2 + 1] = kp;
            }
        }
        // the panel's multipliers, row layout
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const int rs = r + 32 * s;
            if (rs < NP) {
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) s_panh[rs][jj] = pc[s][jj];
            }
        }
        lds_order();

        // ---- panel end: the trailing tile columns of both stencils ---------
        const int first_jt = (rc < 3) ? J0 : J0 + 1;
        if (first_jt < NT) {
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                double *sUh = sU_of(hh);
                double(*s_pan)[5] = reinterpret_cast<double(*)[5]>(sUh + B::PAN);
                double(*s_ub)[4][16] = reinterpret_cast<double(*)[4][16]>(sUh + B::PAN);
                int pr[4] = {0, 0, 0, 0};
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (k < nk) pr[k] = __builtin_amdgcn_readfirstlane(s_rec[(hh * 4 + k) * 2]);
                double l11[4][3];
#pragma unroll
                for (int m2 = 1; m2 < 4; ++m2)
#pragma unroll
                    for (int k2 = 0; k2 < m2; ++k2) l11[m2][k2] = s_pan[pr[m2]][k2];
                double Bop[NT];
#pragma unroll
                for (int I = 0; I < NT; ++I) Bop[I] = s_pan[16 * I + jl][g];
                lds_order();  // the pivot rows below overlay the panel
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int Ipk = pr[k] >> 4, ipk = pr[k] & 15;
                    if (jl == ipk) {
#pragma unroll
                        for (int I = 0; I < NT; ++I) {
                            if (I == Ipk) {
#pragma unroll
                                for (int jt = 0; jt < NT; ++jt)
                                    if (jt >= first_jt) {
#pragma unroll
                                        for (int rr4 = 0; rr4 < 4; ++rr4)
                                            s_ub[jt][k][g + 4 * rr4] = T[hh][I][jt][rr4];
                                    }
                                asm volatile(";tile row %0" ::"i"(I) : "memory");
                            }
                        }
                    }
                }
                lds_order();
#pragma unroll
                for (int jt = 0; jt < NT; ++jt) {
                    if (jt < first_jt) continue;
                    const int i0c = (jt == J0) ? 4 * rc + 4 : 0;
                    const double q0 = s_ub[jt][0][jl], q1 = s_ub[jt][1][jl];
                    const double q2 = s_ub[jt][2][jl], q3 = s_ub[jt][3][jl];
                    const double u0 = q0;
                    const double u1 = fma(-l11[1][0], u0, q1);
                    const double u2 = fma(-l11[2][1], u1, fma(-l11[2][0], u0, q2));
                    const double u3 =
                        fma(-l11[3][2], u2, fma(-l11[3][1], u1, fma(-l11[3][0], u0, q3)));
                    const double ug = g == 0 ? u0 : (g == 1 ? u1 : (g == 2 ? u2 : u3));
                    const int q = 16 * jt + jl;
                    if (jl >= i0c && q <= KP) sUh[L::ubase(c0 + g) + 2 * q] = ug;
                    const double Aop = jl >= i0c ? -ug : 0.0;
#pragma unroll
                    for (int I = 0; I < NT; ++I)
                        T[hh][I][jt] =
                            __builtin_amdgcn_mfma_f64_16x16x4f64(Aop, Bop[I], T[hh][I][jt], 0, 0, 0);
                }
                lds_order();  // s_ub is rewritten at the next panel
            }
        }
    }
    uint32_t fl = seg_all<32, OpOr>(flags, lane);
    lds_order();

    // ---- back substitution, both stencils at once (32-lane segments) -------
    int ub[SL];
    double yb[SL], mb[SL], zm[SL];
    double ur[1][1];
    uint32_t lukey = 0;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int r0 = r + 32 * s;
        const int rr = r0 < KP ? r0 : KP - 1;
        ub[s] = h * B::PER + L::ubase(rr);
        yb[s] = sbase[ub[s] + 2 * KP];
        const double d = sbase[ub[s] + 2 * rr];
        mb[s] = 1.0 / d;
        zm[s] = 0.0;
        const uint32_t f = !isfinite(d) ? L_NONFIN : (d == 0.0 ? L_SING : 0u);
        const uint32_t key = ((uint32_t)(KP - r0) << 2) | f;
        if (r0 < KP && f && key > lukey) lukey = key;
    }
    const uint32_t luflag = seg_all<32, OpMax>(lukey, lane) & 3u;
    bc_step<KP, 32, SL, KP - 1, false>(sbase, ub, ur[0], yb, mb, zm, r, false);

#pragma unroll
    for (int s = 0; s < SL; ++s)
        if (r + 32 * s < K && !isfinite(zm[s])) fl |= F_ZBAD;
    fl = seg_all<32, OpOr>(fl, lane);
    int st = RBFFD_OK;
    if (fl & F_BADIDX) st = RBFFD_BAD_INDEX;
    else if (fl & F_NONFIN) st = RBFFD_NONFINITE;
    else if (fl & F_DUP) st = RBFFD_DUPLICATE;
    else if (luflag == L_NONFIN) st = RBFFD_NONFINITE;
    else if (luflag == L_SING) st = RBFFD_SINGULAR;
    else if (fl & F_ZBAD) st = RBFFD_NONFINITE;
    if (!live) return;
    double *wi = w + i * (int64_t)k_stride;
    const double s2 = OP == 0 ? sc * sc : sc;  // the operator's power of the scale
    const bool good = st == RBFFD_OK;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int rs = r + 32 * s;
        if (rs < n) wi[rs] = good ? zm[s] / s2 : __builtin_nan("");
    }
    for (int q = n + r; q < k_stride; q += 32) wi[q] = 0.0;
    if (r == 0 && status) status[i] = good ? ok_code : st;
}

// One wavefront per pair of stencils; WPB wavefronts (pairs) per block.
template <int KP, int NFIX, int MFIX, int OP, int DIM, int WPB, int OCC>
__global__ __launch_bounds__(WPB * kWave)
__attribute__((amdgpu_waves_per_eu(OCC))) void weights_mf2_kernel(
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
    int64_t n_nodes, const int32_t *__restrict__ nbr, int32_t k_stride,
    const int32_t *__restrict__ rows, int64_t n_rows, double *__restrict__ w,
    int32_t *__restrict__ status, int32_t ok_code) {
    __shared__ __align__(16) char lds[WPB][mf2_lds_bytes<KP, NFIX, MFIX, DIM>()];
    const int wave = threadIdx.x >> 6;
    const int64_t i0 = 2 * ((int64_t)blockIdx.x * WPB + wave);
    if (i0 >= n_rows) return;  // whole wavefront; no block barrier
    weights_mf2_wave<KP, NFIX, MFIX, OP, DIM>(x, y, z, n_nodes, nbr, k_stride, rows, i0, n_rows,
                                              w, status, ok_code, lds[wave]);
}

// The same over a row list counted on the device (a class of a 3-D
// mixed-order batch): two possible list entries per wavefront, the
// wavefronts past the count returning at once.  (A capped grid walking the
// list with a loop took 3.61 ms for 501k stencils of the 1M cube, against
// 2.86 ms for their share of the plain launch.)
template <int KP, int NFIX, int MFIX, int OP, int DIM, int WPB, int OCC>
__global__ __launch_bounds__(WPB * kWave)
__attribute__((amdgpu_waves_per_eu(OCC))) void weights_mf2_list_kernel(
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
    int64_t n_nodes, const int32_t *__restrict__ nbr, int32_t k_stride,
    const int32_t *__restrict__ rows, const int32_t *__restrict__ n_rows_dev,
    double *__restrict__ w, int32_t *__restrict__ status, int32_t ok_code) {
    __shared__ __align__(16) char lds[WPB][mf2_lds_bytes<KP, NFIX, MFIX, DIM>()];
    const int wave = threadIdx.x >> 6;
    const int64_t c = *n_rows_dev;
    const int64_t i0 = 2 * ((int64_t)blockIdx.x * WPB + wave);
    if (i0 >= c) return;  // whole wavefront; no block barrier
    weights_mf2_wave<KP, NFIX, MFIX, OP, DIM>(x, y, z, n_nodes, nbr, k_stride, rows, i0, c, w,
                                              status, ok_code, lds[wave]);
}

}  // namespace wk
}  // namespace rbffd
