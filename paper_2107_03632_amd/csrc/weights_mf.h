#pragma once
// RBF-FD Laplacian stencil weights, FP64: LU blocked by panels of four
// columns with the trailing updates on the matrix cores.  Instances: K = 84
// (m = 6, n = 56; two wavefronts per stencil) and K = 45 (m = 4, n = 30; one
// wavefront per stencil) in two dimensions; in three, K = 105 (m = 4,
// n = 70; several wavefronts per stencil).  weights_mf2.h holds the form
// with two stencils per wavefront (the 3-D K = 30).
//
// v_mfma_f64_16x16x4f64 forms each output as four fused multiply-adds taken
// in k order, fma(a3, b3, fma(a2, b2, fma(a1, b1, fma(a0, b0, c)))).  A
// right-looking LU whose trailing update is L21 x (-U12) on those units
// therefore applies to every element the fused updates of the unblocked
// elimination, in the same order, and the weights are the same bits as
// those of the other kernels (same shift, scale, assembly, pivot rule and
// back substitution).
//
// Layout: the system padded to NP x NP, NP = 16 NT (96 for K = 84, 48 for
// K = 45; right-hand side in column KP, the other padding rows and columns
// zero, padding rows never pivot), in 16 x 16 tiles held transposed as MFMA
// accumulators: in tile (I, J), lane l = 16 g + j, register r holds row
// 16 I + j, column 16 J + g + 4 r.  With NW wavefronts per stencil,
// wavefront w owns the tile columns J = w, w + NW, ... (all tile rows);
// when NW does not divide NT the last wavefronts own one column fewer.
// With more than two wavefronts the wavefront's index is a run-time value
// (one code path for all of them, its branches uniform).
//
// The four columns of a panel [c0, c0 + 4) are register (c0 % 16) / 4 of
// the tiles of column c0 / 16 (column c0 + g in lane group g).  Their owner
// moves them through LDS to row layout (lane l: rows l, l + 64, ...; four
// columns each) and runs the panel's column steps there as the unblocked
// kernels do: pivot search by the exact (|a|, position) key, the pivot
// row's entries by readlane, the multipliers in place of the column, the
// later panel columns updated with fused multiply-adds.  The multipliers go
// back to LDS, where both wavefronts read them in the B-operand layout.
// When KP is not a multiple of 4 the last panel has fewer column steps and
// the right-hand side is one of its columns.
// At the panel's end (a block barrier with two wavefronts) each wavefront
// forms, for its
// trailing tile columns, the pivot rows' entries with the panel's own
// corrections applied in order (U12, the A operand) and updates every tile
// with one MFMA per tile.  Rows of U go to the packed LDS triangle as they
// are completed; wavefront 0 runs the back substitution from there.

#include "weights_ms.h"

namespace rbffd {
namespace wk {

typedef double mf_v4d __attribute__((ext_vector_type(4)));

// 1 / b with the same bits as the general division 1.0 / b.  For |b| in
// [2^-500, 2^501) that division's prescale steps, its scaled fused step and
// its fix-up leave every value unchanged, and what remains is the
// hardware's reciprocal estimate followed by three Newton steps
// y <- y + y (1 - b y), each a pair of fused multiply-adds (the third is
// the division's quotient correction, the quotient of 1 by b being y).
// Other b (also zero, infinities and NaN) go through the division.
__device__ __forceinline__ double recip_div(double b) {
    const uint32_t ex = (uint32_t)((uint64_t)__double_as_longlong(b) >> 52) & 0x7ffu;
    if (__builtin_expect(ex - 523u <= 1000u, 1)) {
        double y = __builtin_amdgcn_rcp(b);
        double e = fma(-b, y, 1.0);
        y = fma(y, e, y);
        e = fma(-b, y, 1.0);
        y = fma(y, e, y);
        e = fma(-b, y, 1.0);
        return fma(e, y, y);
    }
    return 1.0 / b;
}

// LDS traffic of one wavefront is processed in issue order, so a write by
// one lane is seen by a later read of another lane of the same wavefront
// without waiting for the write to complete; this only keeps the compiler
// from reordering the accesses.
__device__ __forceinline__ void lds_order() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Rows of U when one wavefront owns the stencil: row r (entries r .. KP,
// the right-hand side last) packed right after row r - 1, entry q at
// ubase(r) + q.  (Several wavefronts per stencil keep the pair-interleaved
// rows of MsLds, entry q at ubase(r) + 2 q.)
template <int KP, int MM>
struct MfULds {
    static constexpr int US = 1;  // stride of a row's entries
    __host__ __device__ static constexpr int ubase(int r) { return r * KP - r * (r - 1) / 2; }
    static constexpr int USZ = ubase(KP - 1) + KP + 1;
    static constexpr int ASZ = KP * (MM + 2);  // ux, uy, monomials
    static constexpr int SZ = ((USZ > ASZ ? USZ : ASZ) + 1) & ~1;
};

template <bool ONE, int KP, int MM>
struct MfUSel {
    using type = MsLds<KP, MM>;
};
template <int KP, int MM>
struct MfUSel<true, KP, MM> {
    using type = MfULds<KP, MM>;
};

// LDS of one block: doubles first, then int32.  Panel buffers alternate
// between consecutive panels when several wavefronts share them; there a
// panel is row-major with rows padded to five doubles.  With one wavefront
// the panel is column-major (entry (r, j) at j NP + r: a row's four entries
// are four conflict-free reads at fixed offsets, and the tile layout's
// sixteen rows of one column are consecutive), the pivot rows of a panel's
// end overlay its panel buffer (read out before the rows are written), and
// with the packed rows of U that keeps K = 45 under 10 KB per wavefront:
// 16 wavefronts per CU (15 with the interleaved rows and padded panel
// rows).  In three dimensions the assembly tables hold a third offset.
template <int KP, int MM, int NT, int NW, int DIM = 2>
struct MfLds {
    using U = typename MfUSel<NW == 1, KP, MM>::type;  // rows of U
    static constexpr int NP = 16 * NT;
    static constexpr int NPB = NW > 1 ? 2 : 1;       // panel buffers
    static constexpr int PS = NW > 1 ? 5 : 4;        // panel doubles per row
    static constexpr int NJT = (NT + NW - 1) / NW;  // tile columns per wavefront (at most)
    static constexpr int ASZ3 = DIM == 3 ? (KP * (MM + 3) + 1) & ~1 : 0;
    static constexpr int SZ =                        // U triangle / assembly tables
        U::SZ > ASZ3 ? U::SZ : ASZ3;
    static constexpr int PAN = SZ;                  // [NPB][NP][5] or [4][NP] panel
    static constexpr int UB = NW > 1 ? PAN + NPB * NP * PS : PAN;  // [NW][NJT][4][16] pivot rows
    static constexpr int DBL =
        NW > 1 ? UB + NW * NJT * 64 : PAN + (NP * PS > NJT * 64 ? NP * PS : NJT * 64);
    static constexpr int REC = 0;                   // [NPB][4][2] pivot row, its position
    static constexpr int FL = 8 * NPB;              // flags of wavefronts 1 .. NW - 1
    static constexpr int INTS = FL + (NW > 2 ? NW - 1 : 2);
    static constexpr int BYTES = 8 * DBL + 4 * INTS;
};

// SAVE (one wavefront per stencil only) also writes the factors for the
// adjoint: row r of the factors (its multipliers left of its final
// position, its row of U from there on) at row r, the row at each position,
// the unit-scale solution z and the scale s.
// OP: 0 the Laplacian, 1 d/dx, 2 d/dy, 3 d/dz (three dimensions only)
// (right-hand side and power of the scale).
// DIM 3: nodes in three dimensions (z non-null); the polyharmonic spline
// r^3 with lap r^3 = 12 r, the monomials of degree <= MFIX in three
// variables, each evaluated as (u^a v^b) t^c.
// WV: this wavefront's index in the block, or -1 for a run-time index.
// NFIX = 0: the support size is n_arg (K = n_arg + M <= KP), and the rows
// and columns K .. KP - 1 are identity padding: they hold zeros in the
// first K columns and rows, so no real row takes a multiplier from them or
// a pivot from them (a real row holds a lower position), and the real
// unknowns come out as without the padding.
template <int KP, int NFIX, int MFIX, int NW, int WV, bool SAVE, int OP = 0, int DIM = 2>
__device__ __forceinline__ void weights_mf_wave(
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
    int64_t n_nodes, const int32_t *__restrict__ nbr, int32_t k_stride, int64_t i,
    double *__restrict__ w, int32_t *__restrict__ status, const SaveView &sv, int32_t ok_code,
    char *lds, int n_arg = 0) {
    static_assert(!SAVE || (NW == 1 && DIM == 2),
                  "the factors are saved by the one-wavefront 2-D instance");
    static_assert(DIM == 2 || DIM == 3, "two or three dimensions");
    static_assert(OP >= 0 && OP <= DIM, "operator");
    constexpr int MM = DIM == 2 ? (MFIX + 1) * (MFIX + 2) / 2
                                : (MFIX + 1) * (MFIX + 2) * (MFIX + 3) / 6;
    static_assert(NFIX == 0 || NFIX + MM == KP, "identity padding only with a run-time n");
    static_assert(NFIX > 0 || !SAVE, "the factors: fixed supports only");
    const int n = NFIX ? NFIX : n_arg, K = n + MM;
    constexpr int NT = (KP + 1 + 15) / 16;  // tiles per dimension (rhs included)
    constexpr int NP = 16 * NT;
    constexpr int SL = (NP + kWave - 1) / kWave;  // rows per lane in row layout
    static_assert(NW <= 2 ? NT % NW == 0 : WV < 0, "tile columns of the wavefronts");
    using B = MfLds<KP, MM, NT, NW, DIM>;
    using L = typename B::U;
    constexpr int NJT = B::NJT;
    const int wv = WV >= 0 ? WV : __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    // tile columns this wavefront owns: J = NW jt + wv for jt < njt
    const int njt = WV >= 0 ? NJT : (NT - wv + NW - 1) / NW;
    double *sU = reinterpret_cast<double *>(lds);
    double *s_ux = sU;
    double *s_uy = sU + KP;
    double *s_uz = sU + 2 * KP;  // (three dimensions)
    double(*s_P)[MM] = reinterpret_cast<double(*)[MM]>(sU + DIM * KP);
    double *const s_pan0 = sU + B::PAN;
    // entry (r, j) of panel buffer pb
    auto pan = [s_pan0](int pb, int r, int j) -> double & {
        return NW > 1 ? s_pan0[(pb * NP + r) * 5 + j] : s_pan0[j * NP + r];
    };
    double(*s_ub)[4][16] = reinterpret_cast<double(*)[4][16]>(sU + B::UB + wv * NJT * 64);
    int32_t *si = reinterpret_cast<int32_t *>(lds + 8 * B::DBL);
    int32_t(*s_rec)[4][2] = reinterpret_cast<int32_t(*)[4][2]>(si + B::REC);
    uint32_t *s_fl = reinterpret_cast<uint32_t *>(si + B::FL);

    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane >> 4, jl = lane & 15;

    // ---- shift and scale (row order: rows lane, lane + 64) -----------------
    uint32_t flags = 0;
    double dx[SL], dy[SL], dz[SL];
    double d2m = 0.0;
    const double xi = x[i], yi = y[i];
    const double zi = DIM == 3 ? z[i] : 0.0;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int r = lane + kWave * s;
        dx[s] = 0.0;
        dy[s] = 0.0;
        dz[s] = 0.0;
        if (r < n) {
            const int32_t j = nbr[i * (int64_t)k_stride + r];
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
    const double sc = sqrt(seg_all_max_d<kWave>(d2m, lane));
    if (!isfinite(sc)) flags |= F_NONFIN;  // an offset's square overflowed
    if (sc == 0.0) flags |= F_DUP;
    if (wv == 0) {
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const int r = lane + kWave * s;
            if (r < n) {
                const double ux = dx[s] / sc, uy = dy[s] / sc;
                s_ux[r] = ux;
                s_uy[r] = uy;
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
                    for (int j = 0; j < MM; ++j) s_P[r][j] = px[mono_a(j)] * py[mono_b(j)];
                } else {
                    const double uz = dz[s] / sc;
                    s_uz[r] = uz;
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
                        s_P[r][j] = (px[e3.a[j]] * py[e3.b[j]]) * pt[e3.c[j]];
                }
            }
        }
    }
    // one wavefront: its own LDS traffic is ordered, and it may share its
    // block with a wavefront running another stencil, so no block barrier
    if constexpr (NW > 1)
        __syncthreads();
    else
        lds_order();

    // ---- assembly of this wavefront's tile columns (transposed tiles) ------
    mf_v4d T[NT][NJT];
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
        for (int jt = 0; jt < NJT; ++jt) {
            const int J = NW * jt + wv;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int C = 16 * J + g + 4 * r;
                double v = 0.0;
                if (jt >= njt) {
                    // (no such tile column)
                } else if (16 * J < n && C < n) {
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
                        if (prow && C != R && rr == 0.0) flags |= F_DUP;
                        asm volatile("" : "+v"(flags));
                        phs = rr * sqrt(rr);
                    }
                    const double pt = s_P[C][jr];
                    v = prow ? phs : (qrow ? pt : 0.0);
                } else if (16 * J + 15 >= n && 16 * J < K && C >= n && C < K) {
                    v = prow ? s_P[prow ? R : 0][C - n] : 0.0;
                } else if (NFIX == 0 && C >= K && C < KP) {
                    v = C == R ? 1.0 : 0.0;  // identity padding
                } else if (16 * J + 15 >= KP && 16 * J <= KP && C == KP) {
                    double rb, rq;
                    if constexpr (DIM == 2) {
                        const double r0 = uxr * uxr + uyr * uyr;
                        rb = OP == 0 ? 9.0 * sqrt(r0) : -3.0 * sqrt(r0) * (OP == 1 ? uxr : uyr);
                        rq = OP == 0 ? ((jr == 3 || jr == 5) ? 2.0 : 0.0) : (jr == OP ? 1.0 : 0.0);
                    } else {
                        // lap r^3 = 12 r in 3-D; lap of x^2, y^2, z^2 (j = 4, 7, 9) is 2
                        const double r0 = (uxr * uxr + uyr * uyr) + uzr * uzr;
                        rb = OP == 0 ? 12.0 * sqrt(r0)
                                     : -3.0 * sqrt(r0) * (OP == 1 ? uxr : (OP == 2 ? uyr : uzr));
                        rq = OP == 0 ? ((jr == 4 || jr == 7 || jr == 9) ? 2.0 : 0.0)
                                     : (jr == OP ? 1.0 : 0.0);
                    }
                    v = prow ? rb : (qrow ? rq : 0.0);
                }
                T[I][jt][r] = v;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    asm volatile("" : "+v"(flags));
    // the assembly tables' space becomes the rows of U
    if constexpr (NW > 1)
        __syncthreads();
    else
        lds_order();

    // ---- LU, panels of four columns ----------------------------------------
    // Row-layout state (rows lane, lane + 64): done = pivoted already (or
    // padding), pos = current position of the row.
    int pos[SL];
    bool done[SL];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        pos[s] = lane + kWave * s;
        done[s] = pos[s] >= KP;
    }

#pragma unroll
    for (int c0 = 0; c0 < KP; c0 += 4) {
        const int pb = B::NPB > 1 ? (c0 >> 2) & 1 : 0;
        const int J0 = c0 >> 4;                  // tile column of the panel
        const int rc = (c0 & 15) >> 2;           // its register
        const int nk = KP - c0 < 4 ? KP - c0 : 4;  // column steps in the panel
        if (J0 % NW == wv) {
            const int jt0 = J0 / NW;
            // the panel to row layout through LDS: pc[s][j] = row lane + 64 s,
            // column c0 + j
#pragma unroll
            for (int I = 0; I < NT; ++I) pan(pb, 16 * I + jl, g) = T[I][jt0][rc];
            lds_order();
            double pc[SL][4];
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                const int r = lane + kWave * s;
#pragma unroll
                for (int j = 0; j < 4; ++j) pc[s][j] = r < NP ? pan(pb, r < NP ? r : 0, j) : 0.0;
            }
            uint32_t updm[SL];  // bit j: the row took a multiplier in column c0 + j
#pragma unroll
            for (int s = 0; s < SL; ++s) updm[s] = 0u;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k >= nk) break;
                const int c = c0 + k;
                // pivot search over the slots: exact key (|a| bits, position);
                // bb, bp and bv are read only where ba holds
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
                const uint32_t mh = seg_all<kWave, OpMax>(kh, lane);
                // (some row is always left, so mh >= 1 and only rows still in the
                // search can equal it)
                uint64_t chunk = __ballot(kh == mh);
                if (__builtin_expect((chunk & (chunk - 1ull)) != 0ull, 0)) {
                    uint32_t h2 = kh, l2 = ba ? (uint32_t)bb : 0u;
                    int p2 = ba ? bp : 0x7fffffff;
                    seg_argmax_full<kWave>(h2, l2, p2);
                    chunk = __ballot(ba && bp == p2);
                }
                const int win = __builtin_amdgcn_readfirstlane(__ffsll((unsigned long long)chunk) - 1);
                const int bs = __builtin_amdgcn_readlane(bsl, win);
                const int kp = __builtin_amdgcn_readlane(bp, win);
                const double piv = readlane_d(bv, win);
                // (the larger instances keep the division: a fallback copy in
                // every column step measured slower there)
                const double inv = NT <= 3 ? recip_div(piv) : 1.0 / piv;
                const bool b1 = bs != 0;
                // row c of U, panel columns c .. c0 + 3 (up to the rhs)
                if (lane == win) {
#pragma unroll
                    for (int j = k; j < 4; ++j)
                        if (c0 + j <= KP)
                            sU[L::ubase(c) + L::US * (c0 + j)] = b1 ? pc[SL - 1][j] : pc[0][j];
                }
                double uq[4];
#pragma unroll
                for (int j = k + 1; j < 4; ++j)
                    uq[j] = c0 + j <= KP ? readlane_d(b1 ? pc[SL - 1][j] : pc[0][j], win) : 0.0;
                // multipliers, in place (zero for pivoted rows and the pivot)
#pragma unroll
                for (int s = 0; s < SL; ++s) {
                    const bool upd = !done[s] && !(lane == win && bs == s);
                    const double lmv = upd ? pc[s][k] * inv : 0.0;
                    pc[s][k] = lmv;
                    if constexpr (SAVE) updm[s] |= (upd ? 1u : 0u) << k;
#pragma unroll
                    for (int j = k + 1; j < 4; ++j)
                        if (c0 + j <= KP) pc[s][j] = fma(-lmv, uq[j], pc[s][j]);
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
                if (lane == 0) {
                    s_rec[pb][k][0] = win + kWave * bs;
                    s_rec[pb][k][1] = kp;
                }
            }
            // the panel's multipliers, row layout, for both wavefronts
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                const int r = lane + kWave * s;
                if (r < NP) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) pan(pb, r, j) = pc[s][j];
                }
                if constexpr (SAVE) {
                    // the multipliers of L, where the row took them
                    if (r < K) {
                        double *dst = sv.lu + i * (int64_t)sv.kmax * sv.kmax + (int64_t)r * K;
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            if (j < nk && ((updm[s] >> j) & 1u)) dst[c0 + j] = pc[s][j];
                    }
                }
            }
        }
        if constexpr (NW > 1)
            __syncthreads();
        else
            lds_order();

        // ---- panel end: trailing tile columns of this wavefront ------------
        int pr[4] = {0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nk) pr[k] = __builtin_amdgcn_readfirstlane(s_rec[pb][k][0]);
        if (J0 % NW != wv) {
            // the owner's row bookkeeping, replayed
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k >= nk) break;
                const int c = c0 + k;
                const int kp = __builtin_amdgcn_readfirstlane(s_rec[pb][k][1]);
#pragma unroll
                for (int s = 0; s < SL; ++s) {
                    const bool isp = lane + kWave * s == pr[k];
                    pos[s] = isp ? c : ((!done[s] && pos[s] == c) ? kp : pos[s]);
                    done[s] = done[s] || isp;
                    int dn = done[s] ? 1 : 0;
                    asm volatile("" : "+v"(pos[s]), "+v"(dn));
                    done[s] = dn != 0;
                }
            }
        }
        // first tile column of this wavefront that still has trailing columns
        const int first_jt = (J0 % NW == wv) ? ((rc < 3) ? J0 / NW : J0 / NW + 1)
                                             : (J0 - wv + NW) / NW;
        if (first_jt < njt) {  // (a partial panel is the last: nothing trails it)
            // multipliers of the panel's pivot rows in its earlier columns
            double l11[4][3];
#pragma unroll
            for (int m2 = 1; m2 < 4; ++m2)
#pragma unroll
                for (int k2 = 0; k2 < m2; ++k2) l11[m2][k2] = pan(pb, pr[m2], k2);
            // B operands: lane (g, j) holds the multiplier of row 16 I + j in
            // panel column c0 + g
            double Bop[NT];
#pragma unroll
            for (int I = 0; I < NT; ++I) Bop[I] = pan(pb, 16 * I + jl, g);
            lds_order();  // (with one wavefront the rows below overlay the panel)
            // the panel's pivot rows, in every trailing tile column of this
            // wavefront, to LDS (one uniform branch per row)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int Ipk = pr[k] >> 4, ipk = pr[k] & 15;
                if (jl == ipk) {
#pragma unroll
                    for (int I = 0; I < NT; ++I) {
                        if (I == Ipk) {
#pragma unroll
                            for (int jt = 0; jt < NJT; ++jt)
                                // (with a run-time wavefront index every tile
                                // column: fewer branches, the extra rows unread)
                                if (WV < 0 || (jt >= first_jt && jt < njt)) {
#pragma unroll
                                    for (int r = 0; r < 4; ++r)
                                        s_ub[jt][k][g + 4 * r] = T[I][jt][r];
                                }
                            // keeps each case's stores in its own branch
                            // (merged, they would first copy the row
                            // into common registers)
                            asm volatile(";tile row %0" ::"i"(I) : "memory");
                        }
                    }
                }
            }
            lds_order();
            // the tile column of the next panel first: its updates are the
            // ones the next column steps wait for (with a run-time wavefront
            // index simply in order)
            const int J0n = (c0 + 4) >> 4;
            const int jtn = (J0n % NW == wv && c0 + 4 < KP) ? J0n / NW : -1;
#pragma unroll
            for (int pass = 0; pass < (WV < 0 ? 1 : 2); ++pass) {
#pragma unroll
                for (int jt = 0; jt < NJT; ++jt) {
                    if (jt < first_jt || jt >= njt) continue;
                    if (WV >= 0 && (pass == 0) != (jt == jtn)) continue;
                    const int J = NW * jt + wv;
                    const int i0 = (J == J0) ? 4 * rc + 4 : 0;  // first trailing column in the tile
                    const double r0 = s_ub[jt][0][jl], r1 = s_ub[jt][1][jl];
                    const double r2 = s_ub[jt][2][jl], r3 = s_ub[jt][3][jl];
                    const double u0 = r0;
                    const double u1 = fma(-l11[1][0], u0, r1);
                    const double u2 = fma(-l11[2][1], u1, fma(-l11[2][0], u0, r2));
                    const double u3 =
                        fma(-l11[3][2], u2, fma(-l11[3][1], u1, fma(-l11[3][0], u0, r3)));
                    const double ug = g == 0 ? u0 : (g == 1 ? u1 : (g == 2 ? u2 : u3));
                    const int q = 16 * J + jl;
                    if (jl >= i0 && q <= KP) sU[L::ubase(c0 + g) + L::US * q] = ug;
                    const double Aop = jl >= i0 ? -ug : 0.0;
#pragma unroll
                    for (int I = 0; I < NT; ++I)
                        T[I][jt] =
                            __builtin_amdgcn_mfma_f64_16x16x4f64(Aop, Bop[I], T[I][jt], 0, 0, 0);
                }
            }
            lds_order();  // s_ub is rewritten at the next panel
        }
    }
    uint32_t fl = seg_all<kWave, OpOr>(flags, lane);
    if constexpr (NW > 1) {
        // the other wavefronts' flags to wavefront 0
        if (wv != 0 && lane == 0) s_fl[wv - 1] = fl;
        __syncthreads();  // the rows of U and the flags are visible
        if (wv != 0) return;
#pragma unroll
        for (int v = 0; v < NW - 1; ++v) fl |= s_fl[v];
    } else {
        lds_order();
    }

    // ---- back substitution over the rows of U in LDS (wavefront 0) ---------
    int ub[SL];
    double yb[SL], mb[SL], zm[SL];
    double ur[1][1];
    uint32_t lukey = 0;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int r0 = lane + kWave * s;
        const int r = r0 < KP ? r0 : KP - 1;
        ub[s] = L::ubase(r);
        yb[s] = sU[ub[s] + L::US * KP];
        const double d = sU[ub[s] + L::US * r];
        mb[s] = 1.0 / d;
        zm[s] = 0.0;
        const uint32_t f = !isfinite(d) ? L_NONFIN : (d == 0.0 ? L_SING : 0u);
        const uint32_t key = ((uint32_t)(KP - r0) << 2) | f;
        if (r0 < KP && f && key > lukey) lukey = key;
    }
    const uint32_t luflag = seg_all<kWave, OpMax>(lukey, lane) & 3u;
    bc_step<KP, kWave, SL, KP - 1, false, L::US>(sU, ub, ur[0], yb, mb, zm, lane, false);

#pragma unroll
    for (int s = 0; s < SL; ++s)
        if (lane + kWave * s < K && !isfinite(zm[s])) fl |= F_ZBAD;
    fl = seg_all<kWave, OpOr>(fl, lane);
    int st = RBFFD_OK;
    if (fl & F_BADIDX) st = RBFFD_BAD_INDEX;
    else if (fl & F_NONFIN) st = RBFFD_NONFINITE;
    else if (fl & F_DUP) st = RBFFD_DUPLICATE;
    else if (luflag == L_NONFIN) st = RBFFD_NONFINITE;
    else if (luflag == L_SING) st = RBFFD_SINGULAR;
    else if (fl & F_ZBAD) st = RBFFD_NONFINITE;
    double *wi = w + i * (int64_t)k_stride;
    const double s2 = OP == 0 ? sc * sc : sc;  // the operator's power of the scale
    const bool good = st == RBFFD_OK;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int r = lane + kWave * s;
        if (r < n) wi[r] = good ? zm[s] / s2 : __builtin_nan("");
    }
    for (int q = n + lane; q < k_stride; q += kWave) wi[q] = 0.0;
    if (lane == 0 && status) status[i] = good ? ok_code : st;
    if constexpr (SAVE) {
        // the row at each position (in the free panel buffer), then each
        // row of U at its row's index, lanes along the columns
        int32_t *s_row = reinterpret_cast<int32_t *>(s_pan0);
#pragma unroll
        for (int s = 0; s < SL; ++s)
            if (pos[s] < K) s_row[pos[s]] = lane + kWave * s;
        lds_order();
        double *lu = sv.lu + i * (int64_t)sv.kmax * sv.kmax;
        for (int p = 0; p < K; ++p) {
            const int r = __builtin_amdgcn_readfirstlane(s_row[p]);
            for (int q = p + lane; q < K; q += kWave) lu[(int64_t)r * K + q] = sU[L::ubase(p) + L::US * q];
            if (lane == 0) sv.perm[i * (int64_t)sv.kmax + p] = (uint8_t)r;
        }
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const int c = lane + kWave * s;
            if (c < K) sv.z[i * (int64_t)sv.kmax + c] = zm[s];
        }
        if (lane == 0) sv.s[i] = sc;
    }
}

// One block (NW wavefronts) computes stencil `t` of the row list.
template <int KP, int NFIX, int MFIX, int NW, bool SAVE = false, int OP = 0>
__device__ __forceinline__ void weights_mf_body(
    const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
    const int32_t *__restrict__ nbr, int32_t k_stride, const int32_t *__restrict__ rows,
    int64_t n_rows, double *__restrict__ w, int32_t *__restrict__ status, int32_t ok_code,
    int64_t t, char *lds, const SaveView &sv = SaveView{}) {
    if (t >= n_rows) return;  // whole block idle
    const int64_t i = rows ? (int64_t)rows[t] : t;
    static_assert(NW <= 2, "two-dimensional instances: one or two wavefronts");
    if (NW > 1 && ((threadIdx.x >> 6) & 1))
        weights_mf_wave<KP, NFIX, MFIX, NW, NW - 1, SAVE, OP>(x, y, nullptr, n_nodes, nbr,
                                                         k_stride, i, w, status, sv, ok_code, lds);
    else
        weights_mf_wave<KP, NFIX, MFIX, NW, 0, SAVE, OP>(x, y, nullptr, n_nodes, nbr, k_stride, i,
                                                     w, status, sv, ok_code, lds);
}

template <int KP, int NFIX, int MFIX>
__host__ __device__ constexpr int mf_lds_bytes(int nw) {
    constexpr int MM = (MFIX + 1) * (MFIX + 2) / 2;
    constexpr int NT = (KP + 1 + 15) / 16;
    return nw > 1 ? MfLds<KP, MM, NT, 2>::BYTES : MfLds<KP, MM, NT, 1>::BYTES;
}

template <int KP, int NFIX, int MFIX, int NW, int OCC, bool SAVE, int OP = 0>
__global__ __launch_bounds__(NW * kWave)
__attribute__((amdgpu_waves_per_eu(OCC))) void weights_mf_kernel(
    const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
    const int32_t *__restrict__ nbr, int32_t k_stride, const int32_t *__restrict__ rows,
    const int32_t *__restrict__ n_rows_dev, int64_t n_rows, double *__restrict__ w,
    int32_t *__restrict__ status, SaveView sv, int32_t ok_code) {
    __shared__ __align__(16) char lds[mf_lds_bytes<KP, NFIX, MFIX>(NW)];
    if (n_rows_dev) n_rows = *n_rows_dev;
    weights_mf_body<KP, NFIX, MFIX, NW, SAVE, OP>(x, y, n_nodes, nbr, k_stride, rows, n_rows, w,
                                              status, ok_code, (int64_t)blockIdx.x, lds, sv);
}

// A row list counted on the device (the mixed path's fallbacks, the
// per-order lists of a mixed-order batch): the host knows only an upper
// bound, so a grid of at most kListBlocks blocks walks the list with a
// stride.  An empty or short list then costs a few thousand idle blocks, not
// one per node (1M idle blocks took 0.21 ms).
constexpr int64_t kListBlocks = 8192;

template <int KP, int NFIX, int MFIX, int NW, int OCC, int OP>
__global__ __launch_bounds__(NW * kWave)
__attribute__((amdgpu_waves_per_eu(OCC))) void weights_mf_list_kernel(
    const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
    const int32_t *__restrict__ nbr, int32_t k_stride, const int32_t *__restrict__ rows,
    const int32_t *__restrict__ n_rows_dev, double *__restrict__ w,
    int32_t *__restrict__ status, int32_t ok_code) {
    __shared__ __align__(16) char lds[mf_lds_bytes<KP, NFIX, MFIX>(NW)];
    const int64_t c = *n_rows_dev;
    for (int64_t t = blockIdx.x; t < c; t += gridDim.x) {
        // the previous stencil's LDS is free
        if constexpr (NW > 1)
            __syncthreads();
        else
            lds_order();
        weights_mf_body<KP, NFIX, MFIX, NW, false, OP>(x, y, n_nodes, nbr, k_stride, rows, c, w,
                                                   status, ok_code, t, lds);
    }
}

// sv.lu set: the saving instance (one wavefront per stencil only).
// n_rows_dev set: a device-counted list of at most n_rows entries, walked
// by a capped grid, or with per_entry by one block per possible entry (the
// blocks past the count return at once; no loop, so the register allocation
// of the plain kernel).
template <int KP, int NFIX, int MFIX, int NW, int OCC, int OP = 0>
inline int launch_mf(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                     int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev,
                     int64_t n_rows, double *w, int32_t *status, const SaveView &sv,
                     int32_t ok_code, hipStream_t stream, bool per_entry = false) {
    if (n_rows <= 0) return RBFFD_SUCCESS;
    if (n_rows > 0x7fffffff) return RBFFD_ERR_UNSUPPORTED;
    if (sv.lu && OP != 0) return RBFFD_ERR_UNSUPPORTED;  // factors: the Laplacian only
    if constexpr (NW == 1) {
        if (sv.lu) {
            hipLaunchKernelGGL((weights_mf_kernel<KP, NFIX, MFIX, NW, OCC, true>),
                               dim3((unsigned)n_rows), dim3(NW * kWave), 0, stream, x, y,
                               n_nodes, nbr, k_stride, rows, n_rows_dev, n_rows, w, status, sv,
                               ok_code);
            return last_launch_rc();
        }
    } else {
        if (sv.lu) return RBFFD_ERR_UNSUPPORTED;
    }
    if (n_rows_dev && !per_entry) {
        const int64_t blocks = n_rows < kListBlocks ? n_rows : kListBlocks;
        hipLaunchKernelGGL((weights_mf_list_kernel<KP, NFIX, MFIX, NW, OCC, OP>),
                           dim3((unsigned)blocks), dim3(NW * kWave), 0, stream, x, y, n_nodes,
                           nbr, k_stride, rows, n_rows_dev, w, status, ok_code);
        return last_launch_rc();
    }
    hipLaunchKernelGGL((weights_mf_kernel<KP, NFIX, MFIX, NW, OCC, false, OP>),
                       dim3((unsigned)n_rows), dim3(NW * kWave), 0, stream, x, y, n_nodes, nbr,
                       k_stride, rows, n_rows_dev, n_rows, w, status, SaveView{}, ok_code);
    return last_launch_rc();
}

// Three dimensions: one block of NW wavefronts per stencil (node i = block
// index), no row list, no saved factors.
template <int KP, int NFIX, int MFIX, int NW>
__host__ __device__ constexpr int mf3_lds_bytes() {
    constexpr int MM = (MFIX + 1) * (MFIX + 2) * (MFIX + 3) / 6;
    constexpr int NT = (KP + 1 + 15) / 16;
    return MfLds<KP, MM, NT, NW, 3>::BYTES;
}

template <int KP, int NFIX, int MFIX, int NW, int OCC, int OP>
__global__ __launch_bounds__(NW * kWave)
__attribute__((amdgpu_waves_per_eu(OCC))) void weights_mf3_kernel(
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
    int64_t n_nodes, const int32_t *__restrict__ nbr, int32_t k_stride, double *__restrict__ w,
    int32_t *__restrict__ status, int32_t n_arg) {
    __shared__ __align__(16) char lds[mf3_lds_bytes<KP, NFIX, MFIX, NW>()];
    const int64_t i = (int64_t)blockIdx.x;
    if constexpr (NW <= 2) {
        if (NW > 1 && ((threadIdx.x >> 6) & 1))
            weights_mf_wave<KP, NFIX, MFIX, NW, NW - 1, false, OP, 3>(
                x, y, z, n_nodes, nbr, k_stride, i, w, status, SaveView{}, RBFFD_OK, lds, n_arg);
        else
            weights_mf_wave<KP, NFIX, MFIX, NW, 0, false, OP, 3>(
                x, y, z, n_nodes, nbr, k_stride, i, w, status, SaveView{}, RBFFD_OK, lds, n_arg);
    } else {
        weights_mf_wave<KP, NFIX, MFIX, NW, -1, false, OP, 3>(
            x, y, z, n_nodes, nbr, k_stride, i, w, status, SaveView{}, RBFFD_OK, lds, n_arg);
    }
}

// The same over a row list counted on the device (a class of a 3-D
// mixed-order batch): one block per possible entry, block t computing node
// rows[t] or returning at once past the count.  (A capped grid walking the
// list kept more values live across its loop: 256 VGPRs with spills
// against 168; the idle blocks of a half-empty list cost about 0.2 ms per
// million.)
template <int KP, int NFIX, int MFIX, int NW, int OCC, int OP>
__global__ __launch_bounds__(NW * kWave)
__attribute__((amdgpu_waves_per_eu(OCC))) void weights_mf3_list_kernel(
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
    int64_t n_nodes, const int32_t *__restrict__ nbr, int32_t k_stride,
    const int32_t *__restrict__ rows, const int32_t *__restrict__ n_rows_dev,
    double *__restrict__ w, int32_t *__restrict__ status) {
    __shared__ __align__(16) char lds[mf3_lds_bytes<KP, NFIX, MFIX, NW>()];
    static_assert(NFIX > 0, "fixed supports");
    const int64_t t = (int64_t)blockIdx.x;
    if (t >= *n_rows_dev) return;  // whole block idle
    const int64_t i = rows[t];
    if constexpr (NW <= 2) {
        if (NW > 1 && ((threadIdx.x >> 6) & 1))
            weights_mf_wave<KP, NFIX, MFIX, NW, NW - 1, false, OP, 3>(
                x, y, z, n_nodes, nbr, k_stride, i, w, status, SaveView{}, RBFFD_OK, lds);
        else
            weights_mf_wave<KP, NFIX, MFIX, NW, 0, false, OP, 3>(
                x, y, z, n_nodes, nbr, k_stride, i, w, status, SaveView{}, RBFFD_OK, lds);
    } else {
        weights_mf_wave<KP, NFIX, MFIX, NW, -1, false, OP, 3>(
            x, y, z, n_nodes, nbr, k_stride, i, w, status, SaveView{}, RBFFD_OK, lds);
    }
}

// rows, n_rows_dev: a device list of at most max_rows node ids and its
// length.
template <int KP, int NFIX, int MFIX, int NW, int OCC, int OP>
inline int launch_mf3_list(const double *x, const double *y, const double *z, int64_t n_nodes,
                           const int32_t *nbr, int32_t k_stride, const int32_t *rows,
                           const int32_t *n_rows_dev, int64_t max_rows, double *w,
                           int32_t *status, hipStream_t stream) {
    if (max_rows <= 0) return RBFFD_SUCCESS;
    if (max_rows > 0x7fffffff) return RBFFD_ERR_UNSUPPORTED;
    hipLaunchKernelGGL((weights_mf3_list_kernel<KP, NFIX, MFIX, NW, OCC, OP>),
                       dim3((unsigned)max_rows), dim3(NW * kWave), 0, stream, x, y, z, n_nodes,
                       nbr, k_stride, rows, n_rows_dev, w, status);
    return last_launch_rc();
}

// n: the support size when NFIX = 0 (K = n + M <= KP), else ignored.
template <int KP, int NFIX, int MFIX, int NW, int OCC, int OP>
inline int launch_mf3(const double *x, const double *y, const double *z, int64_t n_nodes,
                      const int32_t *nbr, int32_t k_stride, double *w, int32_t *status,
                      hipStream_t stream, int n = NFIX) {
    constexpr int MM = (MFIX + 1) * (MFIX + 2) * (MFIX + 3) / 6;
    if (n_nodes <= 0) return RBFFD_SUCCESS;
    if (n_nodes > 0x7fffffff) return RBFFD_ERR_UNSUPPORTED;
    if (n < 1 || n + MM > KP || (NFIX && n != NFIX)) return RBFFD_ERR_UNSUPPORTED;
    hipLaunchKernelGGL((weights_mf3_kernel<KP, NFIX, MFIX, NW, OCC, OP>),
                       dim3((unsigned)n_nodes), dim3(NW * kWave), 0, stream, x, y, z, n_nodes,
                       nbr, k_stride, w, status, (int32_t)n);
    return last_launch_rc();
}

}  // namespace wk
}  // namespace rbffd
