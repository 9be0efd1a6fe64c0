#pragma once
// RBF-FD Laplacian stencil weights, FP64: several stencils per wavefront,
// several matrix rows per lane.
//
// Same arithmetic as weights_kernel.h (the sequence of IEEE operations of
// the reference definition: shift, scale, r^3 + monomial assembly, LU with
// partial pivoting using pivot reciprocals and fma(-l, u, a) updates,
// forward elimination of the right-hand side, back substitution, w = z/s^2),
// laid out so that the per-column overhead of the elimination (pivot search,
// reciprocal, bookkeeping) is shared by 64/SEG stencils:
//   * a segment of SEG consecutive lanes (8, 16, 32 or 64) owns one stencil;
//     lane l of the segment holds rows l, l+SEG, ..., l+(SL-1)*SEG ("slots")
//     of the augmented matrix in registers; slots past the last row are empty;
//   * reductions inside a segment use DPP: for SEG <= 16 an all-reduce made
//     of row_mirror / row_half_mirror / quad_perm exchanges (every lane gets
//     the result, no LDS and no scalar round trip); wider segments finish
//     with row_bcast and readlane;
//   * the pivot search first compares the slots of a lane exactly (full
//     |a| bits, then position), then takes the segment maximum of the high
//     words; a ballot decides whether that maximum is unique, otherwise a
//     butterfly over the full keys (|a| bits, position) settles ties;
//   * the winning lane writes its pivot row, its right-hand side and its
//     position to LDS; one LDS read of each pivot entry feeds the fused
//     updates of all SL slots of a lane.
// One block is one wavefront, so LDS ordering needs no barrier instruction.

#include "common.h"
#include "weights_kernel.h"

namespace rbffd {
namespace wk {

using lds_f64 = __attribute__((address_space(3))) double;

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
}

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xf, 0xf, false);
}

struct OpMax {
    __device__ static uint32_t f(uint32_t a, uint32_t b) { return a > b ? a : b; }
};
struct OpOr {
    __device__ static uint32_t f(uint32_t a, uint32_t b) { return a | b; }
};

// All-reduce over each SEG-lane segment; every lane receives the result.
// Inside a 16-lane row: DPP exchanges.  Across the rows of a 32-lane
// segment: permlane16_swap (rows 2k <-> 2k+1).  Over the whole wavefront:
// row 0 into row 1 and row 2 into row 3 (row_bcast:15), then lane 31 into
// rows 2 and 3 (row_bcast:31), after which lane 63 holds the result and
// readlane makes it uniform.  All in the VALU (no LDS); zero is the
// identity of both operations, so the rows a broadcast skips see zero.
template <int SEG, class Op>
__device__ __forceinline__ uint32_t seg_all(uint32_t v, int /*lane*/) {
    static_assert(SEG == 4 || SEG == 8 || SEG == 16 || SEG == 32 || SEG == 64, "segment width");
    if constexpr (SEG >= 16) v = Op::f(v, dpp_u32<0x140>(v));  // row_mirror
    if constexpr (SEG >= 8) v = Op::f(v, dpp_u32<0x141>(v));   // row_half_mirror
    v = Op::f(v, dpp_u32<0x4E>(v));                            // quad_perm [2,3,0,1]
    v = Op::f(v, dpp_u32<0xB1>(v));                            // quad_perm [1,0,3,2]
    if constexpr (SEG == 64) {
        v = Op::f(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));
        v = Op::f(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));
        return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
    }
    if constexpr (SEG == 32) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        v = Op::f(r[0], r[1]);
    }
    return v;
}

// Lane SRC of each SEG-lane segment, delivered to every lane of the segment.
template <int SEG, int SRC>
__device__ __forceinline__ uint32_t seg_bcast_u32(uint32_t v, bool upper8) {
    static_assert(SRC >= 0 && SRC < SEG, "source lane");
    if constexpr (SEG == 4) {
        return dpp_mov<SRC | (SRC << 2) | (SRC << 4) | (SRC << 6)>(v);  // quad_perm
    } else if constexpr (SEG == 8) {
        const uint32_t a = dpp_mov<0x150 + SRC>(v);  // row_newbcast
        const uint32_t b = dpp_mov<0x158 + SRC>(v);
        return upper8 ? b : a;
    } else if constexpr (SEG == 16) {
        return dpp_mov<0x150 + SRC>(v);
    } else if constexpr (SEG == 32) {
        const uint32_t t = dpp_mov<0x150 + (SRC & 15)>(v);
        const auto r = __builtin_amdgcn_permlane16_swap(t, t, false, false);
        return (SRC < 16) ? r[0] : r[1];
    } else {
        return (uint32_t)__builtin_amdgcn_readlane((int)v, SRC);
    }
}

template <int SEG, int SRC>
__device__ __forceinline__ double seg_bcast_d(double v, bool upper8) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t hi = seg_bcast_u32<SEG, SRC>((uint32_t)(b >> 32), upper8);
    const uint32_t lo = seg_bcast_u32<SEG, SRC>((uint32_t)b, upper8);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <int SEG>
__device__ __forceinline__ double seg_all_max_d(double v, int lane) {
    // values are >= 0, so their bit patterns order like the values
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    uint32_t hi = (uint32_t)(b >> 32), lo = (uint32_t)b;
    const uint32_t mh = seg_all<SEG, OpMax>(hi, lane);
    lo = (hi == mh) ? lo : 0u;
    const uint32_t ml = seg_all<SEG, OpMax>(lo, lane);
    return __longlong_as_double((long long)(((uint64_t)mh << 32) | ml));
}

template <int SEG>
__device__ __forceinline__ double seg_all_or_d(double v, int lane) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t hi = seg_all<SEG, OpOr>((uint32_t)(b >> 32), lane);
    const uint32_t lo = seg_all<SEG, OpOr>((uint32_t)b, lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// full (|a| bits, position) key butterfly inside a segment (ties only)
template <int SEG>
__device__ __forceinline__ void seg_argmax_full(uint32_t &kh, uint32_t &kl, int &kp) {
#pragma unroll
    for (int o = SEG / 2; o > 0; o >>= 1) {
        const uint32_t oh = (uint32_t)__shfl_xor((int)kh, o, SEG);
        const uint32_t ol = (uint32_t)__shfl_xor((int)kl, o, SEG);
        const int op = __shfl_xor(kp, o, SEG);
        if (key_better(oh, ol, op, kh, kl, kp)) {
            kh = oh;
            kl = ol;
            kp = op;
        }
    }
}

// LDS of one stencil.  During assembly: the scaled offsets and the monomial
// table.  From the elimination on: the rows of U with their right-hand side,
// in pivot order (row c holds columns c..KP-1 and, at KP, the eliminated
// right-hand side).  Rows 2p and 2p+1 share one region, interleaved, so the
// entries of one row lie 16 bytes apart: a row is stored with 64-bit writes
// that never merge into 128-bit ones (which would need contiguous registers).
template <int KP, int MM>
struct MsLds {
    static constexpr int US = 2;  // stride of a row's entries
    // start of the region of rows 2p, 2p+1
    __host__ __device__ static constexpr int region(int p) { return 2 * p * (KP + 2 - p); }
    // entry q of row r sits at ubase(r) + 2 q
    __host__ __device__ static constexpr int ubase(int r) {
        return region(r / 2) - 4 * (r / 2) + (r & 1);
    }
    static constexpr int USZ = region((KP + 1) / 2);
    static constexpr int ASZ = KP * (MM + 2);  // ux, uy, monomials
    static constexpr int SZ = ((USZ > ASZ ? USZ : ASZ) + 1) & ~1;
};

// LDS bytes of weights_ms_body for WPB wavefronts per block.
template <int KP, int SEG, int MFIX, int WPB>
__host__ __device__ constexpr int ms_lds_bytes() {
    constexpr int MM = MFIX ? (MFIX + 1) * (MFIX + 2) / 2 : 28;
    constexpr int GPB = kWave / SEG;
    return (int)sizeof(double) * WPB * GPB * MsLds<KP, MM>::SZ + 4 * WPB * 2 * GPB;
}

// LDS ordering inside one wavefront: this wave's earlier LDS writes are
// complete and visible to its later reads (no barrier with other waves).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// One column of the back substitution (column C, then C-1, ... down to 0):
// the source lane of the broadcast must be a compile-time constant.
// PRE: the lane's rows of U were copied to registers ur[s][q] (row-major,
// stride KP) beforehand.  US: the stride of a row's entries in sU.
template <int KP, int SEG, int SL, int C, bool PRE, int US = 2>
__device__ __forceinline__ void bc_step(const double *sU, const int *ub, const double *ur,
                                        double *yb, const double *mb, double *zm, int l0,
                                        bool upper8) {
    if constexpr (C >= 0) {
        constexpr int S = C / SEG, LC = C % SEG;
        const double zl = yb[S] * mb[S];  // z_C, meaningful in lane LC
        const double z = seg_bcast_d<SEG, LC>(zl, upper8);
        zm[S] = (l0 == LC) ? z : zm[S];
#pragma unroll
        for (int s = 0; s < SL; ++s)
            if (SEG * s < C) {
                const double uc = PRE ? ur[s * KP + C] : sU[ub[s] + US * C];
                yb[s] = fma(-uc, z, yb[s]);
            }
        bc_step<KP, SEG, SL, C - 1, PRE, US>(sU, ub, ur, yb, mb, zm, l0, upper8);
    }
}

// One wavefront computes the stencils of group `grp` (stencils
// grp*GPB .. grp*GPB+GPB-1 of the row list).  WPB wavefronts of a block run
// independent groups; `wave` selects this wavefront's LDS.  SAVE keeps the
// multipliers of L in registers and writes the factors for the adjoint.
// OP: 0 the Laplacian, 1 d/dx, 2 d/dy (the right-hand side of eq. (1) and
// the power of the scale; see rbffd_weights_op).
template <int KP, int SEG, int SL, int NFIX, int MFIX, int WPB, bool SAVE, int OP = 0>
__device__ __forceinline__ void weights_ms_body(
    const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
    const int32_t *__restrict__ nbr, int32_t k_stride, const int32_t *__restrict__ rows,
    int64_t n_rows, int32_t n_arg, int32_t m_arg, double *__restrict__ w,
    int32_t *__restrict__ status, double *__restrict__ sv_lu, double *__restrict__ sv_z,
    double *__restrict__ sv_s, uint8_t *__restrict__ sv_perm, int32_t sv_kmax, int32_t ok_code,
    int64_t grp, int wave, char *lds) {
    static_assert(SEG * SL >= KP, "slots must cover the system");
    constexpr int GPB = kWave / SEG;
    constexpr int MM = MFIX ? (MFIX + 1) * (MFIX + 2) / 2 : 28;
    using L = MsLds<KP, MM>;
    const int n = NFIX ? NFIX : n_arg;
    const int m = MFIX ? MFIX : m_arg;
    const int NM = (m + 1) * (m + 2) / 2;
    const int K = n + NM;

    // block LDS (ms_lds_bytes): [WPB][GPB][SZ] doubles, then the pivot
    // positions [WPB][2][GPB]
    auto s_lds = reinterpret_cast<double(*)[GPB][L::SZ]>(lds);
    auto s_pos_b = reinterpret_cast<int32_t(*)[2][GPB]>(lds + sizeof(double) * WPB * GPB * L::SZ);

    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / SEG;
    const int l0 = lane % SEG;
    double *sU = s_lds[wave][g];
    double *s_ux = sU;                                          // [KP]
    double *s_uy = sU + KP;                                     // [KP]
    double(*s_P)[MM] = reinterpret_cast<double(*)[MM]>(sU + 2 * KP);  // [KP][MM]
    int32_t(*s_pos)[GPB] = s_pos_b[wave];

    if (grp * GPB >= n_rows) return;  // whole wave idle
    const int64_t t = grp * GPB + g;
    const bool valid = t < n_rows;
    const int64_t i = valid ? (rows ? (int64_t)rows[t] : t) : 0;

    // ---- shift: offsets of the support nodes ------------------------------
    uint32_t flags = 0;
    double dx[SL], dy[SL];
    double d2m = 0.0;
    const double xi = x[i], yi = y[i];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int r = l0 + SEG * s;
        dx[s] = 0.0;
        dy[s] = 0.0;
        if (valid && r < n) {
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

    // ---- scale; monomial table --------------------------------------------
    double ux[SL], uy[SL];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int r = l0 + SEG * s;
        ux[s] = 0.0;
        uy[s] = 0.0;
        if (r < n) {
            ux[s] = dx[s] / sc;
            uy[s] = dy[s] / sc;
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
    wave_sync();

    // ---- assemble the rows of every slot -----------------------------------
    double a[SL][KP];
    double yv[SL];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int r = l0 + SEG * s;
        const bool prow = r < n;
        const bool qrow = r >= n && r < K;
        const int jr = qrow ? r - n : 0;
        // slots whose rows all lie past the support rows skip the r^3 block
        const bool any_p = !NFIX || SEG * s < NFIX;
#pragma unroll
        for (int l = 0; l < KP; ++l) {
            if (l < n) {
                double phs = 0.0;
                if (any_p) {
                    const double ex = ux[s] - s_ux[l];
                    const double ey = uy[s] - s_uy[l];
                    const double rr = ex * ex + ey * ey;
                    if (prow && l != r && rr == 0.0) flags |= F_DUP;
                    // settle the check now: sunk past the loop it would keep
                    // every squared distance alive (no instruction emitted)
                    asm volatile("" : "+v"(flags));
                    phs = rr * sqrt(rr);
                }
                const double pt = s_P[l][jr];
                a[s][l] = prow ? phs : (qrow ? pt : 0.0);
            } else if (l < K) {
                a[s][l] = prow ? s_P[r < KP ? r : 0][l - n] : 0.0;
            } else {
                a[s][l] = (l == r) ? 1.0 : 0.0;
            }
            if ((l & 1) == 1) __builtin_amdgcn_sched_barrier(0);
        }
        const double r0 = ux[s] * ux[s] + uy[s] * uy[s];
        const double rb =
            OP == 0 ? 9.0 * sqrt(r0) : -3.0 * sqrt(r0) * (OP == 1 ? ux[s] : uy[s]);
        const double rq = OP == 0 ? ((jr == 3 || jr == 5) ? 2.0 : 0.0) : (jr == OP ? 1.0 : 0.0);
        yv[s] = prow ? rb : (qrow ? rq : 0.0);
    }
    // materialise the flags here: otherwise the duplicate checks sink to the
    // end of the kernel and keep every squared distance alive through the LU
    asm volatile("" : "+v"(flags));
    wave_sync();  // the assembly tables' space becomes the rows of U

    // ---- LU with partial pivoting, right-looking, rhs carried along --------
    int pos[SL];
    bool done[SL];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        pos[s] = l0 + SEG * s;
        done[s] = pos[s] >= KP;
    }
    const uint64_t segmask = SEG == 64 ? ~0ull : ((1ull << (SEG & 63)) - 1ull);
    const int segbase = g * SEG;
#pragma unroll
    for (int c = 0; c < KP; ++c) {
        const int buf = c & 1;
        // best slot of this lane: exact key (|a| bits, position)
        uint64_t bb = 0;
        int bp = 0x7fffffff, bs = 0;
        double bv = 0.0;
        bool ba = false;
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const uint64_t bits = (uint64_t)__double_as_longlong(a[s][c]) & 0x7fffffffffffffffull;
            const bool take = !done[s] && (!ba || bits > bb || (bits == bb && pos[s] < bp));
            bb = take ? bits : bb;
            bp = take ? pos[s] : bp;
            bs = take ? s : bs;
            bv = take ? a[s][c] : bv;
            ba = ba || !done[s];
        }
        const uint32_t kh = ba ? (uint32_t)(bb >> 32) + 1u : 0u;
        const uint32_t mh = seg_all<SEG, OpMax>(kh, lane);
        int win;
        if constexpr (GPB == 1) {
            // one stencil per wavefront: the ballot is the segment's mask
            uint64_t chunk = __ballot(ba && kh == mh);
            if (__builtin_expect((chunk & (chunk - 1ull)) != 0ull, 0)) {
                uint32_t h2 = kh, l2 = ba ? (uint32_t)bb : 0u;
                int p2 = ba ? bp : 0x7fffffff;
                seg_argmax_full<SEG>(h2, l2, p2);
                chunk = __ballot(ba && bp == p2);
            }
            win = __ffsll((unsigned long long)chunk) - 1;
        } else {
            uint64_t chunk = (__ballot(ba && kh == mh) >> segbase) & segmask;
            const bool uniq = (chunk & (chunk - 1ull)) == 0ull;
            if (__builtin_expect(__ballot(!uniq) != 0ull, 0)) {
                uint32_t h2 = kh, l2 = ba ? (uint32_t)bb : 0u;
                int p2 = ba ? bp : 0x7fffffff;
                seg_argmax_full<SEG>(h2, l2, p2);
                chunk = (__ballot(ba && bp == p2) >> segbase) & segmask;
            }
            win = __ffsll((unsigned long long)chunk) - 1;
        }
        const bool is_win = (l0 == win);
        double *u = sU + L::ubase(c);  // row c of U: entry q at u[2q]
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            if (is_win && bs == s) {
#pragma unroll
                for (int q = c; q < KP; ++q) u[2 * q] = a[s][q];
                u[2 * KP] = yv[s];
                if constexpr (GPB > 1) s_pos[buf][g] = pos[s];
            }
        }
        double piv;
        int kp;
        if constexpr (GPB == 1) {
            // the pivot and its position straight from the winning lane
            const uint64_t pb = (uint64_t)__double_as_longlong(bv);
            const uint32_t ph = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(pb >> 32), win);
            const uint32_t pl = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)pb, win);
            piv = __longlong_as_double((long long)(((uint64_t)ph << 32) | pl));
            kp = __builtin_amdgcn_readlane(bp, win);
            wave_sync();
        } else {
            wave_sync();
            piv = u[2 * c];
            kp = s_pos[buf][g];
        }
        const double inv = 1.0 / piv;
        double lm[SL];
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const bool upd = !done[s] && !(is_win && bs == s);
            lm[s] = upd ? a[s][c] * inv : 0.0;
            if constexpr (SAVE) a[s][c] = upd ? lm[s] : a[s][c];
        }
        // Columns c+1 .. KP (KP: the right-hand side) in chunks of CH.  The
        // reads of chunk k go through the row pointer, which an empty asm
        // ties to an update result of chunk k-2: the reads cannot be hoisted
        // further ahead, which bounds the registers they occupy while still
        // overlapping them with two chunks of updates (no instruction is
        // emitted for the tie).
        if constexpr (GPB == 1 && SL == 1) {
            // one stencil per wavefront: the pivot row comes straight from
            // the winning lane's registers into scalar registers (VALU
            // readlane, scalar fma operands), not from LDS reads by every lane
            const int wl = __builtin_amdgcn_readfirstlane(win);
#pragma unroll
            for (int q = c + 1; q <= KP; ++q) {
                const double uqv = readlane_d(q < KP ? a[0][q] : yv[0], wl);
                if (q < KP) a[0][q] = fma(-lm[0], uqv, a[0][q]);
                else yv[0] = fma(-lm[0], uqv, yv[0]);
            }
        } else {
            constexpr int CH = 4;
            lds_f64 *up = (lds_f64 *)u;
            double dep0 = 0.0, dep1 = 0.0;
#pragma unroll
            for (int q0 = c + 1; q0 <= KP; q0 += CH) {
                asm volatile("" : "+v"(up) : "v"(dep0));
                double uq[CH];
#pragma unroll
                for (int j = 0; j < CH; ++j)
                    if (q0 + j <= KP) uq[j] = up[2 * (q0 + j)];
#pragma unroll
                for (int j = 0; j < CH; ++j) {
                    const int q = q0 + j;
                    if (q < KP) {
#pragma unroll
                        for (int s = 0; s < SL; ++s) a[s][q] = fma(-lm[s], uq[j], a[s][q]);
                    } else if (q == KP) {
#pragma unroll
                        for (int s = 0; s < SL; ++s) yv[s] = fma(-lm[s], uq[j], yv[s]);
                    }
                }
                dep0 = dep1;
                dep1 = (q0 < KP) ? a[0][q0] : yv[0];
            }
        }
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const bool isp = is_win && bs == s;
            pos[s] = isp ? c : ((!done[s] && pos[s] == c) ? kp : pos[s]);
            done[s] = done[s] || isp;
            // opaque to the optimiser: keeps it from folding each step's
            // comparisons back through the select chain of all earlier steps
            // (no instruction is emitted)
            int dn = done[s] ? 1 : 0;
            asm volatile("" : "+v"(pos[s]), "+v"(dn));
            done[s] = dn != 0;
        }
    }
    wave_sync();  // the last row of U is visible

    // ---- back substitution over the rows of U in LDS -----------------------
    // Lane l0 takes positions l0 + SEG*s.  z_c = y_c / U_cc is formed in the
    // lane holding position c and broadcast inside the segment; every row
    // then subtracts U_rc z_c (rows at or past c only change values that are
    // no longer read).
    // 8-lane segments: odd segments are the upper halves of 16-lane rows
    const bool upper8 = SEG == 8 && (lane & 8) != 0;
    // The pivots are the diagonal of U; the first zero or non-finite one
    // (lowest column) decides the status.
    constexpr bool PRE = SL * KP <= 64;  // rows of U held in registers
    int ub[SL];
    double yb[SL], mb[SL], zm[SL];
    double ur[PRE ? SL : 1][PRE ? KP : 1];
    uint32_t lukey = 0;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int r0 = l0 + SEG * s;
        const int r = r0 < KP ? r0 : KP - 1;
        ub[s] = L::ubase(r);
        yb[s] = sU[ub[s] + 2 * KP];
        const double d = sU[ub[s] + 2 * r];
        mb[s] = 1.0 / d;
        zm[s] = 0.0;
        const uint32_t f = !isfinite(d) ? L_NONFIN : (d == 0.0 ? L_SING : 0u);
        const uint32_t key = ((uint32_t)(KP - r0) << 2) | f;  // lower column, larger key
        if (r0 < KP && f && key > lukey) lukey = key;
        if constexpr (PRE) {
#pragma unroll
            for (int q = 0; q < KP; ++q) ur[s][q] = sU[ub[s] + 2 * q];
        }
    }
    const uint32_t luflag = seg_all<SEG, OpMax>(lukey, lane) & 3u;
    bc_step<KP, SEG, SL, KP - 1, PRE>(sU, ub, ur[0], yb, mb, zm, l0, upper8);

    // ---- status and outputs -----------------------------------------------
#pragma unroll
    for (int s = 0; s < SL; ++s)
        if (l0 + SEG * s < K && !isfinite(zm[s])) flags |= F_ZBAD;
    flags = seg_all<SEG, OpOr>(flags, lane);
    int st = RBFFD_OK;
    if (flags & F_BADIDX) st = RBFFD_BAD_INDEX;
    else if (flags & F_NONFIN) st = RBFFD_NONFINITE;
    else if (flags & F_DUP) st = RBFFD_DUPLICATE;
    else if (luflag == L_NONFIN) st = RBFFD_NONFINITE;
    else if (luflag == L_SING) st = RBFFD_SINGULAR;
    else if (flags & F_ZBAD) st = RBFFD_NONFINITE;

    if (!valid) return;
    double *wi = w + i * (int64_t)k_stride;
    const double s2 = OP == 0 ? sc * sc : sc;  // the operator's power of the scale
    const bool good = st == RBFFD_OK;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int r = l0 + SEG * s;
        if (r < n) wi[r] = good ? zm[s] / s2 : __builtin_nan("");
    }
    for (int q = n + l0; q < k_stride; q += SEG) wi[q] = 0.0;
    if (l0 == 0 && status) status[i] = good ? ok_code : st;
    if constexpr (SAVE) {
        const int64_t kk = (int64_t)sv_kmax * sv_kmax;
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            // row r of the factors (its multipliers left of its position,
            // U from there on) at row r; the position of each row in perm
            const int r = l0 + SEG * s;
            if (r < K) {
                double *dst = sv_lu + i * kk + (int64_t)r * K;
#pragma unroll
                for (int q = 0; q < KP; ++q)
                    if (q < K) dst[q] = a[s][q];
                sv_z[i * (int64_t)sv_kmax + r] = zm[s];
            }
            if (pos[s] < K) sv_perm[i * (int64_t)sv_kmax + pos[s]] = (uint8_t)r;
        }
        if (l0 == 0) sv_s[i] = sc;
    }
}

template <int KP, int SEG, int SL, int NFIX, int MFIX, int OCC, bool SAVE, int OP = 0>
__global__ __launch_bounds__(kWave)
__attribute__((amdgpu_waves_per_eu(OCC <= 0 ? 1 : (SAVE && OCC > 2 ? 2 : OCC)))) void
weights_ms_kernel(
    const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
    const int32_t *__restrict__ nbr, int32_t k_stride, const int32_t *__restrict__ rows,
    const int32_t *__restrict__ n_rows_dev, int64_t n_rows, int32_t n_arg, int32_t m_arg,
    double *__restrict__ w, int32_t *__restrict__ status, double *__restrict__ sv_lu,
    double *__restrict__ sv_z, double *__restrict__ sv_s, uint8_t *__restrict__ sv_perm,
    int32_t sv_kmax, int32_t ok_code) {
    __shared__ __align__(16) char lds[ms_lds_bytes<KP, SEG, MFIX, 1>()];
    if (n_rows_dev) n_rows = *n_rows_dev;
    weights_ms_body<KP, SEG, SL, NFIX, MFIX, 1, SAVE, OP>(x, y, n_nodes, nbr, k_stride, rows, n_rows,
                                                      n_arg, m_arg, w, status, sv_lu, sv_z, sv_s,
                                                      sv_perm, sv_kmax, ok_code,
                                                      (int64_t)blockIdx.x, 0, lds);
}

// A row list counted on the device: at most kMsListBlocks blocks walk its
// groups with a stride (see weights_mf_list_kernel).
constexpr int64_t kMsListBlocks = 8192;

template <int KP, int SEG, int SL, int NFIX, int MFIX, int OCC, int OP>
__global__ __launch_bounds__(kWave)
__attribute__((amdgpu_waves_per_eu(OCC <= 0 ? 1 : OCC))) void weights_ms_list_kernel(
    const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
    const int32_t *__restrict__ nbr, int32_t k_stride, const int32_t *__restrict__ rows,
    const int32_t *__restrict__ n_rows_dev, int32_t n_arg, int32_t m_arg,
    double *__restrict__ w, int32_t *__restrict__ status, int32_t ok_code) {
    __shared__ __align__(16) char lds[ms_lds_bytes<KP, SEG, MFIX, 1>()];
    constexpr int GPB = kWave / SEG;
    const int64_t c = *n_rows_dev;
    const int64_t groups = (c + GPB - 1) / GPB;
    for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        wave_sync();  // the previous group's LDS is free
        weights_ms_body<KP, SEG, SL, NFIX, MFIX, 1, false, OP>(
            x, y, n_nodes, nbr, k_stride, rows, c, n_arg, m_arg, w, status, nullptr, nullptr,
            nullptr, nullptr, 0, ok_code, g, 0, lds);
    }
}

template <int KP, int SEG, int SL, int NFIX, int MFIX, int OCC = 0, int OP = 0>
inline int launch_ms(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                     int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev,
                     int64_t n_rows, int n, int m, double *w, int32_t *status,
                     const SaveView &sv, int32_t ok_code, hipStream_t stream,
                     bool per_entry = false) {
    constexpr int GPB = kWave / SEG;
    if (n_rows <= 0) return RBFFD_SUCCESS;
    const int64_t blocks = ceil_div(n_rows, GPB);
    if (blocks > 0x7fffffff) return RBFFD_ERR_UNSUPPORTED;
    if (sv.lu && OP != 0) return RBFFD_ERR_UNSUPPORTED;  // factors: the Laplacian only
    if (n_rows_dev && !sv.lu && !per_entry) {  // (per_entry: one group per block)
        const int64_t lb = blocks < kMsListBlocks ? blocks : kMsListBlocks;
        hipLaunchKernelGGL((weights_ms_list_kernel<KP, SEG, SL, NFIX, MFIX, OCC, OP>),
                           dim3((unsigned)lb), dim3(kWave), 0, stream, x, y, n_nodes, nbr,
                           k_stride, rows, n_rows_dev, n, m, w, status, ok_code);
        return last_launch_rc();
    }
    if (sv.lu)
        hipLaunchKernelGGL((weights_ms_kernel<KP, SEG, SL, NFIX, MFIX, OCC, true, OP>),
                           dim3((unsigned)blocks), dim3(kWave), 0, stream, x, y, n_nodes, nbr,
                           k_stride, rows, n_rows_dev, n_rows, n, m, w, status, sv.lu, sv.z, sv.s,
                           sv.perm, sv.kmax, ok_code);
    else
        hipLaunchKernelGGL((weights_ms_kernel<KP, SEG, SL, NFIX, MFIX, OCC, false, OP>),
                           dim3((unsigned)blocks), dim3(kWave), 0, stream, x, y, n_nodes, nbr,
                           k_stride, rows, n_rows_dev, n_rows, n, m, w, status, nullptr, nullptr,
                           nullptr, nullptr, 0, ok_code);
    return last_launch_rc();
}

}  // namespace wk
}  // namespace rbffd
