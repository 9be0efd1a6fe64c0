#pragma once
// RBF-FD Laplacian stencil weights, mixed precision, on the matrix cores:
// the FP64-assembled system M z = rhs (eq. (1): [A P; P^T 0] with
// A_kl = |u_k - u_l|^3, P_kj = p_j(u_k), rhs = [9 |u_k|; lap p_j(0)]) is
// rounded to FP32 and inverted in place by Gauss-Jordan elimination with
// partial pivoting, blocked by panels of four columns with the rank-4
// updates on v_mfma_f32_16x16x4f32; the solution is then refined in FP64.
//
// Per stencil, one wavefront:
//   1. shift and scale in FP64 (u = d / s, s = max |d|), the FP64 entries
//      of M, rounded to FP32 into 16 x 16 tiles held as MFMA accumulators;
//   2. in-place Gauss-Jordan: column c takes as pivot the first row (in the
//      order a row-swapping elimination would have) holding the largest
//      |entry| among the rows not yet pivoted; the pivot row is scaled by
//      the pivot's reciprocal and its multiple is removed from every other
//      row, pivoted or not.  Rows stay in place, so the tiles end up holding
//      S with S[pi(c)][q] = inverse(M)[c][pi(q)], pi(c) the pivot row of
//      column c;
//   3. z0 = S applied to the FP32 right-hand side; then up to 10 times:
//      r = rhs - M z in FP64 (M recomputed from the FP64 offsets, or the
//      FP64 A block kept in registers), d = S applied to (float) r,
//      z += (double) d; stop when max|d| <= 1e-12 max|z|.  A zero or
//      non-finite FP32 pivot, a non-finite value, a correction above half
//      the previous one (the first: half of max|z0|), or no convergence
//      after 10 corrections sends the stencil to the FP64 kernel (appended
//      to a list; that launch reports RBFFD_FELL_BACK_FP64).
//
// The explicit inverse makes every correction two dense products (the
// residual and S d) instead of two sequential triangular sweeps.  The FP32
// arithmetic differs in order from an LU solve, and the products sum in
// another order than a sequential loop, so results agree with the
// reference mixed form to within the refinement's accuracy, not bit for bit.
//
// Tile layout (transposed accumulators): in tile (I, J), lane l = 16 g + j,
// register r holds M[16 I + j][16 J + 4 g + r].  A panel (columns c0 ..
// c0 + 3) is the four registers of lane group g0 = (c0 % 16) / 4 in tile
// column c0 / 16.  The column steps run in row layout (lane l: rows l,
// l + 64) after a transposition through LDS.  At the panel's end, the rank-4
// update M -= G W of every column outside the panel is one MFMA per tile:
// A = -W^T (lane 16 k + i: -W[k][16 J + i], W the panel's pivot rows after
// their own scaling and in-panel eliminations) and B = G^T (lane 16 k + j:
// G[16 I + j][k], the multiple of pivot row k removed from row 16 I + j).

#include "weights_mf.h"
#include "weights_mx.h"

namespace rbffd {
namespace wk {

typedef float gj_v4f __attribute__((ext_vector_type(4)));
typedef double gj_v4d __attribute__((ext_vector_type(4)));

// Sum over the four lane groups (lanes j, 16 + j, 32 + j, 48 + j); every lane
// of the four receives the same value ((v0 + v1) + (v2 + v3)).
__device__ __forceinline__ float gj_sum4(float v) {
    const uint32_t u = __float_as_uint(v);
    const auto a = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    const float s = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    const uint32_t us = __float_as_uint(s);
    const auto b = __builtin_amdgcn_permlane32_swap(us, us, false, false);
    return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}

__device__ __forceinline__ double gj_sum4_d(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
    const auto al = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto ah = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    const double p = __longlong_as_double((long long)(((uint64_t)ah[0] << 32) | al[0]));
    const double q = __longlong_as_double((long long)(((uint64_t)ah[1] << 32) | al[1]));
    const double s = p + q;
    const uint64_t us = (uint64_t)__double_as_longlong(s);
    const uint32_t slo = (uint32_t)us, shi = (uint32_t)(us >> 32);
    const auto bl = __builtin_amdgcn_permlane32_swap(slo, slo, false, false);
    const auto bh = __builtin_amdgcn_permlane32_swap(shi, shi, false, false);
    const double p2 = __longlong_as_double((long long)(((uint64_t)bh[0] << 32) | bl[0]));
    const double q2 = __longlong_as_double((long long)(((uint64_t)bh[1] << 32) | bl[1]));
    return p2 + q2;
}

// sqrt(v) for 0 <= v (no infinities): the hardware reciprocal square root
// refined by one coupled Newton step and one residual correction (within an
// ulp; 0 for v = 0).  The residual's A entries only need FP64 accuracy, not
// the correctly rounded square root of the assembly.
__device__ __forceinline__ double gj_sqrt(double v) {
    const double y = __builtin_amdgcn_rsq(v);
    double g = v * y, h = 0.5 * y;
    const double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, v);
    g = fma(d, h, g);
    return v > 0.0 ? g : 0.0;
}

// LDS of one stencil (bytes).  The FP64 monomial table and the elimination's
// exchange buffers share one region: the table is built for the assembly,
// its space serves the elimination, and it is rebuilt for the refinement.
template <int KP, int NFIX, int MFIX>
struct GjLds {
    static constexpr int MM = (MFIX + 1) * (MFIX + 2) / 2;
    static constexpr int NT = (KP + 15) / 16;
    static constexpr int NP = 16 * NT;
    static constexpr int U = 0;                       // ux[NP], uy[NP] (FP64)
    static constexpr int Z = U + 16 * NP;              // z[NP] (FP64)
    static constexpr int BQ = Z + 8 * NP;              // FP32 right-hand side, by position
    static constexpr int DQ = BQ + 4 * NP;             // FP32 solution, natural order
    static constexpr int POS = DQ + 4 * NP;            // position of each row (int32)
    static constexpr int RA = POS + 4 * NP;            // A-block products (FP64)
    static constexpr int X = RA + 8 * NP;              // shared region
    static constexpr int PTAB = 8 * NFIX * MM;         // monomials [n][MM] (FP64)
    static constexpr int EXCH = 64 * NP;               // panel, G, pivot rows, W (FP32)
    static constexpr int BYTES = X + (PTAB > EXCH ? PTAB : EXCH);
};

// One wavefront computes stencil i.  AREG: keep the FP64 entries of the
// tiles that hold A entries in registers for the residual (else they are
// recomputed from the FP64 offsets at every correction).
// OP: 0 the Laplacian, 1 d/dx, 2 d/dy (the right-hand side of the operator
// and the power of the scale in the weights).
template <int KP, int NFIX, int MFIX, bool AREG, int UNR, int RCP, int OP = 0>
__device__ __forceinline__ void weights_gj_wave(
    const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
    const int32_t *__restrict__ nbr, int32_t k_stride, int64_t i, double *__restrict__ w,
    int32_t *__restrict__ status, int32_t *__restrict__ iters, int32_t *__restrict__ fb_count,
    int32_t *__restrict__ fb_list, char *lds) {
    using L = GjLds<KP, NFIX, MFIX>;
    constexpr int MM = L::MM, n = NFIX, K = NFIX + MM;
    static_assert(K == KP, "exact system size");
    constexpr int NT = L::NT, NP = L::NP;
    constexpr int SL = (NP + kWave - 1) / kWave;    // rows per lane in row layout
    constexpr int NA = (n + 15) / 16;               // tile rows / columns holding A entries
    double *s_ux = reinterpret_cast<double *>(lds + L::U);
    double *s_uy = s_ux + NP;
    double *s_z = reinterpret_cast<double *>(lds + L::Z);
    float *s_bq = reinterpret_cast<float *>(lds + L::BQ);
    float *s_dq = reinterpret_cast<float *>(lds + L::DQ);
    int32_t *s_pos = reinterpret_cast<int32_t *>(lds + L::POS);
    double *s_ra = reinterpret_cast<double *>(lds + L::RA);
    double(*s_P)[MM] = reinterpret_cast<double(*)[MM]>(lds + L::X);
    gj_v4f *s_pan = reinterpret_cast<gj_v4f *>(lds + L::X);             // [NP]
    gj_v4f *s_g = reinterpret_cast<gj_v4f *>(lds + L::X + 16 * NP);     // [NP]
    float(*s_ub)[NP] = reinterpret_cast<float(*)[NP]>(lds + L::X + 32 * NP);  // [4][NP]
    float(*s_w)[NP] = reinterpret_cast<float(*)[NP]>(lds + L::X + 48 * NP);   // [4][NP]

    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane >> 4, jl = lane & 15;

    // ---- shift and scale (FP64; row layout: rows lane, lane + 64) --------
    uint32_t flags = 0;
    double dx[SL], dy[SL];
    double d2m = 0.0;
    const double xi = x[i], yi = y[i];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int r = lane + kWave * s;
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
    const double sc = sqrt(seg_all_max_d<kWave>(d2m, lane));
    if (!isfinite(sc)) flags |= F_NONFIN;  // an offset's square overflowed
    if (sc == 0.0) flags |= F_DUP;
    // the monomials of row r, into the table
    auto monomials = [&](int s) {
        const int r = lane + kWave * s;
        if (r < n) {
            const double ux = s_ux[r], uy = s_uy[r];
            double px[MFIX + 1], py[MFIX + 1];
            px[0] = 1.0;
            py[0] = 1.0;
#pragma unroll
            for (int e = 1; e <= MFIX; ++e) {
                px[e] = px[e - 1] * ux;
                py[e] = py[e - 1] * uy;
            }
#pragma unroll
            for (int j = 0; j < MM; ++j) s_P[r][j] = px[mono_a(j)] * py[mono_b(j)];
        }
    };
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int r = lane + kWave * s;
        if (r < NP) {
            s_ux[r] = r < n ? dx[s] / sc : 0.0;
            s_uy[r] = r < n ? dy[s] / sc : 0.0;
        }
    }
    lds_order();
#pragma unroll
    for (int s = 0; s < SL; ++s) monomials(s);
    lds_order();

    // ---- FP64 entries of M, rounded into the FP32 tiles -----------------
    // entry (R, C) of M in FP64; dup set when two support nodes coincide
    // (the FP32 tiles take these entries rounded once: any FP32 arithmetic
    // in between would put the FP32 system further from the FP64 one and
    // slow the refinement's contraction)
    auto m64 = [&](int I, int J, int r, bool &dup) -> double {
        const int R = 16 * I + jl, C = 16 * J + 4 * g + r;
        double v = 0.0;
        if (16 * I < n && 16 * J < n && R < n && C < n) {
            const double ex = s_ux[R] - s_ux[C];
            const double ey = s_uy[R] - s_uy[C];
            if (C != R && ex == 0.0 && ey == 0.0) dup = true;
            const double rr = ex * ex + ey * ey;
            v = rr * sqrt(rr);
        } else if (16 * I < n && 16 * J + 15 >= n && 16 * J < K && R < n && C >= n && C < K) {
            v = s_P[R][C - n];
        } else if (16 * I + 15 >= n && 16 * I < K && 16 * J < n && R >= n && R < K && C < n) {
            v = s_P[C][R - n];
        }
        return v;
    };
    gj_v4f T[NT][NT];
    gj_v4d A64[AREG ? NA : 1][AREG ? NA : 1];
    {
        bool dup = false;
#pragma unroll
        for (int I = 0; I < NT; ++I)
#pragma unroll
            for (int J = 0; J < NT; ++J) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double v = m64(I, J, r, dup);
                    T[I][J][r] = (float)v;
                    if constexpr (AREG)
                        if (I < NA && J < NA)
                            A64[I < NA ? I : 0][J < NA ? J : 0][r] =
                                (16 * I + jl < n && 16 * J + 4 * g + r < n) ? v : 0.0;
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        if (dup) flags |= F_DUP;
    }
    lds_order();  // the monomial table's space becomes the exchange buffers

    // ---- Gauss-Jordan, panels of four columns --------------------------
    int pos[SL];
    bool done[SL];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        pos[s] = lane + kWave * s;
        done[s] = pos[s] >= KP;
    }
    bool lufail = false;

#pragma unroll
    for (int J0 = 0; J0 < NT; ++J0) {
    // the panels of tile column J0 are the four lane groups' registers:
    // which group is a lane mask, not a register index, so the panel loop
    // can stay rolled here (UNR = 1), which keeps the kernel's code a
    // quarter of the fully unrolled size
    constexpr int kPanMax = 4;
#pragma unroll UNR
    for (int g0 = 0; g0 < kPanMax; ++g0) {
        const int c0 = 16 * J0 + 4 * g0;
        if (c0 >= KP) break;
        const int nk = KP - c0 < 4 ? KP - c0 : 4;
        // no scheduling across panels: overlapping a panel's column steps
        // with the previous panel's products holds both sets of values
        __builtin_amdgcn_sched_barrier(0);
        // the panel to row layout
        if (g == g0) {
#pragma unroll
            for (int I = 0; I < NT; ++I) s_pan[16 * I + jl] = T[I][J0];
        }
        lds_order();
        float pc[SL][4], gk[SL][4];
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const int r = lane + kWave * s;
            const gj_v4f v = r < NP ? s_pan[r < NP ? r : 0] : gj_v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                pc[s][j] = v[j];
                gk[s][j] = 0.f;
            }
        }
        int prow[4] = {0, 0, 0, 0};
        float invk[4] = {0.f, 0.f, 0.f, 0.f};
        float l11[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) l11[a][b] = 0.f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k >= nk) break;
            const int c = c0 + k;
            // pivot search: exact key (|a| bits, position) over the rows not
            // yet pivoted; bb, bp and bv are read only where ba holds
            uint32_t bb = 0;
            int bp = 0, bsl = 0;
            float bv = 0.f;
            bool ba = false;
            if constexpr (SL == 1) {
                bb = __float_as_uint(pc[0][k]) & 0x7fffffffu;
                bp = pos[0];
                bv = pc[0][k];
                ba = !done[0];
            } else {
#pragma unroll
                for (int s = 0; s < SL; ++s) {
                    const uint32_t bits = __float_as_uint(pc[s][k]) & 0x7fffffffu;
                    const bool take =
                        !done[s] && (!ba || bits > bb || (bits == bb && pos[s] < bp));
                    bb = take ? bits : bb;
                    bp = take ? pos[s] : bp;
                    bsl = take ? s : bsl;
                    bv = take ? pc[s][k] : bv;
                    ba = ba || !done[s];
                }
            }
            const uint32_t kh = ba ? bb + 1u : 0u;
            const uint32_t mh = seg_all<kWave, OpMax>(kh, lane);
            // (some row is always left, so mh >= 1 and only rows still in the
            // search can equal it)
            uint64_t chunk = __ballot(kh == mh);
            if (__builtin_expect((chunk & (chunk - 1ull)) != 0ull, 0)) {
                uint32_t h2 = kh, l2 = 0u;
                int p2 = ba ? bp : 0x7fffffff;
                seg_argmax_full<kWave>(h2, l2, p2);
                chunk = __ballot(ba && bp == p2);
            }
            const int win = __builtin_amdgcn_readfirstlane(__ffsll((unsigned long long)chunk) - 1);
            const int bs = __builtin_amdgcn_readlane(bsl, win);
            const int kp = __builtin_amdgcn_readlane(bp, win);
            const float piv = __builtin_bit_cast(
                float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, bv), win));
            if (!(piv != 0.0f) || !isfinite(piv)) lufail = true;
            // the reciprocal: IEEE (RCP = 0) or the hardware's within an ulp
            // (RCP = 1); the refinement, not the factors, sets the accuracy,
            // but a less exact inverse can take more corrections
            const float inv = RCP ? __builtin_amdgcn_rcpf(piv) : 1.0f / piv;
            const bool b1 = bs != 0;
            // the pivot row's other panel entries, scaled
            float wv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (j == k) {
                    wv[j] = 0.f;
                    continue;
                }
                const float pv = __builtin_bit_cast(
                    float, __builtin_amdgcn_readlane(
                               __builtin_bit_cast(int, b1 ? pc[SL - 1][j] : pc[0][j]), win));
                wv[j] = pv * inv;
            }
            // its multiples of the panel's earlier pivot rows
#pragma unroll
            for (int k2 = 0; k2 < k; ++k2)
                l11[k][k2] = __builtin_bit_cast(
                    float, __builtin_amdgcn_readlane(
                               __builtin_bit_cast(int, b1 ? gk[SL - 1][k2] : gk[0][k2]), win));
            invk[k] = inv;
            prow[k] = win + kWave * bs;
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                const bool isp = lane == win && bs == s;
                const float f = pc[s][k];
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (j != k) pc[s][j] = isp ? wv[j] : fmaf(-f, wv[j], pc[s][j]);
                pc[s][k] = isp ? inv : -f * inv;
                gk[s][k] = isp ? 0.f : f;
#pragma unroll
                for (int k2 = 0; k2 < k; ++k2) gk[s][k2] = isp ? 0.f : gk[s][k2];
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
        __builtin_amdgcn_sched_barrier(0);
        // panel values and the multiples G back through LDS
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const int r = lane + kWave * s;
            if (r < NP) {
                s_pan[r] = gj_v4f{pc[s][0], pc[s][1], pc[s][2], pc[s][3]};
                s_g[r] = gj_v4f{gk[s][0], gk[s][1], gk[s][2], gk[s][3]};
            }
        }
        // the panel's pivot rows, every tile column, to LDS (one uniform
        // branch per row: its tile row is wave-uniform)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k >= nk) break;
            const int Ipk = prow[k] >> 4, ipk = prow[k] & 15;
            if (jl == ipk) {
#pragma unroll
                for (int I = 0; I < NT; ++I) {
                    if (I == Ipk) {
#pragma unroll
                        for (int J = 0; J < NT; ++J)
                            *reinterpret_cast<gj_v4f *>(&s_ub[k][16 * J + 4 * g]) = T[I][J];
                        asm volatile(";gj tile row %0" ::"i"(I) : "memory");
                    }
                }
            }
        }
        lds_order();
        if (g == g0) {
#pragma unroll
            for (int I = 0; I < NT; ++I) T[I][J0] = s_pan[16 * I + jl];
        }
        float Bop[NT];
#pragma unroll
        for (int I = 0; I < NT; ++I) Bop[I] = s_g[16 * I + jl][g];
        // W (the pivot rows after the panel's steps), lane (k, i) of the A
        // operand: -W[k][16 J + i], zero in the panel's own columns
        float Aop[NT];
#pragma unroll
        for (int J = 0; J < NT; ++J) {
            const int q = 16 * J + jl;
            float v[4], wk4[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = k < nk ? s_ub[k][q] : 0.f;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float t = v[k];
#pragma unroll
                for (int k2 = 0; k2 < k; ++k2) t = fmaf(-l11[k][k2], wk4[k2], t);
                wk4[k] = k < nk ? t * invk[k] : 0.f;
            }
            const float ws = g == 0 ? wk4[0] : (g == 1 ? wk4[1] : (g == 2 ? wk4[2] : wk4[3]));
            const bool in_panel = J == J0 && (jl >> 2) == g0;
            Aop[J] = in_panel ? 0.f : -ws;
            s_w[g][q] = ws;
        }
        lds_order();
        // W into the pivot rows of the tiles (outside the panel)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k >= nk) break;
            const int Ipk = prow[k] >> 4, ipk = prow[k] & 15;
            if (jl == ipk) {
#pragma unroll
                for (int I = 0; I < NT; ++I) {
                    if (I == Ipk) {
#pragma unroll
                        for (int J = 0; J < NT; ++J) {
                            const gj_v4f wv4 = *reinterpret_cast<const gj_v4f *>(&s_w[k][16 * J + 4 * g]);
                            if (J != J0 || g != g0) T[I][J] = wv4;
                        }
                        asm volatile(";gj w row %0" ::"i"(I) : "memory");
                    }
                }
            }
        }
        // rank-4 update of every tile
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int I = 0; I < NT; ++I)
#pragma unroll
            for (int J = 0; J < NT; ++J)
                T[I][J] = __builtin_amdgcn_mfma_f32_16x16x4f32(Aop[J], Bop[I], T[I][J], 0, 0, 0);
        lds_order();  // the exchange buffers are rewritten by the next panel
    }
    }

    // ---- refinement (vectors in row layout: row R = lane + 64 s) ----------
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int r = lane + kWave * s;
        if (r < NP) s_pos[r] = pos[s];
    }
    for (int q = lane; q < NP; q += kWave) {
        s_bq[q] = 0.f;
        s_z[q] = 0.0;
    }
    lds_order();
#pragma unroll
    for (int s = 0; s < SL; ++s) monomials(s);
    int posT[NT];
#pragma unroll
    for (int I = 0; I < NT; ++I) posT[I] = s_pos[16 * I + jl];
    // right-hand side in FP64
    double rhs_s[SL];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int R = lane + kWave * s;
        double v = 0.0;
        if (kWave * s < n && R < n) {
            const double ux = s_ux[R], uy = s_uy[R];
            const double r0 = ux * ux + uy * uy;
            v = OP == 0 ? 9.0 * sqrt(r0) : -3.0 * sqrt(r0) * (OP == 1 ? ux : uy);
        } else if (R >= n && R < K) {
            v = OP == 0 ? ((R - n == 3 || R - n == 5) ? 2.0 : 0.0) : (R - n == OP ? 1.0 : 0.0);
        }
        rhs_s[s] = v;
    }
    lds_order();

    // d = S v in the natural order: v (FP32) and d in row layout.  Row R's
    // entry of v goes to its position; S's row R then gives d at position
    // pos(R).
    auto apply_inverse = [&](const float *v, float *d) {
#pragma unroll
        for (int s = 0; s < SL; ++s)
            if (lane + kWave * s < K) s_bq[pos[s]] = v[s];
        lds_order();
        float acc[NT];
#pragma unroll
        for (int I = 0; I < NT; ++I) acc[I] = 0.f;
#pragma unroll
        for (int J = 0; J < NT; ++J) {
            const gj_v4f bq = *reinterpret_cast<const gj_v4f *>(&s_bq[16 * J + 4 * g]);
#pragma unroll
            for (int I = 0; I < NT; ++I)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[I] = fmaf(T[I][J][r], bq[r], acc[I]);
        }
#pragma unroll
        for (int I = 0; I < NT; ++I) {
            const float yI = gj_sum4(acc[I]);
            if (g == 0 && 16 * I + jl < K) s_dq[posT[I]] = yI;
        }
        lds_order();
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const int R = lane + kWave * s;
            d[s] = R < K ? s_dq[R < K ? R : 0] : 0.f;
        }
        lds_order();
    };

    // r = rhs - M z in FP64 (z in s_z, natural order), row layout.  The FP64
    // entries are formed anew at every call; an opaque zero in the table
    // addresses keeps the compiler from hoisting them out of the refinement
    // loop (which would hold them all in registers across it).
    auto residual = [&](double *res) {
        int opq = 0;
        asm volatile("" : "+v"(opq));
        const double *ux_o = s_ux + opq, *uy_o = s_uy + opq, *z_o = s_z + opq;
        const double(*P_o)[MM] = s_P + opq;
        double acc[SL];
#pragma unroll
        for (int s = 0; s < SL; ++s) acc[s] = 0.0;
        if constexpr (AREG) {
            // the A block from the FP64 tiles: per tile row, partial sums over
            // the lane's columns, then the sum over the four lane groups
            double accA[NA];
#pragma unroll
            for (int I = 0; I < NA; ++I) accA[I] = 0.0;
#pragma unroll
            for (int J = 0; J < NA; ++J) {
                const gj_v4d zq = *reinterpret_cast<const gj_v4d *>(&z_o[16 * J + 4 * g]);
#pragma unroll
                for (int I = 0; I < NA; ++I)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        accA[I] = fma(A64[AREG ? I : 0][AREG ? J : 0][r], zq[r], accA[I]);
            }
#pragma unroll
            for (int I = 0; I < NA; ++I) {
                const double t = gj_sum4_d(accA[I]);
                if (g == 0) s_ra[16 * I + jl] = t;
            }
            lds_order();
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                const int R = lane + kWave * s;
                if (kWave * s < n && R < n) acc[s] = s_ra[R];
            }
        } else {
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                const int R = lane + kWave * s;
                if (kWave * s < n && R < n) {
                    const double uxr = ux_o[R], uyr = uy_o[R];
                    double a = 0.0;
#pragma unroll 2
                    for (int c = 0; c < n; ++c) {
                        const double ex = uxr - ux_o[c];
                        const double ey = uyr - uy_o[c];
                        const double rr = ex * ex + ey * ey;
                        a = fma(rr * gj_sqrt(rr), z_o[c], a);
                    }
                    acc[s] = a;
                }
            }
        }
        // the P block and its transpose
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const int R = lane + kWave * s;
            if (kWave * s < n && R < n) {
#pragma unroll 4
                for (int j = 0; j < MM; ++j) acc[s] = fma(P_o[R][j], z_o[n + j], acc[s]);
            } else if (kWave * s + kWave > n && R >= n && R < K) {
                const int jj = R - n;
#pragma unroll 2
                for (int c = 0; c < n; ++c) acc[s] = fma(P_o[c][jj], z_o[c], acc[s]);
            }
        }
#pragma unroll
        for (int s = 0; s < SL; ++s) res[s] = rhs_s[s] - acc[s];
    };

    int state = (flags != 0 || lufail) ? 2 : 0;  // 0 iterating, 1 converged, 2 fall back
    int nit = 0;
    double z[SL];
#pragma unroll
    for (int s = 0; s < SL; ++s) z[s] = 0.0;
    if (state == 0) {
        float v[SL], d[SL];
#pragma unroll
        for (int s = 0; s < SL; ++s) v[s] = (float)rhs_s[s];
        apply_inverse(v, d);
        double zmax = 0.0;
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const int R = lane + kWave * s;
            z[s] = (double)d[s];
            zmax = fmax(zmax, fabs(z[s]));
            if (R < NP) s_z[R < NP ? R : 0] = z[s];
        }
        double prev = seg_all_max_d<kWave>(zmax, lane);
        lds_order();
        for (int it = 1; it <= kMixedMaxCorrections; ++it) {
            double res[SL];
            residual(res);
            float v2[SL], d2[SL];
#pragma unroll
            for (int s = 0; s < SL; ++s) v2[s] = (float)res[s];
            apply_inverse(v2, d2);
            double dn = 0.0, zn = 0.0;
            bool bad = false;
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                const int R = lane + kWave * s;
                z[s] = z[s] + (double)d2[s];
                const double ad = fabs((double)d2[s]), az = fabs(z[s]);
                if (!isfinite(ad) || !isfinite(az)) bad = true;
                dn = fmax(dn, ad);
                zn = fmax(zn, az);
                if (R < NP) s_z[R < NP ? R : 0] = z[s];
            }
            lds_order();
            bad = __ballot(bad) != 0ull;
            dn = seg_all_max_d<kWave>(dn, lane);
            zn = seg_all_max_d<kWave>(zn, lane);
            nit = it;
            if (bad) state = 2;
            else if (dn <= kMixedTol * zn) state = 1;
            else if (dn > 0.5 * prev) state = 2;
            prev = dn;
            if (state != 0) break;
        }
        if (state == 0) state = 2;
    }

    // ---- outputs -----------------------------------------------------------
    flags = seg_all<kWave, OpOr>(flags, lane);
    double *wi = w + i * (int64_t)k_stride;
    if (flags != 0) {
        int st = RBFFD_NONFINITE;
        if (flags & F_BADIDX) st = RBFFD_BAD_INDEX;
        else if (flags & F_NONFIN) st = RBFFD_NONFINITE;
        else if (flags & F_DUP) st = RBFFD_DUPLICATE;
        for (int q = lane; q < k_stride; q += kWave) wi[q] = q < n ? __builtin_nan("") : 0.0;
        if (lane == 0) {
            if (status) status[i] = st;
            if (iters) iters[i] = 0;
        }
    } else if (state == 1) {
        const double s2 = OP == 0 ? sc * sc : sc;  // the operator's power of the scale
#pragma unroll
        for (int s = 0; s < SL; ++s)
            if (lane + kWave * s < n) wi[lane + kWave * s] = z[s] / s2;
        for (int q = n + lane; q < k_stride; q += kWave) wi[q] = 0.0;
        if (lane == 0) {
            if (status) status[i] = RBFFD_OK;
            if (iters) iters[i] = nit;
        }
    } else if (lane == 0) {
        fb_list[atomicAdd(fb_count, 1)] = (int32_t)i;
        if (iters) iters[i] = nit;  // the corrections tried
    }
}

template <int KP, int NFIX, int MFIX, bool AREG, int OCC, int UNR, int RCP, int OP = 0>
__global__ __launch_bounds__(kWave)
__attribute__((amdgpu_waves_per_eu(OCC > 0 ? OCC : 1))) void weights_gj_kernel(
    const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
    const int32_t *__restrict__ nbr, int32_t k_stride, const int32_t *__restrict__ rows,
    const int32_t *__restrict__ n_rows_dev, int64_t n_rows, double *__restrict__ w,
    int32_t *__restrict__ status, int32_t *__restrict__ iters, int32_t *__restrict__ fb_count,
    int32_t *__restrict__ fb_list) {
    __shared__ __align__(16) char lds[GjLds<KP, NFIX, MFIX>::BYTES];
    if (n_rows_dev) n_rows = *n_rows_dev;
    const int64_t t = blockIdx.x;
    if (t >= n_rows) return;
    const int64_t i = rows ? (int64_t)rows[t] : t;
    weights_gj_wave<KP, NFIX, MFIX, AREG, UNR, RCP, OP>(x, y, n_nodes, nbr, k_stride, i, w,
                                                   status, iters, fb_count, fb_list, lds);
}

// One block (one wavefront) per listed stencil; no scratch memory.
// UNR: 4 unrolls the panel loop fully, 1 keeps it rolled within a tile column.
template <int KP, int NFIX, int MFIX, bool AREG, int OCC = 0, int UNR = 1, int RCP = 0,
          int OP = 0>
struct GjLaunch {
    static size_t scratch_bytes(int64_t) { return 0; }
    static int run(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                   int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev,
                   int64_t n_rows, double *w, int32_t *status, int32_t *iters, double * /*scratch*/,
                   int32_t *fb_count, int32_t *fb_list, hipStream_t stream) {
        if (n_rows <= 0) return RBFFD_SUCCESS;
        if (n_rows > 0x7fffffff) return RBFFD_ERR_UNSUPPORTED;
        hipLaunchKernelGGL((weights_gj_kernel<KP, NFIX, MFIX, AREG, OCC, UNR, RCP, OP>),
                           dim3((unsigned)n_rows),
                           dim3(kWave), 0, stream, x, y, n_nodes, nbr, k_stride, rows, n_rows_dev,
                           n_rows, w, status, iters, fb_count, fb_list);
        return last_launch_rc();
    }
};

}  // namespace wk
}  // namespace rbffd
