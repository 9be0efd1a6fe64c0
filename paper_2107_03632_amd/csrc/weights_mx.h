#pragma once
// RBF-FD Laplacian stencil weights, mixed precision: FP32 factorisation of
// the FP64-assembled system, FP64 iterative refinement.
//
// Per stencil (the reference definition of the mixed form):
//   1. assemble M and rhs in FP64 exactly as the FP64 path does;
//   2. M32 = (float) M; LU with partial pivoting in FP32 (first largest |a|,
//      reciprocal pivot, fmaf(-l, u, a)), the FP32 right-hand side carried
//      along: z = (double) U^-1 L^-1 P (float) rhs;
//   3. up to 10 times: r = rhs - M z in FP64 (fused, columns ascending),
//      d = FP32 solve of (float) r with the same factors, z += (double) d;
//      converged when max|d| <= 1e-12 max|z|; a correction above half the
//      previous one (the first is compared with max|z| of the initial
//      solve), a non-finite value, an FP32 zero or non-finite pivot, or no
//      convergence after 10 corrections sends the stencil to the FP64 kernel
//      (appended to a list; that launch reports RBFFD_FELL_BACK_FP64); the
//      corrections tried before the fallback are reported.
// Layout: as the FP64 multi-slot kernel (SEG lanes per stencil, SL rows per
// lane) with FP32 rows, i.e. half the registers per row, so more stencils fit
// in a wavefront.  The FP64 matrix rows needed by the residual go to a
// per-block global scratch area (written once, read once per correction, L2
// resident while the block works on the stencil); the kernel loops over
// stencil groups with a grid sized to that scratch area.

#include "weights_ms.h"

namespace rbffd {
namespace wk {

constexpr int kMixedMaxCorrections = 10;
constexpr double kMixedTol = 1e-12;

template <int SEG>
__device__ __forceinline__ float seg_all_or_f(float v, int lane) {
    return __uint_as_float(seg_all<SEG, OpOr>(__float_as_uint(v), lane));
}

// OP: 0 the Laplacian, 1 d/dx, 2 d/dy (right-hand side and scale power).
template <int KP, int SEG, int SL, int NFIX, int MFIX, int OCC, int OP = 0>
__global__ __launch_bounds__(kWave)
__attribute__((amdgpu_waves_per_eu(OCC > 0 ? OCC : 1))) void weights_mx_kernel(
    const double *__restrict__ x, const double *__restrict__ y, int64_t n_nodes,
    const int32_t *__restrict__ nbr, int32_t k_stride, const int32_t *__restrict__ rows,
    const int32_t *__restrict__ n_rows_dev, int64_t n_rows, double *__restrict__ w,
    int32_t *__restrict__ status, int32_t *__restrict__ iters, double *__restrict__ ws_m64,
    int32_t *__restrict__ fb_count, int32_t *__restrict__ fb_list) {
    static_assert(SEG * SL >= KP, "slots must cover the system");
    static_assert(NFIX > 0 && MFIX > 0, "exact sizes only");
    constexpr int GPB = kWave / SEG;
    constexpr int n = NFIX;
    constexpr int NM = (MFIX + 1) * (MFIX + 2) / 2;
    constexpr int K = n + NM;
    static_assert(K == KP, "no padding in the mixed kernel");
    constexpr int MM = NM;

    __shared__ double s_ux[GPB][KP];
    __shared__ double s_uy[GPB][KP];
    __shared__ double s_P[GPB * KP][MM];
    __shared__ float s_row[2][GPB][2 * (KP + 1)];  // entries 8 bytes apart
    __shared__ int32_t s_pos[2][GPB];
    __shared__ double s_z[GPB][KP];

    const int lane = threadIdx.x;
    const int g = lane / SEG;
    const int l0 = lane % SEG;
    if (n_rows_dev) n_rows = *n_rows_dev;
    double *m64 = ws_m64 + ((int64_t)blockIdx.x * GPB + g) * KP * KP;
    const uint64_t segmask = SEG == 64 ? ~0ull : ((1ull << SEG) - 1ull);
    const int segbase = g * SEG;

    for (int64_t tb = blockIdx.x; tb * GPB < n_rows; tb += gridDim.x) {
        const int64_t t = tb * GPB + g;
        const bool valid = t < n_rows;
        const int64_t i = valid ? (rows ? (int64_t)rows[t] : t) : 0;

        // ---- shift / scale / monomials (as the FP64 path) ----------------
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
        double ux[SL], uy[SL];
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const int r = l0 + SEG * s;
            ux[s] = 0.0;
            uy[s] = 0.0;
            if (r < n) {
                ux[s] = dx[s] / sc;
                uy[s] = dy[s] / sc;
                s_ux[g][r] = ux[s];
                s_uy[g][r] = uy[s];
                double px[7], py[7];
                px[0] = 1.0;
                py[0] = 1.0;
#pragma unroll
                for (int e = 1; e < 7; ++e) {
                    px[e] = px[e - 1] * ux[s];
                    py[e] = py[e - 1] * uy[s];
                }
#pragma unroll
                for (int j = 0; j < MM; ++j) s_P[g * KP + r][j] = px[mono_a(j)] * py[mono_b(j)];
            }
        }
        __syncthreads();

        // ---- FP64 rows: to scratch (residuals) and rounded to FP32 --------
        float af[SL][KP];
        float yf[SL];
        double rhs[SL];
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const int r = l0 + SEG * s;
            const bool prow = r < n;
            const bool qrow = r >= n && r < K;
            const int jr = qrow ? r - n : 0;
            const bool any_p = SEG * s < n;
#pragma unroll
            for (int l = 0; l < KP; ++l) {
                double v;
                if (l < n) {
                    double phs = 0.0;
                    if (any_p) {
                        const double ex = ux[s] - s_ux[g][l];
                        const double ey = uy[s] - s_uy[g][l];
                        const double rr = ex * ex + ey * ey;
                        if (prow && l != r && rr == 0.0) flags |= F_DUP;
                        phs = rr * sqrt(rr);
                    }
                    const double pt = s_P[g * KP + l][jr];
                    v = prow ? phs : (qrow ? pt : 0.0);
                } else {
                    v = prow ? s_P[g * KP + (r < KP ? r : 0)][l - n] : 0.0;
                }
                af[s][l] = (float)v;
                if (r < KP) m64[r * KP + l] = v;
                if ((l & 1) == 1) __builtin_amdgcn_sched_barrier(0);
            }
            const double r0 = ux[s] * ux[s] + uy[s] * uy[s];
            const double rb =
                OP == 0 ? 9.0 * sqrt(r0) : -3.0 * sqrt(r0) * (OP == 1 ? ux[s] : uy[s]);
            const bool rq = OP == 0 ? (jr == 3 || jr == 5) : jr == OP;
            rhs[s] = prow ? rb : ((qrow && rq) ? (OP == 0 ? 2.0 : 1.0) : 0.0);
            yf[s] = (float)rhs[s];
        }
        asm volatile("" : "+v"(flags));

        // ---- FP32 LU with partial pivoting, rhs carried ------------------
        int pos[SL];
        bool done[SL];
        float minv[SL];
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            pos[s] = l0 + SEG * s;
            done[s] = pos[s] >= KP;
            minv[s] = 0.0f;
        }
        uint32_t luflag = 0;
#pragma unroll
        for (int c = 0; c < KP; ++c) {
            const int buf = c & 1;
            uint32_t bb = 0;
            int bp = 0x7fffffff, bs = 0;
            bool ba = false;
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                const uint32_t bits = __float_as_uint(af[s][c]) & 0x7fffffffu;
                const bool take = !done[s] && (!ba || bits > bb || (bits == bb && pos[s] < bp));
                bb = take ? bits : bb;
                bp = take ? pos[s] : bp;
                bs = take ? s : bs;
                ba = ba || !done[s];
            }
            const uint32_t kh = ba ? bb + 1u : 0u;
            const uint32_t mh = seg_all<SEG, OpMax>(kh, lane);
            uint64_t chunk = (__ballot(ba && kh == mh) >> segbase) & segmask;
            const bool uniq = (chunk & (chunk - 1ull)) == 0ull;
            if (__builtin_expect(__ballot(!uniq) != 0ull, 0)) {
                uint32_t h2 = kh, l2 = 0u;
                int p2 = ba ? bp : 0x7fffffff;
                seg_argmax_full<SEG>(h2, l2, p2);
                chunk = (__ballot(ba && bp == p2) >> segbase) & segmask;
            }
            const int win = __ffsll((unsigned long long)chunk) - 1;
            const bool is_win = (l0 == win);
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                if (is_win && bs == s) {
#pragma unroll
                    for (int q = c; q < KP; ++q) s_row[buf][g][2 * q] = af[s][q];
                    s_row[buf][g][2 * KP] = yf[s];
                    s_pos[buf][g] = pos[s];
                }
            }
            __syncthreads();
            const float *u = s_row[buf][g];
            const float piv = u[2 * c];
            const int kp = s_pos[buf][g];
            const float inv = 1.0f / piv;
            if (luflag == 0) {
                if (!isfinite(piv)) luflag = L_NONFIN;
                else if (piv == 0.0f) luflag = L_SING;
            }
            float lm[SL];
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                const bool upd = !done[s] && !(is_win && bs == s);
                lm[s] = upd ? af[s][c] * inv : 0.0f;
                af[s][c] = upd ? lm[s] : af[s][c];
            }
#pragma unroll
            for (int q = c + 1; q < KP; ++q) {
                const float uq = u[2 * q];
#pragma unroll
                for (int s = 0; s < SL; ++s) af[s][q] = fmaf(-lm[s], uq, af[s][q]);
            }
            {
                const float uy_ = u[2 * KP];
#pragma unroll
                for (int s = 0; s < SL; ++s) yf[s] = fmaf(-lm[s], uy_, yf[s]);
            }
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                const bool isp = is_win && bs == s;
                pos[s] = isp ? c : ((!done[s] && pos[s] == c) ? kp : pos[s]);
                minv[s] = isp ? inv : minv[s];
                done[s] = done[s] || isp;
                int dn = done[s] ? 1 : 0;
                asm volatile("" : "+v"(pos[s]), "+v"(dn));
                done[s] = dn != 0;
            }
            asm volatile("" : "+v"(luflag));
        }

        // ---- initial FP32 back substitution -------------------------------
        double z[SL];
        {
            float zf[SL];
#pragma unroll
            for (int s = 0; s < SL; ++s) zf[s] = 0.0f;
#pragma unroll
            for (int c = KP - 1; c >= 0; --c) {
                float zl = 0.0f;
#pragma unroll
                for (int s = 0; s < SL; ++s) {
                    const float zc = yf[s] * minv[s];
                    zf[s] = (pos[s] == c) ? zc : zf[s];
                    zl = (pos[s] == c) ? zc : zl;
                }
                const float zb = seg_all_or_f<SEG>(zl, lane);
#pragma unroll
                for (int s = 0; s < SL; ++s) yf[s] = (pos[s] < c) ? fmaf(-af[s][c], zb, yf[s]) : yf[s];
            }
#pragma unroll
            for (int s = 0; s < SL; ++s) z[s] = (double)zf[s];
        }

        // ---- FP64 refinement ----------------------------------------------
        // state: 0 iterating, 1 converged, 2 fall back
        int state = (flags != 0 || luflag != 0) ? 2 : 0;
        state = (int)seg_all<SEG, OpMax>((uint32_t)state, lane);
        double prev = 0.0;
#pragma unroll
        for (int s = 0; s < SL; ++s) prev = fmax(prev, fabs(z[s]));
        prev = seg_all_max_d<SEG>(prev, lane);
        int nit = 0;
        for (int it = 1; it <= kMixedMaxCorrections; ++it) {
            if (__ballot(state == 0) == 0ull) break;
#pragma unroll
            for (int s = 0; s < SL; ++s)
                if (pos[s] < KP) s_z[g][pos[s]] = z[s];
            __syncthreads();
            float yv[SL];
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                const int r = l0 + SEG * s;
                double acc = rhs[s];
                if (r < KP) {
                    const double *mr = m64 + r * KP;
                    for (int l = 0; l < KP; ++l) acc = fma(-mr[l], s_z[g][l], acc);
                }
                yv[s] = (float)acc;
            }
            // forward sweep with unit L (logical positions)
#pragma unroll
            for (int c = 0; c < KP; ++c) {
                float yl = 0.0f;
#pragma unroll
                for (int s = 0; s < SL; ++s) yl = (pos[s] == c) ? yv[s] : yl;
                const float yb = seg_all_or_f<SEG>(yl, lane);
#pragma unroll
                for (int s = 0; s < SL; ++s) yv[s] = (pos[s] > c) ? fmaf(-af[s][c], yb, yv[s]) : yv[s];
            }
            // back sweep
            float dm[SL];
#pragma unroll
            for (int s = 0; s < SL; ++s) dm[s] = 0.0f;
#pragma unroll
            for (int c = KP - 1; c >= 0; --c) {
                float dl = 0.0f;
#pragma unroll
                for (int s = 0; s < SL; ++s) {
                    const float dc = yv[s] * minv[s];
                    dm[s] = (pos[s] == c) ? dc : dm[s];
                    dl = (pos[s] == c) ? dc : dl;
                }
                const float db = seg_all_or_f<SEG>(dl, lane);
#pragma unroll
                for (int s = 0; s < SL; ++s) yv[s] = (pos[s] < c) ? fmaf(-af[s][c], db, yv[s]) : yv[s];
            }
            // update and test (per segment, uniform inside it)
            double dn = 0.0, zn = 0.0;
            uint32_t bad = 0;
            if (state == 0) {
#pragma unroll
                for (int s = 0; s < SL; ++s) z[s] = z[s] + (double)dm[s];
            }
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                const double ad = fabs((double)dm[s]);
                const double az = fabs(z[s]);
                if (!isfinite(ad) || !isfinite(az)) bad = 1u;
                dn = (ad > dn) ? ad : dn;
                zn = (az > zn) ? az : zn;
            }
            bad = seg_all<SEG, OpOr>(bad, lane);
            dn = seg_all_max_d<SEG>(dn, lane);
            zn = seg_all_max_d<SEG>(zn, lane);
            if (state == 0) {
                nit = it;
                if (bad) state = 2;
                else if (dn <= kMixedTol * zn) state = 1;
                else if (dn > 0.5 * prev) state = 2;
                prev = dn;
            }
            asm volatile("" : "+v"(state), "+v"(nit));
            __syncthreads();  // s_z is rewritten by the next correction
        }
        if (state == 0) state = 2;

        // ---- outputs --------------------------------------------------------
        if (valid) {
            flags = seg_all<SEG, OpOr>(flags, lane);
            if (flags != 0) {
                int st = RBFFD_NONFINITE;
                if (flags & F_BADIDX) st = RBFFD_BAD_INDEX;
                else if (flags & F_NONFIN) st = RBFFD_NONFINITE;
                else if (flags & F_DUP) st = RBFFD_DUPLICATE;
                double *wi = w + i * (int64_t)k_stride;
                for (int q = l0; q < k_stride; q += SEG) wi[q] = q < n ? __builtin_nan("") : 0.0;
                if (l0 == 0) {
                    if (status) status[i] = st;
                    if (iters) iters[i] = 0;
                }
            } else if (state == 1) {
                double *wi = w + i * (int64_t)k_stride;
                const double s2 = OP == 0 ? sc * sc : sc;  // the operator's scale power
#pragma unroll
                for (int s = 0; s < SL; ++s)
                    if (pos[s] < n) wi[pos[s]] = z[s] / s2;
                for (int q = n + l0; q < k_stride; q += SEG) wi[q] = 0.0;
                if (l0 == 0) {
                    if (status) status[i] = RBFFD_OK;
                    if (iters) iters[i] = nit;
                }
            } else if (l0 == 0) {
                fb_list[atomicAdd(fb_count, 1)] = (int32_t)i;
                if (iters) iters[i] = nit;  // the corrections tried
            }
        }
        __syncthreads();  // LDS reuse by the next stencil group
    }
}

template <int KP, int SEG, int SL, int NFIX, int MFIX, int OCC = 0, int OP = 0>
struct MixedLaunch {
    static constexpr int GPB = kWave / SEG;
    // blocks of the grid-stride launch: bounded so the scratch stays modest
    static int64_t blocks(int64_t n_rows) {
        const int64_t want = ceil_div(n_rows, GPB);
        return want < 4096 ? want : 4096;
    }
    static size_t scratch_bytes(int64_t n_rows) {
        return (size_t)blocks(n_rows) * GPB * KP * KP * sizeof(double);
    }
    static int run(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                   int32_t k_stride, const int32_t *rows, const int32_t *n_rows_dev,
                   int64_t n_rows, double *w, int32_t *status, int32_t *iters, double *scratch,
                   int32_t *fb_count, int32_t *fb_list, hipStream_t stream) {
        if (n_rows <= 0) return RBFFD_SUCCESS;
        hipLaunchKernelGGL((weights_mx_kernel<KP, SEG, SL, NFIX, MFIX, OCC, OP>),
                           dim3((unsigned)blocks(n_rows)), dim3(kWave), 0, stream, x, y, n_nodes,
                           nbr, k_stride, rows, n_rows_dev, n_rows, w, status, iters, scratch,
                           fb_count, fb_list);
        return last_launch_rc();
    }
};

}  // namespace wk
}  // namespace rbffd
