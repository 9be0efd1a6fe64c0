// Exact k-nearest-neighbour supports (the set N(x) of eq. (1)) for nodes in
// three dimensions, on a uniform cell grid; the 2-D search of knn.hip with a
// third axis.
//
//   1. bounding box of the finite coordinates (two-pass reduction);
//   2. cubic cells sized for ~k/3 nodes each, the cell count bounded by a
//      host-known maximum;
//   3. counting sort of the nodes by cell; queries stream the sorted copy of
//      (x, y, z, id);
//   4. queries in cell order: one thread per query for k <= 32, one
//      wavefront per query above; cells are visited shell by shell around
//      the query's cell (the cells at Chebyshev distance R) and the k best
//      keys (d2, j), d2 = fl(fl(fl(dx*dx) + fl(dy*dy)) + fl(dz*dz)), are kept
//      sorted (in one thread's registers, or spread over the wavefront).
//      The search stops once the k-th key lies strictly inside the visited
//      block (with a margin far above rounding error).  The keys are unique,
//      so the result does not depend on the order in which candidates are
//      met.

#include <float.h>

#include "common.h"
#include "knn_topk.h"

namespace rbffd {
namespace {

constexpr int kT = 256;         // threads of the grid-building kernels
constexpr int kQ = 64;          // queries per block: one wavefront
constexpr int kParts = 512;     // blocks of the bounding-box pass

struct Grid3 {
    double xmin, ymin, zmin, cs, inv_cs;
    int32_t gx, gy, gz;
    int32_t pad;
};

double per_cell3(int32_t k) {
    const double p = (double)k / 3.0;
    return p > 1.0 ? p : 1.0;
}

int64_t max_cells3(int64_t n_nodes, int32_t k) {
    const int64_t per = (int64_t)per_cell3(k) > 1 ? (int64_t)per_cell3(k) : 1;
    return 3 * ceil_div(n_nodes, per) + 2;
}

__global__ __launch_bounds__(kT) void bbox3_partial(const double *__restrict__ x,
                                                    const double *__restrict__ y,
                                                    const double *__restrict__ z, int64_t n,
                                                    double *__restrict__ part) {
    double v[6] = {DBL_MAX, -DBL_MAX, DBL_MAX, -DBL_MAX, DBL_MAX, -DBL_MAX};
    const int64_t stride = (int64_t)gridDim.x * kT;
    for (int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x; q < n; q += stride) {
        const double a = x[q], b = y[q], c = z[q];
        if (isfinite(a) && isfinite(b) && isfinite(c)) {
            v[0] = fmin(v[0], a);
            v[1] = fmax(v[1], a);
            v[2] = fmin(v[2], b);
            v[3] = fmax(v[3], b);
            v[4] = fmin(v[4], c);
            v[5] = fmax(v[5], c);
        }
    }
    __shared__ double sh[6][kT];
#pragma unroll
    for (int c = 0; c < 6; ++c) sh[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int o = kT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
#pragma unroll
            for (int c = 0; c < 6; c += 2) {
                sh[c][threadIdx.x] = fmin(sh[c][threadIdx.x], sh[c][threadIdx.x + o]);
                sh[c + 1][threadIdx.x] = fmax(sh[c + 1][threadIdx.x], sh[c + 1][threadIdx.x + o]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(kT) void grid3_setup(const double *__restrict__ part, int n_parts,
                                                  int64_t n, double per_cell, int64_t cell_cap,
                                                  Grid3 *__restrict__ gp) {
    double v[6] = {DBL_MAX, -DBL_MAX, DBL_MAX, -DBL_MAX, DBL_MAX, -DBL_MAX};
    for (int b = threadIdx.x; b < n_parts; b += kT) {
#pragma unroll
        for (int c = 0; c < 6; c += 2) {
            v[c] = fmin(v[c], part[6 * b + c]);
            v[c + 1] = fmax(v[c + 1], part[6 * b + c + 1]);
        }
    }
    __shared__ double sh[6][kT];
#pragma unroll
    for (int c = 0; c < 6; ++c) sh[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int o = kT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
#pragma unroll
            for (int c = 0; c < 6; c += 2) {
                sh[c][threadIdx.x] = fmin(sh[c][threadIdx.x], sh[c][threadIdx.x + o]);
                sh[c + 1][threadIdx.x] = fmax(sh[c + 1][threadIdx.x], sh[c + 1][threadIdx.x + o]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    double lo[3], wd[3];
    for (int a = 0; a < 3; ++a) {
        double mn = sh[2 * a][0], mx = sh[2 * a + 1][0];
        if (!(mn <= mx)) mn = mx = 0.0;  // no finite node
        lo[a] = mn;
        wd[a] = mx - mn;
    }
    // cube cells of about per_cell nodes over the box (a flat box gets cells
    // sized by its largest extent)
    const double vol = wd[0] * wd[1] * wd[2];
    const double lmax = fmax(wd[0], fmax(wd[1], wd[2]));
    double cs = fmax(cbrt(vol * per_cell / (double)n), lmax * per_cell / (double)n);
    if (cs < lmax * 1e-7) cs = lmax * 1e-7;
    Grid3 p;
    p.xmin = lo[0];
    p.ymin = lo[1];
    p.zmin = lo[2];
    if (!(cs > 0.0) || !isfinite(cs) || !isfinite(lmax)) {
        p.cs = 1.0;
        p.inv_cs = 0.0;  // every node in cell 0
        p.gx = p.gy = p.gz = 1;
    } else {
        double g[3];
        for (int a = 0; a < 3; ++a) g[a] = floor(wd[a] / cs) + 1.0;
        while (g[0] * g[1] * g[2] > (double)cell_cap) {
            cs *= 1.25;
            for (int a = 0; a < 3; ++a) g[a] = floor(wd[a] / cs) + 1.0;
        }
        p.cs = cs;
        p.inv_cs = 1.0 / cs;
        p.gx = (int32_t)g[0];
        p.gy = (int32_t)g[1];
        p.gz = (int32_t)g[2];
    }
    p.pad = 0;
    *gp = p;
}

__device__ __forceinline__ int coord3(double v, double vmin, double inv_cs, int g) {
    const double t = (v - vmin) * inv_cs;
    return (t >= 0.0) ? (t < (double)g ? (int)t : g - 1) : 0;  // NaN -> 0
}

__device__ __forceinline__ int cell3(const Grid3 &gp, double a, double b, double c) {
    const int cx = coord3(a, gp.xmin, gp.inv_cs, gp.gx);
    const int cy = coord3(b, gp.ymin, gp.inv_cs, gp.gy);
    const int cz = coord3(c, gp.zmin, gp.inv_cs, gp.gz);
    return (cz * gp.gy + cy) * gp.gx + cx;
}

__global__ __launch_bounds__(kT) void cell3_count(const double *__restrict__ x,
                                                  const double *__restrict__ y,
                                                  const double *__restrict__ z, int64_t n,
                                                  const Grid3 *__restrict__ gpp,
                                                  int32_t *__restrict__ cell_of,
                                                  int32_t *__restrict__ counts) {
    const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (q >= n) return;
    const Grid3 gp = *gpp;
    const int c = cell3(gp, x[q], y[q], z[q]);
    cell_of[q] = c;
    atomicAdd(&counts[c], 1);
}

__global__ __launch_bounds__(kT) void cell3_scatter(
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
    int64_t n, const int32_t *__restrict__ cell_of, const int32_t *__restrict__ start,
    int32_t *__restrict__ fill, int32_t *__restrict__ ids, double *__restrict__ xs,
    double *__restrict__ ys, double *__restrict__ zs) {
    const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (q >= n) return;
    const int c = cell_of[q];
    const int slot = start[c] + atomicAdd(&fill[c], 1);
    ids[slot] = (int32_t)q;
    xs[slot] = x[q];
    ys[slot] = y[q];
    zs[slot] = z[q];
}

template <int KMAX>
__device__ __forceinline__ void scan3(TopK<KMAX> &top, int p0, int p1, double qx, double qy,
                                      double qz, const int32_t *__restrict__ ids,
                                      const double *__restrict__ xs,
                                      const double *__restrict__ ys,
                                      const double *__restrict__ zs) {
    for (int p = p0; p < p1; ++p) {
        const double dx = xs[p] - qx;
        const double dy = ys[p] - qy;
        const double dz = zs[p] - qz;
        const double dd = (dx * dx + dy * dy) + dz * dz;
        const int32_t cj = ids[p];
        if (key_less(dd, cj, top.wd(), top.wj())) top.insert(dd, cj);
    }
}

template <int KMAX>
__global__ __launch_bounds__(kQ) void knn3_query(const Grid3 *__restrict__ gpp,
                                                 const int32_t *__restrict__ start,
                                                 const int32_t *__restrict__ ids,
                                                 const double *__restrict__ xs,
                                                 const double *__restrict__ ys,
                                                 const double *__restrict__ zs, int64_t n,
                                                 int32_t k, int32_t *__restrict__ nbr) {
    const int64_t t = (int64_t)blockIdx.x * kQ + threadIdx.x;
    if (t >= n) return;
    const Grid3 gp = *gpp;
    const int32_t qi = ids[t];
    const double qx = xs[t], qy = ys[t], qz = zs[t];
    TopK<KMAX> top;
    top.init(k);
    const int cx = coord3(qx, gp.xmin, gp.inv_cs, gp.gx);
    const int cy = coord3(qy, gp.ymin, gp.inv_cs, gp.gy);
    const int cz = coord3(qz, gp.zmin, gp.inv_cs, gp.gz);
    const int max_r = max(gp.gx, max(gp.gy, gp.gz));
    const double margin = 1e-6 * gp.cs;
    for (int R = 0; R <= max_r; ++R) {
        const int x0 = cx - R, x1 = cx + R, y0 = cy - R, y1 = cy + R, z0 = cz - R, z1 = cz + R;
        const int xa = max(x0, 0), xb = min(x1, gp.gx - 1);
        const int ya = max(y0, 0), yb = min(y1, gp.gy - 1);
        const int za = max(z0, 0), zb = min(z1, gp.gz - 1);
        for (int zz = za; zz <= zb; ++zz) {
            for (int yy = ya; yy <= yb; ++yy) {
                const int row = (zz * gp.gy + yy) * gp.gx;
                if (zz == z0 || zz == z1 || yy == y0 || yy == y1) {
                    // a row on the shell's y or z faces: all its cells
                    scan3<KMAX>(top, start[row + xa], start[row + xb + 1], qx, qy, qz, ids, xs,
                                ys, zs);
                } else {
                    if (x0 >= 0)
                        scan3<KMAX>(top, start[row + x0], start[row + x0 + 1], qx, qy, qz, ids,
                                    xs, ys, zs);
                    if (x1 < gp.gx)
                        scan3<KMAX>(top, start[row + x1], start[row + x1 + 1], qx, qy, qz, ids,
                                    xs, ys, zs);
                }
            }
        }
        // distance from the query to the region outside the visited block
        double lb = __builtin_inf();
        if (x0 > 0) lb = fmin(lb, qx - (gp.xmin + x0 * gp.cs));
        if (x1 < gp.gx - 1) lb = fmin(lb, (gp.xmin + (x1 + 1) * gp.cs) - qx);
        if (y0 > 0) lb = fmin(lb, qy - (gp.ymin + y0 * gp.cs));
        if (y1 < gp.gy - 1) lb = fmin(lb, (gp.ymin + (y1 + 1) * gp.cs) - qy);
        if (z0 > 0) lb = fmin(lb, qz - (gp.zmin + z0 * gp.cs));
        if (z1 < gp.gz - 1) lb = fmin(lb, (gp.zmin + (z1 + 1) * gp.cs) - qz);
        if (lb == __builtin_inf()) break;  // the whole grid has been visited
        lb -= margin;
        if (top.wj() != INT32_MAX && lb > 0.0 && top.wd() < lb * lb) break;
    }
    int32_t *out = nbr + (int64_t)qi * k;
#pragma unroll
    for (int s = 0; s < KMAX; ++s)
        if (s >= KMAX - k) out[s - (KMAX - k)] = top.j[s] == INT32_MAX ? -1 : top.j[s];
}

// ---- large k: one wavefront per query -------------------------------------
// The k best keys form one sorted list spread over the wavefront: position
// p = 64 h + lane (h < H, capacity 64 H).  Candidates are examined 64 at a
// time (lane l takes the l-th of the chunk, so the loads are contiguous);
// every candidate of the chunk that precedes the current k-th key is
// inserted in turn: each position compares it with its key, and the keys
// from its place on shift one position up (from the lane below, or from
// lane 63 of the previous h).  The control flow is uniform over the
// wavefront.  A per-lane register list (knn3_query) instead needs three
// registers per slot and, whenever any lane inserts, runs its insertion in
// every lane.

constexpr int kCoopWaves = 4;  // queries (wavefronts) per block

__device__ __forceinline__ double bcast3_d(double v, int lane) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// the value of the lane below (lane 0 receives lane 63's: the caller
// replaces it)
__device__ __forceinline__ int32_t from_below_i(int32_t v, int lane) {
    return __builtin_amdgcn_ds_bpermute(((lane + 63) & 63) << 2, v);
}
__device__ __forceinline__ double from_below_d(double v, int lane) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)from_below_i((int32_t)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)from_below_i((int32_t)(uint32_t)(b >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <int H>
struct WaveList {
    double d[H];
    int32_t j[H];

    __device__ __forceinline__ void init() {
#pragma unroll
        for (int h = 0; h < H; ++h) {
            d[h] = __builtin_inf();
            j[h] = INT32_MAX;
        }
    }
    // key at position q (uniform)
    __device__ __forceinline__ void at(int q, double &kd, int32_t &kj) const {
        const int l = q & 63, hq = q >> 6;
        double vd = d[0];
        int32_t vj = j[0];
#pragma unroll
        for (int h = 1; h < H; ++h)
            if (hq == h) {
                vd = d[h];
                vj = j[h];
            }
        kd = bcast3_d(vd, l);
        kj = __builtin_amdgcn_readlane(vj, l);
    }
    // insert (cd, cj), a key that precedes position k - 1's; keys are
    // unique, so the positions it precedes form a suffix
    __device__ __forceinline__ void insert(double cd, int32_t cj, int lane) {
        bool lt[H];
#pragma unroll
        for (int h = 0; h < H; ++h) lt[h] = key_less(cd, cj, d[h], j[h]);
        double pd[H];
        int32_t pj[H];
        bool plt[H];
#pragma unroll
        for (int h = 0; h < H; ++h) {
            pd[h] = from_below_d(d[h], lane);
            pj[h] = from_below_i(j[h], lane);
            plt[h] = from_below_i(lt[h] ? 1 : 0, lane) != 0;
            if (lane == 0) {
                // position 64 h - 1: lane 63 of the previous h (none for h = 0)
                if (h == 0) {
                    plt[h] = false;
                } else {
                    pd[h] = bcast3_d(d[h - 1], 63);
                    pj[h] = __builtin_amdgcn_readlane(j[h - 1], 63);
                    plt[h] = __builtin_amdgcn_readlane(lt[h - 1] ? 1 : 0, 63) != 0;
                }
            }
        }
#pragma unroll
        for (int h = 0; h < H; ++h) {
            d[h] = plt[h] ? pd[h] : (lt[h] ? cd : d[h]);
            j[h] = plt[h] ? pj[h] : (lt[h] ? cj : j[h]);
        }
    }
};

template <int H>
__device__ __forceinline__ void scan3_wave(WaveList<H> &top, double &wd, int32_t &wj, int kq,
                                           int p0, int p1, double qx, double qy, double qz,
                                           const int32_t *__restrict__ ids,
                                           const double *__restrict__ xs,
                                           const double *__restrict__ ys,
                                           const double *__restrict__ zs, int lane) {
    for (int base = p0; base < p1; base += kWave) {
        const int p = base + lane;
        double cd = __builtin_inf();
        int32_t cj = INT32_MAX;
        bool take = false;
        if (p < p1) {
            const double dx = xs[p] - qx;
            const double dy = ys[p] - qy;
            const double dz = zs[p] - qz;
            cd = (dx * dx + dy * dy) + dz * dz;
            cj = ids[p];
            take = key_less(cd, cj, wd, wj);
        }
        uint64_t m = __ballot(take);
        while (m) {
            const int src = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            const double vd = bcast3_d(cd, src);
            const int32_t vj = __builtin_amdgcn_readlane(cj, src);
            if (!key_less(vd, vj, wd, wj)) continue;  // the k-th key moved since
            top.insert(vd, vj, lane);
            top.at(kq, wd, wj);
        }
    }
}

template <int H>
__global__ __launch_bounds__(kCoopWaves * kWave) void knn3_query_wave(
    const Grid3 *__restrict__ gpp, const int32_t *__restrict__ start,
    const int32_t *__restrict__ ids, const double *__restrict__ xs,
    const double *__restrict__ ys, const double *__restrict__ zs, int64_t n, int32_t k,
    int32_t *__restrict__ nbr) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t t = (int64_t)blockIdx.x * kCoopWaves + (threadIdx.x >> 6);
    if (t >= n) return;  // whole wavefronts
    const Grid3 gp = *gpp;
    const int32_t qi = ids[t];
    const double qx = xs[t], qy = ys[t], qz = zs[t];
    WaveList<H> top;
    top.init();
    double wd = __builtin_inf();  // the current k-th key
    int32_t wj = INT32_MAX;
    const int kq = k - 1;
    const int cx = coord3(qx, gp.xmin, gp.inv_cs, gp.gx);
    const int cy = coord3(qy, gp.ymin, gp.inv_cs, gp.gy);
    const int cz = coord3(qz, gp.zmin, gp.inv_cs, gp.gz);
    const int max_r = max(gp.gx, max(gp.gy, gp.gz));
    const double margin = 1e-6 * gp.cs;
    for (int R = 0; R <= max_r; ++R) {
        const int x0 = cx - R, x1 = cx + R, y0 = cy - R, y1 = cy + R, z0 = cz - R, z1 = cz + R;
        const int xa = max(x0, 0), xb = min(x1, gp.gx - 1);
        const int ya = max(y0, 0), yb = min(y1, gp.gy - 1);
        const int za = max(z0, 0), zb = min(z1, gp.gz - 1);
        for (int zz = za; zz <= zb; ++zz) {
            for (int yy = ya; yy <= yb; ++yy) {
                const int row = (zz * gp.gy + yy) * gp.gx;
                if (zz == z0 || zz == z1 || yy == y0 || yy == y1) {
                    scan3_wave<H>(top, wd, wj, kq, start[row + xa], start[row + xb + 1], qx, qy,
                                  qz, ids, xs, ys, zs, lane);
                } else {
                    if (x0 >= 0)
                        scan3_wave<H>(top, wd, wj, kq, start[row + x0], start[row + x0 + 1], qx,
                                      qy, qz, ids, xs, ys, zs, lane);
                    if (x1 < gp.gx)
                        scan3_wave<H>(top, wd, wj, kq, start[row + x1], start[row + x1 + 1], qx,
                                      qy, qz, ids, xs, ys, zs, lane);
                }
            }
        }
        double lb = __builtin_inf();
        if (x0 > 0) lb = fmin(lb, qx - (gp.xmin + x0 * gp.cs));
        if (x1 < gp.gx - 1) lb = fmin(lb, (gp.xmin + (x1 + 1) * gp.cs) - qx);
        if (y0 > 0) lb = fmin(lb, qy - (gp.ymin + y0 * gp.cs));
        if (y1 < gp.gy - 1) lb = fmin(lb, (gp.ymin + (y1 + 1) * gp.cs) - qy);
        if (z0 > 0) lb = fmin(lb, qz - (gp.zmin + z0 * gp.cs));
        if (z1 < gp.gz - 1) lb = fmin(lb, (gp.zmin + (z1 + 1) * gp.cs) - qz);
        if (lb == __builtin_inf()) break;  // the whole grid has been visited
        lb -= margin;
        if (wj != INT32_MAX && lb > 0.0 && wd < lb * lb) break;
    }
    int32_t *out = nbr + (int64_t)qi * k;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int q = kWave * h + lane;
        if (q < k) out[q] = top.j[h] == INT32_MAX ? -1 : top.j[h];
    }
}

struct Knn3Ws {
    Grid3 *gp;
    double *part;
    int32_t *counts, *fill, *cell_of, *ids;
    double *xs, *ys, *zs;
    void *scan;
    size_t bytes;
};

Knn3Ws carve3(void *base, int64_t n, int32_t k) {
    const int64_t cells = max_cells3(n, k);
    Carver c(base);
    Knn3Ws w;
    w.gp = c.take<Grid3>(1);
    w.part = c.take<double>(kParts * 6);
    w.counts = c.take<int32_t>(cells + 1);
    w.fill = c.take<int32_t>(cells + 1);
    w.cell_of = c.take<int32_t>(n);
    w.ids = c.take<int32_t>(n);
    w.xs = c.take<double>(n);
    w.ys = c.take<double>(n);
    w.zs = c.take<double>(n);
    w.scan = c.take<char>(scan_workspace_bytes(cells + 1));
    w.bytes = c.bytes();
    return w;
}

}  // namespace
}  // namespace rbffd

using namespace rbffd;

extern "C" int rbffd_knn3_workspace_size(int64_t n_nodes, int32_t k, size_t *bytes) {
    if (!bytes || n_nodes < 1 || n_nodes >= INT32_MAX || k < 1 || k > 128 || k > n_nodes)
        return RBFFD_ERR_ARG;
    *bytes = carve3(nullptr, n_nodes, k).bytes;
    return RBFFD_SUCCESS;
}

extern "C" int rbffd_knn3(const double *x, const double *y, const double *z, int64_t n_nodes,
                          int32_t k, int32_t *nbr, void *workspace, size_t workspace_bytes,
                          void *stream) {
    if (!x || !y || !z || !nbr || n_nodes < 1 || n_nodes >= INT32_MAX || k < 1 || k > n_nodes)
        return RBFFD_ERR_ARG;
    if (k > 128) return RBFFD_ERR_UNSUPPORTED;
    Knn3Ws w = carve3(nullptr, n_nodes, k);
    if (!workspace || workspace_bytes < w.bytes) return RBFFD_ERR_WORKSPACE;
    w = carve3(workspace, n_nodes, k);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t cells = max_cells3(n_nodes, k);
    const unsigned nb = (unsigned)ceil_div(n_nodes, kT);
    const int parts = (int)(ceil_div(n_nodes, kT) < kParts ? ceil_div(n_nodes, kT) : kParts);
    int rc;
    hipLaunchKernelGGL(bbox3_partial, dim3(parts), dim3(kT), 0, s, x, y, z, n_nodes, w.part);
    hipLaunchKernelGGL(grid3_setup, dim3(1), dim3(kT), 0, s, (const double *)w.part, parts,
                       n_nodes, per_cell3(k), cells, w.gp);
    if ((rc = fill_i32(w.counts, 0, cells + 1, s)) != 0) return rc;
    if ((rc = fill_i32(w.fill, 0, cells + 1, s)) != 0) return rc;
    hipLaunchKernelGGL(cell3_count, dim3(nb), dim3(kT), 0, s, x, y, z, n_nodes,
                       (const Grid3 *)w.gp, w.cell_of, w.counts);
    if ((rc = exclusive_scan_i32(w.counts, w.counts, cells + 1, w.scan, s)) != 0) return rc;
    hipLaunchKernelGGL(cell3_scatter, dim3(nb), dim3(kT), 0, s, x, y, z, n_nodes,
                       (const int32_t *)w.cell_of, (const int32_t *)w.counts, w.fill, w.ids, w.xs,
                       w.ys, w.zs);
    const unsigned nq = (unsigned)ceil_div(n_nodes, kQ);
    const Grid3 *gp = w.gp;
    const int32_t *start = w.counts, *ids = w.ids;
    const double *xs = w.xs, *ys = w.ys, *zs = w.zs;
    if (k <= 20)
        hipLaunchKernelGGL(knn3_query<20>, dim3(nq), dim3(kQ), 0, s, gp, start, ids, xs, ys, zs,
                           n_nodes, k, nbr);
    else if (k <= 32)
        hipLaunchKernelGGL(knn3_query<32>, dim3(nq), dim3(kQ), 0, s, gp, start, ids, xs, ys, zs,
                           n_nodes, k, nbr);
    else {
        // one wavefront per query (k = 70: the m = 4 support); on the 1M-node
        // cube against per-lane register lists of 64 / 80 slots: k = 33
        // 6.2 ms (8.1), k = 64 11.2 ms (14.4), k = 70 20.5 ms (36.0)
        const unsigned nw = (unsigned)ceil_div(n_nodes, kCoopWaves);
        if (k <= 64)
            hipLaunchKernelGGL(knn3_query_wave<1>, dim3(nw), dim3(kCoopWaves * kWave), 0, s, gp,
                               start, ids, xs, ys, zs, n_nodes, k, nbr);
        else
            hipLaunchKernelGGL(knn3_query_wave<2>, dim3(nw), dim3(kCoopWaves * kWave), 0, s, gp,
                               start, ids, xs, ys, zs, n_nodes, k, nbr);
    }
    return last_launch_rc();
}
