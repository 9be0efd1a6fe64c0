// Exact k-nearest-neighbour supports (the set N(x) of eq. (1)) on a uniform
// cell grid.
//
//   1. bounding box of the finite coordinates (two-pass reduction);
//   2. square cells sized for ~k/3 or k/6 nodes each, the cell count bounded by a
//      host-known maximum so no host round trip is needed;
//   3. counting sort of the nodes by cell (histogram, scan, scatter); the
//      sorted copy of (x, y, id) is what the queries stream through;
//   4. one thread per query, queries in cell order so a wave's lanes search
//      overlapping cells; cells are visited ring by ring around the query's
//      cell and the k best keys (d2, j) are kept sorted in registers.  The
//      search stops once the k-th key is strictly below the squared distance
//      to the unvisited region (minus a safety margin far above rounding
//      error), so every node that could precede the k-th key has been seen.
// Keys are compared lexicographically on (d2, j) with d2 = fl(fl(dx*dx) +
// fl(dy*dy)) (no contraction), hence the result is independent of the order
// in which candidates are visited.

#include <float.h>

#include <mutex>

#include "common.h"
#include "knn_topk.h"

namespace rbffd {
namespace {

constexpr int kBBoxBlocks = 512;
constexpr int kThreads = 256;
// Queries per block.  One wavefront per block spreads the few query
// wavefronts of a 100k-node set evenly over the 256 compute units.
#ifndef RBFFD_KNN_QUERY_THREADS
#define RBFFD_KNN_QUERY_THREADS 64
#endif
constexpr int kQueryThreads = RBFFD_KNN_QUERY_THREADS;

struct GridParams {
    double xmin, ymin, cs, inv_cs;
    int32_t gx, gy;
    int32_t pad[2];
};

// Target nodes per cell: k/3 for lists of up to 16, k/6 for longer ones
// (finer rings cut the candidates scanned past the k-th distance; measured
// on a 100k-node disk at k = 30 and a 1M-node square at k = 12 and 56).
double per_cell(int32_t k) {
    const double p = (double)k / (k > 16 ? 6.0 : 3.0);
    return p > 1.0 ? p : 1.0;
}

// Upper bound on the cell count: three times the target (room for a
// bounding box larger than the node cloud; past it the cells grow)
int64_t max_cells(int64_t n_nodes, int32_t k) {
    const int64_t per = (int64_t)per_cell(k) > 1 ? (int64_t)per_cell(k) : 1;
    return 3 * ceil_div(n_nodes, per) + 2;
}

// Per-block bounding box of the finite nodes; the blocks also clear the two
// cell histograms z0, z1 [nz] (one launch fewer than a separate fill).
__global__ __launch_bounds__(kThreads) void bbox_partial(const double *__restrict__ x,
                                                         const double *__restrict__ y,
                                                         int64_t n, double *__restrict__ part,
                                                         int32_t *__restrict__ z0,
                                                         int32_t *__restrict__ z1, int64_t nz) {
    double v[4] = {DBL_MAX, -DBL_MAX, DBL_MAX, -DBL_MAX};
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < nz; q += stride) {
        z0[q] = 0;
        z1[q] = 0;
    }
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < n; q += stride) {
        const double a = x[q], b = y[q];
        if (isfinite(a) && isfinite(b)) {
            v[0] = fmin(v[0], a);
            v[1] = fmax(v[1], a);
            v[2] = fmin(v[2], b);
            v[3] = fmax(v[3], b);
        }
    }
    __shared__ double sh[4][kThreads];
#pragma unroll
    for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sh[0][threadIdx.x] = fmin(sh[0][threadIdx.x], sh[0][threadIdx.x + o]);
            sh[1][threadIdx.x] = fmax(sh[1][threadIdx.x], sh[1][threadIdx.x + o]);
            sh[2][threadIdx.x] = fmin(sh[2][threadIdx.x], sh[2][threadIdx.x + o]);
            sh[3][threadIdx.x] = fmax(sh[3][threadIdx.x], sh[3][threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(kThreads) void grid_setup(const double *__restrict__ part,
                                                       int n_parts, int64_t n, double per_cell,
                                                       int64_t cell_cap,
                                                       GridParams *__restrict__ gp) {
    // min/max of the per-block boxes (exact, so the order does not matter)
    double v[4] = {DBL_MAX, -DBL_MAX, DBL_MAX, -DBL_MAX};
    for (int b = threadIdx.x; b < n_parts; b += kThreads) {
        v[0] = fmin(v[0], part[4 * b + 0]);
        v[1] = fmax(v[1], part[4 * b + 1]);
        v[2] = fmin(v[2], part[4 * b + 2]);
        v[3] = fmax(v[3], part[4 * b + 3]);
    }
    __shared__ double sh[4][kThreads];
#pragma unroll
    for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sh[0][threadIdx.x] = fmin(sh[0][threadIdx.x], sh[0][threadIdx.x + o]);
            sh[1][threadIdx.x] = fmax(sh[1][threadIdx.x], sh[1][threadIdx.x + o]);
            sh[2][threadIdx.x] = fmin(sh[2][threadIdx.x], sh[2][threadIdx.x + o]);
            sh[3][threadIdx.x] = fmax(sh[3][threadIdx.x], sh[3][threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    double xmn = sh[0][0], xmx = sh[1][0], ymn = sh[2][0], ymx = sh[3][0];
    if (!(xmn <= xmx)) xmn = xmx = 0.0;  // no finite node
    if (!(ymn <= ymx)) ymn = ymx = 0.0;
    const double wx = xmx - xmn, wy = ymx - ymn;
    double cs = fmax(sqrt(wx * wy * per_cell / (double)n), fmax(wx, wy) * per_cell / (double)n);
    GridParams p;
    p.xmin = xmn;
    p.ymin = ymn;
    if (!(cs > 0.0) || !isfinite(cs) || !isfinite(wx) || !isfinite(wy)) {
        p.cs = 1.0;
        p.inv_cs = 0.0;  // every node in cell 0
        p.gx = p.gy = 1;
    } else {
        double gxd = floor(wx / cs) + 1.0, gyd = floor(wy / cs) + 1.0;
        while (gxd * gyd > (double)cell_cap) {
            cs *= 1.25;
            gxd = floor(wx / cs) + 1.0;
            gyd = floor(wy / cs) + 1.0;
        }
        p.cs = cs;
        p.inv_cs = 1.0 / cs;
        p.gx = (int32_t)gxd;
        p.gy = (int32_t)gyd;
    }
    p.pad[0] = p.pad[1] = 0;
    *gp = p;
}

__device__ __forceinline__ int cell_coord(double v, double vmin, double inv_cs, int g) {
    const double t = (v - vmin) * inv_cs;
    return (t >= 0.0) ? (t < (double)g ? (int)t : g - 1) : 0;  // NaN -> 0
}

__global__ __launch_bounds__(kThreads) void cell_count(const double *__restrict__ x,
                                                       const double *__restrict__ y, int64_t n,
                                                       const GridParams *__restrict__ gpp,
                                                       int32_t *__restrict__ cell_of,
                                                       int32_t *__restrict__ counts) {
    const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (q >= n) return;
    const GridParams gp = *gpp;
    const int cx = cell_coord(x[q], gp.xmin, gp.inv_cs, gp.gx);
    const int cy = cell_coord(y[q], gp.ymin, gp.inv_cs, gp.gy);
    const int c = cy * gp.gx + cx;
    cell_of[q] = c;
    atomicAdd(&counts[c], 1);
}

__global__ __launch_bounds__(kThreads) void cell_scatter(
    const double *__restrict__ x, const double *__restrict__ y, int64_t n,
    const int32_t *__restrict__ cell_of, const int32_t *__restrict__ start,
    int32_t *__restrict__ fill, int32_t *__restrict__ ids, double *__restrict__ xs,
    double *__restrict__ ys) {
    const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (q >= n) return;
    const int c = cell_of[q];
    const int slot = start[c] + atomicAdd(&fill[c], 1);
    ids[slot] = (int32_t)q;
    xs[slot] = x[q];
    ys[slot] = y[q];
}

// Candidates whose coordinates are loaded together before any of them is
// tested, so that the loads' latencies overlap: 4 for k <= 32 (measured
// 8-12% faster), 1 for the 64-slot list, whose registers leave no room.
// The insertion order does not change the result (the k smallest keys are a
// set, and the keys are unique).
template <int KMAX>
constexpr int knn_batch() {
    return KMAX <= 32 ? 4 : 1;
}

template <int KMAX>
__device__ __forceinline__ void scan_range(TopK<KMAX> &top, int p0, int p1, double qx,
                                           double qy, const int32_t *__restrict__ ids,
                                           const double *__restrict__ xs,
                                           const double *__restrict__ ys) {
    constexpr int kKnnBatch = knn_batch<KMAX>();
    int p = p0;
    if constexpr (kKnnBatch > 1) {
        for (; p + kKnnBatch <= p1; p += kKnnBatch) {
            double cx[kKnnBatch], cy[kKnnBatch];
            int32_t cj[kKnnBatch];
#pragma unroll
            for (int u = 0; u < kKnnBatch; ++u) {
                cx[u] = xs[p + u];
                cy[u] = ys[p + u];
                cj[u] = ids[p + u];
            }
#pragma unroll
            for (int u = 0; u < kKnnBatch; ++u) {
                const double dx = cx[u] - qx;
                const double dy = cy[u] - qy;
                const double dd = dx * dx + dy * dy;
                if (key_less(dd, cj[u], top.wd(), top.wj())) top.insert(dd, cj[u]);
            }
        }
    }
    for (; p < p1; ++p) {
        const double dx = xs[p] - qx;
        const double dy = ys[p] - qy;
        const double dd = dx * dx + dy * dy;
        const int32_t cj = ids[p];
        if (key_less(dd, cj, top.wd(), top.wj())) top.insert(dd, cj);
    }
}

template <int KMAX>
__global__ __launch_bounds__(kQueryThreads) void knn_query(
    const GridParams *__restrict__ gpp, const int32_t *__restrict__ start,
    const int32_t *__restrict__ ids, const double *__restrict__ xs,
    const double *__restrict__ ys, int64_t n, int32_t k, int32_t *__restrict__ nbr) {
    const int64_t t = (int64_t)blockIdx.x * kQueryThreads + threadIdx.x;
    if (t >= n) return;
    const GridParams gp = *gpp;
    const int32_t qi = ids[t];
    const double qx = xs[t], qy = ys[t];
    TopK<KMAX> top;
    top.init(k);
    const int cx = cell_coord(qx, gp.xmin, gp.inv_cs, gp.gx);
    const int cy = cell_coord(qy, gp.ymin, gp.inv_cs, gp.gy);
    const int max_r = gp.gx > gp.gy ? gp.gx : gp.gy;
    const double margin = 1e-6 * gp.cs;
    for (int R = 0; R <= max_r; ++R) {
        const int x0 = cx - R, x1 = cx + R, y0 = cy - R, y1 = cy + R;
        const int xa = x0 > 0 ? x0 : 0;
        const int xb = x1 < gp.gx - 1 ? x1 : gp.gx - 1;
        const int ya = y0 > 0 ? y0 : 0;
        const int yb = y1 < gp.gy - 1 ? y1 : gp.gy - 1;
        for (int yy = ya; yy <= yb; ++yy) {
            const int row = yy * gp.gx;
            if (yy == y0 || yy == y1) {
                scan_range<KMAX>(top, start[row + xa], start[row + xb + 1], qx, qy, ids, xs,
                                 ys);
            } else {
                if (x0 >= 0)
                    scan_range<KMAX>(top, start[row + x0], start[row + x0 + 1], qx, qy, ids,
                                     xs, ys);
                if (x1 < gp.gx)
                    scan_range<KMAX>(top, start[row + x1], start[row + x1 + 1], qx, qy, ids,
                                     xs, ys);
            }
        }
        // distance from the query to the region outside the visited block
        double lb = __builtin_inf();
        if (x0 > 0) lb = fmin(lb, qx - (gp.xmin + x0 * gp.cs));
        if (x1 < gp.gx - 1) lb = fmin(lb, (gp.xmin + (x1 + 1) * gp.cs) - qx);
        if (y0 > 0) lb = fmin(lb, qy - (gp.ymin + y0 * gp.cs));
        if (y1 < gp.gy - 1) lb = fmin(lb, (gp.ymin + (y1 + 1) * gp.cs) - qy);
        if (lb == __builtin_inf()) break;  // the whole grid has been visited
        lb -= margin;
        if (top.wj() != INT32_MAX && lb > 0.0 && top.wd() < lb * lb) break;
    }
    int32_t *out = nbr + (int64_t)qi * k;
#pragma unroll
    for (int s = 0; s < KMAX; ++s)
        if (s >= KMAX - k) out[s - (KMAX - k)] = top.j[s] == INT32_MAX ? -1 : top.j[s];
}

struct KnnWs {
    GridParams *gp;
    double *part;
    int32_t *counts;
    int32_t *fill;
    int32_t *cell_of;
    int32_t *ids;
    double *xs, *ys;
    void *scan;
    size_t bytes;
};

KnnWs carve(void *base, int64_t n, int32_t k) {
    const int64_t cells = max_cells(n, k);
    Carver c(base);
    KnnWs w;
    w.gp = c.take<GridParams>(1);
    w.part = c.take<double>(kBBoxBlocks * 4);
    w.counts = c.take<int32_t>(cells + 1);
    w.fill = c.take<int32_t>(cells + 1);
    w.cell_of = c.take<int32_t>(n);
    w.ids = c.take<int32_t>(n);
    w.xs = c.take<double>(n);
    w.ys = c.take<double>(n);
    w.scan = c.take<char>(scan_workspace_bytes(cells + 1));
    w.bytes = c.bytes();
    return w;
}

}  // namespace
}  // namespace rbffd

using namespace rbffd;

extern "C" int rbffd_knn_workspace_size(int64_t n_nodes, int32_t k, size_t *bytes) {
    if (!bytes || n_nodes < 1 || n_nodes >= INT32_MAX || k < 1 || k > 64 || k > n_nodes)
        return RBFFD_ERR_ARG;
    *bytes = carve(nullptr, n_nodes, k).bytes;
    return RBFFD_SUCCESS;
}

namespace rbffd {
namespace {

// The whole search on stream s with the workspace carved as w.  Everything
// that must start at zero (the two cell histograms) is cleared by the first
// kernel (bbox_partial); the rest of the workspace is written before it is
// read.
int knn_launch(const double *x, const double *y, int64_t n_nodes, int32_t k, int32_t *nbr,
               const KnnWs &w, hipStream_t s) {
    const int64_t cells = max_cells(n_nodes, k);
    const unsigned nb = (unsigned)ceil_div(n_nodes, kThreads);
    const int parts = (int)(ceil_div(n_nodes, kThreads) < kBBoxBlocks ? ceil_div(n_nodes, kThreads)
                                                                       : kBBoxBlocks);
    int rc;
    hipLaunchKernelGGL(bbox_partial, dim3(parts), dim3(kThreads), 0, s, x, y, n_nodes, w.part,
                       w.counts, w.fill, cells + 1);
    hipLaunchKernelGGL(grid_setup, dim3(1), dim3(kThreads), 0, s, (const double *)w.part, parts,
                       n_nodes, per_cell(k), cells, w.gp);
    hipLaunchKernelGGL(cell_count, dim3(nb), dim3(kThreads), 0, s, x, y, n_nodes,
                       (const GridParams *)w.gp, w.cell_of, w.counts);
    if ((rc = exclusive_scan_i32(w.counts, w.counts, cells + 1, w.scan, s)) != 0) return rc;
    hipLaunchKernelGGL(cell_scatter, dim3(nb), dim3(kThreads), 0, s, x, y, n_nodes,
                       (const int32_t *)w.cell_of, (const int32_t *)w.counts, w.fill, w.ids, w.xs,
                       w.ys);
    const unsigned nq = (unsigned)ceil_div(n_nodes, kQueryThreads);
    const GridParams *gp = w.gp;
    const int32_t *start = w.counts, *ids = w.ids;
    const double *xs = w.xs, *ys = w.ys;
    // exact list lengths for the standard supports (12, 30, 56), else the
    // next of 16, 32, 64
    switch (k) {
    case 12:
        hipLaunchKernelGGL(knn_query<12>, dim3(nq), dim3(kQueryThreads), 0, s, gp, start, ids, xs,
                           ys, n_nodes, k, nbr);
        break;
    case 30:
        hipLaunchKernelGGL(knn_query<30>, dim3(nq), dim3(kQueryThreads), 0, s, gp, start, ids, xs,
                           ys, n_nodes, k, nbr);
        break;
    case 56:
        hipLaunchKernelGGL(knn_query<56>, dim3(nq), dim3(kQueryThreads), 0, s, gp, start, ids, xs,
                           ys, n_nodes, k, nbr);
        break;
    default:
        if (k <= 16)
            hipLaunchKernelGGL(knn_query<16>, dim3(nq), dim3(kQueryThreads), 0, s, gp, start, ids,
                               xs, ys, n_nodes, k, nbr);
        else if (k <= 32)
            hipLaunchKernelGGL(knn_query<32>, dim3(nq), dim3(kQueryThreads), 0, s, gp, start, ids,
                               xs, ys, n_nodes, k, nbr);
        else
            hipLaunchKernelGGL(knn_query<64>, dim3(nq), dim3(kQueryThreads), 0, s, gp, start, ids,
                               xs, ys, n_nodes, k, nbr);
    }
    return last_launch_rc();
}

// Scratch of rbffd_knn_noalloc, used in place of a caller workspace.  Each
// GPU the library runs on holds its own copy of this array until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// is a stand-in, not a device address): it uses the per-device address from
// hipGetSymbolAddress below.
static __device__ __align__(256) char scratch[RBFFD_KNN_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch`, looked up once per device (with
// that device current) and kept.
int scratch_for_current_device(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_rc(e);
    if (dev < 0 || dev >= kMaxDevices) return RBFFD_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_rc(e);
        if (!p) return RBFFD_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RBFFD_SUCCESS;
}

}  // namespace
}  // namespace rbffd

extern "C" int rbffd_knn(const double *x, const double *y, int64_t n_nodes, int32_t k,
                         int32_t *nbr, void *workspace, size_t workspace_bytes, void *stream) {
    if (!x || !y || !nbr || n_nodes < 1 || n_nodes >= INT32_MAX || k < 1 || k > n_nodes)
        return RBFFD_ERR_ARG;
    if (k > 64) return RBFFD_ERR_UNSUPPORTED;
    KnnWs w = carve(nullptr, n_nodes, k);
    if (!workspace || workspace_bytes < w.bytes) return RBFFD_ERR_WORKSPACE;
    w = carve(workspace, n_nodes, k);
    return knn_launch(x, y, n_nodes, k, nbr, w, static_cast<hipStream_t>(stream));
}

extern "C" int rbffd_knn_noalloc(const double *x, const double *y, int64_t n_nodes, int32_t k,
                                 int32_t *nbr, void *stream) {
    if (!x || !y || !nbr || n_nodes < 1 || n_nodes >= INT32_MAX || k < 1 || k > n_nodes)
        return RBFFD_ERR_ARG;
    if (k > 64) return RBFFD_ERR_UNSUPPORTED;
    KnnWs w = carve(nullptr, n_nodes, k);
    if (w.bytes > (size_t)RBFFD_KNN_NOALLOC_SCRATCH_BYTES) return RBFFD_ERR_TOO_LARGE;
    void *base = nullptr;
    const int rc = scratch_for_current_device(&base);
    if (rc) return rc;
    w = carve(base, n_nodes, k);
    return knn_launch(x, y, n_nodes, k, nbr, w, static_cast<hipStream_t>(stream));
}
