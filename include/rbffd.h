/*
 * rbffd.h - C ABI of the MI355X (gfx950) RBF-FD Laplacian stencil library.
 *
 * The library computes, for every scattered 2-D node x_i, the weights w_ik of
 * the local operator approximation  (lap u)(x_i) ~ sum_k w_ik u(x_{nbr_ik})
 * (paper: eq. (1), section II), using the polyharmonic spline phi(r) = r^3
 * augmented with all monomials of degree <= m (sections I and V), and the
 * pieces around it: support selection, the CSR form of the operator with
 * Dirichlet identity rows (section IV) and its product with a field.
 *
 * Conventions shared by every entry point
 *   - Pointers are DEVICE pointers unless marked "host".  All arrays are
 *     dense, row-major, owned by the caller; the library never allocates,
 *     frees or keeps caller memory.  Scratch memory is passed in as a
 *     workspace whose size the matching *_workspace_size query returns.
 *   - stream is a hipStream_t (NULL = the default stream).  Work is enqueued
 *     asynchronously on it; no entry point synchronises the host.
 *   - Return value: RBFFD_SUCCESS (0) or a negative RBFFD_ERR_* code.
 *     Arguments are checked before anything is enqueued, so a negative return
 *     means nothing ran.  RBFFD_ERR_HIP - e signals a HIP launch error e.
 *   - Numerical trouble is reported per stencil in a status array (values
 *     RBFFD_OK ... RBFFD_DUPLICATE below) and the failed stencil's weights
 *     are NaN, so it cannot be used silently.
 *   - Calls on different streams are independent; the only process-wide
 *     state is the batch tuning table (rbffd_batch_tuning_set) and the fixed
 *     scratch array of rbffd_knn_noalloc.
 */
#ifndef RBFFD_H
#define RBFFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---------------------------------------------------- */
#define RBFFD_SUCCESS 0
#define RBFFD_ERR_ARG (-1)          /* invalid argument (null, size, range) */
#define RBFFD_ERR_WORKSPACE (-2)    /* workspace missing or too small */
#define RBFFD_ERR_UNSUPPORTED (-3)  /* valid but not built (e.g. K > 96) */
#define RBFFD_ERR_TOO_LARGE (-4)    /* input too large for a no-allocation call */
#define RBFFD_ERR_HIP (-100)        /* RBFFD_ERR_HIP - hipError_t */

/* ---- per-stencil status codes ------------------------------------------ */
#define RBFFD_OK 0
#define RBFFD_SINGULAR 1        /* a pivot of the LU is exactly zero */
#define RBFFD_FELL_BACK_FP64 2  /* mixed precision: refinement failed, the
                                   stencil was redone in FP64 (weights valid) */
#define RBFFD_NONFINITE 3       /* non-finite coordinate, pivot or solution */
#define RBFFD_BAD_INDEX 4       /* a support index lies outside [0, n_nodes) */
#define RBFFD_DUPLICATE 5       /* two support nodes coincide */
#define RBFFD_BAD_ORDER 6       /* per-node order not in {2,4,6} ({2,4} in 3-D) */

/* ---- precision ---------------------------------------------------------- */
/* outcome of rbffd_solve (its `info` output) */
#define RBFFD_SOLVE_CONVERGED 0  /* ||b - W x|| <= rtol ||b|| by the recurrence */
#define RBFFD_SOLVE_MAX_ITER 1   /* max_iter iterations without converging */
#define RBFFD_SOLVE_BREAKDOWN 2  /* (r0, v) = 0, (r0, r) = 0 or omega = 0 */
#define RBFFD_SOLVE_NONFINITE 3  /* a non-finite scalar (NaN or Inf in W, b, x) */

#define RBFFD_FP64 0   /* FP64 assembly, factorisation and solves */
#define RBFFD_MIXED 1  /* FP32 factorisation + FP64 iterative refinement */

/* Text for a return code or a status code (host, static storage). */
const char *rbffd_error_string(int code);

/* Library version, major * 10000 + minor * 100 + patch. */
int rbffd_version(void);

/* ==========================================================================
 * Support selection: N(x) of eq. (1), the k nearest nodes (section II; the
 * support sizes of section V).
 *
 * nbr[i*k + s] (int32, [n_nodes][k]) lists, for node i, the k nodes j with the
 * smallest keys (d2, j) in lexicographic order, ascending, where
 * d2 = fl(fl(dx*dx) + fl(dy*dy)), dx = x[j] - x[i], dy = y[j] - y[i], with no
 * fused multiply-add.  Node i itself comes first unless a coincident node has
 * a smaller index.  Nodes whose key is NaN are never selected; slots that
 * cannot be filled for that reason hold -1.
 *
 * x, y: [n_nodes] FP64.  1 <= k <= 64, k <= n_nodes, n_nodes < 2^31.
 * The search is exact (a uniform cell grid visited ring by ring, stopped
 * only when no unvisited cell can hold a smaller key).
 * ======================================================================== */
int rbffd_knn_workspace_size(int64_t n_nodes, int32_t k, size_t *bytes /* host */);
int rbffd_knn(const double *x, const double *y, int64_t n_nodes, int32_t k,
              int32_t *nbr, void *workspace, size_t workspace_bytes, void *stream);

/* --------------------------------------------------------------------------
 * rbffd_knn without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments (minus the workspace), same kernels and
 * the same nbr, bit for bit.  Its scratch is a fixed array of
 * RBFFD_KNN_NOALLOC_SCRATCH_BYTES in device memory that the library holds on
 * every GPU it runs on, until the process ends; the call itself allocates
 * nothing and frees nothing.
 *
 * Size limit: the call is accepted when rbffd_knn_workspace_size(n_nodes, k)
 * is at most RBFFD_KNN_NOALLOC_SCRATCH_BYTES: every k <= 64 up to at least
 * 1,397,396 nodes, and the standard supports k = 12, 30, 56 up to 2,236,160,
 * 2,329,376 and 2,515,808 nodes.  Larger inputs return RBFFD_ERR_TOO_LARGE
 * before anything is enqueued.
 * Device: the scratch used is the current device's (hipGetDevice); the
 * stream must belong to that device.  The first call on a device looks the
 * array up (hipGetSymbolAddress) and keeps its address.
 * Concurrency: every call on one GPU shares that GPU's array, so calls that
 * overlap in time on one GPU (other streams, other host threads) race and
 * corrupt each other's results; serialise them (one stream, or events).
 * Each call clears what it needs cleared (a fill kernel, no memset) and
 * overwrites the rest, so the previous call's contents do no harm.
 * ------------------------------------------------------------------------ */
#define RBFFD_KNN_NOALLOC_SCRATCH_BYTES (64u << 20)
int rbffd_knn_noalloc(const double *x, const double *y, int64_t n_nodes, int32_t k,
                      int32_t *nbr, void *stream);

/* ==========================================================================
 * Stencil weights: w of eq. (1) for L = Laplacian with phi(r) = r^3 and all
 * 2-D monomials of degree <= m (sections I, II, V).
 *
 * For stencil i with support idx_k = nbr[i*k_stride + k], k < n:
 *   d_k  = (x[idx_k] - x[i], y[idx_k] - y[i]),  s = max_k |d_k|,  u_k = d_k / s
 *   M    = [A P; P^T 0],  A_kl = |u_k - u_l|^3,  P_kj = p_j(u_k)
 *          (monomials in graded order 1, x, y, x^2, xy, y^2, x^3, ...)
 *   rhs  = [9 |u_k| ; lap p_j(0)]        (lap r^3 = 9 r in 2-D)
 *   M z  = rhs by LU with partial pivoting (first largest |entry| wins ties),
 *   w_ik = z_k / s^2   for k < n;   w_ik = 0 for n <= k < k_stride.
 * The FP64 path performs exactly this sequence of IEEE operations (the
 * elimination uses fma(-l, u, a) and the reciprocal of each pivot).  For
 * (m, n) = (4, 30) and (6, 56) the elimination is blocked by four columns
 * and the trailing updates run as FP64 matrix-core instructions, which
 * apply the same fused updates in the same order, so the result is the
 * same bits.
 *
 * Order: order == NULL -> every node uses (m, n), m in {2,4,6},
 *        (m+1)(m+2)/2 <= n <= k_stride, n + (m+1)(m+2)/2 <= 96.
 *        order != NULL -> order[i] (int8, device, [n_nodes]) in {2,4,6}
 *        selects m per node and n = n_for_order[m/2 - 1] (host, [3]); nodes
 *        are bucketed by system size inside the call.
 * precision: RBFFD_FP64, or RBFFD_MIXED (standard supports (m, n) = (2, 12),
 *   (4, 30), (6, 56) only; RBFFD_ERR_UNSUPPORTED otherwise): the same M and
 *   rhs, factorised in FP32 (same pivoting rule, fmaf updates), then refined:
 *   r = rhs - M z in FP64 (fused, columns ascending), d = FP32 solve of
 *   (float) r, z += d, converged when max|d| <= 1e-12 max|z|.  An FP32 zero
 *   or non-finite pivot, a correction above half the previous one (the first
 *   is compared with max|z| of the initial solve), a non-finite value or 10
 *   corrections without convergence redo the stencil in FP64; its status is
 *   then RBFFD_FELL_BACK_FP64 (weights valid).
 * w: [n_nodes][k_stride] FP64 out.  status: [n_nodes] int32 out (may be NULL).
 * refine_steps: [n_nodes] int32 out (may be NULL; mixed only): corrections
 * applied; for a stencil that fell back, the corrections tried before it
 * did (0 when the FP32 factorisation or the assembly failed).
 * save (may be NULL): factors for rbffd_weights_backward; see
 * rbffd_weights_save_size.  Only with RBFFD_FP64.
 * ======================================================================== */
int rbffd_weights_workspace_size(int64_t n_nodes, int32_t has_order, int32_t precision,
                                 size_t *bytes /* host */);
/* Bytes of the save buffer for the largest system size kmax = n + M(m) in
 * the call: n_nodes * (8*kmax*kmax + 8*kmax + 8 + kmax) rounded up. */
int rbffd_weights_save_size(int64_t n_nodes, int32_t kmax, size_t *bytes /* host */);
int rbffd_weights(const double *x, const double *y, int64_t n_nodes,
                  const int32_t *nbr, int32_t k_stride,
                  const int8_t *order, int32_t m, int32_t n,
                  const int32_t *n_for_order /* host [3] or NULL */,
                  int32_t precision,
                  double *w, int32_t *status, int32_t *refine_steps,
                  void *save, size_t save_bytes,
                  void *workspace, size_t workspace_bytes, void *stream);

/* ==========================================================================
 * Weights of eq. (1) for other operators L (an extension the conclusions
 * name): the same system M, the right-hand side [L phi_k; L p_j] at the
 * centre in unit-scale coordinates, and the scale's power of L:
 *   RBFFD_OP_LAPLACIAN  exactly rbffd_weights with (m, n), FP64;
 *   RBFFD_OP_DX         rhs_k = -3 * sqrt(fl(u_kx^2 + u_ky^2)) * u_kx
 *                       (d/dx of r^3 at the centre), rhs_{n+j} = 1 for the
 *                       monomial x, else 0; w_ik = z_k / s;
 *   RBFFD_OP_DY         likewise with u_ky and the monomial y.
 * Same operation sequence, pivoting, status codes and layouts as
 * rbffd_weights (x, y [n_nodes]; nbr [n_nodes][k_stride]; w out
 * [n_nodes][k_stride], zero past n; status [n_nodes] or NULL).  The
 * derivative operators take any support with K = n + (m+1)(m+2)/2 <= 96
 * (RBFFD_ERR_UNSUPPORTED above), FP64, all nodes.
 * Errors: RBFFD_ERR_ARG for null pointers, an op outside the list, m not in
 * {2, 4, 6}, n < (m+1)(m+2)/2 or n > k_stride.  No workspace.
 * ======================================================================== */
#define RBFFD_OP_LAPLACIAN 0
#define RBFFD_OP_DX 1
#define RBFFD_OP_DY 2
int rbffd_weights_op(const double *x, const double *y, int64_t n_nodes, const int32_t *nbr,
                     int32_t k_stride, int32_t m, int32_t n, int32_t op, double *w,
                     int32_t *status, void *stream);
/* rbffd_weights_op_batch: the d/dx or d/dy weights of rbffd_weights_op for
 * nodes of mixed order (the batching form of section V applied to the
 * derivative operators): order [n_nodes] int8 (device), m_i in {2, 4, 6}
 * on the standard supports n = 12 / 30 / 56; nbr [n_nodes][k_stride] with
 * k_stride >= 56; op RBFFD_OP_DX or RBFFD_OP_DY.  Bucketed by order on the
 * device, then one launch per order (K = 84 first) of rbffd_weights_op's
 * kernels with a block per possible list entry, so each node's weights and
 * status are rbffd_weights_op's at its order, bit for bit; a node whose
 * order is not 2, 4 or 6 gets NaN weights and RBFFD_BAD_ORDER.
 * workspace: rbffd_weights_op_batch_workspace_size bytes of device memory
 * (RBFFD_ERR_WORKSPACE if short).  No host synchronisation. */
int rbffd_weights_op_batch_workspace_size(int64_t n_nodes, size_t *bytes /* host */);
int rbffd_weights_op_batch(const double *x, const double *y, int64_t n_nodes,
                           const int32_t *nbr, int32_t k_stride, const int8_t *order,
                           int32_t op, double *w, int32_t *status, void *workspace,
                           size_t workspace_bytes, void *stream);
/* rbffd_weights_op_mixed: the d/dx or d/dy weights of rbffd_weights_op in
 * the mixed-precision form of rbffd_weights (section V: FP32 factorisation
 * of the FP64-assembled system, FP64 iterative refinement of the
 * operator's right-hand side, the same stopping and fallback rules; a
 * stencil that cannot be refined is solved in FP64 with status
 * RBFFD_FELL_BACK_FP64), on the standard supports (m, n) = (2, 12),
 * (4, 30), (6, 56) (RBFFD_ERR_UNSUPPORTED otherwise).  refine_steps
 * [n_nodes] int32 or NULL receives the corrections per stencil.
 * workspace: rbffd_weights_op_mixed_workspace_size bytes (device).  No
 * host synchronisation. */
int rbffd_weights_op_mixed_workspace_size(int64_t n_nodes, int32_t m, size_t *bytes /* host */);
int rbffd_weights_op_mixed(const double *x, const double *y, int64_t n_nodes,
                           const int32_t *nbr, int32_t k_stride, int32_t m, int32_t n,
                           int32_t op, double *w, int32_t *status, int32_t *refine_steps,
                           void *workspace, size_t workspace_bytes, void *stream);

/* ==========================================================================
 * Three-dimensional nodes (eq. (1) and eq. (2) hold for any dimension d; the
 * paper's experiments are 2-D).  Node coordinates x, y, z: [n_nodes] FP64,
 * device.
 *
 * rbffd_knn3: N(x) in R^3, as rbffd_knn: the k nearest nodes (self first),
 * ascending by (d2, index) with d2 = fl(fl(fl(dx^2) + fl(dy^2)) + fl(dz^2)),
 * NaN keys never taken, -1 for unfillable slots.  nbr: [n_nodes][k] int32
 * out.  1 <= k <= min(128, n_nodes) (k > 128: RBFFD_ERR_UNSUPPORTED from
 * rbffd_knn3, RBFFD_ERR_ARG from the workspace query).
 * Workspace from rbffd_knn3_workspace_size (cell grid, cell-sorted copy of
 * the nodes).
 *
 * rbffd_weights3: Laplacian weights of eq. (1) in d = 3: phi(r) = r^3 with
 * lap r^3 = 12 r, the M = (m+1)(m+2)(m+3)/6 monomials of degree <= m in
 * graded order (inside a degree the x exponent descending, then the y
 * exponent: 1, x, y, z, x^2, xy, xz, y^2, yz, z^2, x^3, ...; each evaluated
 * as (u^a v^b) t^c with powers by repeated multiplication; rhs 2 for x^2,
 * y^2, z^2), the scale s = max |x_k - x_i| (IEEE division by s,
 * w_ik = z_k / s^2), dense LU with partial pivoting (first maximum |entry|
 * in the current order), multipliers a * (1 / pivot), fma updates, the rhs
 * carried along, back substitution with the pivot reciprocals, as in two
 * dimensions.  Status codes and their precedence as in rbffd_weights.
 * nbr: [n_nodes][k_stride] int32, first n columns used; w:
 * [n_nodes][k_stride] FP64 out, zero past n; status: [n_nodes] int32 out or
 * NULL.  m = 2 with 10 <= n <= k_stride, or m = 4 with 35 <= n <= k_stride
 * (RBFFD_ERR_ARG otherwise); m = 2 with n > 54 (K = n + 10 > 64) and m = 4
 * with n > 76 (K = n + 35 > 111) return RBFFD_ERR_UNSUPPORTED.  No
 * workspace.
 *
 * rbffd_weights3_op: the same for the operator op: RBFFD_OP_LAPLACIAN (as
 * rbffd_weights3), RBFFD_OP_DX, RBFFD_OP_DY, RBFFD_OP3_DZ: rhs_k =
 * -3 * sqrt(fl(fl(u^2 + v^2) + t^2)) * (u_k, v_k or t_k) (the derivative of
 * r^3 of node k at the centre), rhs_{n+j} = 1 for the monomial x, y or z,
 * else 0; w_ik = z_k / s.  An op outside the list is RBFFD_ERR_ARG.
 * ======================================================================== */
#define RBFFD_OP3_DZ 3
/* rbffd_weights3_batch: the Laplacian weights of rbffd_weights3 for nodes
 * of mixed order (the batching form of section V, in d = 3): order
 * [n_nodes] int8 (device) gives each node's m, 2 or 4, on the supports
 * n = 20 (m = 2, K = 30) and n = 70 (m = 4, K = 105); nbr [n_nodes]
 * [k_stride] with k_stride >= 70 (the first n_i columns of row i are
 * used); w [n_nodes][k_stride] FP64 out, zero past n_i; status [n_nodes]
 * or NULL.  The nodes are bucketed by order on the device and each class
 * runs its single-order kernel over its list, so every node's weights and
 * status are those of rbffd_weights3 at its order, bit for bit.  A node
 * whose order is neither 2 nor 4 gets NaN weights and RBFFD_BAD_ORDER.
 * workspace: rbffd_weights3_batch_workspace_size bytes of device memory
 * (owned by the caller, RBFFD_ERR_WORKSPACE if short); no host
 * synchronisation.  Argument errors as in rbffd_weights3. */
int rbffd_weights3_batch_workspace_size(int64_t n_nodes, size_t *bytes /* host */);
int rbffd_weights3_batch(const double *x, const double *y, const double *z, int64_t n_nodes,
                         const int32_t *nbr, int32_t k_stride, const int8_t *order, double *w,
                         int32_t *status, void *workspace, size_t workspace_bytes,
                         void *stream);
int rbffd_knn3_workspace_size(int64_t n_nodes, int32_t k, size_t *bytes /* host */);
int rbffd_knn3(const double *x, const double *y, const double *z, int64_t n_nodes, int32_t k,
               int32_t *nbr, void *workspace, size_t workspace_bytes, void *stream);
int rbffd_weights3(const double *x, const double *y, const double *z, int64_t n_nodes,
                   const int32_t *nbr, int32_t k_stride, int32_t m, int32_t n, double *w,
                   int32_t *status, void *stream);
int rbffd_weights3_op(const double *x, const double *y, const double *z, int64_t n_nodes,
                      const int32_t *nbr, int32_t k_stride, int32_t m, int32_t n, int32_t op,
                      double *w, int32_t *status, void *stream);

/* ==========================================================================
 * Tuning of the mixed-order batch (rbffd_weights with a per-node order and
 * the standard supports n = 12/30/56, FP64), in one of three forms:
 *   per_order = 0: one persistent launch: blocks_per_cu blocks of 128
 *     threads per compute unit pull tiles from a work queue, largest
 *     systems first; groups_per_tile[q] sets the tile size of order
 *     m = 2q+2 (in stencils for m = 6, in 2-stencil / 8-stencil wavefront
 *     groups for m = 4 / m = 2);
 *   per_order = 1: one persistent launch per order on the same stream
 *     (m = 6, 4, 2), each with its single-order kernel's block shape and
 *     occupancy, order_blocks_per_cu[q] blocks per compute unit walking
 *     that order's list; nothing is cleared between calls;
 *   per_order = 2: one launch per order (m = 6, 4, 2) of the single-order
 *     kernels themselves, one block (or one 8-stencil group at m = 2) per
 *     possible list entry, those past the list's length returning at once.
 * When the factors are saved (the adjoint's forward) the one-launch form
 * runs.  The values only change speed, never results.  This table is the
 * library's only process-wide state; set it before launching (e.g. from
 * the autotuner's saved choice).  NULL restores the defaults
 * {2, {1, 1, 1}, 0, {12, 16, 4}} (the per-order grids: one block per wavefront
 * slot of each kernel's occupancy).
 * ======================================================================== */
typedef struct rbffd_batch_tuning {
    int32_t blocks_per_cu;          /* 1..64 */
    int32_t groups_per_tile[3];     /* 1..64 each, for m = 2, 4, 6 */
    int32_t per_order;              /* 0, 1 or 2 */
    int32_t order_blocks_per_cu[3]; /* 1..64 each, for m = 2, 4, 6 */
} rbffd_batch_tuning;
int rbffd_batch_tuning_set(const rbffd_batch_tuning *tuning /* host, or NULL */);
int rbffd_batch_tuning_get(rbffd_batch_tuning *tuning /* host */);

/* ==========================================================================
 * Adjoint of rbffd_weights (FP64): given G = dL/dw ([n_nodes][k_stride]),
 * returns dL/dx, dL/dy ([n_nodes], overwritten) for all node coordinates,
 * with the supports held fixed.  Uses the factors that rbffd_weights stored
 * in save (same nodes, supports and orders): mu = M^{-1} [G/s^2; 0] (M is
 * symmetric), then per support node
 *   dL/du_k = 9 mu_k u_k/|u_k| - sum_l 3|u_k-u_l|(u_k-u_l)(mu_k w_l + mu_l w_k)
 *             - sum_j grad p_j(u_k)(mu_k lambda_j + w_k mu_{n+j})
 * (w, lambda: the unit-scale solution z), dL/dx_{idx_k} += dL/du_k / s and
 * dL/dx_i -= dL/du_k / s.  The sum over stencils is gathered per node in a
 * fixed order, so results are deterministic.  Stencils whose forward status
 * was not RBFFD_OK contribute nothing.
 * ======================================================================== */
int rbffd_weights_backward_workspace_size(int64_t n_nodes, int32_t k_stride,
                                          size_t *bytes /* host */);
int rbffd_weights_backward(const double *x, const double *y, int64_t n_nodes,
                           const int32_t *nbr, int32_t k_stride,
                           const int8_t *order, int32_t m, int32_t n,
                           const int32_t *n_for_order /* host [3] or NULL */,
                           const double *grad_w, const void *save, size_t save_bytes,
                           const int32_t *status,
                           double *grad_x, double *grad_y,
                           void *workspace, size_t workspace_bytes, void *stream);

/* ==========================================================================
 * CSR form of the discrete operator (eq. (1) rows; Dirichlet rows of
 * section IV become identity rows).
 *
 * Row i: is_boundary[i] != 0 -> the single entry (i, 1.0); otherwise the
 * pairs (nbr[i][k], w[i][k]), k < n_i, sorted by (column, k).  n_i is n, or
 * n_for_order[order[i]/2 - 1] when order != NULL.  is_boundary may be NULL
 * (all rows interior).  row_ptr: [n_nodes + 1] int64 out; col (int32),
 * val (FP64): capacity entries, capacity >= n_nodes * max n_i (the exact
 * nnz is row_ptr[n_nodes], known only on the device).
 * ======================================================================== */
int rbffd_assemble_csr_workspace_size(int64_t n_nodes, size_t *bytes /* host */);
int rbffd_assemble_csr(int64_t n_nodes, const int32_t *nbr, int32_t k_stride,
                       const int8_t *order, int32_t n,
                       const int32_t *n_for_order /* host [3] or NULL */,
                       const double *w, const uint8_t *is_boundary,
                       int64_t *row_ptr, int32_t *col, double *val, int64_t capacity,
                       void *workspace, size_t workspace_bytes, void *stream);

/* ==========================================================================
 * The explicit pseudo-time loop of section IV, eq. (3), n_steps times:
 *   u(x_i) <- u(x_i) + dt (f(x_i) + sum_{k < n} w[i][k] u(x_nbr[i][k]))
 * for interior nodes (is_boundary[i] == 0); Dirichlet nodes
 * (is_boundary[i] != 0) keep their values.  is_boundary may be NULL (no
 * boundary).  The sum runs with fma over k ascending from 0, then
 * t = f + sum and u + dt * t (two roundings).  Supports and weights are the
 * ELL rows of rbffd_knn / rbffd_weights: nbr, w [n_nodes][k_stride], the
 * first n entries of each row used.  u [n_nodes] holds the initial values
 * (boundary values included) and receives the values after the last step;
 * u_work [n_nodes] is caller-owned scratch (must differ from u).  The
 * workspace (size from rbffd_time_steps_workspace_size) receives a k-major
 * copy of the first n columns of nbr and w, made once per call.  A support
 * index outside [0, n_nodes) turns the node's value into NaN.
 * Errors: RBFFD_ERR_ARG for null pointers, n < 1, k_stride < n,
 * n_steps < 0, dt NaN or a short workspace.  n_steps = 0 leaves u unchanged.
 * ======================================================================== */
int rbffd_time_steps_workspace_size(int64_t n_nodes, int32_t n, size_t *bytes /* host */);
int rbffd_time_steps(int64_t n_nodes, const int32_t *nbr, int32_t k_stride, int32_t n,
                     const double *w, const uint8_t *is_boundary, const double *f, double dt,
                     int64_t n_steps, double *u, double *u_work, void *workspace,
                     size_t workspace_bytes, void *stream);

/* ==========================================================================
 * y = W u - f for a CSR matrix (the operator product of eq. (3)); f may be
 * NULL (then y = W u).  Each row is summed in CSR order with fma, starting
 * from 0.  The operator is square: row_ptr [n_rows+1] int64, col int32,
 * val FP64, u/f/y [n_rows] FP64; a row holding a column outside [0, n_rows)
 * yields NaN (such an entry is never read).
 * ======================================================================== */
int rbffd_spmv(int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
               const double *val, const double *u, const double *f, double *y,
               void *stream);

/* ==========================================================================
 * Implicit solve of the assembled operator, W x = b: the steady Dirichlet
 * Poisson problem of eq. (2) with the boundary rows of section IV (an
 * extension the conclusions name).  W is a square CSR matrix as built by
 * rbffd_assemble_csr (row_ptr [n_rows+1] int64, col int32, val FP64); b and
 * x are [n_rows] FP64 device vectors; x holds the initial guess on entry and
 * the solution on return.  Method: BiCGSTAB (van der Vorst 1992) without a
 * preconditioner, stopped when the recurrence residual satisfies
 * ||r|| <= rtol ||b|| or after max_iter iterations.  Dot products are
 * reduced in a fixed order, so a call is reproducible bit for bit.
 * Host outputs: iters (iterations run), relres = ||b - W x|| / ||b|| of the
 * returned x (recomputed, not the recurrence value; ||b - W x|| when b = 0),
 * info = RBFFD_SOLVE_*.  Unlike the other calls this one synchronizes the
 * stream (it reads the convergence flag every 8 iterations), so it cannot
 * be captured into a graph.  workspace: rbffd_solve_workspace_size bytes
 * (six vectors, the Jacobi scaling and the reduction partials).
 * Errors: RBFFD_ERR_ARG for null pointers, n_rows < 1, rtol < 0 or NaN,
 * max_iter < 0; RBFFD_ERR_WORKSPACE for a short workspace.  A column
 * outside [0, n_rows) makes its row NaN and the solve ends with
 * RBFFD_SOLVE_NONFINITE.
 * ======================================================================== */
int rbffd_solve_workspace_size(int64_t n_rows, size_t *bytes /* host */);
int rbffd_solve(int64_t n_rows, const int64_t *row_ptr, const int32_t *col, const double *val,
                const double *b, double *x, double rtol, int32_t max_iter,
                int32_t *iters /* host */, double *relres /* host */, int32_t *info /* host */,
                void *workspace, size_t workspace_bytes, void *stream);

/* --------------------------------------------------------------------------
 * The same solve with an optional preconditioner and no host
 * synchronisation, so that it can be captured into a graph.
 * precond: RBFFD_PRECOND_NONE (the iteration of rbffd_solve, the same bits)
 * or RBFFD_PRECOND_JACOBI: right preconditioning by the diagonal of W
 * (W D^-1 y = b, x = D^-1 y; the residual and the stopping test stay those
 * of W x = b).  The interior rows of the assembled operator scale as 1/h^2
 * and its Dirichlet rows as 1; the scaling puts every row on the unit
 * diagonal.  A row without a non-zero finite diagonal entry is left
 * unscaled.
 * All max_iter iterations are enqueued (five launches each); once the solve
 * has ended every later launch returns at once.  result (device) receives
 * {iters, info, relres} as rbffd_solve returns them, after the last launch;
 * read it after synchronising the stream.  Same workspace and errors as
 * rbffd_solve, and RBFFD_ERR_ARG for an unknown precond.
 * ------------------------------------------------------------------------ */
#define RBFFD_PRECOND_NONE 0
#define RBFFD_PRECOND_JACOBI 1
typedef struct {
    int32_t iters;
    int32_t info;
    double relres;
} rbffd_solve_result;
int rbffd_solve_async(int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
                      const double *val, const double *b, double *x, double rtol,
                      int32_t max_iter, int32_t precond, rbffd_solve_result *result,
                      void *workspace, size_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RBFFD_H */
