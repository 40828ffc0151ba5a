/*
 * rs.h -- C ABI of the MI355X recursive-skeletonization solver.
 *
 * Method: K. L. Ho and L. Greengard, "A fast direct solver for structured linear
 * systems by recursive skeletonization".  Given nodes x_i, quadrature weights w_i
 * and a Green's function K, the library builds the Nystrom system
 *     A_ij = c delta_ij + K(x_i, x_j) w_j      (Section 2, Section 6.2)
 * compresses it level by level over a quadtree/octree with proxy surfaces and
 * interpolative decompositions (Sections 2.2, 3.1, 3.2), factors the compressed
 * inverse (Section 3.4, eq. (multilevel-inverse)), and applies it to right-hand
 * sides (the solution phase of Section 3.4).  All arithmetic is IEEE binary64: real
 * for the Laplace kernels, complex (complex128, re/im pairs of binary64) for the
 * Helmholtz kernel.
 *
 * Conventions shared by every entry point
 *   - Indices are 0-based.  Point arrays are point-major: x0,y0[,z0],x1,... in the
 *     caller's order; the tree permutation is internal.
 *   - "host" pointers are read during the call only; the caller keeps ownership and
 *     may free them on return.  "device" pointers are HIP device memory on the
 *     current device; the library reads/writes them in stream order.
 *   - Every call returns rs_status; no C++ exception crosses this boundary.  On
 *     error, outputs are left untouched and rs_last_error() (thread-local) holds a
 *     message; for RS_ESINGULAR it names the tree depth and box.
 *   - Trees and factor handles are opaque and owned by the library until
 *     rs_tree_free / rs_free.
 */
#ifndef RS_H
#define RS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RS_OK = 0,
  RS_EINVAL = 1,     /* bad argument: NULL, n < 1, non-finite data, eps < 0, ... */
  RS_ENOMEM = 2,     /* device or host allocation failed */
  RS_ESINGULAR = 3,  /* zero or non-finite pivot in a box or root elimination */
  RS_EDEVICE = 4,    /* HIP runtime error, or no device */
  RS_EBUSY = 5,      /* the object is in use by queued work */
  RS_ENOTSUP = 6     /* kernel / dimension combination not built */
} rs_status;

/* Green's functions (Section 2.1 eqs. (2d-laplace), (3d-laplace), (double-layer);
 * Section 6.1 eq. (2d-helmholtz)). */
typedef enum {
  RS_LAP2D_SL = 1,   /* -(1/2pi) log|x-y|,  dim 2 */
  RS_LAP2D_DL = 2,   /* (x-y).nu_y / (2pi |x-y|^2), dim 2, needs normals + curvature */
  RS_LAP3D_SL = 3,   /* 1/(4pi |x-y|), dim 3 */
  RS_HELM2D_CFIE = 4, /* combined field dG_k/dnu_y - i eta G_k, G_k = (i/4) H0(k|x-y|),
                        dim 2, complex128; needs normals + curvature (Section 6.1
                        eq. (2d-helmholtz), combined layer of Section 3.2) */
  RS_HELM3D_SL = 5   /* exp(i k |x-y|) / (4 pi |x-y|), dim 3, complex128 (Section 6.1
                        eq. (3d-helmholtz)) */
} rs_kernel_kind;

/* Kernel description.  The diagonal entries A_ii follow a per-kernel rule:
 *   LAP2D_SL: c - (w_i/2pi) log(w_i/2pi);   LAP2D_DL: c - kappa_i w_i/(4pi);
 *   LAP3D_SL: c + sqrt(w_i/pi)/2;
 *   HELM2D_CFIE: c - kappa_i w_i/(4pi) - i eta s_i with the single-layer self term
 *     s_i = w_i (i/4 - (log(k/2) + gamma)/(2pi)) - (w_i/2pi) log(w_i/2pi)
 *     (gamma = Euler's constant; the smooth part of G_k at coincidence plus the
 *     LAP2D_SL rule for its logarithm);
 *   HELM3D_SL: c + (exp(i k R) - 1) / (2 i k), R = sqrt(w_i/pi) (the kernel integrated
 *     over a flat disc of area w_i; k -> 0 gives the LAP3D_SL rule). */
typedef struct {
  int32_t kind;             /* rs_kernel_kind */
  int32_t dim;              /* 2 or 3, must match kind */
  double identity;          /* c: -0.5 for the interior double-layer equation
                               (eq. (2k-integral-eqn)), 0 for first kind */
  double wavenumber;        /* Helmholtz: k > 0 (unused otherwise) */
  double eta;               /* HELM2D_CFIE: combined-field coupling, e.g. k (unused otherwise) */
  const double *normals;    /* host, N x dim, caller order; LAP2D_DL and HELM2D_CFIE */
  const double *curvature;  /* host, N, caller order; LAP2D_DL and HELM2D_CFIE */
  int32_t proxy_points;     /* proxy-surface points per box (Section 3.2), >= 8 */
  double proxy_ratio;       /* proxy radius / box side; > 0.5*sqrt(dim), e.g. 1.5 */
  int32_t id_mode;          /* rs_id_mode: how each box's block M (m x n) is compressed */
  int32_t oversample;       /* RS_ID_SKETCH: sketch rows ell = min(m, n + oversample), 0..4096 */
  uint64_t sketch_seed;     /* RS_ID_SKETCH: seed of the sign generator */
} rs_kernel;

/* Interpolative decomposition of a box's block (Section 2.2). */
typedef enum {
  RS_ID_CPQR = 0,     /* column-pivoted QR of M itself (deterministic) */
  RS_ID_SKETCH = 1    /* column-pivoted QR of the row sketch Y = Omega M (the randomized
                         ID of Section 2.2): Omega is ell x m with entries +-1, entry (a, i)
                         of tree box b set by the top bit of SplitMix64 (Steele, Lea and
                         Flood, OOPSLA 2014) at the counter
                         seed ^ (b << 40) ^ (a << 20) ^ i  (sign -1 when the bit is set);
                         no sketch when ell = m.  Every box is compressed through its
                         sketch, so a factorization depends on the seed. */
} rs_id_mode;

typedef struct rs_tree_s *rs_tree;
typedef struct rs_factor_s *rs_handle;

/* Launch organisation of the factor and solve passes. */
typedef enum {
  RS_LAUNCH_LEVEL = 0,   /* one launch per kernel per tree level, all boxes of the
                            level (and of every problem of a batch) together */
  RS_LAUNCH_PER_BOX = 1  /* the same kernels launched once per box (reference path) */
} rs_launch_mode;

typedef struct {
  int32_t launch_mode;   /* rs_launch_mode */
  void *stream;          /* hipStream_t for all work of the call; NULL = default */
} rs_options;

/* ---------------------------------------------------------------- tree ---- */

/* Quadtree (dim 2) / octree (dim 3) over n points (Section 2.1; tree rule of
 * Section 6: uniform subdivision of the bounding square/cube until a box holds
 * at most leaf_size points, empty boxes dropped).  points: host, n x dim.
 * Root = bounding box (centre (lo+hi)/2, side max extent); child code bit a set
 * iff x_a >= centre_a; children in code order; stable order inside a child;
 * boxes numbered breadth-first.  Errors: RS_EINVAL (dim not 2/3, n < 1,
 * leaf_size < 1, non-finite coordinate), RS_ENOMEM. */
rs_status rs_build_tree(int32_t dim, int64_t n, const double *points, int32_t leaf_size,
                        rs_tree *out);

/* Box count and maximum depth of a tree. */
rs_status rs_tree_info(rs_tree t, int64_t *nbox, int32_t *maxdepth);

/* Copies the tree into caller arrays (host; any may be NULL to skip):
 * perm[n] (tree position i holds caller point perm[i]), depth/parent/begin/end
 * [nbox] (parent -1 at the root; [begin,end) tree positions), center[nbox*dim],
 * side[nbox]. */
rs_status rs_tree_export(rs_tree t, int64_t *perm, int32_t *depth, int32_t *parent,
                         int64_t *begin, int64_t *end, double *center, double *side);

void rs_tree_free(rs_tree t);

/* -------------------------------------------------------------- factor ---- */

/* Compression + factorization (Sections 3.1, 3.2, 3.4) of the system defined by
 * kernel k on the tree's points.  points (n x dim) and weights (n) are host
 * arrays in caller order and must be the points the tree was built on.
 * eps >= 0 is the relative ID precision (eps = 0: no compression, exact dense
 * elimination).  The returned handle holds the compressed inverse in device
 * memory and is immutable; it stays valid after the tree is freed.
 * Errors: RS_EINVAL, RS_ENOTSUP, RS_ENOMEM, RS_ESINGULAR, RS_EDEVICE. */
rs_status rs_factor(const rs_kernel *k, rs_tree t, const double *points,
                    const double *weights, double eps, rs_handle *out);

/* rs_factor with explicit options (launch mode, stream).  opts may be NULL. */
rs_status rs_factor_ex(const rs_kernel *k, rs_tree t, const double *points,
                       const double *weights, double eps, const rs_options *opts,
                       rs_handle *out);

/* ---------------------------------------------------------------- solve ---- */

/* B := A_eps^{-1} B in place (the solution phase, Section 3.4).  B is column-major
 * n x nrhs with leading dimension ldb >= n (in entries), caller order; entries are
 * doubles for the Laplace kernels and complex128 (re, im pairs of doubles) for the
 * Helmholtz kernels.  B may be
 *   - device memory of the current device: the work is enqueued on stream
 *     (hipStream_t, NULL = default stream) and the result is valid once the stream
 *     has reached this point; the whole n x nrhs range must lie inside one device
 *     allocation as the HIP runtime reports it (RS_EINVAL otherwise; for memory of a
 *     pool allocator such as PyTorch's that is the pool's segment, so the check cannot
 *     see a range that overruns a sub-allocation);
 *   - host memory (pageable or pinned): the call stages B through device memory on
 *     stream and returns when the result is back in B (synchronous).
 * nrhs = 0 is a no-op.  Concurrent calls on one handle from different streams are
 * allowed; each call takes its own workspace.  Errors: RS_EINVAL (including device
 * memory of another device), RS_ENOMEM, RS_EDEVICE. */
rs_status rs_solve(rs_handle h, void *B, int64_t ldb, int32_t nrhs, void *stream);

/* rs_solve with a launch mode (RS_LAUNCH_LEVEL or RS_LAUNCH_PER_BOX). */
rs_status rs_solve_ex(rs_handle h, void *B, int64_t ldb, int32_t nrhs,
                      const rs_options *opts);

/* Y := A_eps X, the compressed forward operator that the handle's compression defines
 * (Section 3.3: an upward pass applying each level's interpolation R, the dense block of
 * the remaining skeletons, and a downward pass applying L and adding each level's
 * diagonal blocks; Section 6.1 uses it as a generalized FMM).  A_eps agrees with A to
 * the compression precision and is exactly the matrix rs_solve inverts, so
 * |A_eps x - b| measures a solve's rounding in O(N) work.  X and Y: device memory of
 * the current device, column-major n x nrhs, leading dimensions ldx, ldy >= n, doubles
 * or complex128 as for rs_solve, caller order; they must not overlap.  Enqueued on
 * stream (NULL = default stream).  The diagonal blocks are evaluated from the kernel on
 * each call; the first call on a handle uploads its descriptors (synchronous once).
 * Errors: RS_EINVAL (host pointers, overlap, ld < n), RS_ENOMEM, RS_EDEVICE. */
rs_status rs_matvec(rs_handle h, const void *X, int64_t ldx, void *Y, int64_t ldy,
                    int32_t nrhs, void *stream);

/* rs_solve for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same solve,
 * bitwise equal to rs_solve, with its workspace (the tree-ordered copy of B and the
 * staging of large boxes) in a fixed 64 MiB scratch array that each device holds
 * from the library's first such call until the process ends.  No hipMalloc, hipFree
 * or other allocating call is made, and no profiler events are recorded.
 * B: device memory of the current device, column-major n x nrhs, ldb >= n, doubles or
 * complex128 as for rs_solve; enqueued on stream (NULL = default stream).
 * Limit: n * nrhs scalars (times 2 for complex128) plus the staging of the largest
 * box must fit 64 MiB; larger requests fail with RS_EINVAL and a message giving the
 * size needed (split the columns over several calls).
 * Every call on a device shares that device's scratch: calls that overlap on one
 * device (different streams, or host threads) race and give wrong results; order
 * them on one stream or synchronize between them.
 * Errors: RS_EINVAL (host pointer, range past the allocation, size over the limit),
 * RS_EDEVICE. */
rs_status rs_solve_noalloc(rs_handle h, void *B, int64_t ldb, int32_t nrhs, void *stream);

/* ------------------------------------------------- batched (many problems) ---- */

/* Factors `count` independent problems together (arrays of length count): every
 * launch covers one tree level of all problems, aligned at each problem's finest
 * depth, and all roots share one launch (real and complex problems in separate
 * launch groups).  Each problem's result is bitwise identical
 * to rs_factor on it alone (same per-box kernels and reduction order).  On success
 * out[i] receives problem i's handle; on error no handle is returned.  Errors as
 * rs_factor. */
rs_status rs_factor_batched(int32_t count, const rs_kernel *kernels, const rs_tree *trees,
                            const double *const *points, const double *const *weights,
                            const double *eps, const rs_options *opts, rs_handle *out);

/* Solves request i (handle h[i], device block B[i] of nrhs[i] columns, leading
 * dimension ldb[i]) for i < count in place, with shared per-level sweep launches
 * across the handles; requests may repeat a handle only on disjoint B blocks.
 * Asynchronous on opts->stream; per-request results are bitwise identical to
 * rs_solve.  launch_mode must be RS_LAUNCH_LEVEL.  Errors: RS_EINVAL, RS_EDEVICE. */
rs_status rs_solve_batched(int32_t count, const rs_handle *h, void *const *B,
                           const int64_t *ldb, const int32_t *nrhs, const rs_options *opts);

/* --------------------------------------------- captured solves (HIP graphs) ---- */

/* A solve plan: the launches of rs_solve_batched for fixed requests (handles h[i],
 * device blocks B[i] with leading dimension ldb[i] and nrhs[i] >= 1 columns) captured
 * once into a HIP graph, with a workspace and launch tables of its own.  Each
 * rs_plan_launch replays the graph on `stream`, solving the current contents of the
 * same B blocks in place; results are bitwise identical to rs_solve_batched and
 * rs_solve.  For callers that solve into fixed buffers in a loop (launch overhead of
 * the per-level sweeps paid once).  The handles stay busy (rs_free returns RS_EBUSY)
 * until rs_plan_free.  Replays on one plan must not overlap (they share the plan's
 * workspace).  Errors: RS_EINVAL, RS_ENOMEM, RS_EDEVICE. */
typedef struct rs_plan_s *rs_plan;
rs_status rs_plan_create(int32_t count, const rs_handle *h, void *const *B, const int64_t *ldb,
                         const int32_t *nrhs, rs_plan *out);
rs_status rs_plan_launch(rs_plan p, void *stream);
/* Waits for the device, then frees the plan; RS_OK for NULL. */
rs_status rs_plan_free(rs_plan p);

/* ----------------------------------------------------------- autotuner ---- */

/* Times every valid tile width of the solve sweeps of small boxes (16, 32, 64
 * right-hand sides per workgroup; boxes with n <= 512 real, 256 complex -- larger ones
 * go through row-tiled GEMMs with nothing to tune) on handle h's own levels for each
 * nrhs in nrhs_list[count], reps timed repetitions each, and records the fastest width
 * per bucket -- (real/complex, ceil(log2 nrhs), largest box of the launch in steps of
 * 32) -- in a process-wide table that every later solve consults.  A width
 * changes the work distribution only: results are bitwise the same with any table.
 * Synchronous on `stream`.  Errors: RS_EINVAL, RS_EDEVICE. */
rs_status rs_autotune(rs_handle h, const int32_t *nrhs_list, int32_t count, int32_t reps,
                      void *stream);
/* Copies the table (bucket keys and widths, cap entries at most); *count receives its
 * size.  Key bits: 0 MFMA class, 1 complex, 2..7 ceil(log2 nrhs), 8..15 box bucket. */
rs_status rs_tune_entries(uint32_t *keys, int32_t *widths, int32_t cap, int32_t *count);
rs_status rs_tune_clear(void);
/* Text file of "key width" lines; load merges into the current table and rejects
 * widths that do not exist.  Errors: RS_EINVAL (unreadable, malformed). */
rs_status rs_tune_save(const char *path);
rs_status rs_tune_load(const char *path);

/* Factors one problem and solves one block of right-hand sides with the new factors in
 * the same call (Sections 3.4 and 4: the factorization, then the multilevel inverse
 * applied to B in place).  Arguments as rs_factor_ex, plus B: device memory,
 * column-major n x nrhs with leading dimension ldb >= n, scalars of the operator's type
 * (complex128 as interleaved pairs), overwritten with the solution.  The solve's
 * permutation and upward sweeps through the compressed levels run while the root block
 * is inverted; the results are those of rs_factor_ex followed by rs_solve_ex, bit for
 * bit.  Returns when both are complete (errors of either, as those calls report them;
 * on an error no handle is returned and B is unspecified).  The caller owns *out. */
rs_status rs_factor_solve_ex(const rs_kernel *k, rs_tree t, const double *points,
                             const double *weights, double eps, const rs_options *opts,
                             void *B, int64_t ldb, int32_t nrhs, rs_handle *out);

/* Releases a handle.  RS_EBUSY (handle untouched) while a solve enqueued on it has not
 * completed on its stream, or while a call, a plan or the server uses it; synchronize
 * the solve's stream first.  RS_OK for NULL. */
rs_status rs_free(rs_handle h);

/* Thread-local message for the last failed call on this thread ("" if none). */
const char *rs_last_error(void);

/* Number of HIP devices visible to the library (0 if none or the runtime fails). */
int32_t rs_device_count(void);

/* -------------------------------------------------------------- queries ---- */

typedef struct {
  int64_t n;                /* unknowns */
  int64_t nbox;             /* boxes in the tree (root included) */
  int32_t maxdepth;         /* finest depth; compressed depths are maxdepth..1 */
  int32_t dim;
  int64_t root_size;        /* unknowns left at the root (dense block) */
  int64_t total_skeletons;  /* sum of k over all compressed boxes */
  int64_t factor_doubles;   /* doubles stored for the compressed inverse (2 per complex) */
  int64_t max_box_n;        /* largest active set of a box */
  int64_t max_box_m;        /* largest compression block row count */
  double factor_ms;         /* host wall time of the factor call */
  double plan_ms;           /* of which: host planning (active sets, near lists, descriptors) */
  double wait_ms;           /* of which: host blocked waiting for the device */
  int32_t complex_values;   /* 1: complex128 operator and right-hand sides (HELM2D_CFIE) */
  int32_t pad;
} rs_stats;

rs_status rs_query(rs_handle h, rs_stats *out);

/* Per level of a factorization (compressed levels finest first, then the root). */
typedef struct {
  int32_t depth;            /* tree depth (0 = the root) */
  int32_t boxes;            /* boxes factored at this level */
  int64_t n_total;          /* sum over the boxes of the active DOFs n */
  int64_t k_total;          /* sum of the ranks k (skeletons passed to the parent; 0 at the root) */
  int32_t max_n;            /* largest active set */
  int32_t max_m;            /* largest compression block (rows; 0 at the root) */
  int64_t factor_doubles;   /* doubles stored for the level's compressed inverse (2 per complex) */
  double device_ms;         /* compressed levels: device time of the level's compression
                               launches (assembly, sketch, ID; from the first launch to the
                               join of its streams); root: its factorization */
  double plan_ms;           /* host planning time of the level (active sets, near lists,
                               descriptors).  A batched factorization processes the same
                               level step of all its problems together: both times are then
                               those of the step, shared by the problems */
} rs_level_stats;

/* Copies up to cap level records into out (finest level first, the root last) and sets
 * *count to the number of levels.  out may be NULL with cap = 0 to query the count.
 * Errors: RS_EINVAL. */
rs_status rs_query_levels(rs_handle h, rs_level_stats *out, int32_t cap, int32_t *count);

/* Per-box ranks and skeletons (tree positions, ascending per box), for
 * inspection and testing.  k_out[nbox] receives k per box (-1 for boxes with no
 * compression step, i.e. the root); skel_out receives the concatenation of all
 * boxes' skeleton lists in box order and must hold cap entries; *total receives
 * the number written.  RS_EINVAL if cap is too small. */
rs_status rs_box_skeletons(rs_handle h, int32_t *k_out, int64_t *skel_out, int64_t cap,
                           int64_t *total);

/* Copies box b's active set (n tree positions, ascending) and its interpolation
 * matrix T (k x (n-k), column-major; rows follow the sorted skeletons, columns the
 * sorted redundant DOFs) to host arrays.  Either output may be NULL.  n_out/k_out
 * receive the sizes.  The root (b = 0 unless the tree is a single box) reports
 * k = 0 and no T.  For HELM2D_CFIE, T_out receives complex128 entries (2 doubles each). */
rs_status rs_box_export(rs_handle h, int64_t b, int32_t *n_out, int32_t *k_out,
                        int64_t *J_out, double *T_out);

/* -------------------------------------------------------------- serving ---- */

/* A request server: factorizations stay resident in device memory; solve requests
 * (any handle, any nrhs) are batched continuously into shared per-level sweeps, with
 * up to two batches on the device at once on separate streams, so requests that
 * arrive while a batch runs join the next one; factor requests are admitted in
 * arrival order when their estimated device footprint fits the free budget, and run
 * on their own stream concurrently with the solves.  Per-request results are
 * bitwise identical to rs_solve / rs_factor on the same inputs.
 * For callers that keep many factors resident and serve streams of right-hand sides
 * (the regime the paper's fast solve phase targets). */
typedef struct rs_server_s *rs_server;

typedef struct {
  size_t hbm_budget;            /* bytes the server's own factorizations may occupy */
  int32_t max_batch_requests;   /* solve requests per batch (<= 0: 64) */
  int32_t max_batch_rhs;        /* right-hand-side columns per batch (<= 0: 4096) */
} rs_server_opts;

typedef struct {
  int64_t solves_done, rhs_done, factors_done, rejected, batches;
  int64_t resident_bytes;       /* device bytes held by the server's factorizations */
  int64_t queued_solves, queued_factors;
  double p50_ms, p99_ms, mean_ms;  /* solve latency: submission -> completion event */
  double window_ms;             /* first submission -> last completion */
} rs_server_stats;

/* Device footprint of rs_factor(k, t, points, weights, eps) before it runs, from the
 * tree, the kernel and eps only (host computation; no device needed): a rank model
 * (skeletons per box growing with the box's height and the decades of eps, never more
 * than its active set), giving the bytes the handle keeps (*resident) and the bytes the
 * factorization needs besides while it runs (*transient).  The server admits factor
 * requests by resident * c + transient, where c >= 1 is the ratio of kept to predicted
 * bytes of its earlier factorizations of the same kernel and decade of eps.
 * Errors: RS_EINVAL. */
rs_status rs_factor_estimate(const rs_kernel *k, rs_tree t, double eps, size_t *resident,
                             size_t *transient);

/* Creates a server on the current device.  Errors: RS_EINVAL, RS_EDEVICE. */
rs_status rs_server_create(const rs_server_opts *opts, rs_server *out);

/* Queues a factorization (arguments as rs_factor; inputs are copied, so they may be
 * freed on return).  It is admitted when its estimated footprint (rs_factor_estimate,
 * corrected as described there) fits the budget left by the resident factorizations and
 * the admitted ones; a request whose estimate exceeds the whole budget completes at once
 * with RS_ENOMEM.  *ticket identifies the request. */
rs_status rs_server_submit_factor(rs_server s, const rs_kernel *k, rs_tree t,
                                  const double *points, const double *weights, double eps,
                                  uint64_t *ticket);

/* Queues B := A^{-1} B (device memory of the server's device, column-major, ldb >= n,
 * nrhs >= 1; RS_EINVAL for a host pointer or a range past the end of B's allocation).
 * stream (hipStream_t, NULL = default stream) is the producer's stream: the request
 * runs after all work queued on it before this call (an event is recorded on it here),
 * so B may still be being written there.  B must not be touched until the ticket
 * completes; concurrent requests need disjoint B. */
rs_status rs_server_submit_solve(rs_server s, rs_handle h, void *B, int64_t ldb,
                                 int32_t nrhs, void *stream, uint64_t *ticket);

/* Waits up to timeout_ms (0: no wait, < 0: forever) for a ticket.  *done = 1 when it
 * completed; then *status holds its outcome, *factor_out the new handle of a factor
 * request, and the ticket is forgotten.  Handles created by the server are owned by
 * it: release them with rs_server_release (not rs_free); the rest are freed by
 * rs_server_destroy. */
rs_status rs_server_poll(rs_server s, uint64_t ticket, int32_t timeout_ms, int32_t *done,
                         rs_status *status, rs_handle *factor_out);

/* Frees a server-created handle and returns its memory to the budget.  RS_EBUSY if
 * solves on it are queued or running. */
rs_status rs_server_release(rs_server s, rs_handle h);

rs_status rs_server_query(rs_server s, rs_server_stats *out);
rs_status rs_server_reset_stats(rs_server s);

/* Waits for queued and running solves, drops queued factor requests, stops the
 * threads and frees the server's handles. */
void rs_server_destroy(rs_server s);

/* ------------------------------------------------------------ profiling ---- */

/* Kernel families of the library, for rs_profile_read. */
typedef enum {
  RS_K_ASSEMBLE = 0,   /* proxy + near compression block (Section 3.2) */
  RS_K_ID = 1,         /* column-pivoted QR interpolative decomposition (Section 2.2) */
  RS_K_FACTOR = 2,     /* diagonal block + box factorization (Section 3.4) */
  RS_K_SWEEP_UP = 3,   /* upward solve sweep */
  RS_K_SWEEP_DOWN = 4, /* downward solve sweep */
  RS_K_PERMUTE = 5,    /* caller <-> tree order of right-hand sides */
  RS_K_COUNT = 6
} rs_kernel_family;

/* When enabled (process-wide), every kernel launch of the library is bracketed by
 * two HIP events recorded on the launch's own stream, and the algorithmic work of
 * the launch is counted from the box sizes: flops (FP64 operations the algorithm
 * needs; one kernel evaluation counts as one "entry", reported separately) and
 * bytes (the minimum HBM traffic: operands read once, results written once).
 * Enabling adds a host-side event record per launch. */
rs_status rs_profile_enable(int32_t on);

/* Clears all counters (waits for pending events first). */
rs_status rs_profile_reset(void);

/* Accumulated totals of one kernel family since the last reset; waits for the
 * recorded events.  Any output may be NULL. */
rs_status rs_profile_read(int32_t family, int64_t *launches, double *total_ms,
                          double *flops, double *bytes, double *entries);

#ifdef __cplusplus
}
#endif

#endif /* RS_H */
