// Internal data structures shared by the host runtime and the HIP kernels.
// Plain-old-data only: these structs are copied to device memory verbatim.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/rs.h"

namespace rs {

// Per-problem device view: geometry in tree order, structure-of-arrays.
struct ProbDev {
  const double *x[3];      // coordinates, x[a][i]
  const double *nrm[3];    // unit normals (double-layer kernels) or null
  const double *w;         // quadrature weights
  const double *kappa;     // curvature (2D double layer) or null
  int32_t kind;            // rs_kernel_kind
  int32_t dim;
  double c;                // identity coefficient
  int32_t npx;             // proxy points
  int32_t log_kernel;      // 1: append the charge and constant rows
  double eps;              // relative ID precision
  double ratio;            // proxy radius / box side
  double kwave;            // Helmholtz wavenumber
  double eta;              // Helmholtz combined-field coupling
  int32_t id_mode;         // rs_id_mode
  int32_t oversample;      // sketch rows beyond n (RS_ID_SKETCH)
  uint64_t sketch_seed;
};

// One box of one level, for the compression kernels (assembly + ID).
struct CompBox {
  int32_t prob;            // index into the ProbDev table
  int32_t n;               // active DOFs
  int32_t nn;              // near DOFs
  int32_t m;               // rows of M = 2 nn + 2 npx (+2)
  int64_t J_off;           // int32 tree positions in the index pool
  int64_t N_off;           // near tree positions in the index pool
  int64_t M_off;           // scalars, column-major m x n, ld = m
  double cen[3];
  double rho;              // proxy radius
  int64_t order_off;       // ints: out, sorted skeleton then redundant local positions
  int32_t kslot;           // index of this box's rank in the rank array
  int32_t box;             // tree box index (the sketch's counter)
  double *T;               // out: T (k x (n-k)), the head of the box's factor slot
};

// One box of one level for the diagonal-block assembly and box factorization.
struct FacBox {
  int32_t prob;
  int32_t n;
  int32_t kslot;           // rank index (ignored if force_k0)
  int32_t force_k0;        // root: eliminate everything (k = 0)
  int32_t leaf;            // D = A(J, J) with the diagonal rule
  int32_t nchild;
  int64_t J_off;           // tree positions (int32) of the active DOFs (local order)
  int64_t order_off;       // sorted s then r local positions (int32), from the ID
  double *slot;            // T | G | E | F | Lambda (layout below; scalars of the problem)
  int64_t work_off;        // scalars of workspace (n*n)
  int32_t child_lo[8];     // segment of each child in the local order
  int32_t child_k[8];
  const double *child_lam[8];  // Lambda of each child (k_c x k_c, column-major)
};

// One box for the solve sweeps.  Matrix pointers address scalars of the problem's type
// (binary64, or complex128 as re/im pairs).
struct SweepBox {
  int32_t k, r;            // skeleton / redundant counts
  const int32_t *idx;      // k skeleton tree positions, then r redundant ones
  const double *T;         // k x r
  const double *G;         // r x r  (X_rr^{-1})
  const double *E;         // k x r  (X_sr G)
  const double *F;         // r x k  (G X_rs)
};

// One box of one level for the compressed forward operator (rs_matvec).  idx lists the
// box's active DOFs as in SweepBox (k skeletons, then r redundant); save_off is the
// box's first row in the buffer that keeps the level's skeleton values for the
// downward pass.  Children's tree ranges start at child_begin[0..nchild) (ascending):
// above the leaves a DOF belongs to the child whose range holds its tree position.
struct MvBox {
  int32_t k, r;
  const int32_t *idx;
  const double *T;         // k x r, scalars of the problem's type (null when k or r is 0)
  int64_t save_off;
  int32_t prob;
  int32_t leaf;
  int32_t nchild;
  int32_t pad;
  int64_t child_begin[8];
};

// A run of consecutive blocks of a multi-handle sweep launch: boxes[0..count) of one
// handle's level, applied to that handle's workspace W (nrhs columns).
struct SweepSeg {
  const SweepBox *boxes;
  double *W;               // scalars of the handle's type
  int32_t count;
  int32_t nrhs;
  int32_t block0;          // first block of the launch that belongs to this segment
  int32_t pad;
};

// One right-hand-side block of a multi-handle permutation launch.
struct PermSeg {
  double *B;               // caller order, column-major, leading dimension ldb
  int64_t ldb;
  double *W;               // tree order, row-major n x nrhs
  const int64_t *perm;
  int64_t n;
  int32_t nrhs;
  int32_t pad;
};

// Slot layout of a factored box with n = k + r, in scalars (a complex scalar occupies
// two doubles).
__host__ __device__ inline int64_t slot_T(int k, int r) { (void)k; (void)r; return 0; }
__host__ __device__ inline int64_t slot_G(int k, int r) { return (int64_t)k * r; }
__host__ __device__ inline int64_t slot_E(int k, int r) { return (int64_t)k * r + (int64_t)r * r; }
__host__ __device__ inline int64_t slot_F(int k, int r) { return 2 * (int64_t)k * r + (int64_t)r * r; }
__host__ __device__ inline int64_t slot_L(int k, int r) { return 3 * (int64_t)k * r + (int64_t)r * r; }
__host__ __device__ inline int64_t slot_size(int k, int r) {
  return 3 * (int64_t)k * r + (int64_t)r * r + (int64_t)k * k;
}
// Upper bound of slot_size over k + r = n (maximum 5n^2/4 at k = n/2 ... bounded by
// 1.25 n^2 + n for every split).
__host__ __device__ inline int64_t slot_bound(int n) { return (5 * (int64_t)n * n) / 4 + n + 8; }

// ------------------------------------------------------------------ launchers
// All launchers enqueue on `st`; grid = one workgroup per box in [first, first+count).
// `cplx` selects the scalar type of the arrays behind the double pointers: binary64, or
// complex128 (re/im pairs) for the Helmholtz kernel.
// Blocks with more than kThreads * 16 entries are assembled by several workgroups per
// box (assemble_chunks(max_n, max_m) of them; `partials` holds count * chunks doubles);
// smaller ones by one workgroup per box.  The entries are the same either way.
constexpr int kAssembleMaxChunks = 1024;
int assemble_chunks(int max_n, int max_m);
void launch_assemble(bool cplx, const CompBox *boxes, int first, int count, const ProbDev *probs,
                     const int32_t *pool, double *Marena, int max_npx, int max_n, int max_m,
                     double *partials, hipStream_t st);
void launch_cpqr_id(bool cplx, const CompBox *boxes, int first, int count, const ProbDev *probs,
                    double *Marena, int32_t *order_pool, int32_t *ranks, int max_n, int max_m,
                    hipStream_t st);
// Box factorizations (one workgroup per box).  The roots' launches pass no order and no
// ranks (force_k0 boxes).
void launch_diag_factor(bool cplx, const FacBox *boxes, int first, int count,
                        const ProbDev *probs, const int32_t *pool, const int32_t *order_pool,
                        const int32_t *ranks, double *work, int32_t *err, int err_base,
                        int max_n, hipStream_t st);
size_t cpqr_lds_bytes(bool cplx, int max_n, int max_m);
// Small real boxes (n <= kFusedMaxN, m <= kFusedMaxM) are assembled and compressed by one
// fused kernel with the block held in registers; their M_off region holds n x n scalars
// (the first k rows of R).  The class depends on the box alone.
constexpr int kFusedMaxN = 80;
constexpr int kFusedMaxM = 512;
bool fused_class(bool cplx, int n, int m);
// Randomized ID: comp_id[i] is comp[i] with m the sketch's row count and M_off its
// sketch Y (ell x n, column-major, in the same arena); boxes with ell = m are skipped
// (their comp_id entry points at M itself).  max_tiles bounds ceil(ell/16) ceil(n/16).
void launch_sketch(bool cplx, const CompBox *comp, const CompBox *comp_id, int first, int count,
                   const ProbDev *probs, double *Marena, int max_tiles, hipStream_t st);
int fused_variant_of(int n, int m);     // register-resident variant of a launch's largest box
bool fused_small(int n, int m);         // fits the 256-thread variants
void launch_compress_fused(const CompBox *boxes, int first, int count, const ProbDev *probs,
                           const int32_t *pool, int32_t *order_pool, int32_t *ranks, int max_n,
                           int max_m, int max_npx, hipStream_t st);
// Real boxes beyond the fused class up to 832 rows and 112 columns are assembled and
// compressed in the registers of ceil(n / 48) workgroups per box that exchange each pivot
// step's offers through device memory (k_compress_split); same outputs as the fused
// class.
bool split_class(bool cplx, int n, int m);
void launch_compress_split(const CompBox *boxes, int first, int count, const ProbDev *probs,
                           const int32_t *pool, int32_t *order_pool, int32_t *ranks, int max_n,
                           int max_m, int max_npx, hipStream_t st);
// Roots with at least kWideRootMinN unknowns are skipped by k_diag_factor and factored
// by launch_root_wide instead: assembly by many workgroups, then a blocked Gauss-Jordan
// inversion with one launch per panel of 16 pivot steps and one launch of many
// workgroups per rank-16 update.  box: the root's device descriptor; work + work_off:
// its workspace (n^2 + 16 n scalars); G: its slot (n x n inverse); err: the factor's
// error index (err_idx written on a zero or non-finite pivot).
constexpr int kWideRootMinN = 1536;
void launch_root_wide(bool cplx, const FacBox *box, int n, const ProbDev *probs,
                      const int32_t *pool, double *work, int64_t work_off, double *G,
                      int32_t *err, int err_idx, hipStream_t st);
// Real roots of kRegRootMinN .. kGjRegRootMax unknowns are skipped by k_diag_factor too and
// factored by launch_root_regs: assembly by many workgroups into the workspace, then the
// Gauss-Jordan inversion held in the registers of one 512-thread workgroup.  Arguments as
// for launch_root_wide.
constexpr int kRegRootMinN = 65;
constexpr int kGjRegRootMax = 200;
__host__ __device__ constexpr bool root_in_regs(bool cplx, int n) {
  return !cplx && n >= kRegRootMinN && n <= kGjRegRootMax;
}
void launch_root_regs(const FacBox *box, int n, const ProbDev *probs, const int32_t *pool,
                      double *work, int64_t work_off, double *G, int32_t *err, int err_idx,
                      hipStream_t st);
// Global workspace scalars reserved for a box of n DOFs in k_diag_factor.
size_t diag_work_elems(int n);
void launch_permute_in(bool cplx, const double *B, int64_t ldb, double *W, const int64_t *perm,
                       int64_t n, int nrhs, hipStream_t st);
void launch_permute_out(bool cplx, double *B, int64_t ldb, const double *W, const int64_t *perm,
                        int64_t n, int nrhs, hipStream_t st);
void launch_permute_seg(bool cplx, const PermSeg *segs, int nseg, int64_t max_elems,
                        int max_nrhs, bool to_tree, hipStream_t st);
// Boxes with n = k + r <= mfma_max_n are swept with FP64 MFMA tiles, one workgroup per
// box and column tile (any nrhs); larger boxes by the wide path (launch_wide_level), each
// product a row-tiled MFMA GEMM over many workgroups.  The class of a box never depends
// on the launch.
constexpr int kMfmaMaxN = 512;
constexpr int kMfmaMaxNComplex = 256;
int mfma_max_n(bool cplx);
// nt = 0: tile width from the tuning table, else the built-in choice; nt > 0 forces a
// width (used by the autotuner; must be valid for the LDS budget).
void launch_sweep_mfma(bool cplx, bool up, const SweepBox *boxes, int first, int count,
                       double *W, int nrhs, int max_n, hipStream_t st, int nt = 0);
void launch_sweep_seg(bool cplx, bool up, const SweepSeg *segs, int nseg, int nblocks,
                      int max_nrhs, int max_n, hipStream_t st);
// Wide path over count boxes of one level (device descriptors): gathers each box's rows
// of W (nrhs columns) into scratch, then up: t = b_r - T^T b_s, b_r <- G t,
// b_s <- b_s - E t; down: u = y_r - F z, b_r <- u, b_s <- z - T u; one launch per stage
// for all boxes.  max_n, max_k, max_r bound the boxes' n = k + r, k and r.  Boxes are
// processed in chunks whose scratch fits scratch_doubles (at least one box's).
int64_t wide_scratch_doubles(int count, int max_n, int max_r, int nrhs, bool cplx);
void launch_wide_level(bool cplx, bool up, const SweepBox *boxes, int count, int max_n,
                       int max_k, int max_r, double *W, int nrhs, double *scratch,
                       int64_t scratch_doubles, hipStream_t st);

// Compressed forward operator (one launch per kernel per level; grid.x = boxes, grid.y
// = row blocks of 256, grid.z = column tiles of 16).  W, Y, save: tree order, row-major
// (n x nrhs and total-skeletons x nrhs), scalars of the problem's type.
//   up:   save[box rows] <- W[s];  W[s] <- W[s] + T W[r]
//   lift: Y[r] <- T^T Y[s]
//   diag: Y[J] += S_d(J, J) x_J with x_s from save (x_J = W[J] when k = 0)
void launch_mv_up(bool cplx, const MvBox *boxes, int count, int max_k, double *W, int nrhs,
                  double *save, hipStream_t st);
void launch_mv_lift(bool cplx, const MvBox *boxes, int count, int max_r, double *Y, int nrhs,
                    hipStream_t st);
void launch_mv_diag(bool cplx, const MvBox *boxes, int count, int max_n, const ProbDev *probs,
                    const double *W, const double *save, double *Y, int nrhs, hipStream_t st);

// ------------------------------------------------------------------ tuning table
// Tile widths of the MFMA-class sweep kernels per bucket (class flag, scalar size,
// ceil(log2 nrhs), largest box in steps of 32); only MFMA-class keys are valid.  Every width computes each output element with the same
// arithmetic, so a table changes speed only, never results.
bool sweep_nt_valid(bool mfma, int nt, int max_n, int es);
uint32_t tune_key(bool mfma, int es, int nrhs, int max_n);
int tune_lookup(bool mfma, int es, int nrhs, int max_n);
void tune_set(uint32_t key, int nt);
std::vector<std::pair<uint32_t, int>> tune_entries();
void tune_clear();

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);

#define RS_HIP_CHECK(expr)                                                   \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess) throw rs::DeviceError(#expr, e_);                  \
  } while (0)

struct DeviceError {
  std::string what;
  DeviceError(const char *expr, hipError_t e)
      : what(std::string(expr) + ": " + hipGetErrorString(e)) {}
};

struct Status {
  rs_status code;
  std::string msg;
};

}  // namespace rs
