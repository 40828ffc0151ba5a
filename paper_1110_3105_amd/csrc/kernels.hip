// HIP kernels of the recursive-skeletonization factor and solve passes (gfx950).
//
// Every kernel processes one box per workgroup (256 threads = 4 wave64s); a launch
// covers all boxes of one tree level (of every problem of a batch), or a single box
// in the per-box reference mode.  All arithmetic is binary64.
#include <float.h>
#include <limits.h>

#include "rs_internal.h"

namespace rs {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr double kPi = 3.14159265358979323846;
constexpr double kInv2Pi = 0.15915494309189533577;   // 1 / (2 pi)
constexpr double kInv4Pi = 0.07957747154594766788;   // 1 / (4 pi)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Green's function K(t, s) with the unit normal ns at the source (double layer):
// eqs. (2d-laplace), (3d-laplace) and the double-layer kernel of eq. (double-layer).
__device__ __forceinline__ double green(int kind, const double *t, const double *s,
                                        const double *ns) {
  const double dx = t[0] - s[0], dy = t[1] - s[1];
  if (kind == RS_LAP2D_SL) {
    return -0.5 * kInv2Pi * log(dx * dx + dy * dy);
  } else if (kind == RS_LAP2D_DL) {
    return (dx * ns[0] + dy * ns[1]) * kInv2Pi / (dx * dx + dy * dy);
  } else {
    const double dz = t[2] - s[2];
    return kInv4Pi / sqrt(dx * dx + dy * dy + dz * dz);
  }
}

__device__ __forceinline__ void load_pt(const ProbDev &P, int g, double *x) {
  x[0] = P.x[0][g];
  x[1] = P.x[1][g];
  x[2] = P.dim == 3 ? P.x[2][g] : 0.0;
}

__device__ __forceinline__ void load_nrm(const ProbDev &P, int g, double *nv) {
  if (P.nrm[0]) {
    nv[0] = P.nrm[0][g];
    nv[1] = P.nrm[1][g];
    nv[2] = P.dim == 3 ? P.nrm[2][g] : 0.0;
  } else {
    nv[0] = nv[1] = nv[2] = 0.0;
  }
}

// Diagonal entry A_ii: identity coefficient plus the kernel's diagonal rule.
__device__ __forceinline__ double diag_entry(const ProbDev &P, int g) {
  const double w = P.w[g];
  double d;
  if (P.kind == RS_LAP2D_SL) {
    d = -(w * kInv2Pi) * log(w * kInv2Pi);
  } else if (P.kind == RS_LAP2D_DL) {
    d = -P.kappa[g] * w * (0.25 / kPi);
  } else {
    d = 0.5 * sqrt(w / kPi);
  }
  return P.c + d;
}

// A(gi, gj) = c delta + K(x_gi, x_gj) w_gj.
__device__ __forceinline__ double entry(const ProbDev &P, int gi, int gj) {
  if (gi == gj) return diag_entry(P, gi);
  double t[3], s[3], ns[3];
  load_pt(P, gi, t);
  load_pt(P, gj, s);
  load_nrm(P, gj, ns);
  return green(P.kind, t, s, ns) * P.w[gj];
}

__device__ __forceinline__ void proxy_unit(int dim, int p, int npx, double *u) {
  if (dim == 2) {
    double sn, cs;
    sincos(2.0 * kPi * (double)p / (double)npx, &sn, &cs);
    u[0] = cs;
    u[1] = sn;
    u[2] = 0.0;
  } else {
    const double z = 1.0 - (2.0 * p + 1.0) / (double)npx;
    const double rr = sqrt(fmax(0.0, 1.0 - z * z));
    double sn, cs;
    sincos((double)p * (kPi * (3.0 - sqrt(5.0))), &sn, &cs);
    u[0] = rr * cs;
    u[1] = rr * sn;
    u[2] = z;
  }
}

__device__ double block_max(double v, double *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_max(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double r = red[0];
  for (int i = 1; i < kWaves; ++i) r = fmax(r, red[i]);
  __syncthreads();
  return r;
}

// --------------------------------------------------------------------------
// Compression block M_B (Section 3.2), column-major m x n:
//   rows [0, nn)            near DOFs as targets      A(N, J)
//   rows [nn, 2nn)          near DOFs as sources      A(J, N)^T
//   rows [2nn, 2nn+np)      proxies as targets        K(Gamma, J) W_J
//   rows [2nn+np, 2nn+2np)  proxies as sources        (K(J, Gamma) W_Gamma)^T
//   rows m-2, m-1 (log kernels): total charge and constant field, scaled to the
//                           largest proxy entry.
__global__ __launch_bounds__(kThreads) void k_assemble(const CompBox *__restrict__ boxes,
                                                       int first,
                                                       const ProbDev *__restrict__ probs,
                                                       const int32_t *__restrict__ pool,
                                                       double *__restrict__ Marena) {
  extern __shared__ double sh_u[];   // npx * 3 proxy unit vectors
  __shared__ double red[kWaves];
  const CompBox &B = boxes[first + blockIdx.x];
  const ProbDev &P = probs[B.prob];
  const int n = B.n, nn = B.nn, m = B.m, npx = P.npx, dim = P.dim;
  if (n == 0) return;
  const int32_t *J = pool + B.J_off;
  const int32_t *N = pool + B.N_off;
  double *M = Marena + B.M_off;
  for (int p = threadIdx.x; p < npx; p += kThreads) proxy_unit(dim, p, npx, sh_u + 3 * p);
  double wmax = 0.0;
  for (int j = threadIdx.x; j < n; j += kThreads) wmax = fmax(wmax, P.w[J[j]]);
  wmax = block_max(wmax, red);   // includes a barrier: proxy vectors are visible
  const double wG = dim == 2 ? 2.0 * kPi * B.rho / npx : 4.0 * kPi * B.rho * B.rho / npx;
  const int rows = 2 * nn + 2 * npx;
  double pmax = 0.0;
  const int64_t total = (int64_t)rows * n;
  for (int64_t e = threadIdx.x; e < total; e += kThreads) {
    const int j = (int)(e / rows), i = (int)(e - (int64_t)j * rows);
    const int g = J[j];
    double xs[3], ns[3], v;
    load_pt(P, g, xs);
    if (i < nn) {
      double xq[3];
      load_nrm(P, g, ns);
      load_pt(P, N[i], xq);
      v = green(P.kind, xq, xs, ns) * P.w[g];
    } else if (i < 2 * nn) {
      const int q = N[i - nn];
      double xq[3], nq[3];
      load_pt(P, q, xq);
      load_nrm(P, q, nq);
      v = green(P.kind, xs, xq, nq) * P.w[q];
    } else if (i < 2 * nn + npx) {
      const double *u = sh_u + 3 * (i - 2 * nn);
      double y[3] = {B.cen[0] + B.rho * u[0], B.cen[1] + B.rho * u[1], B.cen[2] + B.rho * u[2]};
      load_nrm(P, g, ns);
      v = green(P.kind, y, xs, ns) * P.w[g];
      pmax = fmax(pmax, fabs(v));
    } else {
      const double *u = sh_u + 3 * (i - 2 * nn - npx);
      double y[3] = {B.cen[0] + B.rho * u[0], B.cen[1] + B.rho * u[1], B.cen[2] + B.rho * u[2]};
      v = green(P.kind, xs, y, u) * wG;
      pmax = fmax(pmax, fabs(v));
    }
    M[(int64_t)j * m + i] = v;
  }
  if (P.log_kernel) {
    pmax = block_max(pmax, red);
    for (int j = threadIdx.x; j < n; j += kThreads) {
      M[(int64_t)j * m + rows] = pmax * P.w[J[j]] / wmax;
      M[(int64_t)j * m + rows + 1] = pmax;
    }
  }
}

// --------------------------------------------------------------------------
// Interpolative decomposition (Section 2.2) of M_B by column-pivoted Householder QR:
// pivot = largest remaining column norm (recomputed after every reflection, ties to
// the lowest original column), stop at the first |R_jj| <= eps |R_00|, then
// T = R11^{-1} R12 and the skeleton / redundant sets sorted ascending.
// Outputs: ranks[kslot] = k, order (n ints: sorted s, then sorted r), T (k x (n-k)).
//
// Trailing update: each wave takes CB columns at a time; a lane holds up to RT rows of
// each of them in registers, so one step reads and writes the trailing matrix once
// (dot product with the reflector, update, and the recomputed norm in one pass).  The
// reflector is staged in LDS when VLDS.  Rows beyond 64*RT are streamed in two passes.
template <int NTH, int RT, int CB, bool VLDS>
__global__ __launch_bounds__(NTH) void k_cpqr_id(const CompBox *__restrict__ boxes, int first,
                                                 const ProbDev *__restrict__ probs,
                                                 double *__restrict__ Marena,
                                                 int32_t *__restrict__ order_pool,
                                                 int32_t *__restrict__ ranks) {
  constexpr int NW = NTH / 64;
  extern __shared__ double smem[];
  __shared__ double s_best, s_tau;
  __shared__ int s_p;
  const CompBox &B = boxes[first + blockIdx.x];
  const int m = B.m, n = B.n;
  const double eps = probs[B.prob].eps;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (n == 0) {
    if (threadIdx.x == 0) ranks[B.kslot] = 0;
    return;
  }
  double *M = Marena + B.M_off;
  const int kmax = min(m, n);
  double *norms = smem;                                    // n
  int *perm = reinterpret_cast<int *>(norms + n);          // n
  int *rk = perm + n;                                      // n
  double *wbuf = reinterpret_cast<double *>(rk + n);       // NW * kmax (16n bytes in)
  double *sv = wbuf + NW * kmax;                           // m (VLDS only)

  for (int c = threadIdx.x; c < n; c += NTH) perm[c] = c;
  for (int c = wave; c < n; c += NW) {
    const double *col = M + (int64_t)c * m;
    double s = 0.0;
    for (int i = lane; i < m; i += 64) s += col[i] * col[i];
    s = wave_sum(s);
    if (lane == 0) norms[c] = sqrt(s);
  }
  __syncthreads();

  int k = kmax;
  double r00 = 0.0;
  for (int j = 0; j < kmax; ++j) {
    if (wave == 0) {
      double best = -1.0;
      int bperm = INT_MAX, bc = -1;
      for (int c = j + lane; c < n; c += 64) {
        const double v = norms[c];
        const int pc = perm[c];
        if (v > best || (v == best && pc < bperm)) { best = v; bperm = pc; bc = c; }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int op = __shfl_xor(bperm, off, 64);
        const int oc = __shfl_xor(bc, off, 64);
        if (ob > best || (ob == best && op < bperm)) { best = ob; bperm = op; bc = oc; }
      }
      if (lane == 0) { s_best = best; s_p = bc; }
    }
    __syncthreads();
    const double best = s_best;
    const int p = s_p;
    if (j == 0) r00 = best;
    if (best == 0.0 || best <= eps * r00) { k = j; break; }
    if (p != j) {
      double *cj = M + (int64_t)j * m, *cp = M + (int64_t)p * m;
      for (int i = threadIdx.x; i < m; i += NTH) {
        const double a = cj[i];
        cj[i] = cp[i];
        cp[i] = a;
      }
      if (threadIdx.x == 0) {
        const double t = norms[j]; norms[j] = norms[p]; norms[p] = t;
        const int q = perm[j]; perm[j] = perm[p]; perm[p] = q;
      }
    }
    __syncthreads();
    if (wave == 0) {   // Householder reflector of column j, rows j..m-1
      double *cj = M + (int64_t)j * m;
      double s = 0.0;
      for (int i = j + lane; i < m; i += 64) s += cj[i] * cj[i];
      s = wave_sum(s);
      const double alpha = sqrt(s);
      const double x0 = cj[j];
      const double beta = x0 >= 0.0 ? -alpha : alpha;
      const double scale = 1.0 / (x0 - beta);
      for (int i = j + 1 + lane; i < m; i += 64) {
        const double v = cj[i] * scale;
        cj[i] = v;
        if (VLDS) sv[i] = v;
      }
      if (lane == 0) {
        s_tau = (beta - x0) / beta;
        cj[j] = beta;
        if (VLDS) sv[j] = 1.0;
      }
    }
    __syncthreads();
    const double tau = s_tau;
    const double *vg = M + (int64_t)j * m;
    auto vload = [&](int i) -> double { return i == j ? 1.0 : (VLDS ? sv[i] : vg[i]); };
    const int rows = m - j;
    for (int c0 = j + 1 + wave * CB; c0 < n; c0 += NW * CB) {
      double dot[CB], nrm[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) { dot[cb] = 0.0; nrm[cb] = 0.0; }
      if (rows <= 64 * RT) {
        double val[CB][RT], vi[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          const int i = j + lane + 64 * t;
          const bool ok = i < m;
          vi[t] = ok ? vload(i) : 0.0;
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
            const int c = c0 + cb;
            val[cb][t] = (ok && c < n) ? M[(int64_t)c * m + i] : 0.0;
            dot[cb] += vi[t] * val[cb][t];
          }
        }
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) dot[cb] = wave_sum(dot[cb]) * tau;
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          const int i = j + lane + 64 * t;
          if (i < m) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
              const int c = c0 + cb;
              if (c < n) {
                const double nv = val[cb][t] - dot[cb] * vi[t];
                M[(int64_t)c * m + i] = nv;
                if (i > j) nrm[cb] += nv * nv;
              }
            }
          }
        }
      } else {
        for (int base = j; base < m; base += 64 * RT) {
#pragma unroll
          for (int t = 0; t < RT; ++t) {
            const int i = base + lane + 64 * t;
            if (i < m) {
              const double v = vload(i);
#pragma unroll
              for (int cb = 0; cb < CB; ++cb) {
                const int c = c0 + cb;
                if (c < n) dot[cb] += v * M[(int64_t)c * m + i];
              }
            }
          }
        }
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) dot[cb] = wave_sum(dot[cb]) * tau;
        for (int base = j; base < m; base += 64 * RT) {
#pragma unroll
          for (int t = 0; t < RT; ++t) {
            const int i = base + lane + 64 * t;
            if (i < m) {
              const double v = vload(i);
#pragma unroll
              for (int cb = 0; cb < CB; ++cb) {
                const int c = c0 + cb;
                if (c < n) {
                  double *pc = M + (int64_t)c * m + i;
                  const double nv = *pc - dot[cb] * v;
                  *pc = nv;
                  if (i > j) nrm[cb] += nv * nv;
                }
              }
            }
          }
        }
      }
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const double s = wave_sum(nrm[cb]);
        if (lane == 0 && c0 + cb < n) norms[c0 + cb] = sqrt(s);
      }
    }
    __syncthreads();
  }

  // T = R11^{-1} R12, one column per wave, column held in the wave's LDS buffer.
  double *buf = wbuf + wave * kmax;
  for (int c = k + wave; c < n; c += NW) {
    double *col = M + (int64_t)c * m;
    for (int i = lane; i < k; i += 64) buf[i] = col[i];
    for (int i = k - 1; i >= 0; --i) {
      const double xi = buf[i] / M[(int64_t)i * m + i];
      const double *ri = M + (int64_t)i * m;
      for (int l = lane; l < i; l += 64) buf[l] -= xi * ri[l];
      if (lane == 0) buf[i] = xi;
    }
    for (int i = lane; i < k; i += 64) col[i] = buf[i];
  }
  // Sorted skeleton and redundant sets.
  int32_t *order = order_pool + B.order_off;
  for (int c = threadIdx.x; c < n; c += NTH) {
    const int pc = perm[c];
    const int lo = c < k ? 0 : k, hi = c < k ? k : n;
    int r = 0;
    for (int c2 = lo; c2 < hi; ++c2) r += perm[c2] < pc;
    rk[c] = r;
    order[lo + r] = pc;
  }
  __syncthreads();
  double *T = B.T;
  for (int c = k + wave; c < n; c += NW) {
    const double *col = M + (int64_t)c * m;
    double *Tc = T + (int64_t)k * rk[c];
    for (int i = lane; i < k; i += 64) Tc[rk[i]] = col[i];
  }
  if (threadIdx.x == 0) ranks[B.kslot] = k;

}

// --------------------------------------------------------------------------
// Diagonal block and box factorization (Section 3.4 in Schur form).
// With the box's DOFs ordered (s, r), X = P D Q where P = [[I, 0], [-T^T, I]] and
// Q = [[I, -T], [0, I]] remove the skeleton-interpolated part; then
//   G = X_rr^{-1},  F = G X_rs,  E = X_sr G,  Lambda = X_ss - X_sr F,
// and Lambda = (R D^{-1} L)^{-1} is the box's block of the next level's matrix.
// D is A(J, J) at a leaf; above, Lambda of each child on its diagonal block and
// A between siblings.  The root (force_k0) eliminates everything: G = D^{-1}.
// X_rr is inverted in place by Gauss-Jordan elimination with partial pivoting (row
// interchanges, undone as column interchanges at the end).  INLDS: the whole n x n
// block lives in LDS (small boxes); otherwise in the global workspace.
// Index loops are two-level (waves over columns, lanes over rows): no integer division.
template <int NTH, bool INLDS>
__global__ __launch_bounds__(NTH) void k_diag_factor(const FacBox *__restrict__ boxes, int first,
                                                     const ProbDev *__restrict__ probs,
                                                     const int32_t *__restrict__ pool,
                                                     const int32_t *__restrict__ order_pool,
                                                     const int32_t *__restrict__ ranks,
                                                     double *__restrict__ workbase,
                                                     int32_t *__restrict__ err, int err_base) {
  constexpr int NW = NTH / 64;
  constexpr int CB = 4;    // columns per wave in the elimination
  constexpr int RB = 4;    // rows per lane per chunk in the elimination
  extern __shared__ double sh[];
  __shared__ double s_inv;
  __shared__ int s_prow, s_bad;
  const FacBox &B = boxes[first + blockIdx.x];
  const ProbDev &P = probs[B.prob];
  const int n = B.n;
  if (n == 0) return;
  const int k = B.force_k0 ? 0 : ranks[B.kslot];
  const int r = n - k;
  const int32_t *J = pool + B.J_off;
  const int32_t *ord = B.force_k0 ? nullptr : order_pool + B.order_off;
  double *slot = B.slot;
  const double *T = slot + slot_T(k, r);
  double *X = INLDS ? sh : workbase + B.work_off;            // n x n, (s, r) order
  double *fac = INLDS ? sh + (int64_t)n * n : sh;            // r
  int *ipiv = reinterpret_cast<int *>(fac + r);              // r
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  // D in (s, r) order.
  for (int b = wave; b < n; b += NW) {
    const int lj = ord ? ord[b] : b;
    int cb = 0;
    if (!B.leaf)
      for (int c = 1; c < B.nchild; ++c) cb += lj >= B.child_lo[c];
    double *Xb = X + (int64_t)b * n;
    for (int a = lane; a < n; a += 64) {
      const int li = ord ? ord[a] : a;
      double v;
      if (B.leaf) {
        v = entry(P, J[li], J[lj]);
      } else {
        int ca = 0;
        for (int c = 1; c < B.nchild; ++c) ca += li >= B.child_lo[c];
        if (ca == cb) {
          v = B.child_lam[ca][(li - B.child_lo[ca]) +
                              (int64_t)B.child_k[ca] * (lj - B.child_lo[ca])];
        } else {
          v = entry(P, J[li], J[lj]);
        }
      }
      Xb[a] = v;
    }
  }
  __syncthreads();
  if (k > 0 && r > 0) {
    // Y = D Q: redundant columns minus the skeleton columns times T.
    for (int jr = wave; jr < r; jr += NW) {
      const double *Tj = T + (int64_t)k * jr;
      double *Xc = X + (int64_t)(k + jr) * n;
      for (int a = lane; a < n; a += 64) {
        double s = Xc[a];
        for (int i = 0; i < k; ++i) s -= X[(int64_t)i * n + a] * Tj[i];
        Xc[a] = s;
      }
    }
    __syncthreads();
    // X = P Y: redundant rows minus T^T times the skeleton rows.
    for (int b = wave; b < n; b += NW) {
      double *Xb = X + (int64_t)b * n;
      for (int jr = lane; jr < r; jr += 64) {
        const double *Tj = T + (int64_t)k * jr;
        double s = Xb[k + jr];
        for (int i = 0; i < k; ++i) s -= Tj[i] * Xb[i];
        Xb[k + jr] = s;
      }
    }
    __syncthreads();
  }
  // In-place Gauss-Jordan inversion of A = X_rr, A(i, c) = X[(k + c) n + k + i].
  double *A = X + (int64_t)k * n + k;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();      // every thread reads s_bad below, also when r == 0
  for (int j = 0; j < r; ++j) {
    if (wave == 0) {
      double best = -1.0;
      int brow = INT_MAX;
      const double *Aj = A + (int64_t)j * n;
      for (int i = j + lane; i < r; i += 64) {
        const double v = fabs(Aj[i]);
        if (v > best || (v == best && i < brow)) { best = v; brow = i; }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int orow = __shfl_xor(brow, off, 64);
        if (ob > best || (ob == best && orow < brow)) { best = ob; brow = orow; }
      }
      if (lane == 0) {
        s_prow = brow;
        ipiv[j] = brow;
        if (!(best > 0.0) || !isfinite(best)) s_bad = 1;
      }
    }
    __syncthreads();
    if (s_bad) break;
    const int pr = s_prow;
    if (pr != j) {
      for (int c = threadIdx.x; c < r; c += NTH) {
        double *Ac = A + (int64_t)c * n;
        const double a = Ac[j];
        Ac[j] = Ac[pr];
        Ac[pr] = a;
      }
      __syncthreads();
    }
    {
      const double *Aj = A + (int64_t)j * n;
      for (int i = threadIdx.x; i < r; i += NTH) fac[i] = Aj[i];
      if (threadIdx.x == 0) s_inv = 1.0 / Aj[j];
    }
    __syncthreads();
    const double inv = s_inv;
    for (int c = threadIdx.x; c < r; c += NTH) {
      double *Ac = A + (int64_t)c * n;
      Ac[j] = c == j ? inv : Ac[j] * inv;
    }
    __syncthreads();
    // A(i, c) <- [c != j] A(i, c) - fac[i] A(j, c) for i != j.  All loads of a chunk of
    // RB rows x CB columns are issued before its stores, so they overlap in flight.
    for (int c0 = wave * CB; c0 < r; c0 += NW * CB) {
      double aj[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) aj[cb] = c0 + cb < r ? A[(int64_t)(c0 + cb) * n + j] : 0.0;
      for (int i0 = 0; i0 < r; i0 += 64 * RB) {
        double v[RB][CB], f[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const int i = i0 + lane + 64 * rb;
          const bool ok = i < r && i != j;
          f[rb] = ok ? fac[i] : 0.0;
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
            v[rb][cb] = (ok && c0 + cb < r && c0 + cb != j) ? A[(int64_t)(c0 + cb) * n + i] : 0.0;
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const int i = i0 + lane + 64 * rb;
          if (i < r && i != j) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
              if (c0 + cb < r) A[(int64_t)(c0 + cb) * n + i] = v[rb][cb] - f[rb] * aj[cb];
          }
        }
      }
    }
    __syncthreads();
  }
  if (s_bad) {
    if (threadIdx.x == 0) atomicMin(reinterpret_cast<unsigned int *>(err),
                                    (unsigned int)(err_base + first + (int)blockIdx.x));
    return;
  }
  for (int j = r - 1; j >= 0; --j) {      // undo the row interchanges on the columns
    const int pr = ipiv[j];
    if (pr != j) {
      double *Aj = A + (int64_t)j * n, *Ap = A + (int64_t)pr * n;
      for (int i = threadIdx.x; i < r; i += NTH) {
        const double a = Aj[i];
        Aj[i] = Ap[i];
        Ap[i] = a;
      }
      __syncthreads();
    }
  }
  double *G = slot + slot_G(k, r);
  for (int c = wave; c < r; c += NW)
    for (int a = lane; a < r; a += 64) G[(int64_t)c * r + a] = A[(int64_t)c * n + a];
  if (k == 0) return;
  double *E = slot + slot_E(k, r);
  double *F = slot + slot_F(k, r);
  double *L = slot + slot_L(k, r);
  // F = G X_rs (r x k); X_rs(l, i) = X[i n + k + l]
  for (int i = wave; i < k; i += NW) {
    const double *Xi = X + (int64_t)i * n + k;
    for (int a = lane; a < r; a += 64) {
      double s = 0.0;
      for (int l = 0; l < r; ++l) s += A[(int64_t)l * n + a] * Xi[l];
      F[(int64_t)i * r + a] = s;
    }
  }
  // E = X_sr G (k x r); X_sr(i, l) = X[(k + l) n + i]
  for (int a = wave; a < r; a += NW) {
    const double *Ga = A + (int64_t)a * n;
    for (int i = lane; i < k; i += 64) {
      double s = 0.0;
      for (int l = 0; l < r; ++l) s += X[(int64_t)(k + l) * n + i] * Ga[l];
      E[(int64_t)a * k + i] = s;
    }
  }
  __syncthreads();
  // Lambda = X_ss - X_sr F (k x k)
  for (int i2 = wave; i2 < k; i2 += NW) {
    const double *Fi = F + (int64_t)i2 * r;
    for (int i = lane; i < k; i += 64) {
      double s = X[(int64_t)i2 * n + i];
      for (int a = 0; a < r; ++a) s -= X[(int64_t)(k + a) * n + i] * Fi[a];
      L[(int64_t)i2 * k + i] = s;
    }
  }
}

// --------------------------------------------------------------------------
// Solve sweeps.  W is the tree-ordered right-hand side / solution, row-major
// (n x nrhs): the values of DOF g are W[g*nrhs .. g*nrhs+nrhs).  A box reads and
// writes only its own DOFs; a parent reads its children's skeleton outputs in place.
//
// Up (finest level first):  t = b_r - T^T b_s;  b_r <- G t;  b_s <- b_s - E t.
// Down (root side first):   u = y_r - F z_s;   b_r <- u;     b_s <- z_s - T u.
template <int NT>
__device__ __forceinline__ void sweep_up_box(const SweepBox &B, double *__restrict__ W, int nrhs,
                                             int col0, double *sh) {
  const int k = B.k, r = B.r;
  const int nt = min(NT, nrhs - col0);
  double *bs = sh;              // k x NT
  double *t = sh + k * NT;      // r x NT
  const int32_t *idx = B.idx;
  for (int e = threadIdx.x; e < k * NT; e += kThreads) {
    const int i = e / NT, c = e - i * NT;
    bs[e] = c < nt ? W[(int64_t)idx[i] * nrhs + col0 + c] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < r * NT; e += kThreads) {
    const int j = e / NT, c = e - j * NT;
    double s = c < nt ? W[(int64_t)idx[k + j] * nrhs + col0 + c] : 0.0;
    const double *Tj = B.T + (int64_t)k * j;
    for (int i = 0; i < k; ++i) s -= Tj[i] * bs[i * NT + c];
    t[e] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < r * NT; e += kThreads) {
    const int j = e / NT, c = e - j * NT;
    double s = 0.0;
    for (int l = 0; l < r; ++l) s += B.G[j + (int64_t)r * l] * t[l * NT + c];
    if (c < nt) W[(int64_t)idx[k + j] * nrhs + col0 + c] = s;
  }
  for (int e = threadIdx.x; e < k * NT; e += kThreads) {
    const int i = e / NT, c = e - i * NT;
    double s = bs[e];
    for (int l = 0; l < r; ++l) s -= B.E[i + (int64_t)k * l] * t[l * NT + c];
    if (c < nt) W[(int64_t)idx[i] * nrhs + col0 + c] = s;
  }
}

template <int NT>
__device__ __forceinline__ void sweep_down_box(const SweepBox &B, double *__restrict__ W,
                                               int nrhs, int col0, double *sh) {
  const int k = B.k, r = B.r;
  const int nt = min(NT, nrhs - col0);
  double *z = sh;              // k x NT
  double *u = sh + k * NT;     // r x NT
  const int32_t *idx = B.idx;
  for (int e = threadIdx.x; e < k * NT; e += kThreads) {
    const int i = e / NT, c = e - i * NT;
    z[e] = c < nt ? W[(int64_t)idx[i] * nrhs + col0 + c] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < r * NT; e += kThreads) {
    const int j = e / NT, c = e - j * NT;
    double s = c < nt ? W[(int64_t)idx[k + j] * nrhs + col0 + c] : 0.0;
    for (int i = 0; i < k; ++i) s -= B.F[j + (int64_t)r * i] * z[i * NT + c];
    u[e] = s;
    if (c < nt) W[(int64_t)idx[k + j] * nrhs + col0 + c] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < k * NT; e += kThreads) {
    const int i = e / NT, c = e - i * NT;
    double s = z[e];
    for (int j = 0; j < r; ++j) s -= B.T[i + (int64_t)k * j] * u[j * NT + c];
    if (c < nt) W[(int64_t)idx[i] * nrhs + col0 + c] = s;
  }
}

template <int NT>
__global__ __launch_bounds__(kThreads) void k_sweep_up(const SweepBox *__restrict__ boxes,
                                                       int first, double *__restrict__ W,
                                                       int nrhs) {
  extern __shared__ double sh[];
  const SweepBox &B = boxes[first + blockIdx.x];
  if (B.r == 0) return;
  sweep_up_box<NT>(B, W, nrhs, blockIdx.y * NT, sh);
}

template <int NT>
__global__ __launch_bounds__(kThreads) void k_sweep_down(const SweepBox *__restrict__ boxes,
                                                         int first, double *__restrict__ W,
                                                         int nrhs) {
  extern __shared__ double sh[];
  const SweepBox &B = boxes[first + blockIdx.x];
  if (B.r == 0 || B.k == 0) return;
  sweep_down_box<NT>(B, W, nrhs, blockIdx.y * NT, sh);
}

// ---- FP64 MFMA variants of the sweeps (boxes with n <= kMfmaMaxN) -----------------
// v_mfma_f64_16x16x4f64 (wave64): lane l supplies A[l & 15][l >> 4] and
// B[l >> 4][l & 15]; element v of its result holds D[(l >> 4) + 4 v][l & 15].
// Every 16 x 16 output tile is produced by one wave with the full K loop, so the
// arithmetic of a column does not depend on how many columns share the launch.
typedef double dbl4 __attribute__((ext_vector_type(4)));

// acc += A(r0 + i, kk) * Bs(kk, c0 + j) over kk in [0, K); A(i, kk) = a(i, kk) for
// i < M (zero beyond), Bs row-major with leading dimension ldb (LDS).
template <class AF>
__device__ __forceinline__ dbl4 tile_gemm(AF a, const double *Bs, int ldb, int K, int M, int r0,
                                          int c0) {
  const int lane = threadIdx.x & 63, i = lane & 15, kq = lane >> 4;
  dbl4 acc = {0.0, 0.0, 0.0, 0.0};
  const bool rowok = r0 + i < M;
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int kk = k0 + kq;
    const bool kok = kk < K;
    const double av = (rowok && kok) ? a(r0 + i, kk) : 0.0;
    const double bv = kok ? Bs[kk * ldb + c0 + i] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
  }
  return acc;
}

template <int NT>
__device__ __forceinline__ void sweep_up_box_mfma(const SweepBox &B, double *__restrict__ W,
                                                  int nrhs, int col0, double *sh) {
  constexpr int TN = NT / 16;
  const int k = B.k, r = B.r;
  const int nt = min(NT, nrhs - col0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, kq = lane >> 4, cj = lane & 15;
  double *bs = sh;              // k x NT
  double *t = sh + k * NT;      // r x NT
  const int32_t *idx = B.idx;
  for (int e = threadIdx.x; e < (k + r) * NT; e += kThreads) {
    const int i = e / NT, c = e - i * NT;
    sh[e] = c < nt ? W[(int64_t)idx[i] * nrhs + col0 + c] : 0.0;
  }
  __syncthreads();
  const double *T = B.T;
  const int tm_r = (r + 15) >> 4, tm_k = (k + 15) >> 4;
  if (k > 0) {   // t = b_r - T^T b_s
    for (int tile = wave; tile < tm_r * TN; tile += kWaves) {
      const int tm = tile / TN, tn = tile - tm * TN;
      const dbl4 acc = tile_gemm([&](int i, int kk) { return T[kk + (int64_t)k * i]; }, bs, NT,
                                 k, r, tm * 16, tn * 16);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = tm * 16 + kq + 4 * v;
        if (row < r) t[row * NT + tn * 16 + cj] -= acc[v];
      }
    }
    __syncthreads();
  }
  const double *G = B.G;
  for (int tile = wave; tile < tm_r * TN; tile += kWaves) {   // b_r <- G t
    const int tm = tile / TN, tn = tile - tm * TN;
    const dbl4 acc = tile_gemm([&](int i, int l) { return G[i + (int64_t)r * l]; }, t, NT, r, r,
                               tm * 16, tn * 16);
    const int c = tn * 16 + cj;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = tm * 16 + kq + 4 * v;
      if (row < r && c < nt) W[(int64_t)idx[k + row] * nrhs + col0 + c] = acc[v];
    }
  }
  const double *E = B.E;
  for (int tile = wave; tile < tm_k * TN; tile += kWaves) {   // b_s <- b_s - E t
    const int tm = tile / TN, tn = tile - tm * TN;
    const dbl4 acc = tile_gemm([&](int i, int l) { return E[i + (int64_t)k * l]; }, t, NT, r, k,
                               tm * 16, tn * 16);
    const int c = tn * 16 + cj;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = tm * 16 + kq + 4 * v;
      if (row < k && c < nt) W[(int64_t)idx[row] * nrhs + col0 + c] = bs[row * NT + c] - acc[v];
    }
  }
}

template <int NT>
__device__ __forceinline__ void sweep_down_box_mfma(const SweepBox &B, double *__restrict__ W,
                                                    int nrhs, int col0, double *sh) {
  constexpr int TN = NT / 16;
  const int k = B.k, r = B.r;
  const int nt = min(NT, nrhs - col0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, kq = lane >> 4, cj = lane & 15;
  double *z = sh;              // k x NT
  double *u = sh + k * NT;     // r x NT
  const int32_t *idx = B.idx;
  for (int e = threadIdx.x; e < (k + r) * NT; e += kThreads) {
    const int i = e / NT, c = e - i * NT;
    sh[e] = c < nt ? W[(int64_t)idx[i] * nrhs + col0 + c] : 0.0;
  }
  __syncthreads();
  const int tm_r = (r + 15) >> 4, tm_k = (k + 15) >> 4;
  const double *F = B.F;
  for (int tile = wave; tile < tm_r * TN; tile += kWaves) {   // u = y_r - F z
    const int tm = tile / TN, tn = tile - tm * TN;
    const dbl4 acc = tile_gemm([&](int j, int i) { return F[j + (int64_t)r * i]; }, z, NT, k, r,
                               tm * 16, tn * 16);
    const int c = tn * 16 + cj;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = tm * 16 + kq + 4 * v;
      if (row < r) {
        const double val = u[row * NT + c] - acc[v];
        u[row * NT + c] = val;
        if (c < nt) W[(int64_t)idx[k + row] * nrhs + col0 + c] = val;
      }
    }
  }
  __syncthreads();
  const double *T = B.T;
  for (int tile = wave; tile < tm_k * TN; tile += kWaves) {   // x_s = z - T u
    const int tm = tile / TN, tn = tile - tm * TN;
    const dbl4 acc = tile_gemm([&](int i, int j) { return T[i + (int64_t)k * j]; }, u, NT, r, k,
                               tm * 16, tn * 16);
    const int c = tn * 16 + cj;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = tm * 16 + kq + 4 * v;
      if (row < k && c < nt) W[(int64_t)idx[row] * nrhs + col0 + c] = z[row * NT + c] - acc[v];
    }
  }
}

template <int NT>
__global__ __launch_bounds__(kThreads) void k_sweep_up_mfma(const SweepBox *__restrict__ boxes,
                                                            int first, double *__restrict__ W,
                                                            int nrhs) {
  extern __shared__ double sh[];
  const SweepBox &B = boxes[first + blockIdx.x];
  if (B.r == 0) return;
  sweep_up_box_mfma<NT>(B, W, nrhs, blockIdx.y * NT, sh);
}

template <int NT>
__global__ __launch_bounds__(kThreads) void k_sweep_down_mfma(const SweepBox *__restrict__ boxes,
                                                              int first, double *__restrict__ W,
                                                              int nrhs) {
  extern __shared__ double sh[];
  const SweepBox &B = boxes[first + blockIdx.x];
  if (B.r == 0 || B.k == 0) return;
  sweep_down_box_mfma<NT>(B, W, nrhs, blockIdx.y * NT, sh);
}

// Segment lookup for launches that cover the boxes of several handles: the last
// segment whose first block is <= blockIdx.x.
__device__ __forceinline__ int find_seg(const SweepSeg *segs, int nseg) {
  int lo = 0, hi = nseg - 1;
  const int b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].block0 <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int NT>
__global__ __launch_bounds__(kThreads) void k_sweep_up_seg(const SweepSeg *__restrict__ segs,
                                                           int nseg) {
  extern __shared__ double sh[];
  const SweepSeg &S = segs[find_seg(segs, nseg)];
  const SweepBox &B = S.boxes[blockIdx.x - S.block0];
  const int col0 = blockIdx.y * NT;
  if (B.r == 0 || col0 >= S.nrhs) return;
  sweep_up_box<NT>(B, S.W, S.nrhs, col0, sh);
}

template <int NT>
__global__ __launch_bounds__(kThreads) void k_sweep_down_seg(const SweepSeg *__restrict__ segs,
                                                             int nseg) {
  extern __shared__ double sh[];
  const SweepSeg &S = segs[find_seg(segs, nseg)];
  const SweepBox &B = S.boxes[blockIdx.x - S.block0];
  const int col0 = blockIdx.y * NT;
  if (B.r == 0 || B.k == 0 || col0 >= S.nrhs) return;
  sweep_down_box<NT>(B, S.W, S.nrhs, col0, sh);
}

template <int NT>
__global__ __launch_bounds__(kThreads) void k_sweep_up_seg_mfma(const SweepSeg *__restrict__ segs,
                                                                int nseg) {
  extern __shared__ double sh[];
  const SweepSeg &S = segs[find_seg(segs, nseg)];
  const SweepBox &B = S.boxes[blockIdx.x - S.block0];
  const int col0 = blockIdx.y * NT;
  if (B.r == 0 || col0 >= S.nrhs) return;
  sweep_up_box_mfma<NT>(B, S.W, S.nrhs, col0, sh);
}

template <int NT>
__global__ __launch_bounds__(kThreads) void k_sweep_down_seg_mfma(
    const SweepSeg *__restrict__ segs, int nseg) {
  extern __shared__ double sh[];
  const SweepSeg &S = segs[find_seg(segs, nseg)];
  const SweepBox &B = S.boxes[blockIdx.x - S.block0];
  const int col0 = blockIdx.y * NT;
  if (B.r == 0 || B.k == 0 || col0 >= S.nrhs) return;
  sweep_down_box_mfma<NT>(B, S.W, S.nrhs, col0, sh);
}

// Caller order <-> tree order for several right-hand-side blocks (grid.y = block).
__global__ void k_permute_seg(const PermSeg *__restrict__ segs, int to_tree) {
  const PermSeg &S = segs[blockIdx.y];
  const int64_t total = S.n * S.nrhs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / S.nrhs;
    const int c = (int)(e - i * S.nrhs);
    if (to_tree) S.W[e] = S.B[S.perm[i] + S.ldb * c];
    else S.B[S.perm[i] + S.ldb * c] = S.W[e];
  }
}

__global__ void k_permute_in(const double *__restrict__ B, int64_t ldb, double *__restrict__ W,
                             const int64_t *__restrict__ perm, int64_t n, int nrhs) {
  const int64_t total = n * nrhs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / nrhs;
    const int c = (int)(e - i * nrhs);
    W[e] = B[perm[i] + ldb * c];
  }
}

__global__ void k_permute_out(double *__restrict__ B, int64_t ldb, const double *__restrict__ W,
                              const int64_t *__restrict__ perm, int64_t n, int nrhs) {
  const int64_t total = n * nrhs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / nrhs;
    const int c = (int)(e - i * nrhs);
    B[perm[i] + ldb * c] = W[e];
  }
}

void check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw DeviceError(what, e);
}

template <int NT>
void sweep_up_nt(const SweepBox *boxes, int first, int count, double *W, int nrhs, int max_n,
                 hipStream_t st) {
  dim3 grid(count, (nrhs + NT - 1) / NT);
  hipLaunchKernelGGL(k_sweep_up<NT>, grid, dim3(kThreads), (size_t)max_n * NT * sizeof(double),
                     st, boxes, first, W, nrhs);
  check_launch("k_sweep_up");
}

template <int NT>
void sweep_down_nt(const SweepBox *boxes, int first, int count, double *W, int nrhs,
                   int max_n, hipStream_t st) {
  dim3 grid(count, (nrhs + NT - 1) / NT);
  hipLaunchKernelGGL(k_sweep_down<NT>, grid, dim3(kThreads),
                     (size_t)max_n * NT * sizeof(double), st, boxes, first, W, nrhs);
  check_launch("k_sweep_down");
}

int pick_nt(int nrhs, int max_n) {
  // LDS holds max_n x NT doubles; keep it within 64 KiB.
  int nt = nrhs <= 1 ? 1 : nrhs <= 4 ? 4 : nrhs <= 16 ? 16 : 32;
  while (nt > 1 && (int64_t)max_n * nt * 8 > 65536) nt = nt == 32 ? 16 : nt == 16 ? 4 : 1;
  return nt;
}

constexpr size_t kMaxLds = 160 * 1024;
// Dynamic LDS requested per workgroup.
constexpr size_t kLdsLimit = 64 * 1024;

}  // namespace

void launch_assemble(const CompBox *boxes, int first, int count, const ProbDev *probs,
                     const int32_t *pool, double *Marena, int max_npx, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_assemble, dim3(count), dim3(kThreads),
                     (size_t)max_npx * 3 * sizeof(double), st, boxes, first, probs, pool, Marena);
  check_launch("k_assemble");
}

constexpr int kVldsMaxRows = 8192;

size_t cpqr_lds_bytes_nt(int nth, int max_n, int max_m) {
  const int nw = nth / 64;
  size_t b = (size_t)max_n * sizeof(double) + (size_t)2 * max_n * sizeof(int) +
             (size_t)nw * max_n * sizeof(double);
  if (max_m <= kVldsMaxRows) b += (size_t)max_m * sizeof(double);
  return b;
}

size_t cpqr_lds_bytes(int max_n, int max_m) { return cpqr_lds_bytes_nt(256, max_n, max_m); }

template <int NTH, int RT, int CB, bool VLDS>
void cpqr_variant(const CompBox *boxes, int first, int count, const ProbDev *probs,
                  double *Marena, int32_t *order_pool, int32_t *ranks, size_t lds,
                  hipStream_t st) {
  auto kern = k_cpqr_id<NTH, RT, CB, VLDS>;
  if (lds > 64 * 1024)
    RS_HIP_CHECK(hipFuncSetAttribute((const void *)kern,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(kern, dim3(count), dim3(NTH), lds, st, boxes, first, probs, Marena,
                     order_pool, ranks);
  check_launch("k_cpqr_id");
}

template <int NTH>
void cpqr_bucket(const CompBox *boxes, int first, int count, const ProbDev *probs,
                 double *Marena, int32_t *order_pool, int32_t *ranks, int max_n, int max_m,
                 hipStream_t st) {
  const size_t lds = cpqr_lds_bytes_nt(NTH, max_n, max_m);
  const size_t lds_nov = cpqr_lds_bytes_nt(NTH, max_n, kVldsMaxRows + 1);
  if (lds_nov > kMaxLds)
    throw DeviceError("k_cpqr_id: box too large for LDS", hipErrorInvalidValue);
  // size buckets: rows held per lane (RT) and columns per wave (CB); 1024-thread
  // workgroups have half the registers per lane, so they hold fewer columns
  constexpr int CB4 = NTH >= 1024 ? 2 : 4;
  constexpr int CB16 = NTH >= 1024 ? 1 : 2;
  if (max_m <= 256 && lds <= kLdsLimit)
    cpqr_variant<NTH, 4, CB4, true>(boxes, first, count, probs, Marena, order_pool, ranks, lds,
                                    st);
  else if (max_m <= 512 && lds <= kLdsLimit)
    cpqr_variant<NTH, 8, CB4 / 2 * (NTH >= 1024 ? 1 : 2), true>(
        boxes, first, count, probs, Marena, order_pool, ranks, lds, st);
  else if (lds <= kLdsLimit)
    cpqr_variant<NTH, 16, CB16, true>(boxes, first, count, probs, Marena, order_pool, ranks, lds,
                                      st);
  else
    cpqr_variant<NTH, 16, CB16, false>(boxes, first, count, probs, Marena, order_pool, ranks,
                                       lds_nov, st);
}

void launch_cpqr_id(const CompBox *boxes, int first, int count, const ProbDev *probs,
                    double *Marena, int32_t *order_pool, int32_t *ranks, int max_n, int max_m,
                    hipStream_t st) {
  if (count <= 0) return;
  // Wide levels of small boxes: 256 threads, so several boxes share a CU; a few large
  // boxes: 1024 threads, so more trailing columns are updated at once.
  if (count >= 512 && max_n <= 96)
    cpqr_bucket<256>(boxes, first, count, probs, Marena, order_pool, ranks, max_n, max_m, st);
  else if (count <= 64 && max_m <= 512 &&
           cpqr_lds_bytes_nt(1024, max_n, kVldsMaxRows + 1) <= kLdsLimit)
    cpqr_bucket<1024>(boxes, first, count, probs, Marena, order_pool, ranks, max_n, max_m, st);
  else
    cpqr_bucket<512>(boxes, first, count, probs, Marena, order_pool, ranks, max_n, max_m, st);
}

// Dynamic LDS per workgroup is kept within 64 KiB: n^2 doubles + 12n bytes <= 64 KiB.
constexpr int kDiagLdsMaxN = 88;

template <int NTH, bool INLDS>
void diag_factor_nt(const FacBox *boxes, int first, int count, const ProbDev *probs,
                    const int32_t *pool, const int32_t *order_pool, const int32_t *ranks,
                    double *work, int32_t *err, int err_base, size_t lds, hipStream_t st) {
  auto kern = k_diag_factor<NTH, INLDS>;
  if (lds > 64 * 1024)
    RS_HIP_CHECK(hipFuncSetAttribute((const void *)kern,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(kern, dim3(count), dim3(NTH), lds, st, boxes, first, probs, pool,
                     order_pool, ranks, work, err, err_base);
  check_launch("k_diag_factor");
}

// Every box gets its own n x n workspace: the variant (LDS or global) is chosen per
// launch from the largest box, so the smaller boxes of a launch need one too.
size_t diag_work_doubles(int n) { return (size_t)n * n; }

void launch_diag_factor(const FacBox *boxes, int first, int count, const ProbDev *probs,
                        const int32_t *pool, const int32_t *order_pool, const int32_t *ranks,
                        double *work, int32_t *err, int err_base, int max_n, hipStream_t st) {
  if (count <= 0) return;
  if (max_n <= kDiagLdsMaxN) {
    const size_t lds = (size_t)max_n * max_n * sizeof(double) + (size_t)max_n * 12;
    diag_factor_nt<256, true>(boxes, first, count, probs, pool, order_pool, ranks, work, err,
                              err_base, lds, st);
    return;
  }
  const size_t lds = (size_t)max_n * 12;
  if (lds > kLdsLimit) throw DeviceError("k_diag_factor: box too large", hipErrorInvalidValue);
  // Few large boxes (the root): one 1024-thread workgroup each; otherwise 256 threads.
  if (count <= 64)
    diag_factor_nt<1024, false>(boxes, first, count, probs, pool, order_pool, ranks, work, err,
                                err_base, lds, st);
  else
    diag_factor_nt<256, false>(boxes, first, count, probs, pool, order_pool, ranks, work, err,
                               err_base, lds, st);
}

void launch_permute_in(const double *B, int64_t ldb, double *W, const int64_t *perm, int64_t n,
                       int nrhs, hipStream_t st) {
  const int64_t total = n * nrhs;
  if (total == 0) return;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_permute_in, dim3(blocks), dim3(256), 0, st, B, ldb, W, perm, n, nrhs);
  check_launch("k_permute_in");
}

void launch_permute_out(double *B, int64_t ldb, const double *W, const int64_t *perm,
                        int64_t n, int nrhs, hipStream_t st) {
  const int64_t total = n * nrhs;
  if (total == 0) return;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_permute_out, dim3(blocks), dim3(256), 0, st, B, ldb, W, perm, n, nrhs);
  check_launch("k_permute_out");
}

template <int NT>
void sweep_seg_nt(bool up, const SweepSeg *segs, int nseg, int nblocks, int max_nrhs, int max_n,
                  hipStream_t st) {
  dim3 grid(nblocks, (max_nrhs + NT - 1) / NT);
  const size_t lds = (size_t)max_n * NT * sizeof(double);
  if (up)
    hipLaunchKernelGGL(k_sweep_up_seg<NT>, grid, dim3(kThreads), lds, st, segs, nseg);
  else
    hipLaunchKernelGGL(k_sweep_down_seg<NT>, grid, dim3(kThreads), lds, st, segs, nseg);
  check_launch("k_sweep_seg");
}

void launch_sweep_seg(bool up, const SweepSeg *segs, int nseg, int nblocks, int max_nrhs,
                      int max_n, hipStream_t st) {
  if (nseg <= 0 || nblocks <= 0 || max_nrhs <= 0) return;
  switch (pick_nt(max_nrhs, max_n)) {
    case 1: sweep_seg_nt<1>(up, segs, nseg, nblocks, max_nrhs, max_n, st); break;
    case 4: sweep_seg_nt<4>(up, segs, nseg, nblocks, max_nrhs, max_n, st); break;
    case 16: sweep_seg_nt<16>(up, segs, nseg, nblocks, max_nrhs, max_n, st); break;
    default: sweep_seg_nt<32>(up, segs, nseg, nblocks, max_nrhs, max_n, st); break;
  }
}

void launch_permute_seg(const PermSeg *segs, int nseg, int64_t max_elems, bool to_tree,
                        hipStream_t st) {
  if (nseg <= 0 || max_elems <= 0) return;
  const int blocks = (int)std::min<int64_t>((max_elems + 255) / 256, 2048);
  hipLaunchKernelGGL(k_permute_seg, dim3(blocks, nseg), dim3(256), 0, st, segs, to_tree ? 1 : 0);
  check_launch("k_permute_seg");
}

int pick_nt_mfma(int nrhs, int max_n) {
  int nt = nrhs <= 16 ? 16 : nrhs <= 32 ? 32 : 64;
  while (nt > 16 && (int64_t)max_n * nt * 8 > 65536) nt /= 2;
  return nt;
}

template <int NT>
void sweep_mfma_nt(bool up, const SweepBox *boxes, int first, int count, double *W, int nrhs,
                   int max_n, hipStream_t st) {
  dim3 grid(count, (nrhs + NT - 1) / NT);
  const size_t lds = (size_t)max_n * NT * sizeof(double);
  if (up)
    hipLaunchKernelGGL(k_sweep_up_mfma<NT>, grid, dim3(kThreads), lds, st, boxes, first, W, nrhs);
  else
    hipLaunchKernelGGL(k_sweep_down_mfma<NT>, grid, dim3(kThreads), lds, st, boxes, first, W,
                       nrhs);
  check_launch("k_sweep_mfma");
}

void launch_sweep_mfma(bool up, const SweepBox *boxes, int first, int count, double *W, int nrhs,
                       int max_n, hipStream_t st) {
  if (count <= 0 || nrhs <= 0) return;
  if (max_n > kMfmaMaxN) throw DeviceError("k_sweep_mfma: box too large", hipErrorInvalidValue);
  switch (pick_nt_mfma(nrhs, max_n)) {
    case 16: sweep_mfma_nt<16>(up, boxes, first, count, W, nrhs, max_n, st); break;
    case 32: sweep_mfma_nt<32>(up, boxes, first, count, W, nrhs, max_n, st); break;
    default: sweep_mfma_nt<64>(up, boxes, first, count, W, nrhs, max_n, st); break;
  }
}

template <int NT>
void sweep_seg_mfma_nt(bool up, const SweepSeg *segs, int nseg, int nblocks, int max_nrhs,
                       int max_n, hipStream_t st) {
  dim3 grid(nblocks, (max_nrhs + NT - 1) / NT);
  const size_t lds = (size_t)max_n * NT * sizeof(double);
  if (up)
    hipLaunchKernelGGL(k_sweep_up_seg_mfma<NT>, grid, dim3(kThreads), lds, st, segs, nseg);
  else
    hipLaunchKernelGGL(k_sweep_down_seg_mfma<NT>, grid, dim3(kThreads), lds, st, segs, nseg);
  check_launch("k_sweep_seg_mfma");
}

void launch_sweep_seg_mfma(bool up, const SweepSeg *segs, int nseg, int nblocks, int max_nrhs,
                           int max_n, hipStream_t st) {
  if (nseg <= 0 || nblocks <= 0 || max_nrhs <= 0) return;
  if (max_n > kMfmaMaxN) throw DeviceError("k_sweep_seg_mfma: box too large", hipErrorInvalidValue);
  switch (pick_nt_mfma(max_nrhs, max_n)) {
    case 16: sweep_seg_mfma_nt<16>(up, segs, nseg, nblocks, max_nrhs, max_n, st); break;
    case 32: sweep_seg_mfma_nt<32>(up, segs, nseg, nblocks, max_nrhs, max_n, st); break;
    default: sweep_seg_mfma_nt<64>(up, segs, nseg, nblocks, max_nrhs, max_n, st); break;
  }
}

void launch_sweep_up(const SweepBox *boxes, int first, int count, double *W, int nrhs,
                     int max_n, hipStream_t st) {
  if (count <= 0 || nrhs <= 0) return;
  switch (pick_nt(nrhs, max_n)) {
    case 1: sweep_up_nt<1>(boxes, first, count, W, nrhs, max_n, st); break;
    case 4: sweep_up_nt<4>(boxes, first, count, W, nrhs, max_n, st); break;
    case 16: sweep_up_nt<16>(boxes, first, count, W, nrhs, max_n, st); break;
    default: sweep_up_nt<32>(boxes, first, count, W, nrhs, max_n, st); break;
  }
}

void launch_sweep_down(const SweepBox *boxes, int first, int count, double *W, int nrhs,
                       int max_n, hipStream_t st) {
  if (count <= 0 || nrhs <= 0) return;
  switch (pick_nt(nrhs, max_n)) {
    case 1: sweep_down_nt<1>(boxes, first, count, W, nrhs, max_n, st); break;
    case 4: sweep_down_nt<4>(boxes, first, count, W, nrhs, max_n, st); break;
    case 16: sweep_down_nt<16>(boxes, first, count, W, nrhs, max_n, st); break;
    default: sweep_down_nt<32>(boxes, first, count, W, nrhs, max_n, st); break;
  }
}

}  // namespace rs
