// HIP kernels of the recursive-skeletonization factor and solve passes (gfx950).
//
// Every kernel processes one box per workgroup; a launch covers all boxes of one tree
// level (of every problem of a batch), or a single box in the per-box reference mode.
// Every kernel is a template over the scalar type S: binary64 (`double`) for the
// Laplace kernels, complex128 (`Cplx`, stored as re/im pairs of binary64) for the
// Helmholtz combined-field kernel.
#include <float.h>
#include <limits.h>

#include <map>
#include <mutex>
#include <type_traits>
#include <utility>
#include <vector>

#include "rs_internal.h"

namespace rs {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr double kPi = 3.14159265358979323846;
constexpr double kInv2Pi = 0.15915494309189533577;   // 1 / (2 pi)
constexpr double kInv4Pi = 0.07957747154594766788;   // 1 / (4 pi)
constexpr double kEulerGamma = 0.57721566490153286061;

// ---------------------------------------------------------------- scalar types
struct Cplx {
  double re, im;
  Cplx() = default;
  __host__ __device__ constexpr Cplx(double r, double i = 0.0) : re(r), im(i) {}
};
__device__ __forceinline__ Cplx operator+(Cplx a, Cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ Cplx operator-(Cplx a, Cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ Cplx operator-(Cplx a) { return {-a.re, -a.im}; }
__device__ __forceinline__ Cplx operator*(Cplx a, Cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ Cplx operator*(double a, Cplx b) { return {a * b.re, a * b.im}; }
__device__ __forceinline__ Cplx operator*(Cplx a, double b) { return {a.re * b, a.im * b}; }
__device__ __forceinline__ Cplx &operator+=(Cplx &a, Cplx b) { return a = a + b; }
__device__ __forceinline__ Cplx &operator-=(Cplx &a, Cplx b) { return a = a - b; }
__device__ __forceinline__ double abs2(double a) { return a * a; }
__device__ __forceinline__ double abs2(Cplx a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ double mag(double a) { return fabs(a); }
__device__ __forceinline__ double mag(Cplx a) { return hypot(a.re, a.im); }
__device__ __forceinline__ double conjg(double a) { return a; }
__device__ __forceinline__ Cplx conjg(Cplx a) { return {a.re, -a.im}; }
__device__ __forceinline__ double re_part(double a) { return a; }
__device__ __forceinline__ double re_part(Cplx a) { return a.re; }
__device__ __forceinline__ double recip(double a) { return 1.0 / a; }
// 1 / (a + ib) by Smith's scaling (R. L. Smith, CACM 5 (1962)), no intermediate overflow.
__device__ __forceinline__ Cplx recip(Cplx a) {
  if (fabs(a.re) >= fabs(a.im)) {
    const double q = a.im / a.re, d = a.re + a.im * q;
    return {1.0 / d, -q / d};
  }
  const double q = a.re / a.im, d = a.re * q + a.im;
  return {q / d, -1.0 / d};
}
__device__ __forceinline__ double sdiv(double a, double b) { return a / b; }
__device__ __forceinline__ Cplx sdiv(Cplx a, double b) { return {a.re / b, a.im / b}; }
__device__ __forceinline__ Cplx sdiv(Cplx a, Cplx b) { return a * recip(b); }

__device__ __forceinline__ double shfl_xor(double v, int off) { return __shfl_xor(v, off, 64); }
__device__ __forceinline__ Cplx shfl_xor(Cplx v, int off) {
  return {__shfl_xor(v.re, off, 64), __shfl_xor(v.im, off, 64)};
}

// ---- wave64 reductions: DPP steps inside each row of 16 lanes (xor 1, xor 2, half-row
// mirror, row mirror: every lane ends with its row's total), then the four row totals
// read with readlane and combined in a fixed order.  The result is uniform across the
// wave and its rounding does not depend on anything but the 64 inputs.
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = dpp_i32<CTRL>(__double2loint(v));
  const int hi = dpp_i32<CTRL>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

__device__ __forceinline__ double wave_sum_f64(double v) {
  v += dpp_f64<kDppXor1>(v);
  v += dpp_f64<kDppXor2>(v);
  v += dpp_f64<kDppHalfMirror>(v);
  v += dpp_f64<kDppMirror>(v);
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}
__device__ __forceinline__ double wave_sum(double v) { return wave_sum_f64(v); }

// Eight sums over the wave at once: lane 8 g + 0..7 receive the sum of slot g.  Three
// transposing stages halve the slots while pairing lanes across bit 5, bit 4 and bit 3
// of the lane index -- gfx950's v_permlane32_swap and v_permlane16_swap exchange the
// halves and rows in registers, DPP row_ror:8 the half rows -- then DPP adds over lane
// bits 0-2.  Every slot is summed over the same pairing tree (and IEEE addition is
// commutative), so a column's sum does not depend on its slot.
constexpr int kDppRor8 = 0x128;
__device__ __forceinline__ void permlane32_swap_f64(double &a, double &b) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false,
                                                   false);
  a = __hiloint2double(hi[0], lo[0]);
  b = __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ void permlane16_swap_f64(double &a, double &b) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false,
                                                   false);
  a = __hiloint2double(hi[0], lo[0]);
  b = __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ double wave_sum8(const double (&x)[8]) {
  const int lane = threadIdx.x & 63;
  const bool b3 = lane & 8;
  double y[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {      // lanes 0-31: slot j over lanes l, l+32; 32-63: slot j+4
    double a = x[j], b = x[j + 4];
    permlane32_swap_f64(a, b);
    y[j] = a + b;
  }
  double z[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {      // rows of 16: even rows keep slot j, odd rows slot j+2
    double a = y[j], b = y[j + 2];
    permlane16_swap_f64(a, b);
    z[j] = a + b;
  }
  double w = (b3 ? z[1] : z[0]) + dpp_f64<kDppRor8>(b3 ? z[0] : z[1]);
  w += dpp_f64<kDppXor1>(w);
  w += dpp_f64<kDppXor2>(w);
  w += dpp_f64<kDppHalfMirror>(w);
  return w;
}
__device__ __forceinline__ Cplx wave_sum(Cplx v) { return {wave_sum_f64(v.re), wave_sum_f64(v.im)}; }

// Largest value over the wave with its key; ties (and NaN-free equal values) go to the
// smallest key.  `val` carries a payload chosen with the winner.  Uniform result.
struct ArgMax {
  double v;
  int key, val;
};
__device__ __forceinline__ void argmax_merge(ArgMax &a, double ov, int ok, int oval) {
  if (ov > a.v || (ov == a.v && ok < a.key)) { a.v = ov; a.key = ok; a.val = oval; }
}
template <int CTRL>
__device__ __forceinline__ void argmax_step(ArgMax &a) {
  const double ov = dpp_f64<CTRL>(a.v);
  const int ok = dpp_i32<CTRL>(a.key);
  const int oval = dpp_i32<CTRL>(a.val);
  argmax_merge(a, ov, ok, oval);
}
__device__ __forceinline__ ArgMax wave_argmax(double v, int key, int val) {
  ArgMax a{v, key, val};
  argmax_step<kDppXor1>(a);
  argmax_step<kDppXor2>(a);
  argmax_step<kDppHalfMirror>(a);
  argmax_step<kDppMirror>(a);
  ArgMax r{readlane_f64(a.v, 0), __builtin_amdgcn_readlane(a.key, 0),
           __builtin_amdgcn_readlane(a.val, 0)};
#pragma unroll
  for (int row = 16; row < 64; row += 16)
    argmax_merge(r, readlane_f64(a.v, row), __builtin_amdgcn_readlane(a.key, row),
                 __builtin_amdgcn_readlane(a.val, row));
  return r;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// ---------------------------------------------------------------- FP64 MFMA tiles
// v_mfma_f64_16x16x4f64 (wave64): lane l supplies A[l & 15][l >> 4] and
// B[l >> 4][l & 15]; element v of its result holds D[(l >> 4) + 4 v][l & 15].
// Complex tiles use four real products per step: (ar br - ai bi, ar bi + ai br).
typedef double dbl4 __attribute__((ext_vector_type(4)));

template <class S>
struct Acc;
template <>
struct Acc<double> {
  dbl4 v = {0.0, 0.0, 0.0, 0.0};
  __device__ __forceinline__ void mma(double a, double b) {
    v = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, v, 0, 0, 0);
  }
  __device__ __forceinline__ double get(int e) const { return v[e]; }
};
template <>
struct Acc<Cplx> {
  dbl4 re = {0.0, 0.0, 0.0, 0.0}, im = {0.0, 0.0, 0.0, 0.0};
  __device__ __forceinline__ void mma(Cplx a, Cplx b) {
    re = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, b.re, re, 0, 0, 0);
    re = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.im, b.im, re, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, b.im, im, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f64_16x16x4f64(a.im, b.re, im, 0, 0, 0);
  }
  __device__ __forceinline__ Cplx get(int e) const { return {re[e], im[e]}; }
};


// ---------------------------------------------------------------- kernels K(t, s)
// Laplace: eqs. (2d-laplace), (3d-laplace) and the double-layer kernel of eq.
// (double-layer), with the unit normal ns at the source.
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

// Helmholtz combined field (eq. (2d-helmholtz) with the combined layer of Section 3.2):
// K = dG/dnu_s - i eta G with G = (i/4) H0(kr).  With H_n = J_n + i Y_n,
//   dG/dnu_s = (k (d.nu)/(4 r)) (-Y1 + i J1),   -i eta G = (eta/4) (J0 + i Y0).
__device__ __noinline__ Cplx green_cfie(double kw, double eta, const double *t,
                                     const double *s, const double *ns) {
  const double dx = t[0] - s[0], dy = t[1] - s[1];
  const double r = sqrt(dx * dx + dy * dy);
  const double z = kw * r;
  const double j0v = j0(z), y0v = y0(z), j1v = j1(z), y1v = y1(z);
  const double dl = 0.25 * kw * (dx * ns[0] + dy * ns[1]) / r;
  return {-dl * y1v + 0.25 * eta * j0v, dl * j1v + 0.25 * eta * y0v};
}

template <class S>
__device__ __forceinline__ S kernel_val(const ProbDev &P, const double *t, const double *s,
                                        const double *ns);
template <>
__device__ __forceinline__ double kernel_val<double>(const ProbDev &P, const double *t,
                                                     const double *s, const double *ns) {
  return green(P.kind, t, s, ns);
}
// 3D Helmholtz (eq. (3d-helmholtz)): exp(i k r) / (4 pi r).
__device__ __forceinline__ Cplx green_helm3d(double kw, const double *t, const double *s) {
  const double dx = t[0] - s[0], dy = t[1] - s[1], dz = t[2] - s[2];
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  double sn, cs;
  sincos(kw * r, &sn, &cs);
  const double a = kInv4Pi / r;
  return {a * cs, a * sn};
}

template <>
__device__ __forceinline__ Cplx kernel_val<Cplx>(const ProbDev &P, const double *t,
                                                 const double *s, const double *ns) {
  if (P.kind == RS_HELM3D_SL) return green_helm3d(P.kwave, t, s);
  return green_cfie(P.kwave, P.eta, t, s, ns);
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
template <class S>
__device__ __forceinline__ S diag_entry(const ProbDev &P, int g);
template <>
__device__ __forceinline__ double diag_entry<double>(const ProbDev &P, int g) {
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
// Combined field: double-layer limit -kappa w / (4 pi) minus i eta times the
// single-layer self term w (i/4 - (log(k/2) + gamma)/(2 pi)) - (w/2pi) log(w/2pi).
template <>
__device__ __forceinline__ Cplx diag_entry<Cplx>(const ProbDev &P, int g) {
  const double w = P.w[g];
  if (P.kind == RS_HELM3D_SL) {
    // (exp(i k R) - 1) / (2 i k) = (sin kR + i (1 - cos kR)) / (2k), R = sqrt(w / pi);
    // 1 - cos kR written as 2 sin^2(kR/2) (no cancellation for small kR)
    const double kr = P.kwave * sqrt(w / kPi);
    const double sh = sin(0.5 * kr);
    return {P.c + sin(kr) / (2.0 * P.kwave), sh * sh / P.kwave};
  }
  const double dl = -P.kappa[g] * w * (0.25 / kPi);
  const double sl_re = -w * (log(0.5 * P.kwave) + kEulerGamma) * kInv2Pi -
                       (w * kInv2Pi) * log(w * kInv2Pi);
  const double sl_im = 0.25 * w;
  // -i eta (sl_re + i sl_im) = eta sl_im - i eta sl_re
  return {P.c + dl + P.eta * sl_im, -P.eta * sl_re};
}

// A(gi, gj) = c delta + K(x_gi, x_gj) w_gj.
template <class S>
__device__ __forceinline__ S entry(const ProbDev &P, int gi, int gj) {
  if (gi == gj) return diag_entry<S>(P, gi);
  double t[3], s[3], ns[3];
  load_pt(P, gi, t);
  load_pt(P, gj, s);
  load_nrm(P, gj, ns);
  return kernel_val<S>(P, t, s, ns) * P.w[gj];
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
//   rows m-2, m-1 (kernels with a logarithmic part): total charge and constant field,
//                           scaled to the largest proxy entry.
// Entry (i, j) of M_B for the rows i < 2 nn + 2 np (the two log rows are separate).
template <class S>
__device__ __forceinline__ S comp_entry(const ProbDev &P, const CompBox &B, const int32_t *J,
                                        const int32_t *N, const double *sh_u, double wG, int i,
                                        int j) {
  const int nn = B.nn, npx = P.npx;
  const int g = J[j];
  double xs[3], ns[3];
  load_pt(P, g, xs);
  if (i < nn) {
    double xq[3];
    load_nrm(P, g, ns);
    load_pt(P, N[i], xq);
    return kernel_val<S>(P, xq, xs, ns) * P.w[g];
  } else if (i < 2 * nn) {
    const int q = N[i - nn];
    double xq[3], nq[3];
    load_pt(P, q, xq);
    load_nrm(P, q, nq);
    return kernel_val<S>(P, xs, xq, nq) * P.w[q];
  } else if (i < 2 * nn + npx) {
    const double *u = sh_u + 3 * (i - 2 * nn);
    double y[3] = {B.cen[0] + B.rho * u[0], B.cen[1] + B.rho * u[1], B.cen[2] + B.rho * u[2]};
    load_nrm(P, g, ns);
    return kernel_val<S>(P, y, xs, ns) * P.w[g];
  } else {
    const double *u = sh_u + 3 * (i - 2 * nn - npx);
    double y[3] = {B.cen[0] + B.rho * u[0], B.cen[1] + B.rho * u[1], B.cen[2] + B.rho * u[2]};
    return kernel_val<S>(P, xs, y, u) * wG;
  }
}

// The same entry with the box's active points (index j) and near points (index i or
// i - nn) staged in LDS as structure of arrays: x[a][idx], nrm[a][idx], w[idx].
struct StagedPts {
  const double *x[3], *nrm[3], *w;
  __device__ __forceinline__ void load(int dim, int idx, double *p, double *nv) const {
    p[0] = x[0][idx];
    p[1] = x[1][idx];
    p[2] = dim == 3 ? x[2][idx] : 0.0;
    if (nrm[0]) {
      nv[0] = nrm[0][idx];
      nv[1] = nrm[1][idx];
      nv[2] = dim == 3 ? nrm[2][idx] : 0.0;
    } else {
      nv[0] = nv[1] = nv[2] = 0.0;
    }
  }
};

template <class S>
__device__ __forceinline__ S comp_entry_staged(const ProbDev &P, const CompBox &B,
                                               const StagedPts &Jp, const StagedPts &Np,
                                               const double *sh_u, double wG, int i, int j) {
  const int nn = B.nn, npx = P.npx, dim = P.dim;
  double xs[3], ns[3];
  Jp.load(dim, j, xs, ns);
  if (i < nn) {
    double xq[3], nq[3];
    Np.load(dim, i, xq, nq);
    return kernel_val<S>(P, xq, xs, ns) * Jp.w[j];
  } else if (i < 2 * nn) {
    double xq[3], nq[3];
    Np.load(dim, i - nn, xq, nq);
    return kernel_val<S>(P, xs, xq, nq) * Np.w[i - nn];
  } else if (i < 2 * nn + npx) {
    const double *u = sh_u + 3 * (i - 2 * nn);
    double y[3] = {B.cen[0] + B.rho * u[0], B.cen[1] + B.rho * u[1], B.cen[2] + B.rho * u[2]};
    return kernel_val<S>(P, y, xs, ns) * Jp.w[j];
  } else {
    const double *u = sh_u + 3 * (i - 2 * nn - npx);
    double y[3] = {B.cen[0] + B.rho * u[0], B.cen[1] + B.rho * u[1], B.cen[2] + B.rho * u[2]};
    return kernel_val<S>(P, xs, y, u) * wG;
  }
}

// Copies the points of idx[0..cnt) into LDS arrays at `base` (7 cnt doubles: x, y, z,
// three normal components (zero without normals), weight); returns the view.
__device__ __forceinline__ StagedPts stage_points(const ProbDev &P, const int32_t *idx, int cnt,
                                                  double *base, int nth) {
  StagedPts v;
  for (int a = 0; a < 3; ++a) v.x[a] = base + a * cnt;
  for (int a = 0; a < 3; ++a) v.nrm[a] = P.nrm[0] ? base + (3 + a) * cnt : nullptr;
  v.w = base + 6 * cnt;
  for (int e = threadIdx.x; e < cnt; e += nth) {
    const int g = idx[e];
    base[e] = P.x[0][g];
    base[cnt + e] = P.x[1][g];
    base[2 * cnt + e] = P.dim == 3 ? P.x[2][g] : 0.0;
    if (P.nrm[0]) {
      base[3 * cnt + e] = P.nrm[0][g];
      base[4 * cnt + e] = P.nrm[1][g];
      base[5 * cnt + e] = P.dim == 3 ? P.nrm[2][g] : 0.0;
    }
    base[6 * cnt + e] = P.w[g];
  }
  return v;
}

template <class S>
__global__ __launch_bounds__(kThreads) void k_assemble(const CompBox *__restrict__ boxes,
                                                       int first,
                                                       const ProbDev *__restrict__ probs,
                                                       const int32_t *__restrict__ pool,
                                                       S *__restrict__ Marena) {
  extern __shared__ double sh_u[];   // npx * 3 proxy unit vectors
  __shared__ double red[kWaves];
  const CompBox &B = boxes[first + blockIdx.x];
  const ProbDev &P = probs[B.prob];
  const int n = B.n, nn = B.nn, m = B.m, npx = P.npx, dim = P.dim;
  if (n == 0) return;
  const int32_t *J = pool + B.J_off;
  const int32_t *N = pool + B.N_off;
  S *M = Marena + B.M_off;
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
    const S v = comp_entry<S>(P, B, J, N, sh_u, wG, i, j);
    if (i >= 2 * nn) pmax = fmax(pmax, mag(v));
    M[(int64_t)j * m + i] = v;
  }
  if (P.log_kernel) {
    pmax = block_max(pmax, red);
    for (int j = threadIdx.x; j < n; j += kThreads) {
      M[(int64_t)j * m + rows] = S(pmax * P.w[J[j]] / wmax);
      M[(int64_t)j * m + rows + 1] = S(pmax);
    }
  }
}


// Chunked assembly of large blocks: blockIdx.x = box * CH + chunk; each chunk writes
// every CH-th group of kThreads entries of its box (column-major, rows fastest) and the
// largest proxy-row magnitude it saw into partials[box * CH + chunk]; k_assemble_tail
// then adds the two rows of the log kernels.  The entries and both maxima equal those
// of k_assemble.
template <class S>
__global__ __launch_bounds__(kThreads) void k_assemble_chunks(const CompBox *__restrict__ boxes,
                                                              int first, int CH,
                                                              const ProbDev *__restrict__ probs,
                                                              const int32_t *__restrict__ pool,
                                                              S *__restrict__ Marena,
                                                              double *__restrict__ partials) {
  extern __shared__ double sh_u[];   // npx * 3 proxy unit vectors
  __shared__ double red[kWaves];
  const int bi = blockIdx.x / CH, ch = blockIdx.x - bi * CH;
  const CompBox &B = boxes[first + bi];
  const ProbDev &P = probs[B.prob];
  const int n = B.n, nn = B.nn, m = B.m, npx = P.npx, dim = P.dim;
  if (n == 0) return;
  const int32_t *J = pool + B.J_off;
  const int32_t *N = pool + B.N_off;
  S *M = Marena + B.M_off;
  for (int p = threadIdx.x; p < npx; p += kThreads) proxy_unit(dim, p, npx, sh_u + 3 * p);
  __syncthreads();
  const double wG = dim == 2 ? 2.0 * kPi * B.rho / npx : 4.0 * kPi * B.rho * B.rho / npx;
  const int rows = 2 * nn + 2 * npx;
  double pmax = 0.0;
  const int64_t total = (int64_t)rows * n;
  for (int64_t e = (int64_t)ch * kThreads + threadIdx.x; e < total; e += (int64_t)CH * kThreads) {
    const int j = (int)(e / rows), i = (int)(e - (int64_t)j * rows);
    const S v = comp_entry<S>(P, B, J, N, sh_u, wG, i, j);
    if (i >= 2 * nn) pmax = fmax(pmax, mag(v));
    M[(int64_t)j * m + i] = v;
  }
  pmax = block_max(pmax, red);
  if (threadIdx.x == 0) partials[(int64_t)bi * CH + ch] = pmax;
}

template <class S>
__global__ __launch_bounds__(kThreads) void k_assemble_tail(const CompBox *__restrict__ boxes,
                                                            int first, int CH,
                                                            const ProbDev *__restrict__ probs,
                                                            const int32_t *__restrict__ pool,
                                                            S *__restrict__ Marena,
                                                            const double *__restrict__ partials) {
  __shared__ double red[kWaves];
  const CompBox &B = boxes[first + blockIdx.x];
  const ProbDev &P = probs[B.prob];
  const int n = B.n, m = B.m;
  if (n == 0 || !P.log_kernel) return;
  const int32_t *J = pool + B.J_off;
  S *M = Marena + B.M_off;
  double wmax = 0.0;
  for (int j = threadIdx.x; j < n; j += kThreads) wmax = fmax(wmax, P.w[J[j]]);
  wmax = block_max(wmax, red);
  double pmax = 0.0;
  for (int c = 0; c < CH; ++c) pmax = fmax(pmax, partials[(int64_t)blockIdx.x * CH + c]);
  const int rows = 2 * B.nn + 2 * P.npx;
  for (int j = threadIdx.x; j < n; j += kThreads) {
    M[(int64_t)j * m + rows] = S(pmax * P.w[J[j]] / wmax);
    M[(int64_t)j * m + rows + 1] = S(pmax);
  }
}

// --------------------------------------------------------------------------
// Fused compression of small boxes (real data, n <= 16 CPW, m <= 64 RT): M_B is evaluated
// into registers and factored there by column-pivoted Householder QR with the same rules
// as k_cpqr_id (largest recomputed norm, ties to the lowest column, stop at
// |R_jj| <= eps |R_00|).  With NW = NTH / 64 waves, wave w holds columns c = w + NW q
// (q < CPW), lane l rows l + 64 t (t < RT); a column's reductions stay inside its wave,
// so a pivot step needs two workgroup barriers (reflector ready, norms ready) and
// touches no global memory.  Columns are not moved: piv[j] is the column of pivot step
// j.  The first k rows of R are then staged in LDS and T = R11^{-1} R12 is solved by one wave
// per redundant column.  The arithmetic of a box does not depend on NTH, RT or CPW (a
// column's sums run over its rows in the same lanes and order; rows and columns beyond
// the box are zeros).
template <int NW>
__device__ __forceinline__ double block_max_w(double v, double *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_max(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double r = red[0];
  for (int i = 1; i < NW; ++i) r = fmax(r, red[i]);
  __syncthreads();
  return r;
}

// LDS doubles of the staging region: the assembly tiles, then rows < k <= min(m, n) of R
__host__ __device__ __forceinline__ int fused_tile_doubles(int nw, int n, int m) {
  const int kmax = n < m ? n : m;
  return nw * m > n * kmax ? nw * m : n * kmax;
}

template <int NTH, int RT, int CPW>
__global__ __launch_bounds__(NTH, 2) void k_compress_fused(
    const CompBox *__restrict__ boxes, int first, const ProbDev *__restrict__ probs,
    const int32_t *__restrict__ pool, int32_t *__restrict__ order_pool,
    int32_t *__restrict__ ranks) {
  constexpr int NW = NTH / 64;
  extern __shared__ double smem[];
  __shared__ double red[NW];
  __shared__ double s_ctau;
  const CompBox &B = boxes[first + blockIdx.x];
  const ProbDev &P = probs[B.prob];
  const int n = B.n, nn = B.nn, m = B.m, npx = P.npx, dim = P.dim;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (n == 0) {
    if (tid == 0) ranks[B.kslot] = 0;
    return;
  }
  const int32_t *J = pool + B.J_off;
  const int32_t *N = pool + B.N_off;
  double *sh_u = smem;                                 // 3 npx
  double *norms = sh_u + 3 * npx;                      // n
  double *sv = norms + n;                              // m
  double *wbuf = sv + m;                               // NW * n
  double *tile = wbuf + NW * n;   // NW m (assembly staging), later k n (rows < k of R)
  double *pts = tile + fused_tile_doubles(NW, n, m);   // 7 (n + nn): staged points
  int *piv = reinterpret_cast<int *>(pts + 7 * (n + nn));   // n
  int *rk = piv + n;                                   // n
  int *done = rk + n;                                  // n

  // ---- assembly
  for (int p = tid; p < npx; p += NTH) proxy_unit(dim, p, npx, sh_u + 3 * p);
  const StagedPts Jp = stage_points(P, J, n, pts, NTH);
  const StagedPts Np = stage_points(P, N, nn, pts + 7 * n, NTH);
  double wmax = 0.0;
  for (int j = tid; j < n; j += NTH) wmax = fmax(wmax, P.w[J[j]]);
  wmax = block_max_w<NW>(wmax, red);      // barrier: proxy vectors and points visible
  const double wG = dim == 2 ? 2.0 * kPi * B.rho / npx : 4.0 * kPi * B.rho * B.rho / npx;
  const int rows = 2 * nn + 2 * npx;
  double pmax = 0.0;
  double val[CPW][RT];
  // each wave evaluates its own columns into its LDS column, then every lane takes its
  // rows.  Symmetric kernels (the single layers, K(x, y) = K(y, x) bit for bit: the
  // distance is formed from squared differences) evaluate each point pair once for both
  // of its rows: near row i and its transpose nn + i, proxy row 2 nn + p and 2 nn + npx + p.
  double *mytile = tile + wave * m;
  const bool sym = P.kind == RS_LAP2D_SL || P.kind == RS_LAP3D_SL;
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    const int c = wave + NW * q;
    if (c < n && sym) {
      double xs[3], ns[3];
      Jp.load(dim, c, xs, ns);
      const double wc = Jp.w[c];
      for (int i = lane; i < nn; i += 64) {
        double xq[3], nq[3];
        Np.load(dim, i, xq, nq);
        const double g = kernel_val<double>(P, xq, xs, ns);
        mytile[i] = g * wc;
        mytile[nn + i] = g * Np.w[i];
      }
      for (int p = lane; p < npx; p += 64) {
        const double *u = sh_u + 3 * p;
        const double y[3] = {B.cen[0] + B.rho * u[0], B.cen[1] + B.rho * u[1],
                             B.cen[2] + B.rho * u[2]};
        const double g = kernel_val<double>(P, y, xs, ns);
        const double a = g * wc, b = g * wG;
        pmax = fmax(pmax, fmax(fabs(a), fabs(b)));
        mytile[2 * nn + p] = a;
        mytile[2 * nn + npx + p] = b;
      }
      wave_sync();     // rows were written by other lanes of the wave
    } else if (c < n) {
      for (int i = lane; i < rows; i += 64) {
        const double v = comp_entry_staged<double>(P, B, Jp, Np, sh_u, wG, i, c);
        if (i >= 2 * nn) pmax = fmax(pmax, fabs(v));
        mytile[i] = v;
      }
    }
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int i = lane + 64 * t;
      val[q][t] = (c < n && i < rows) ? mytile[i] : 0.0;
    }
  }
  if (P.log_kernel) {
    pmax = block_max_w<NW>(pmax, red);
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      const int c = wave + NW * q;
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int i = lane + 64 * t;
        if (c < n && i == rows) val[q][t] = pmax * P.w[J[c]] / wmax;
        if (c < n && i == rows + 1) val[q][t] = pmax;
      }
    }
  }

  // ---- column-pivoted QR in registers.  Column sums are taken eight columns at a
  // time (wave_sum8); lane 8 g + 0 holds the result for column slot g of the group.
  constexpr int NG = (CPW + 7) / 8;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    double x[8];
#pragma unroll
    for (int qq = 0; qq < 8; ++qq) {
      const int q = 8 * g + qq;
      double s = 0.0;
      if (q < CPW) {
#pragma unroll
        for (int t = 0; t < RT; ++t)
          if (64 * t < m) s += val[q][t] * val[q][t];
      }
      x[qq] = s;
    }
    const double tot = wave_sum8(x);
    const int q = 8 * g + (lane >> 3), c = wave + NW * q;
    if ((lane & 7) == 0 && q < CPW && c < n) norms[c] = sqrt(tot);
  }
  for (int c = tid; c < n; c += NTH) done[c] = 0;
  __syncthreads();
  const double eps = P.eps;
  const int kmax = min(m, n);
  int k = kmax;
  double r00 = 0.0;
  unsigned mine_done = 0;
  for (int j = 0; j < kmax; ++j) {
    double lbest = -1.0;
    int lbc = INT_MAX;
    for (int c = lane; c < n; c += 64) {
      if (done[c]) continue;
      const double v = norms[c];
      if (v > lbest || (v == lbest && c < lbc)) { lbest = v; lbc = c; }
    }
    const ArgMax am = wave_argmax(lbest, lbc, lbc);
    const double best = am.v;
    const int bc = am.key;
    if (j == 0) r00 = best;
    if (best == 0.0 || best <= eps * r00) { k = j; break; }
    const int p = bc, pw = p & (NW - 1), pq = p / NW;
    if (wave == pw) {   // reflector of column p, rows j..m-1
      // its norm over rows j..m-1 is the pivot search's value (recomputed after the
      // previous step over exactly these rows)
      double mine = 0.0;
#pragma unroll
      for (int q = 0; q < CPW; ++q)
        if (q == pq)
#pragma unroll
          for (int t = 0; t < RT; ++t)
            if (t == (j >> 6)) mine = val[q][t];
      const double alpha = best;
      const double x0 = readlane_f64(mine, j & 63);
      const double beta = x0 >= 0.0 ? -alpha : alpha;
      const double scale = 1.0 / (x0 - beta);
#pragma unroll
      for (int q = 0; q < CPW; ++q)
        if (q == pq)
#pragma unroll
          for (int t = 0; t < RT; ++t) {
            if (64 * t >= m) continue;
            const int i = lane + 64 * t;
            if (i > j && i < m) {
              val[q][t] *= scale;
              sv[i] = val[q][t];
            } else if (i == j) {
              val[q][t] = beta;
              sv[j] = 1.0;
            }
          }
      mine_done |= 1u << pq;
      if (lane == 0) s_ctau = (beta - x0) / beta;
    }
    __syncthreads();
    // every wave has finished this step's pivot search: the pivot can be marked
    if (tid == 0) {
      done[p] = 1;
      piv[j] = p;
    }
    const double ctau = s_ctau;
    double vi[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int i = lane + 64 * t;
      vi[t] = (i >= j && i < m) ? sv[i] : 0.0;
    }
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      double x[8];
#pragma unroll
      for (int qq = 0; qq < 8; ++qq) {
        const int q = 8 * g + qq;
        double dot = 0.0;
        if (q < CPW && wave + NW * q < n && !((mine_done >> q) & 1u)) {
#pragma unroll
          for (int t = 0; t < RT; ++t) dot += vi[t] * val[q][t];
        }
        x[qq] = dot;
      }
      const double dots = wave_sum8(x);
#pragma unroll
      for (int qq = 0; qq < 8; ++qq) {
        const int q = 8 * g + qq;
        double nr = 0.0;
        if (q < CPW && wave + NW * q < n && !((mine_done >> q) & 1u)) {
          const double dot = readlane_f64(dots, 8 * qq) * ctau;
#pragma unroll
          for (int t = 0; t < RT; ++t) {
            const int i = lane + 64 * t;
            const double nv = val[q][t] - dot * vi[t];
            val[q][t] = nv;
            if (i > j) nr += nv * nv;
          }
        }
        x[qq] = nr;
      }
      const double nrs = wave_sum8(x);
      const int q = 8 * g + (lane >> 3), c = wave + NW * q;
      if ((lane & 7) == 0 && q < CPW && c < n && !((mine_done >> q) & 1u)) norms[c] = sqrt(nrs);
    }
    __syncthreads();
  }

  // every wave has left the pivot search (the loop ends at a break without a barrier)
  // before its norms' space is reused
  __syncthreads();
  // ---- rows < k of R to LDS (column c at c k; the assembly staging is free now), and
  // the sorted positions of the columns within their class (skeleton or redundant)
  double *Rl = tile;
  int *ordl = reinterpret_cast<int *>(norms);          // n ints (the norms are done)
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    const int c = wave + NW * q;
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int i = lane + 64 * t;
      if (c < n && i < k) Rl[c * k + i] = val[q][t];
    }
  }
  if (wave == 0) {
    // n <= 128: two 64-column masks of the skeleton columns
    const bool s0 = lane < n && done[lane] != 0;
    const bool s1 = lane + 64 < n && done[lane + 64] != 0;
    const uint64_t m0 = __ballot(s0), m1 = __ballot(s1);
    const uint64_t v0 = n >= 64 ? ~0ull : ((1ull << n) - 1ull);
    const uint64_t v1 = n >= 128 ? ~0ull : (n > 64 ? ((1ull << (n - 64)) - 1ull) : 0ull);
    const uint64_t below = (1ull << lane) - 1ull;
    int32_t *order = order_pool + B.order_off;
    if (lane < n) {
      const int c = lane;
      const int r = s0 ? __popcll(m0 & below) : __popcll(~m0 & v0 & below);
      const int pos = s0 ? r : k + r;
      order[pos] = c;
      ordl[pos] = c;
      rk[c] = r;
    }
    if (lane + 64 < n) {
      const int c = lane + 64;
      const int r = s1 ? __popcll(m0) + __popcll(m1 & below)
                       : __popcll(~m0 & v0) + __popcll(~m1 & v1 & below);
      const int pos = s1 ? r : k + r;
      order[pos] = c;
      ordl[pos] = c;
      rk[c] = r;
    }
  }
  __syncthreads();
  // T = R11^{-1} R12, one wave per redundant column (two at a time): lane l keeps rows l
  // and l + 64 of the column; for i = k-1 down to 0, x_i = b_i / R(i, piv_i), then
  // b_l -= R(l, piv_i) x_i for l < i.  x_l goes to T(rk[piv_l], r) (skeletons sorted).
  double *T = B.T;
  const int nr = n - k;
  const int pv0 = lane < k ? piv[lane] : 0, pv1 = lane + 64 < k ? piv[lane + 64] : 0;
  for (int r0 = wave; r0 < nr; r0 += 2 * NW) {
    const int r1 = r0 + NW;
    const bool two = r1 < nr;
    const int ca = ordl[k + r0], cb = two ? ordl[k + r1] : ca;
    double a0 = lane < k ? Rl[ca * k + lane] : 0.0;
    double a1 = lane + 64 < k ? Rl[ca * k + lane + 64] : 0.0;
    double b0 = lane < k ? Rl[cb * k + lane] : 0.0;
    double b1 = lane + 64 < k ? Rl[cb * k + lane + 64] : 0.0;
    for (int i = k - 1; i >= 0; --i) {
      const int pi = i < 64 ? __builtin_amdgcn_readlane(pv0, i) : __builtin_amdgcn_readlane(pv1, i - 64);
      const double *Rc = Rl + pi * k;
      const double rii = Rc[i];
      const double ra0 = lane < k ? Rc[lane] : 0.0;
      const double ra1 = lane + 64 < k ? Rc[lane + 64] : 0.0;
      const double xa = (i < 64 ? readlane_f64(a0, i) : readlane_f64(a1, i - 64)) / rii;
      const double xb = (i < 64 ? readlane_f64(b0, i) : readlane_f64(b1, i - 64)) / rii;
      if (lane < i) {
        a0 -= ra0 * xa;
        b0 -= ra0 * xb;
      } else if (lane == i) {
        a0 = xa;
        b0 = xb;
      }
      if (lane + 64 < i) {
        a1 -= ra1 * xa;
        b1 -= ra1 * xb;
      } else if (lane + 64 == i) {
        a1 = xa;
        b1 = xb;
      }
    }
    double *Ta = T + (int64_t)k * r0;
    double *Tb = T + (int64_t)k * r1;
    if (lane < k) {
      Ta[rk[pv0]] = a0;
      if (two) Tb[rk[pv0]] = b0;
    }
    if (lane + 64 < k) {
      Ta[rk[pv1]] = a1;
      if (two) Tb[rk[pv1]] = b1;
    }
  }
  if (tid == 0) ranks[B.kslot] = k;
}

// Boxes with m n >= kCoopMinEntries take the multi-workgroup ID (k_cpqr_coop).
// (below ~1M entries the two box-wide barriers of every pivot step cost more than the
// single workgroup's streaming of the block: the 2D benchmark's top levels, 776 x 112,
// ran 0.6 ms per launch slower across workgroups)
constexpr int64_t kCoopMinEntries = int64_t(1) << 20;
constexpr int kCoopThreads = 256;
constexpr int kCoopMaxG = 64;
constexpr unsigned kCoopSpinLimit = 1u << 22;   // polls (each one L2 round trip plus a sleep): seconds

__host__ __device__ __forceinline__ bool coop_class(int m, int n) {
  return (int64_t)m * n >= kCoopMinEntries;
}

// ---------------------------------------------------------------------------------
// Register-resident ID of blocks beyond one workgroup's registers (the top levels' boxes,
// up to 64 RT rows and kSplitMaxN columns), spread over G workgroups per box in one
// cooperative launch.  Workgroup g of a box holds the columns c = g + G (w + 8 q) (wave
// w, slot q) in the layout of k_compress_fused (lane l: rows l + 64 t) and assembles them
// itself.  Per pivot step every workgroup offers its best column (norm, index and rows
// j..m-1) in the box's exchange area -- agent-coherent stores, then its step count --
// and, once all G offers are in, takes the same winner (largest norm, ties to the lowest
// column), forms the same Householder reflector from the offered column and updates its
// own columns.  After the last step the pivot columns' rows < k are exchanged the same
// way and each workgroup solves T = R11^{-1} R12 for its redundant columns from LDS.  A
// box's arithmetic does not depend on the launch (G follows from n).  Waits are bounded:
// past kCoopSpinLimit polls the launch's abort flag is raised, every workgroup stops and
// the box's rank is left at -1 for the host to report.
constexpr int kSplitRT = 13, kSplitCPW = 6, kSplitThreads = 512;
constexpr int kSplitCols = (kSplitThreads / 64) * kSplitCPW;      // columns per workgroup
constexpr int kSplitMaxN = 112;      // k <= 112: R11 fits LDS, rows < k in two registers
constexpr int kSplitMaxG = (kSplitMaxN + kSplitCols - 1) / kSplitCols;
constexpr int kSplitWideG = 8;       // workgroups per box on levels of few boxes

__host__ __device__ __forceinline__ int split_groups(int n) {
  return (n + kSplitCols - 1) / kSplitCols;
}
// exchange area of one box (doubles): step counts (one per 64-byte line), offers of both
// step parities (value, column), the proxy-row maxima, the offered columns of both
// parities, then R11 (k x k, in pivot order)
__host__ __device__ __forceinline__ int64_t split_xarea(int G) {
  const int64_t mp = 64 * kSplitRT;
  return 8 * G + 4 * G + G + 2 * G * mp + (int64_t)kSplitMaxN * kSplitMaxN + 8;
}

__device__ __forceinline__ void xstore(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double xload(const double *p) {
  return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publishes the workgroup's stores of the exchange (all of them completed first), then
// waits until every workgroup of the box has published `seq`: lane h of wave 0 polls
// workgroup h's count, so one poll is one round trip whatever G (G <= 64).  False on
// abort.
__device__ __forceinline__ bool split_exchange(unsigned *cnt, int g, int G, unsigned seq,
                                               int *abort_flag, int *s_ok) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    if (lane == 0)
      __hip_atomic_store(cnt + 16 * g, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool ready = lane >= G;
    bool ok = true;
    unsigned spins = 0;
    while (true) {
      if (!ready)
        ready = __hip_atomic_load(cnt + 16 * lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= seq;
      if (__all(ready)) break;
      const bool ab = lane == 0 &&
          __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
      if (__any(ab) || ++spins > kCoopSpinLimit) {
        if (lane == 0) __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = false;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (lane == 0) *s_ok = ok ? 1 : 0;
  }
  __syncthreads();
  return *s_ok != 0;
}

template <int RT, int CPW>
__global__ __launch_bounds__(kSplitThreads) void k_compress_split(
    const CompBox *__restrict__ boxes, int first, int G, const ProbDev *__restrict__ probs,
    const int32_t *__restrict__ pool, int32_t *__restrict__ order_pool,
    int32_t *__restrict__ ranks, double *__restrict__ xbase, int *__restrict__ abort_flag) {
  constexpr int NTH = kSplitThreads, NW = NTH / 64;
  extern __shared__ double smem[];
  __shared__ double red[NW];
  __shared__ int s_ok;
  __shared__ double s_best;
  __shared__ int s_bc, s_gw;
  const int bi = blockIdx.x / G, g = blockIdx.x - bi * G;
  const CompBox &B = boxes[first + bi];
  const ProbDev &P = probs[B.prob];
  const int n = B.n, nn = B.nn, m = B.m, npx = P.npx, dim = P.dim;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double *X = xbase + split_xarea(G) * bi;
  unsigned *cnt = reinterpret_cast<unsigned *>(X);
  double *offer = X + 8 * G;                 // [parity][h]: value, column
  double *xpmax = offer + 4 * G;             // [h]
  double *xcol = xpmax + G;                  // [parity][h][64 RT]
  double *xR = xcol + 2 * G * 64 * RT;       // k x k
  if (n == 0) {
    if (g == 0 && tid == 0) ranks[B.kslot] = 0;
    return;
  }
  const int32_t *J = pool + B.J_off;
  const int32_t *N = pool + B.N_off;
  // LDS: proxy vectors, then the assembly region (staged points and per-wave column
  // tiles) which the T solve later reuses for R11, then the column state
  double *sh_u = smem;                                        // 3 npx
  double *reg = sh_u + 3 * npx;
  const int assemble_d = 7 * (n + nn) + NW * m;
  const int kmax = min(m, n);
  double *pts = reg;                                          // 7 (n + nn)
  double *tile = pts + 7 * (n + nn);                          // NW m
  double *Rl = reg;                                           // kmax^2 (T solve)
  double *norms = reg + max(assemble_d, kmax * kmax);         // NW CPW (own columns)
  int *gdone = reinterpret_cast<int *>(norms + NW * CPW);     // n: pivoted, any group
  int *piv = gdone + n;                                       // kmax: column of step j
  int *stepof = piv + kmax;                                   // n: step of a pivot column
  int *rk = stepof + n;                                       // n: sorted class position

  // ---- assembly of this group's columns (as in k_compress_fused)
  for (int p = tid; p < npx; p += NTH) proxy_unit(dim, p, npx, sh_u + 3 * p);
  const StagedPts Jp = stage_points(P, J, n, pts, NTH);
  const StagedPts Np = stage_points(P, N, nn, pts + 7 * n, NTH);
  for (int c = tid; c < n; c += NTH) gdone[c] = 0;
  double wmax = 0.0;
  for (int j = tid; j < n; j += NTH) wmax = fmax(wmax, P.w[J[j]]);
  wmax = block_max_w<NW>(wmax, red);
  const double wG = dim == 2 ? 2.0 * kPi * B.rho / npx : 4.0 * kPi * B.rho * B.rho / npx;
  const int rows = 2 * nn + 2 * npx;
  double pmax = 0.0;
  double val[CPW][RT];
  double *mytile = tile + wave * m;
  const bool sym = P.kind == RS_LAP2D_SL || P.kind == RS_LAP3D_SL;
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    const int c = g + G * (wave + NW * q);
    if (c < n && sym) {
      double xs[3], ns[3];
      Jp.load(dim, c, xs, ns);
      const double wc = Jp.w[c];
      for (int i = lane; i < nn; i += 64) {
        double xq[3], nq[3];
        Np.load(dim, i, xq, nq);
        const double gv = kernel_val<double>(P, xq, xs, ns);
        mytile[i] = gv * wc;
        mytile[nn + i] = gv * Np.w[i];
      }
      for (int p = lane; p < npx; p += 64) {
        const double *u = sh_u + 3 * p;
        const double y[3] = {B.cen[0] + B.rho * u[0], B.cen[1] + B.rho * u[1],
                             B.cen[2] + B.rho * u[2]};
        const double gv = kernel_val<double>(P, y, xs, ns);
        const double a = gv * wc, b = gv * wG;
        pmax = fmax(pmax, fmax(fabs(a), fabs(b)));
        mytile[2 * nn + p] = a;
        mytile[2 * nn + npx + p] = b;
      }
      wave_sync();
    } else if (c < n) {
      for (int i = lane; i < rows; i += 64) {
        const double v = comp_entry_staged<double>(P, B, Jp, Np, sh_u, wG, i, c);
        if (i >= 2 * nn) pmax = fmax(pmax, fabs(v));
        mytile[i] = v;
      }
    }
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int i = lane + 64 * t;
      val[q][t] = (c < n && i < rows) ? mytile[i] : 0.0;
    }
  }
  unsigned seq = 0;
  if (P.log_kernel) {
    // the proxy-row maximum over the whole box, through the exchange
    pmax = block_max_w<NW>(pmax, red);
    if (tid == 0) xstore(xpmax + g, pmax);
    if (!split_exchange(cnt, g, G, ++seq, abort_flag, &s_ok)) {
      if (g == 0 && tid == 0) ranks[B.kslot] = -1;
      return;
    }
    pmax = wave_max(lane < G ? xload(xpmax + lane) : 0.0);
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      const int c = g + G * (wave + NW * q);
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int i = lane + 64 * t;
        if (c < n && i == rows) val[q][t] = pmax * P.w[J[c]] / wmax;
        if (c < n && i == rows + 1) val[q][t] = pmax;
      }
    }
  }
  // ---- initial column norms (one wave_sum8 group: CPW <= 8)
  static_assert(CPW <= 8, "one reduction group per wave");
  {
    double x[8];
#pragma unroll
    for (int qq = 0; qq < 8; ++qq) {
      double s = 0.0;
      if (qq < CPW) {
#pragma unroll
        for (int t = 0; t < RT; ++t) s += val[qq][t] * val[qq][t];
      }
      x[qq] = s;
    }
    const double tot = wave_sum8(x);
    const int q = lane >> 3;
    if ((lane & 7) == 0 && q < CPW) norms[wave + NW * q] = sqrt(tot);
  }
  __syncthreads();

  // ---- pivot steps
  const double eps = P.eps;
  int k = kmax;
  double r00 = 0.0;
  unsigned mine_done = 0;
  bool aborted = false;
  for (int j = 0; j < kmax; ++j) {
    const int par = j & 1;
    // this group's best column (every wave scans the group's norms)
    double lbest = -1.0;
    int lbc = INT_MAX;
    for (int cl = lane; cl < NW * CPW; cl += 64) {
      const int c = g + G * cl;
      if (c >= n || gdone[c]) continue;
      const double v = norms[cl];
      if (v > lbest || (v == lbest && c < lbc)) { lbest = v; lbc = c; }
    }
    const ArgMax am = wave_argmax(lbest, lbc, lbc);
    // offer it: value and column, and its rows j..m-1
    if (am.key != INT_MAX) {
      const int cl = (am.key - g) / G, ow = cl % NW, oq = cl / NW;
      if (wave == ow) {
#pragma unroll
        for (int q = 0; q < CPW; ++q)
          if (q == oq)
#pragma unroll
            for (int t = 0; t < RT; ++t) {
              const int i = lane + 64 * t;
              if (i >= j && i < m) xstore(xcol + ((int64_t)(par * G + g) * RT * 64) + i, val[q][t]);
            }
      }
    }
    if (tid == 0) {
      xstore(offer + 2 * (par * G + g), am.v);
      xstore(offer + 2 * (par * G + g) + 1, (double)am.key);
    }
    if (!split_exchange(cnt, g, G, ++seq, abort_flag, &s_ok)) {
      aborted = true;      // leaves the loop (returning from inside it costs registers)
      break;
    }
    if (wave == 0) {       // the offers, one lane each: largest norm, ties to the lowest column
      const double v = lane < G ? xload(offer + 2 * (par * G + lane)) : -2.0;
      const int c = lane < G ? (int)xload(offer + 2 * (par * G + lane) + 1) : INT_MAX;
      const ArgMax w = wave_argmax(v, c, lane);
      if (lane == 0) {
        s_best = w.v;
        s_bc = w.key;
        s_gw = w.val;
      }
    }
    __syncthreads();
    const double best = s_best;
    const int bc = s_bc, gw = s_gw;
    if (j == 0) r00 = best;
    if (best <= 0.0 || best <= eps * r00) { k = j; break; }
    // the reflector of the winning column, rows j..m-1, formed by every wave
    const double *xc = xcol + (int64_t)(par * G + gw) * RT * 64;
    double vi[RT];
    double xj = 0.0;
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int i = lane + 64 * t;
      vi[t] = (i >= j && i < m) ? xload(xc + i) : 0.0;
      if (t == (j >> 6)) xj = vi[t];
    }
    const double alpha = best;
    const double x0 = readlane_f64(xj, j & 63);
    const double beta = x0 >= 0.0 ? -alpha : alpha;
    const double scale = 1.0 / (x0 - beta);
    const double ctau = (beta - x0) / beta;
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int i = lane + 64 * t;
      vi[t] = i > j ? vi[t] * scale : (i == j ? 1.0 : 0.0);
    }
    if (tid == 0) {
      gdone[bc] = 1;
      piv[j] = bc;
      stepof[bc] = j;
    }
    // the winning column itself (its group): R(j, bc) = beta, Householder vector below
    if (gw == g) {
      const int cl = (bc - g) / G, ow = cl % NW, oq = cl / NW;
      if (wave == ow) {
#pragma unroll
        for (int q = 0; q < CPW; ++q)
          if (q == oq) {
#pragma unroll
            for (int t = 0; t < RT; ++t) {
              const int i = lane + 64 * t;
              if (i == j) val[q][t] = beta;
              else if (i > j && i < m) val[q][t] = vi[t];
            }
          }
        mine_done |= 1u << oq;
      }
    }
    // update of the group's other columns and their norms over rows > j
    {
      double x[8];
#pragma unroll
      for (int qq = 0; qq < 8; ++qq) {
        double dot = 0.0;
        if (qq < CPW && g + G * (wave + NW * qq) < n && !((mine_done >> qq) & 1u)) {
#pragma unroll
          for (int t = 0; t < RT; ++t) dot += vi[t] * val[qq][t];
        }
        x[qq] = dot;
      }
      const double dots = wave_sum8(x);
#pragma unroll
      for (int qq = 0; qq < 8; ++qq) {
        double nr = 0.0;
        if (qq < CPW && g + G * (wave + NW * qq) < n && !((mine_done >> qq) & 1u)) {
          const double dot = readlane_f64(dots, 8 * qq) * ctau;
#pragma unroll
          for (int t = 0; t < RT; ++t) {
            const int i = lane + 64 * t;
            const double nv = val[qq][t] - dot * vi[t];
            val[qq][t] = nv;
            if (i > j) nr += nv * nv;
          }
        }
        x[qq] = nr;
      }
      const double nrs = wave_sum8(x);
      const int q = lane >> 3;
      if ((lane & 7) == 0 && q < CPW && g + G * (wave + NW * q) < n && !((mine_done >> q) & 1u))
        norms[wave + NW * q] = sqrt(nrs);
    }
    __syncthreads();
  }
  if (aborted) {
    if (g == 0 && tid == 0) ranks[B.kslot] = -1;
    return;
  }
  __syncthreads();
  // ---- rows < k of the group's pivot columns to the exchange (R11 in pivot order)
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    const int c = g + G * (wave + NW * q);
    if (c < n && ((mine_done >> q) & 1u)) {
      const int s = stepof[c];
      if (s < k) {
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          const int i = lane + 64 * t;
          if (i < k) xstore(xR + i + (int64_t)k * s, val[q][t]);
        }
      }
    }
  }
  if (!split_exchange(cnt, g, G, ++seq, abort_flag, &s_ok)) {
    if (g == 0 && tid == 0) ranks[B.kslot] = -1;
    return;
  }
  for (int e = tid; e < k * k; e += NTH) Rl[e] = xload(xR + e);
  // sorted positions of the columns within their class (n <= 128: two masks)
  if (wave == 0) {
    const bool s0 = lane < n && gdone[lane] != 0 && stepof[lane] < k;
    const bool s1 = lane + 64 < n && gdone[lane + 64] != 0 && stepof[lane + 64] < k;
    const uint64_t m0 = __ballot(s0), m1 = __ballot(s1);
    const uint64_t v0 = n >= 64 ? ~0ull : ((1ull << n) - 1ull);
    const uint64_t v1 = n >= 128 ? ~0ull : (n > 64 ? ((1ull << (n - 64)) - 1ull) : 0ull);
    const uint64_t below = (1ull << lane) - 1ull;
    int32_t *order = order_pool + B.order_off;
    if (lane < n) {
      const int r = s0 ? __popcll(m0 & below) : __popcll(~m0 & v0 & below);
      if (g == 0) order[s0 ? r : k + r] = lane;
      rk[lane] = r;
    }
    if (lane + 64 < n) {
      const int r = s1 ? __popcll(m0) + __popcll(m1 & below)
                       : __popcll(~m0 & v0) + __popcll(~m1 & v1 & below);
      if (g == 0) order[s1 ? r : k + r] = lane + 64;
      rk[lane + 64] = r;
    }
  }
  __syncthreads();
  // ---- T = R11^{-1} R12 for this group's redundant columns: one wave per column,
  // right-looking substitution as in k_compress_fused (k <= 128: rows l and l + 64)
  double *T = B.T;
  const int pv0 = lane < k ? piv[lane] : 0, pv1 = lane + 64 < k ? piv[lane + 64] : 0;
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    const int c = g + G * (wave + NW * q);
    if (c >= n || (gdone[c] && stepof[c] < k)) continue;
    double b0 = lane < k ? val[q][0] : 0.0;
    double b1 = lane + 64 < k ? val[q][1] : 0.0;
    for (int i = k - 1; i >= 0; --i) {
      const double *Rc = Rl + (int64_t)k * i;        // R11 column of step i
      const double rii = Rc[i];
      const double ra0 = lane < k ? Rc[lane] : 0.0;
      const double ra1 = lane + 64 < k ? Rc[lane + 64] : 0.0;
      const double x = (i < 64 ? readlane_f64(b0, i) : readlane_f64(b1, i - 64)) / rii;
      if (lane < i) b0 -= ra0 * x;
      else if (lane == i) b0 = x;
      if (lane + 64 < i) b1 -= ra1 * x;
      else if (lane + 64 == i) b1 = x;
    }
    double *Tc = T + (int64_t)k * rk[c];
    if (lane < k) Tc[rk[pv0]] = b0;
    if (lane + 64 < k) Tc[rk[pv1]] = b1;
  }
  if (g == 0 && tid == 0) ranks[B.kslot] = k;
}

// --------------------------------------------------------------------------
// Row sketch Y = Omega M of a compression block for the randomized ID (Section 2.2):
// Omega is ell x m with entries +-1, entry (a, i) of tree box b set by the top bit of
// SplitMix64 (published by Steele, Lea and Flood, OOPSLA 2014) at the counter
// seed ^ (b << 40) ^ (a << 20) ^ i.  Each wave produces 16 x 16 tiles of Y with FP64
// MFMA over the rows of M in order.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <class S>
__global__ __launch_bounds__(kThreads) void k_sketch(const CompBox *__restrict__ comp,
                                                     const CompBox *__restrict__ comp_id,
                                                     int first, const ProbDev *__restrict__ probs,
                                                     S *__restrict__ Marena) {
  const CompBox &B = comp[first + blockIdx.x];
  const CompBox &Bi = comp_id[first + blockIdx.x];
  const int m = B.m, n = B.n, ell = Bi.m;
  if (ell >= m || n == 0) return;
  const ProbDev &P = probs[B.prob];
  const uint64_t key = P.sketch_seed ^ ((uint64_t)(uint32_t)B.box << 40);
  const S *M = Marena + B.M_off;
  S *Y = Marena + Bi.M_off;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ta = (ell + 15) / 16, tc = (n + 15) / 16;
  for (int tile = blockIdx.y * kWaves + wave; tile < ta * tc; tile += gridDim.y * kWaves) {
    const int a0 = (tile / tc) * 16, c0 = (tile % tc) * 16;
    const int a = a0 + li, c = c0 + li;
    const uint64_t ka = key ^ ((uint64_t)a << 20);
    Acc<S> acc;
    for (int i0 = 0; i0 < m; i0 += 4) {
      const int i = i0 + lk;
      double w = 0.0;
      if (a < ell && i < m) w = (splitmix64(ka ^ (uint64_t)i) >> 63) ? -1.0 : 1.0;
      const S x = (c < n && i < m) ? M[(int64_t)c * m + i] : S(0.0);
      acc.mma(S(w), x);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ar = a0 + lk + 4 * v;
      if (ar < ell && c < n) Y[(int64_t)c * ell + ar] = acc.get(v);
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
// Reflector of column x (rows j..m-1): beta = -sign(Re x_0) |x|, v = x / (x_0 - beta)
// with v_0 = 1, tau = (beta - x_0) / beta; the trailing columns are multiplied by
// I - conj(tau) v v^H, which maps x to beta e_0 (beta real; for real data this is the
// usual Householder reflector).
//
// Trailing update: each wave takes CB columns at a time; a lane holds up to RT rows of
// each of them in registers, so one step reads and writes the trailing matrix once
// (dot product with the reflector, update, and the recomputed norm in one pass).  The
// reflector is staged in LDS when VLDS.  Rows beyond 64*RT are streamed in two passes.
template <class S, int NTH, int RT, int CB, bool VLDS>
__global__ __launch_bounds__(NTH) void k_cpqr_id(const CompBox *__restrict__ boxes, int first,
                                                 const ProbDev *__restrict__ probs,
                                                 S *__restrict__ Marena,
                                                 int32_t *__restrict__ order_pool,
                                                 int32_t *__restrict__ ranks) {
  constexpr int NW = NTH / 64;
  extern __shared__ double smem[];
  __shared__ double s_best;
  __shared__ S s_ctau;
  __shared__ int s_p;
  const CompBox &B = boxes[first + blockIdx.x];
  const int m = B.m, n = B.n;
  const double eps = probs[B.prob].eps;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (n == 0) {
    if (threadIdx.x == 0) ranks[B.kslot] = 0;
    return;
  }
  if (coop_class(m, n)) return;                    // factored by k_cpqr_coop
  S *M = Marena + B.M_off;
  const int kmax = min(m, n);
  double *norms = smem;                                    // n
  int *perm = reinterpret_cast<int *>(norms + n);          // n
  int *rk = perm + n;                                      // n
  S *wbuf = reinterpret_cast<S *>(rk + n);                 // NW * kmax (16n bytes in)
  S *sv = wbuf + NW * kmax;                                // m (VLDS only)

  for (int c = threadIdx.x; c < n; c += NTH) perm[c] = c;
  for (int c = wave; c < n; c += NW) {
    const S *col = M + (int64_t)c * m;
    double s = 0.0;
    for (int i = lane; i < m; i += 64) s += abs2(col[i]);
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
      const ArgMax a = wave_argmax(best, bperm, bc);
      if (lane == 0) { s_best = a.v; s_p = a.val; }
    }
    __syncthreads();
    const double best = s_best;
    const int p = s_p;
    if (j == 0) r00 = best;
    if (best == 0.0 || best <= eps * r00) { k = j; break; }
    if (p != j) {
      S *cj = M + (int64_t)j * m, *cp = M + (int64_t)p * m;
      for (int i = threadIdx.x; i < m; i += NTH) {
        const S a = cj[i];
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
      S *cj = M + (int64_t)j * m;
      double s = 0.0;
      // real data with at most 512 threads: the column's rows j + lane + 64 t are held
      // in registers between the norm and the scaling, when they fit
      constexpr bool kHhRegs = sizeof(S) == sizeof(double) && NTH <= 512;
      const bool in_regs = kHhRegs && m - j <= 64 * RT;
      S xv[RT];
      if (in_regs) {
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          const int i = j + lane + 64 * t;
          xv[t] = i < m ? cj[i] : S(0.0);
        }
#pragma unroll
        for (int t = 0; t < RT; ++t)
          if (j + lane + 64 * t < m) s += abs2(xv[t]);
      } else {
        for (int i = j + lane; i < m; i += 64) s += abs2(cj[i]);
      }
      s = wave_sum(s);
      const double alpha = sqrt(s);
      const S x0 = cj[j];
      const double beta = re_part(x0) >= 0.0 ? -alpha : alpha;
      const S scale = recip(x0 - S(beta));
      if (in_regs) {
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          const int i = j + lane + 64 * t;
          if (i > j && i < m) {
            const S v = xv[t] * scale;
            cj[i] = v;
            if (VLDS) sv[i] = v;
          }
        }
      } else {
        for (int i = j + 1 + lane; i < m; i += 64) {
          const S v = cj[i] * scale;
          cj[i] = v;
          if (VLDS) sv[i] = v;
        }
      }
      if (lane == 0) {
        s_ctau = conjg(sdiv(S(beta) - x0, beta));
        cj[j] = S(beta);
        if (VLDS) sv[j] = S(1.0);
      }
    }
    __syncthreads();
    const S ctau = s_ctau;
    const S *vg = M + (int64_t)j * m;
    auto vload = [&](int i) -> S { return i == j ? S(1.0) : (VLDS ? sv[i] : vg[i]); };
    const int rows = m - j;
    // Pipelined rounds of CBP columns: the next round's columns are loaded while the
    // current one is reduced and written (software pipelining over the L2 latency), the
    // reflector once per step; register budget: two rounds plus the reflector in at most
    // 48 doubles per lane (half that with 1024 threads).  Per column the arithmetic is
    // that of the plain rounds: one fused multiply-add per real term.  Complex data keeps
    // the plain rounds, so that each complex product is contracted the same way in every
    // variant a box can be launched with.
    constexpr int ES = (int)(sizeof(S) / sizeof(double));
    constexpr bool PIPE = ES == 1 && RT * (NTH >= 1024 ? 2 : 1) <= 16;
    constexpr int CBP0 = RT * ES >= 16 ? 1 : 16 / (RT * ES);
    constexpr int CBP = CBP0 < CB ? CBP0 : CB;
    if (PIPE && rows <= 64 * RT) {
      S vi[RT];
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int i = j + lane + 64 * t;
        vi[t] = i < m ? vload(i) : S(0.0);
      }
      S nxt[CBP][RT];
      auto load_round = [&](int c0) {
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          const int i = j + lane + 64 * t;
#pragma unroll
          for (int cb = 0; cb < CBP; ++cb) {
            const int c = c0 + cb;
            nxt[cb][t] = (i < m && c < n) ? M[(int64_t)c * m + i] : S(0.0);
          }
        }
      };
      const int c_first = j + 1 + wave * CBP;
      if (c_first < n) load_round(c_first);
      for (int c0 = c_first; c0 < n; c0 += NW * CBP) {
        S val[CBP][RT];
#pragma unroll
        for (int cb = 0; cb < CBP; ++cb)
#pragma unroll
          for (int t = 0; t < RT; ++t) val[cb][t] = nxt[cb][t];
        if (c0 + NW * CBP < n) load_round(c0 + NW * CBP);
        S dot[CBP];
        double nrm[CBP];
#pragma unroll
        for (int cb = 0; cb < CBP; ++cb) { dot[cb] = S(0.0); nrm[cb] = 0.0; }
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int cb = 0; cb < CBP; ++cb) dot[cb] += conjg(vi[t]) * val[cb][t];
#pragma unroll
        for (int cb = 0; cb < CBP; ++cb) dot[cb] = wave_sum(dot[cb]) * ctau;
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          const int i = j + lane + 64 * t;
          if (i < m) {
#pragma unroll
            for (int cb = 0; cb < CBP; ++cb) {
              const int c = c0 + cb;
              if (c < n) {
                const S nv = val[cb][t] - dot[cb] * vi[t];
                M[(int64_t)c * m + i] = nv;
                if (i > j) nrm[cb] += abs2(nv);
              }
            }
          }
        }
#pragma unroll
        for (int cb = 0; cb < CBP; ++cb) {
          const double sn = wave_sum(nrm[cb]);
          if (lane == 0 && c0 + cb < n) norms[c0 + cb] = sqrt(sn);
        }
      }
    } else
    for (int c0 = j + 1 + wave * CB; c0 < n; c0 += NW * CB) {
      S dot[CB];
      double nrm[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) { dot[cb] = S(0.0); nrm[cb] = 0.0; }
      if (rows <= 64 * RT) {
        S val[CB][RT], vi[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          const int i = j + lane + 64 * t;
          const bool ok = i < m;
          vi[t] = ok ? vload(i) : S(0.0);
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
            const int c = c0 + cb;
            val[cb][t] = (ok && c < n) ? M[(int64_t)c * m + i] : S(0.0);
            dot[cb] += conjg(vi[t]) * val[cb][t];
          }
        }
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) dot[cb] = wave_sum(dot[cb]) * ctau;
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          const int i = j + lane + 64 * t;
          if (i < m) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
              const int c = c0 + cb;
              if (c < n) {
                const S nv = val[cb][t] - dot[cb] * vi[t];
                M[(int64_t)c * m + i] = nv;
                if (i > j) nrm[cb] += abs2(nv);
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
              const S v = conjg(vload(i));
#pragma unroll
              for (int cb = 0; cb < CB; ++cb) {
                const int c = c0 + cb;
                if (c < n) dot[cb] += v * M[(int64_t)c * m + i];
              }
            }
          }
        }
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) dot[cb] = wave_sum(dot[cb]) * ctau;
        for (int base = j; base < m; base += 64 * RT) {
#pragma unroll
          for (int t = 0; t < RT; ++t) {
            const int i = base + lane + 64 * t;
            if (i < m) {
              const S v = vload(i);
#pragma unroll
              for (int cb = 0; cb < CB; ++cb) {
                const int c = c0 + cb;
                if (c < n) {
                  S *pc = M + (int64_t)c * m + i;
                  const S nv = *pc - dot[cb] * v;
                  *pc = nv;
                  if (i > j) nrm[cb] += abs2(nv);
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
  S *buf = wbuf + wave * kmax;
  for (int c = k + wave; c < n; c += NW) {
    S *col = M + (int64_t)c * m;
    for (int i = lane; i < k; i += 64) buf[i] = col[i];
    for (int i = k - 1; i >= 0; --i) {
      const S xi = sdiv(buf[i], M[(int64_t)i * m + i]);
      const S *ri = M + (int64_t)i * m;
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
  S *T = reinterpret_cast<S *>(B.T);
  for (int c = k + wave; c < n; c += NW) {
    const S *col = M + (int64_t)c * m;
    S *Tc = T + (int64_t)k * rk[c];
    for (int i = lane; i < k; i += 64) Tc[rk[i]] = col[i];
  }
  if (threadIdx.x == 0) ranks[B.kslot] = k;
}


// --------------------------------------------------------------------------
// Blocked Gauss-Jordan inversion with partial pivoting (the box inversions of Section
// 3.4).  Pivot rows are not swapped: piv[j] records the row that eliminates column j.
// Columns are processed in panels of kPB: the panel's steps run on the panel's columns
// only (in place when A is in LDS, else on an LDS or workspace copy); their combined
// effect on every other column q is the rank-kPB update
//   A(i, q) <- [i not a pivot of the panel] A(i, q) + P(i, :) W(:, q),
// where P is the panel after its steps and W(s, q) = A(piv[p0 + s], q) before them
// (the panel's columns equal those of the accumulated row-operation matrix), done with
// FP64 MFMA tiles.  At the end the in-place array Y holds the inverse as
// A^{-1}(a, b) = Y(piv[a], q[b]) with q = piv^{-1}; it is written to G (r x r) in that
// order.  Returns false on a zero or non-finite pivot.
//
// For r <= kWavePanelMaxR with the panel in LDS one wave runs a panel's steps alone
// (lanes over rows, no workgroup barrier between steps; the other waves wait once per
// panel); otherwise each step is spread over the workgroup.  Both perform the same operations on every
// element, so the result depends on the block alone.
constexpr int kPB = 16;           // panel width
constexpr int kQC = 128;          // columns per chunk of the deferred update
constexpr int kWavePanelMaxR = 512;

template <class S>
__host__ __device__ constexpr size_t gj_panel_lds_max() { return 64 * 1024; }

// LDS bytes of the blocked inversion's buffers for up to r unknowns; with a_in_lds the
// panel needs no copy, otherwise the copy is in LDS when it fits gj_panel_lds_max.  A
// launch reserves for its largest box, and any smaller box whose copy fits must find
// room too: the reservation is min(copy, gj_panel_lds_max), never zero.
template <class S>
__host__ __device__ inline size_t gj_blocked_lds(int r, int nw, bool a_in_lds) {
  const size_t panel = (size_t)r * kPB * sizeof(S);
  size_t b = a_in_lds ? 0 : (panel <= gj_panel_lds_max<S>() ? panel : gj_panel_lds_max<S>());
  b += (size_t)kPB * kQC * sizeof(S) + (size_t)kPB * sizeof(S);
  b += (size_t)nw * (sizeof(double) + sizeof(int));
  b += (size_t)3 * r * sizeof(int) + 2 * sizeof(int);
  return (b + 15) & ~(size_t)15;
}

// Orders the memory operations of the lanes of one wave (no workgroup barrier).

// --------------------------------------------------------------------------
// The same interpolative decomposition for large blocks, spread over G workgroups per
// box in one cooperative launch (every workgroup of the grid resident at once).  A box
// is in this class when m n >= kCoopMinEntries (its own size only, so its result never
// depends on the launch it shares); k_cpqr_id skips such boxes.  The rules and outputs
// are those of k_cpqr_id: pivot = largest recomputed norm of the remaining part (rows
// j..m-1), ties to the lowest column, stop at |R_jj| <= eps |R_00|, T = R11^{-1} R12,
// sorted skeleton and redundant sets.
//
// Columns are not moved: step j's pivot is column piv[j], and R's row j ends in row j of
// every column.  Workgroup g owns the columns c = g (mod G) and is the only one to write
// them.  A step: each workgroup offers its best column; box-wide barrier; all pick the
// same pivot from the G offers; the pivot's owner forms the reflector in place (v below
// the diagonal, beta on it) and publishes conj(tau); box-wide barrier; every workgroup
// applies the reflector to its remaining columns and recomputes their norms.  A column's
// sums always run over the same lanes in the same order (one wave per column), so the
// result does not depend on G.
//
// Barriers count arrivals on a per-box counter with agent-scope release/acquire; a wait
// is bounded: past kCoopSpinLimit polls a workgroup raises the launch's abort flag and
// every workgroup leaves at its next barrier (the box's rank is then reported as -1).
// Box-wide barrier number `seq` (1, 2, ...) of G workgroups.  Returns false if the launch
// was aborted (uniform over the workgroup).
__device__ __forceinline__ bool coop_barrier(unsigned *cnt, unsigned target, int *abort_flag,
                                             int *s_ok) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    unsigned spins = 0;
    while (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        ok = 0;
        break;
      }
      if (++spins > kCoopSpinLimit) {
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
    *s_ok = ok;
  }
  __syncthreads();
  __threadfence();
  return *s_ok != 0;
}

template <class S>
__global__ __launch_bounds__(kCoopThreads) void k_cpqr_coop(
    const CompBox *__restrict__ boxes, int first, int count, int nbox_al, int G,
    const ProbDev *__restrict__ probs, S *__restrict__ Marena, int32_t *__restrict__ order_pool,
    int32_t *__restrict__ ranks, unsigned *__restrict__ bar, double *__restrict__ cval,
    int *__restrict__ ccol, double *__restrict__ ctau_g, int *__restrict__ abort_flag,
    int vlds) {
  constexpr int NW = kCoopThreads / 64;
  extern __shared__ double smem[];
  __shared__ int s_ok, s_p, s_k;
  __shared__ double s_best;
  const int bl = blockIdx.x % nbox_al, g = blockIdx.x / nbox_al;
  if (bl >= count) return;
  const CompBox &B = boxes[first + bl];
  const int m = B.m, n = B.n;
  if (!coop_class(m, n)) return;                    // not in this class: no barriers
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double eps = probs[B.prob].eps;
  S *M = Marena + B.M_off;
  const int kmax = min(m, n);
  const int nq = g < n ? (n - g + G - 1) / G : 0;   // columns g, g + G, ...
  const int nqmax = (n + G - 1) / G;
  char *lb0 = reinterpret_cast<char *>(smem);
  double *nrm = reinterpret_cast<double *>(lb0);                     // nqmax
  int *dn = reinterpret_cast<int *>(lb0 + (size_t)nqmax * 8);        // nqmax
  int *piv = dn + nqmax;                                             // kmax
  int *rs = piv + kmax;                                              // kmax (sorted rank of step i)
  const size_t vb_off = ((size_t)nqmax * 12 + (size_t)kmax * 8 + 15) & ~size_t(15);
  S *vb = reinterpret_cast<S *>(lb0 + vb_off);       // m (reflector) when vlds, then T buffers
  unsigned *cnt = bar + bl;
  unsigned seq = 0;
  double *cv = cval + (int64_t)bl * 2 * kCoopMaxG;
  int *cc = ccol + (int64_t)bl * 2 * kCoopMaxG;
  double *ct = ctau_g + (int64_t)bl * 2;

  for (int q = wave; q < nq; q += NW) {
    const S *col = M + (int64_t)(g + q * G) * m;
    double sum = 0.0;
    for (int i = lane; i < m; i += 64) sum += abs2(col[i]);
    sum = wave_sum(sum);
    if (lane == 0) {
      nrm[q] = sqrt(sum);
      dn[q] = 0;
    }
  }
  __syncthreads();
  int k = kmax;
  double r00 = 0.0;
  bool aborted = false;
  for (int j = 0; j < kmax; ++j) {
    const int par = j & 1;
    if (wave == 0) {           // this workgroup's offer: largest norm, lowest column
      double lb = -1.0;
      int lc = INT_MAX;
      for (int q = lane; q < nq; q += 64) {
        if (dn[q]) continue;
        const double v = nrm[q];
        const int c = g + q * G;
        if (v > lb || (v == lb && c < lc)) { lb = v; lc = c; }
      }
      const ArgMax a = wave_argmax(lb, lc, lc);
      if (lane == 0) {
        cv[par * kCoopMaxG + g] = a.v;
        cc[par * kCoopMaxG + g] = a.key;
      }
    }
    if (!coop_barrier(cnt, ++seq * (unsigned)G, abort_flag, &s_ok)) { aborted = true; break; }
    if (wave == 0) {
      const double v = lane < G ? cv[par * kCoopMaxG + lane] : -1.0;
      const int c = lane < G ? cc[par * kCoopMaxG + lane] : INT_MAX;
      const ArgMax a = wave_argmax(v, c, c);
      if (lane == 0) { s_best = a.v; s_p = a.key; }
    }
    __syncthreads();
    const double best = s_best;
    const int p = s_p;
    if (j == 0) r00 = best;
    if (best == 0.0 || best <= eps * r00) { k = j; break; }
    if (threadIdx.x == 0) piv[j] = p;
    if (p % G == g && wave == 0) {     // owner: reflector of column p, rows j..m-1
      S *cp = M + (int64_t)p * m;
      double sum = 0.0;
      for (int i = j + lane; i < m; i += 64) sum += abs2(cp[i]);
      sum = wave_sum(sum);
      const double alpha = sqrt(sum);
      const S x0 = cp[j];
      const double beta = re_part(x0) >= 0.0 ? -alpha : alpha;
      const S scale = recip(x0 - S(beta));
      for (int i = j + 1 + lane; i < m; i += 64) cp[i] = cp[i] * scale;
      if (lane == 0) {
        const S ctau = conjg(sdiv(S(beta) - x0, beta));
        ct[0] = re_part(ctau);
        if constexpr (sizeof(S) != sizeof(double)) ct[1] = reinterpret_cast<const double *>(&ctau)[1];
        cp[j] = S(beta);
        dn[(p - g) / G] = 1;
      }
    }
    if (!coop_barrier(cnt, ++seq * (unsigned)G, abort_flag, &s_ok)) { aborted = true; break; }
    S ctau;
    if constexpr (sizeof(S) == sizeof(double)) {
      ctau = ct[0];
    } else {
      reinterpret_cast<double *>(&ctau)[0] = ct[0];
      reinterpret_cast<double *>(&ctau)[1] = ct[1];
    }
    const S *vg = M + (int64_t)p * m;
    if (vlds) {
      for (int i = j + threadIdx.x; i < m; i += kCoopThreads) vb[i] = i == j ? S(1.0) : vg[i];
      __syncthreads();
    }
    auto vload = [&](int i) -> S { return vlds ? vb[i] : (i == j ? S(1.0) : vg[i]); };
    for (int q = wave; q < nq; q += NW) {
      if (dn[q]) continue;
      S *col = M + (int64_t)(g + q * G) * m;
      S dot = S(0.0);
      for (int i0 = j; i0 < m; i0 += 256) {
        S xv[4], vv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 + lane + 64 * u;
          xv[u] = i < m ? col[i] : S(0.0);
          vv[u] = i < m ? vload(i) : S(0.0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) dot += conjg(vv[u]) * xv[u];
      }
      dot = wave_sum(dot) * ctau;
      double ns = 0.0;
      for (int i0 = j; i0 < m; i0 += 256) {
        S xv[4], vv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 + lane + 64 * u;
          xv[u] = i < m ? col[i] : S(0.0);
          vv[u] = i < m ? vload(i) : S(0.0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 + lane + 64 * u;
          if (i < m) {
            const S nv = xv[u] - dot * vv[u];
            col[i] = nv;
            if (i > j) ns += abs2(nv);
          }
        }
      }
      ns = wave_sum(ns);
      if (lane == 0) nrm[q] = sqrt(ns);
    }
    __syncthreads();
  }
  if (aborted) {
    if (g == 0 && threadIdx.x == 0) ranks[B.kslot] = -1;
    return;
  }
  if (threadIdx.x == 0) s_k = k;
  __syncthreads();
  k = s_k;
  // sorted position of each skeleton (pivot step i) among the skeletons
  for (int i = threadIdx.x; i < k; i += kCoopThreads) {
    const int pc = piv[i];
    int r = 0;
    for (int l = 0; l < k; ++l) r += piv[l] < pc;
    rs[i] = r;
  }
  __syncthreads();
  int32_t *order = order_pool + B.order_off;
  S *T = reinterpret_cast<S *>(B.T);
  for (int i = threadIdx.x; i < k; i += kCoopThreads)
    if (piv[i] % G == g) order[rs[i]] = piv[i];
  // T = R11^{-1} R12 for this workgroup's redundant columns, one column per wave; the
  // column is solved in the wave's share of the LDS after the reflector buffer
  S *buf = vb + (int64_t)wave * kmax;
  for (int q = wave; q < nq; q += NW) {
    if (dn[q]) continue;
    const int c = g + q * G;
    // redundant rank: columns below c that are not skeletons
    int below = 0;
    for (int l = lane; l < k; l += 64) below += piv[l] < c;
    for (int off = 32; off > 0; off >>= 1) below += __shfl_xor(below, off, 64);
    const int rr = c - below;
    if (lane == 0) order[k + rr] = c;
    const S *col = M + (int64_t)c * m;
    for (int i = lane; i < k; i += 64) buf[i] = col[i];
    wave_sync();
    for (int i = k - 1; i >= 0; --i) {
      const S *ri = M + (int64_t)piv[i] * m;        // R11 column i: rows 0..i
      const S xi = sdiv(buf[i], ri[i]);
      for (int l = lane; l < i; l += 64) buf[l] -= xi * ri[l];
      wave_sync();
      if (lane == 0) buf[i] = xi;
      wave_sync();
    }
    S *Tc = T + (int64_t)k * rr;
    for (int i = lane; i < k; i += 64) Tc[rs[i]] = buf[i];
    wave_sync();
  }
  if (g == 0 && threadIdx.x == 0) ranks[B.kslot] = k;
}


// One non-pivot row of a panel step: A(i, c) <- A(i, c) - f prow[c] (c != jj) and
// A(i, jj) <- -f inv with f = A(i, jj).  The row's entries and those of prow are loaded
// in groups (8 real, 4 complex) before any store, so the loads are in flight together.
template <class S>
__device__ __forceinline__ void gj_row_update(S *row, int ldp, int pb, int jj, S inv,
                                              const S *prow) {
  constexpr int G = sizeof(S) == sizeof(double) ? 8 : 4;
  const S f = row[jj * ldp];
#pragma unroll
  for (int h = 0; h < kPB; h += G) {
    S v[G], pv[G];
#pragma unroll
    for (int c = 0; c < G; ++c) {
      v[c] = h + c < pb ? row[(h + c) * ldp] : S(0.0);
      pv[c] = h + c < pb ? prow[h + c] : S(0.0);
    }
#pragma unroll
    for (int c = 0; c < G; ++c)
      if (h + c < pb) row[(h + c) * ldp] = h + c == jj ? S(0.0) - f * inv : v[c] - f * pv[c];
  }
}

// All rows i = i0, i0 + stride, ... < r of one panel step: the pivot row pr becomes
// prow, every other row gets gj_row_update's values.  Full panels (pb = kPB) take a
// branch-free path: each group of a row's entries is loaded together with the matching
// entries of prow before any store (a store to a row could alias prow, so a prow read
// after a store would wait for it: one LDS round trip per entry).
template <class S>
__device__ __forceinline__ void gj_step_rows(S *PN, int ldp, int r, int i0, int stride, int pr,
                                             int pb, int jj, S inv, const S *prow) {
  if (pb == kPB) {
    constexpr int G = sizeof(S) == sizeof(double) ? kPB / 2 : kPB / 4;
    for (int i = i0; i < r; i += stride) {
      S *row = PN + i;
      if (i == pr) {
#pragma unroll
        for (int c = 0; c < kPB; ++c) row[c * ldp] = prow[c];
      } else {
        const S f = row[jj * ldp];
        const S fj = S(0.0) - f * inv;
#pragma unroll
        for (int h = 0; h < kPB; h += G) {
          S v[G], pv[G];
#pragma unroll
          for (int c = 0; c < G; ++c) {
            v[c] = row[(h + c) * ldp];
            pv[c] = prow[h + c];
          }
#pragma unroll
          for (int c = 0; c < G; ++c) {
            const S u = v[c] - f * pv[c];
            row[(h + c) * ldp] = h + c == jj ? fj : u;
          }
        }
      }
    }
    return;
  }
  for (int i = i0; i < r; i += stride) {
    S *row = PN + i;
    if (i == pr) {
      for (int c = 0; c < pb; ++c) row[c * ldp] = prow[c];
    } else {
      gj_row_update<S>(row, ldp, pb, jj, inv, prow);
    }
  }
}

template <class S, int NTH>
__device__ __forceinline__ bool gj_blocked(S *__restrict__ A, int lda, int r,
                                           S *__restrict__ G, char *lds,
                                           S *__restrict__ pn_work, bool a_in_lds) {
  constexpr int NW = NTH / 64;
  static_assert(NW <= 64, "one lane per wave in the combine");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool pn_lds = !a_in_lds && (size_t)r * kPB * sizeof(S) <= gj_panel_lds_max<S>();
  char *p = lds;
  S *PNl = reinterpret_cast<S *>(p);                              // panel copy in LDS, ld = r
  if (!a_in_lds) p += std::min((size_t)r * kPB * sizeof(S), gj_panel_lds_max<S>());
  S *Wt = reinterpret_cast<S *>(p);                               // kPB x kQC
  p += (size_t)kPB * kQC * sizeof(S);
  S *prow = reinterpret_cast<S *>(p);                             // kPB
  p += (size_t)kPB * sizeof(S);
  double *red_v = reinterpret_cast<double *>(p);
  p += (size_t)NW * sizeof(double);
  int *red_i = reinterpret_cast<int *>(p);
  p += (size_t)NW * sizeof(int);
  int *piv = reinterpret_cast<int *>(p);                          // r
  int *qinv = piv + r;                                            // r
  int *ustep = qinv + r;                                          // r: step that used row
  int *s_fail = ustep + r;

  // Steps p0 .. p0 + pb - 1 on the panel PN (ld ldp; in LDS when pn_on_chip).  Returns
  // false on a bad pivot (uniform over the workgroup).
  // Real data: panels of at most NTH rows are held in registers (complex rows would
  // need twice the registers; they keep the LDS paths).
  constexpr bool kRegPanel = sizeof(S) == sizeof(double);
  auto panel = [&](S *PN, int ldp, int p0, int pb, bool pn_on_chip) -> bool {
    if (kRegPanel && r <= NTH) {
      // One panel row per thread, held in registers through the pb steps: per step a
      // block-wide argmax (two barriers) and a register update of every row, the same
      // operations as gj_step_rows.
      const int i = tid;
      const bool own = i < r;
      S rowv[kPB];
#pragma unroll
      for (int c = 0; c < kPB; ++c) rowv[c] = (own && c < pb) ? PN[i + c * ldp] : S(0.0);
      bool used = !own || ustep[i] >= 0;
      for (int jj = 0; jj < pb; ++jj) {
        const int j = p0 + jj;
        S x = rowv[0];
#pragma unroll
        for (int c = 1; c < kPB; ++c)
          if (c == jj) x = rowv[c];
        const double mv = mag(x);
        const bool cand = !used && mv > -1.0;          // NaN rows are never chosen
        const ArgMax am = wave_argmax(cand ? mv : -1.0, cand ? i : INT_MAX, 0);
        if (lane == 0) { red_v[wave] = am.v; red_i[wave] = am.key; }
        __syncthreads();
        const ArgMax g = wave_argmax(lane < NW ? red_v[lane] : -1.0,
                                     lane < NW ? red_i[lane] : INT_MAX, 0);
        if (!(g.v > 0.0) || !isfinite(g.v)) return false;
        const int pr = g.key;
        if (i == pr) {
          const S inv = recip(x);
#pragma unroll
          for (int c = 0; c < kPB; ++c)
            if (c < pb) prow[c] = c == jj ? inv : rowv[c] * inv;
          ustep[pr] = j;
          piv[j] = pr;
          used = true;
        }
        __syncthreads();
        if (i == pr) {
#pragma unroll
          for (int c = 0; c < kPB; ++c)
            if (c < pb) rowv[c] = prow[c];
        } else if (own) {
          const S inv = prow[jj];
          const S fj = S(0.0) - x * inv;
#pragma unroll
          for (int c = 0; c < kPB; ++c)
            if (c < pb) rowv[c] = c == jj ? fj : rowv[c] - x * prow[c];
        }
      }
      if (own) {
#pragma unroll
        for (int c = 0; c < kPB; ++c)
          if (c < pb) PN[i + c * ldp] = rowv[c];
      }
      __syncthreads();
      return true;
    }
    if ((!kRegPanel || NTH < kWavePanelMaxR) && r <= kWavePanelMaxR && pn_on_chip) {
      if (wave == 0) {
        for (int jj = 0; jj < pb; ++jj) {
          const int j = p0 + jj;
          double lb = -1.0;
          int li = INT_MAX;
          // rows in groups of 4 per lane, loaded before they are compared (r <= 512)
          for (int i0 = lane; i0 < r; i0 += 256) {
            int us[4];
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int i = i0 + 64 * u;
              us[u] = i < r ? ustep[i] : 0;
              v[u] = i < r ? mag(PN[i + jj * ldp]) : -1.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int i = i0 + 64 * u;
              if (us[u] < 0 && (v[u] > lb || (v[u] == lb && i < li))) { lb = v[u]; li = i; }
            }
          }
          const ArgMax am = wave_argmax(lb, li, li);
          if (!(am.v > 0.0) || !isfinite(am.v)) {
            if (lane == 0) *s_fail = 1;
            break;
          }
          const int pr = am.key;
          const S inv = recip(PN[pr + jj * ldp]);
          if (lane < pb) prow[lane] = lane == jj ? inv : PN[pr + lane * ldp] * inv;
          wave_sync();                 // the scaled pivot row is complete and visible
          gj_step_rows<S>(PN, ldp, r, lane, 64, pr, pb, jj, inv, prow);
          if (lane == 0) {
            ustep[pr] = j;
            piv[j] = pr;
          }
          wave_sync();
        }
      }
      __syncthreads();
      return *s_fail == 0;
    }
    for (int jj = 0; jj < pb; ++jj) {
      const int j = p0 + jj;
      double lb = -1.0;
      int li = INT_MAX;
      for (int i = tid; i < r; i += NTH) {
        if (ustep[i] >= 0) continue;
        const double v = mag(PN[i + jj * ldp]);
        if (v > lb || (v == lb && i < li)) { lb = v; li = i; }
      }
      const ArgMax am = wave_argmax(lb, li, li);
      if (lane == 0) { red_v[wave] = am.v; red_i[wave] = am.key; }
      __syncthreads();
      // every wave combines the per-wave winners (uniform result, no broadcast needed)
      const ArgMax g = wave_argmax(lane < NW ? red_v[lane] : -1.0, lane < NW ? red_i[lane] : INT_MAX, 0);
      if (!(g.v > 0.0) || !isfinite(g.v)) return false;
      const int pr = g.key;
      if (wave == 0) {     // scaled pivot row (old values) into LDS, lanes in parallel
        const S inv = recip(PN[pr + jj * ldp]);
        if (lane < pb) prow[lane] = lane == jj ? inv : PN[pr + lane * ldp] * inv;
        if (lane == 0) {
          ustep[pr] = j;
          piv[j] = pr;
        }
      }
      __syncthreads();
      const S inv = prow[jj];
      gj_step_rows<S>(PN, ldp, r, tid, NTH, pr, pb, jj, inv, prow);
      __syncthreads();
    }
    return true;
  };

  // Deferred update of every column outside the panel, kQC columns at a time.
  auto update = [&](const S *PN, int ldp, int p0, int pb) {
    for (int q0 = 0; q0 < r; q0 += kQC) {
      const int qc = min(kQC, r - q0);
      for (int sidx = wave; sidx < pb; sidx += NW) {
        const int prw = piv[p0 + sidx];
        for (int c = lane; c < qc; c += 64) {
          const int q = q0 + c;
          Wt[sidx * kQC + c] = (q >= p0 && q < p0 + pb) ? S(0.0) : A[q * lda + prw];
        }
      }
      __syncthreads();
      const int tr = (r + 15) >> 4, tq = (qc + 15) >> 4;
      const int ci = lane & 15, kq = lane >> 4;
      for (int tile = wave; tile < tr * tq; tile += NW) {
        const int ti = tile / tq, tc = tile - ti * tq;
        const int i = ti * 16 + ci;
        const int cc = tc * 16 + ci;
        const int q = q0 + cc;
        const bool colok = cc < qc && !(q >= p0 && q < p0 + pb);
        // the tile's current values are loaded before the products, so their latency
        // overlaps the MFMA steps
        S cur[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = ti * 16 + kq + 4 * v;
          cur[v] = (colok && row < r) ? A[q * lda + row] : S(0.0);
        }
        Acc<S> acc;
        if (sizeof(S) == sizeof(double) && pb == kPB) {   // real full panel: the four
                                                           // steps' operands first
          S av[4], bv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int kk = 4 * u + kq;
            av[u] = i < r ? PN[i + kk * ldp] : S(0.0);
            bv[u] = cc < qc ? Wt[kk * kQC + cc] : S(0.0);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) acc.mma(av[u], bv[u]);
        } else {
          for (int k0 = 0; k0 < pb; k0 += 4) {
            const int kk = k0 + kq;
            const S av = (i < r && kk < pb) ? PN[i + kk * ldp] : S(0.0);
            const S bv = (kk < pb && cc < qc) ? Wt[kk * kQC + cc] : S(0.0);
            acc.mma(av, bv);
          }
        }
        if (colok) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = ti * 16 + kq + 4 * v;
            if (row < r) {
              const int us = ustep[row];
              A[q * lda + row] = ((us >= p0 && us < p0 + pb) ? S(0.0) : cur[v]) + acc.get(v);
            }
          }
        }
      }
      __syncthreads();
    }
  };

  // One panel through a copy PN (ld r): copy in, steps, write back, update.
  auto via_copy = [&](S *PN, int p0, int pb, bool pn_on_chip) -> bool {
    for (int c = wave; c < pb; c += NW) {
      const S *Ac = A + (p0 + c) * lda;
      for (int i = lane; i < r; i += 64) PN[i + c * r] = Ac[i];
    }
    __syncthreads();
    if (!panel(PN, r, p0, pb, pn_on_chip)) return false;
    for (int c = wave; c < pb; c += NW) {
      S *Ac = A + (p0 + c) * lda;
      for (int i = lane; i < r; i += 64) Ac[i] = PN[i + c * r];
    }
    update(PN, r, p0, pb);
    return true;
  };

  for (int i = tid; i < r; i += NTH) ustep[i] = -1;
  if (tid == 0) *s_fail = 0;
  __syncthreads();
  for (int p0 = 0; p0 < r; p0 += kPB) {
    const int pb = min(kPB, r - p0);
    if (a_in_lds) {            // in place
      if (!panel(A + p0 * lda, lda, p0, pb, true)) return false;
      update(A + p0 * lda, lda, p0, pb);
    } else if (pn_lds) {
      if (!via_copy(PNl, p0, pb, true)) return false;
    } else {
      if (!via_copy(pn_work, p0, pb, false)) return false;
    }
  }
  for (int j = tid; j < r; j += NTH) qinv[piv[j]] = j;
  __syncthreads();
  for (int b = wave; b < r; b += NW) {
    const S *col = A + qinv[b] * lda;
    for (int a = lane; a < r; a += 64) G[b * r + a] = col[piv[a]];
  }
  __syncthreads();
  return true;
}

// --------------------------------------------------------------------------
// Unblocked Gauss-Jordan inversion with partial pivoting held in registers (real
// blocks of up to RS * 64 rows and NW * CPL columns; the box inversions of Section 3.4).
// Lane l of wave w holds rows s * 64 + l (s < RS) of columns cc * NW + w (cc < CPL).
// Rows are kept unscaled: the array holds S(i, c) = A_j(i, c) d_i, where A_j is the
// matrix after j steps and d_i = 1 until row i is a pivot, then the pivot value that
// eliminated it.  Step j: the wave owning column j picks the pivot row p among the
// unused rows (largest magnitude, ties to the lowest row; a NaN is never chosen) and
// publishes the column and 1 / S(p, j) in LDS (two buffers, so one barrier per step
// suffices); with x_i = S(i, j) / S(p, j) for i != p and x_p = 0 every wave then applies
//   S(i, c) <- S(i, c) - x_i S(p, c)   (c != j),   S(i, j) <- -x_i,   S(p, j) <- 1,
// the row of p reaching each wave through LDS.  The entry S(p, j) is held as S(p, j) - 1
// (only later steps update it; nothing reads it), so that column j takes the common
// update from zeroed registers.  At the end A^{-1}(ustep[i], piv[c]) = S(i, c) / d_i
// (ustep[i]: the step at which row i was the pivot).  Each element sees the
// same operations in every layout, so the result depends on the block alone.  The
// inverse is written to G (ld r) and, when Ginv is given, to Ginv (ld ldi); A is read at
// the start only, so Ginv may alias it.  Returns false (uniformly) on a zero or
// non-finite pivot.  LDS: gj_regs_lds(RS, NW, CPL, r) bytes.
__host__ __device__ constexpr size_t gj_regs_lds(int rs, int nw, int cpl, int r) {
  return (size_t)(2 * (rs * 64 + 1) + nw * cpl + r) * sizeof(double) +
         (size_t)(4 + 2 * r) * sizeof(int);
}
static_assert(gj_regs_lds(4, 8, (kGjRegRootMax + 7) / 8, kGjRegRootMax) <=
                  (size_t)kPB * kQC * sizeof(double),
              "the register inversion fits the LDS reserved for the blocked one");

template <int NTH, int RS, int CPL>
__device__ __forceinline__ bool gj_regs(const double *A, int lda, int r,
                                        double *__restrict__ G, double *Ginv, int ldi,
                                        char *lds) {
  constexpr int NW = NTH / 64;
  constexpr int CB = RS * 64 + 1;              // doubles per column buffer (column, 1/pivot)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double *colbuf = reinterpret_cast<double *>(lds);
  double *prw = colbuf + 2 * CB + wave * CPL;  // this wave's columns of the pivot row
  double *rinv = colbuf + 2 * CB + NW * CPL;   // 1 / d_i per row
  int *pv = reinterpret_cast<int *>(rinv + r);  // pivot row per buffer (-1: failed)
  int *piv = pv + 4;                            // pivot row of each step
  int *ustep = piv + r;                         // step of each row (-1: not yet a pivot)
  double a[RS][CPL];
#pragma unroll
  for (int s = 0; s < RS; ++s)
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
      const int i = s * 64 + lane, c = cc * NW + wave;
      a[s][cc] = (i < r && c < r) ? A[(int64_t)c * lda + i] : 0.0;
    }
  for (int i = threadIdx.x; i < r; i += NTH) ustep[i] = -1;
  // Column j reaches its owner through LDS: column 0 from the start, column j + 1 from
  // the wave that applies step j to it (so no register is indexed by j).
  if (wave == 0) {
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      colbuf[s * 64 + lane] = a[s][0];
      a[s][0] = 0.0;
    }
  }
  __syncthreads();
  for (int j = 0; j < r; ++j) {
    double *col = colbuf + (j & 1) * CB;
    if (wave == j % NW) {
      double x[RS];
      double lb = -1.0;
      int li = INT_MAX;
#pragma unroll
      for (int s = 0; s < RS; ++s) {
        x[s] = col[s * 64 + lane];
        const int i = s * 64 + lane;
        const double v = fabs(x[s]);
        if (i < r && ustep[i] < 0 && v > lb) { lb = v; li = i; }
      }
      const ArgMax am = wave_argmax(lb, li, li);
      const bool ok = am.v > 0.0 && isfinite(am.v);
      const int p = ok ? am.key : 0;
      double xp = x[0];
#pragma unroll
      for (int s = 1; s < RS; ++s)
        if ((p >> 6) == s) xp = x[s];
      const double inv = recip(readlane_f64(xp, p & 63));
      if (lane == 0) {
        col[RS * 64] = inv;
        pv[j & 1] = ok ? p : -1;
        piv[j] = p;
        ustep[p] = j;
        rinv[p] = inv;
      }
    }
    __syncthreads();
    const int p = pv[j & 1];
    if (p < 0) return false;
    const double inv = col[RS * 64];
    double xi[RS];
#pragma unroll
    for (int s = 0; s < RS; ++s) xi[s] = s * 64 + lane == p ? 0.0 : col[s * 64 + lane] * inv;
    // the pivot row's values of this wave's columns, from the lane that holds them (its
    // slot p / 64 a constant of each copy of the branch); column j, whose registers
    // were cleared when it went to LDS, takes the value 1, so that the common update
    // below leaves -x_i in it and 0 in row p (the entry S(p, j) - 1)
    const int jc = j % NW == wave ? j / NW : -1;
    const int jn = (j + 1) % NW == wave && j + 1 < r ? (j + 1) / NW : -1;
#pragma unroll
    for (int ps = 0; ps < RS; ++ps)
      if ((p >> 6) == ps && lane == (p & 63)) {
#pragma unroll
        for (int c2 = 0; c2 < CPL; ++c2) prw[c2] = a[ps][c2];
      }
    if (jc >= 0 && lane == 0) prw[jc] = 1.0;
    wave_sync();
    // one branch-free pass over the columns in groups of GC, the pivot-row values of the
    // next group read from LDS while the current group is updated (two groups in
    // registers)
    constexpr int GC = CPL > 8 ? 5 : CPL, NG = (CPL + GC - 1) / GC;
    double vb[2][GC];
#pragma unroll
    for (int u = 0; u < GC; ++u) vb[0][u] = u < CPL ? prw[u] : 0.0;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      if (g + 1 < NG) {
#pragma unroll
        for (int u = 0; u < GC; ++u)
          vb[(g + 1) & 1][u] = (g + 1) * GC + u < CPL ? prw[(g + 1) * GC + u] : 0.0;
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < GC; ++u) {
        const int c2 = g * GC + u;
        if (c2 < CPL) {
#pragma unroll
          for (int s = 0; s < RS; ++s) a[s][c2] = a[s][c2] - xi[s] * vb[g & 1][u];
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // every updated value is complete here (keeps the products out of the branches below)
#pragma unroll
    for (int s = 0; s < RS; ++s)
#pragma unroll
      for (int c2 = 0; c2 < CPL; ++c2) asm volatile("" : "+v"(a[s][c2]));
    // column j + 1 to its owner, its registers cleared
    double *nxt = colbuf + ((j + 1) & 1) * CB;
#pragma unroll
    for (int c2 = 0; c2 < CPL; ++c2)
      if (c2 == jn) {
#pragma unroll
        for (int s = 0; s < RS; ++s) {
          nxt[s * 64 + lane] = a[s][c2];
          a[s][c2] = 0.0;
        }
      }
  }
  __syncthreads();                   // piv, ustep and rinv complete
  int us[RS];
  double dinv[RS];
#pragma unroll
  for (int s = 0; s < RS; ++s) {
    const int i = min(s * 64 + lane, r - 1);
    us[s] = ustep[i];
    dinv[s] = rinv[i];
  }
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) {
    const int c = cc * NW + wave;
    if (c >= r) continue;
    const int b = piv[c];
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      const int i = s * 64 + lane;
      if (i < r) {
        const double g = (c == us[s] ? a[s][cc] + 1.0 : a[s][cc]) * dinv[s];
        G[(int64_t)b * r + us[s]] = g;
        if (Ginv) Ginv[(int64_t)b * ldi + us[s]] = g;
      }
    }
  }
  __syncthreads();
  return true;
}

// --------------------------------------------------------------------------
// Small dense products of a box factorization with FP64 MFMA tiles (16 x 16 per wave,
// the full K loop in k order): out(i, j) = c0(i, j) - sum_l a(i, l) b(l, j) when
// subtract (c0 defaults to out's current value), else the plain product.  Each output
// element is read and written by one lane only, so out may overlap c0 element-wise.
template <class S, int NW, class FA, class FB, class FO>
__device__ __forceinline__ void block_gemm(int M, int N, int K, FA a, FB b, FO out,
                                           bool subtract) {
  block_gemm<S, NW>(M, N, K, a, b, out, subtract, [&](int i, int j) { return out(i, j); });
}

template <class S, int NW, class FA, class FB, class FO, class FC>
__device__ __forceinline__ void block_gemm(int M, int N, int K, FA a, FB b, FO out,
                                           bool subtract, FC c0) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, ci = lane & 15, kq = lane >> 4;
  const int tn = (N + 15) >> 4, nt = ((M + 15) >> 4) * tn;
  for (int tile = wave; tile < nt; tile += NW) {
    const int ti = tile / tn, tj = tile - ti * tn;
    const int i = ti * 16 + ci, j = tj * 16 + ci;
    Acc<S> acc;
    int k0 = 0;
    if constexpr (sizeof(S) == sizeof(double)) {
      // real data: four K steps' operands loaded before their products (same order)
      for (; k0 + 16 <= K; k0 += 16) {
        S av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int kk = k0 + 4 * u + kq;
          av[u] = i < M ? a(i, kk) : S(0.0);
          bv[u] = j < N ? b(kk, j) : S(0.0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc.mma(av[u], bv[u]);
      }
    }
    for (; k0 < K; k0 += 4) {
      const int kk = k0 + kq;
      const S av = (i < M && kk < K) ? a(i, kk) : S(0.0);
      const S bv = (kk < K && j < N) ? b(kk, j) : S(0.0);
      acc.mma(av, bv);
    }
    if (j < N) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = ti * 16 + kq + 4 * v;
        if (row < M) {
          S &o = out(row, j);
          o = subtract ? c0(row, j) - acc.get(v) : acc.get(v);
        }
      }
    }
  }
}

// --------------------------------------------------------------------------
// Diagonal block and box factorization (Section 3.4 in Schur form).
// With the box's DOFs ordered (s, r), X = P D Q where P = [[I, 0], [-T^T, I]] and
// Q = [[I, -T], [0, I]] remove the skeleton-interpolated part; then
//   G = X_rr^{-1},  F = G X_rs,  E = X_sr G,  Lambda = X_ss - X_sr F,
// and Lambda = (R D^{-1} L)^{-1} is the box's block of the next level's matrix.
// (T^T is the plain transpose also for complex data: the row and column IDs share T.)
// D is A(J, J) at a leaf; above, Lambda of each child on its diagonal block and
// A between siblings.  The root (force_k0) eliminates everything: G = D^{-1}.
// X_rr is inverted in place by Gauss-Jordan elimination with partial pivoting (row
// interchanges, undone as column interchanges at the end).  INLDS: the whole n x n
// block lives in LDS (small boxes); otherwise in the global workspace.
// Index loops are two-level (waves over columns, lanes over rows): no integer division.
template <class S, int NTH, bool INLDS>
__global__ __launch_bounds__(NTH, 4) void k_diag_factor(const FacBox *__restrict__ boxes, int first,
                                                     const ProbDev *__restrict__ probs,
                                                     const int32_t *__restrict__ pool,
                                                     const int32_t *__restrict__ order_pool,
                                                     const int32_t *__restrict__ ranks,
                                                     S *__restrict__ workbase,
                                                     int32_t *__restrict__ err, int err_base) {
  constexpr int NW = NTH / 64;
  extern __shared__ double sh_raw[];
  S *sh = reinterpret_cast<S *>(sh_raw);
  const FacBox &B = boxes[first + blockIdx.x];
  const ProbDev &P = probs[B.prob];
  const int n = B.n;
  if (n == 0) return;
  // roots factored by the wide-root or register-root launches
  if (B.force_k0 && (n >= kWideRootMinN || root_in_regs(sizeof(S) != sizeof(double), n))) return;
  const int k = B.force_k0 ? 0 : ranks[B.kslot];
  if (k < 0 || k > n) {            // the box's ID did not complete: nothing to factor
    if (threadIdx.x == 0)
      atomicMin(reinterpret_cast<unsigned int *>(err), (unsigned int)(err_base + first + (int)blockIdx.x));
    return;
  }
  const int r = n - k;
  const int32_t *J = pool + B.J_off;
  const int32_t *ord = B.force_k0 ? nullptr : order_pool + B.order_off;
  S *slot = reinterpret_cast<S *>(B.slot);
  const S *T = slot + slot_T(k, r);
  S *X = INLDS ? sh : workbase + B.work_off;                 // n x n, (s, r) order
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  // D in (s, r) order.  Real data: a lane takes its rows four at a time; their indices,
  // child and target point are loaded once and reused for every column of the wave, and
  // the four entries of a column are formed before they are stored.  Complex data (whose
  // kernel is an out-of-line call) takes one entry at a time.  Either way each entry is
  // entry()'s value, or the child's Lambda entry.
  if constexpr (sizeof(S) != sizeof(double)) {
    for (int b = wave; b < n; b += NW) {
      const int lj = ord ? ord[b] : b;
      int cb = 0;
      if (!B.leaf)
        for (int c = 1; c < B.nchild; ++c) cb += lj >= B.child_lo[c];
      S *Xb = X + (int64_t)b * n;
      for (int a = lane; a < n; a += 64) {
        const int li = ord ? ord[a] : a;
        S v;
        if (B.leaf) {
          v = entry<S>(P, J[li], J[lj]);
        } else {
          int ca = 0;
          for (int c = 1; c < B.nchild; ++c) ca += li >= B.child_lo[c];
          if (ca == cb) {
            v = reinterpret_cast<const S *>(B.child_lam[ca])[(li - B.child_lo[ca]) +
                (int64_t)B.child_k[ca] * (lj - B.child_lo[ca])];
          } else {
            v = entry<S>(P, J[li], J[lj]);
          }
        }
        Xb[a] = v;
      }
    }
  } else
  for (int a0 = lane; a0 < n; a0 += 256) {
    int li[4], gi[4], ca[4];
    double tx[4][3];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int a = min(a0 + 64 * u, n - 1);
      li[u] = ord ? ord[a] : a;
      gi[u] = J[li[u]];
      ca[u] = 0;
      if (!B.leaf)
        for (int c = 1; c < B.nchild; ++c) ca[u] += li[u] >= B.child_lo[c];
      load_pt(P, gi[u], tx[u]);
    }
    for (int b = wave; b < n; b += NW) {
      const int lj = ord ? ord[b] : b;
      int cb = 0;
      if (!B.leaf)
        for (int c = 1; c < B.nchild; ++c) cb += lj >= B.child_lo[c];
      const int gj = J[lj];
      double sx[3], ns[3];
      load_pt(P, gj, sx);
      load_nrm(P, gj, ns);
      const double wj = P.w[gj];
      S v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (!B.leaf && ca[u] == cb) {
          v[u] = reinterpret_cast<const S *>(B.child_lam[cb])[(li[u] - B.child_lo[cb]) +
                 (int64_t)B.child_k[cb] * (lj - B.child_lo[cb])];
        } else if (gi[u] == gj) {
          v[u] = diag_entry<S>(P, gj);
        } else {
          v[u] = kernel_val<S>(P, tx[u], sx, ns) * wj;
        }
      }
      S *Xb = X + (int64_t)b * n;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (a0 + 64 * u < n) Xb[a0 + 64 * u] = v[u];
    }
  }
  __syncthreads();
  if (k > 0 && r > 0) {
    // Y = D Q: redundant columns minus the skeleton columns times T (n x r).
    block_gemm<S, NW>(n, r, k, [&](int a, int i) { return X[i * n + a]; },
                      [&](int i, int jr) { return T[i + k * jr]; },
                      [&](int a, int jr) -> S & { return X[(k + jr) * n + a]; }, true);
    __syncthreads();
    // X = P Y: redundant rows minus T^T times the skeleton rows (r x n).
    block_gemm<S, NW>(r, n, k, [&](int jr, int i) { return T[i + k * jr]; },
                      [&](int i, int b) { return X[b * n + i]; },
                      [&](int jr, int b) -> S & { return X[b * n + k + jr]; }, true);
    __syncthreads();
  }
  // Inversion of A = X_rr, A(i, c) = X[(k + c) n + k + i], into G (blocked
  // Gauss-Jordan).  With the block in LDS the inverse is copied back over A, so the
  // products below read it from LDS.
  S *A = X + (int64_t)k * n + k;
  S *G = slot + slot_G(k, r);
  const S *Gi = G;                 // the inverse as the products below read it
  int ldg = r;
  if (r > 0) {
    char *gl = INLDS ? reinterpret_cast<char *>(sh + (int64_t)n * n) : reinterpret_cast<char *>(sh_raw);
    // Real blocks of up to 64 unknowns are inverted in registers, larger ones by the
    // blocked elimination.  The choice depends on r alone, so a box's arithmetic is the
    // same in every variant and launch mode.
    bool ok, in_regs = false;
    if constexpr (sizeof(S) == sizeof(double)) {
      double *gd = reinterpret_cast<double *>(G);
      double *ad = INLDS ? reinterpret_cast<double *>(A) : nullptr;
      if (r <= 64) {
        ok = gj_regs<NTH, 1, 64 / NW>(reinterpret_cast<const double *>(A), n, r, gd, ad, n, gl);
        in_regs = true;
      }
    }
    if (!in_regs) ok = gj_blocked<S, NTH>(A, n, r, G, gl, workbase + B.work_off + (int64_t)n * n, INLDS);
    if (!ok) {
      if (threadIdx.x == 0) atomicMin(reinterpret_cast<unsigned int *>(err),
                                      (unsigned int)(err_base + first + (int)blockIdx.x));
      return;
    }
    if (INLDS) {
      if (!in_regs) {
        for (int c = wave; c < r; c += NW)
          for (int a = lane; a < r; a += 64) A[(int64_t)c * n + a] = G[(int64_t)c * r + a];
        __syncthreads();
      }
      Gi = A;
      ldg = n;
    }
  }
  if (k == 0) return;
  S *E = slot + slot_E(k, r);
  S *F = slot + slot_F(k, r);
  S *L = slot + slot_L(k, r);
  // F = G X_rs (r x k); X_rs(l, i) = X[i n + k + l]
  block_gemm<S, NW>(r, k, r, [&](int a, int l) { return Gi[l * ldg + a]; },
                    [&](int l, int i) { return X[i * n + k + l]; },
                    [&](int a, int i) -> S & { return F[i * r + a]; }, false);
  // E = X_sr G (k x r); X_sr(i, l) = X[(k + l) n + i]
  block_gemm<S, NW>(k, r, r, [&](int i, int l) { return X[(k + l) * n + i]; },
                    [&](int l, int a) { return Gi[a * ldg + l]; },
                    [&](int i, int a) -> S & { return E[a * k + i]; }, false);
  __syncthreads();
  // Lambda = X_ss - X_sr F (k x k)
  block_gemm<S, NW>(k, k, r, [&](int i, int a) { return X[(k + a) * n + i]; },
                    [&](int a, int i2) { return F[i2 * r + a]; },
                    [&](int i, int i2) -> S & { return L[i2 * k + i]; }, true,
                    [&](int i, int i2) { return X[i2 * n + i]; });
}

// --------------------------------------------------------------------------
// Solve sweeps.  W is the tree-ordered right-hand side / solution, row-major
// (n x nrhs): the values of DOF g are W[g*nrhs .. g*nrhs+nrhs).  A box reads and
// writes only its own DOFs; a parent reads its children's skeleton outputs in place.
//
// Up (finest level first):  t = b_r - T^T b_s;  b_r <- G t;  b_s <- b_s - E t.
// Down (root side first):   u = y_r - F z_s;   b_r <- u;     b_s <- z_s - T u.
// ---------------------------------------------------------------------------------
// Large roots across the GPU (the dense root block of Section 3.4, eq.
// (multilevel-inverse), when it has kWideRootMinN unknowns or more): the block is
// assembled by many workgroups, then inverted by the blocked Gauss-Jordan elimination of
// gj_blocked spread over launches -- per panel of kPB columns one workgroup runs the
// panel's pivot steps on those columns (partial pivoting over the unused rows, ties to
// the lowest row), copies the panel's pivot rows, and a launch of many workgroups
// applies the panel's rank-kPB update to every other column with FP64 MFMA tiles:
//   A(i, q) <- [i not a pivot of the panel] A(i, q) + P(i, :) W(:, q).
// At the end G(a, b) = A(piv[a], ustep[b]) (ustep is the inverse permutation of piv).
// A zero or non-finite pivot sets the root's failure flag and the error index; every
// later launch of the root sees the flag and does nothing.
constexpr int kWidePanelThreads = 1024;

// Entry (a, b) of a factored box's diagonal block D in its local order (the order ord,
// or the active-set order when ord is null): a child's Lambda inside a child, else A.
template <class S>
__device__ __forceinline__ S fac_entry(const FacBox &B, const ProbDev &P, const int32_t *J,
                                       const int32_t *ord, int a, int b) {
  const int li = ord ? ord[a] : a, lj = ord ? ord[b] : b;
  if (!B.leaf) {
    int ca = 0, cb = 0;
    for (int c = 1; c < B.nchild; ++c) {
      ca += li >= B.child_lo[c];
      cb += lj >= B.child_lo[c];
    }
    if (ca == cb)
      return reinterpret_cast<const S *>(B.child_lam[ca])[(li - B.child_lo[ca]) +
                                                          (int64_t)B.child_k[ca] * (lj - B.child_lo[ca])];
  }
  return entry<S>(P, J[li], J[lj]);
}

// Root block (k = 0) into the box's workspace, column-major n x n: grid.x column groups
// of 16, 256 threads over the rows.
template <class S>
__global__ __launch_bounds__(kThreads) void k_root_assemble(const FacBox *__restrict__ box,
                                                            const ProbDev *__restrict__ probs,
                                                            const int32_t *__restrict__ pool,
                                                            S *__restrict__ workbase) {
  const FacBox &B = *box;
  const ProbDev &P = probs[B.prob];
  const int n = B.n;
  const int32_t *J = pool + B.J_off;
  S *X = workbase + B.work_off;
  const int b0 = blockIdx.x * 16;
  for (int bb = 0; bb < 16; ++bb) {
    const int b = b0 + bb;
    if (b >= n) break;
    for (int a = threadIdx.x; a < n; a += kThreads) X[(int64_t)b * n + a] = fac_entry<S>(B, P, J, nullptr, a, b);
  }
}

// Real roots of kRegRootMinN .. kGjRegRootMax unknowns: the block assembled in the
// workspace by k_root_assemble is inverted in the registers of one 512-thread workgroup
// (two waves per SIMD, up to 256 registers each), G = D^{-1} in the root's slot.
template <int RS, int CPL>
__global__ __launch_bounds__(512, 1) void k_root_regs(const double *__restrict__ X, int n,
                                                       double *__restrict__ G,
                                                       int32_t *__restrict__ err, int err_idx) {
  extern __shared__ double sh_raw[];
  if (!gj_regs<512, RS, CPL>(X, n, n, G, nullptr, 0, reinterpret_cast<char *>(sh_raw)) &&
      threadIdx.x == 0)
    atomicMin(reinterpret_cast<unsigned int *>(err), (unsigned int)err_idx);
}

// Control block of a wide root: piv[r], ustep[r] (rows), fail flag.
struct WideCtl {
  int *piv;
  int *ustep;
  int *fail;
};

template <class S>
__global__ __launch_bounds__(kWidePanelThreads) void k_gj_wide_panel(
    S *__restrict__ A, int lda, int r, int p0, int pb, WideCtl ctl, S *__restrict__ W,
    int32_t *__restrict__ err, int err_idx) {
  constexpr int NTH = kWidePanelThreads, NW = NTH / 64;
  __shared__ S prow[kPB];
  __shared__ double red_v[NW];
  __shared__ int red_i[NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (*ctl.fail) return;
  for (int jj = 0; jj < pb; ++jj) {
    const int j = p0 + jj;
    double lb = -1.0;
    int li = INT_MAX;
    for (int i = tid; i < r; i += NTH) {
      if (ctl.ustep[i] >= 0) continue;
      const double v = mag(A[(int64_t)j * lda + i]);
      if (v > lb || (v == lb && i < li)) { lb = v; li = i; }
    }
    const ArgMax am = wave_argmax(lb, li, li);
    if (lane == 0) { red_v[wave] = am.v; red_i[wave] = am.key; }
    __syncthreads();
    const ArgMax gm = wave_argmax(lane < NW ? red_v[lane] : -1.0, lane < NW ? red_i[lane] : INT_MAX, 0);
    if (!(gm.v > 0.0) || !isfinite(gm.v)) {
      if (tid == 0) {
        *ctl.fail = 1;
        atomicMin(reinterpret_cast<unsigned int *>(err), (unsigned int)err_idx);
      }
      return;
    }
    const int pr = gm.key;
    if (wave == 0) {
      const S inv = recip(A[(int64_t)j * lda + pr]);
      if (lane < pb) prow[lane] = lane == jj ? inv : A[(int64_t)(p0 + lane) * lda + pr] * inv;
      if (lane == 0) {
        ctl.ustep[pr] = j;
        ctl.piv[j] = pr;
      }
    }
    __syncthreads();
    const S inv = prow[jj];
    for (int i = tid; i < r; i += NTH) {
      S *row = A + (int64_t)p0 * lda + i;
      if (i == pr) {
        for (int c = 0; c < pb; ++c) row[(int64_t)c * lda] = prow[c];
      } else {
        const S f = row[(int64_t)jj * lda];
        for (int c = 0; c < pb; ++c) {
          const S v = row[(int64_t)c * lda];
          row[(int64_t)c * lda] = c == jj ? S(0.0) - f * inv : v - f * prow[c];
        }
      }
    }
    __syncthreads();
  }
  // the panel's pivot rows outside the panel, before the update: W(s, q), ld kPB
  for (int e = tid; e < pb * r; e += NTH) {
    const int sidx = e % pb, q = e / pb;
    W[(int64_t)q * kPB + sidx] = (q >= p0 && q < p0 + pb) ? S(0.0)
                                                          : A[(int64_t)q * lda + ctl.piv[p0 + sidx]];
  }
}

// Rank-pb update of every column outside the panel: 64 x 64 tiles, wave w takes rows
// 16 w .. 16 w + 15 of the tile and its four 16 x 16 column tiles.
template <class S>
__global__ __launch_bounds__(kThreads) void k_gj_wide_update(S *__restrict__ A, int lda, int r,
                                                             int p0, int pb, WideCtl ctl,
                                                             const S *__restrict__ W) {
  if (*ctl.fail) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i0 = blockIdx.x * 64 + wave * 16, q0 = blockIdx.y * 64;
  const int li = lane & 15, lk = lane >> 4;
  const int ia = i0 + li;
  for (int t = 0; t < 4; ++t) {
    const int qt = q0 + 16 * t;
    if (qt >= r) break;
    Acc<S> acc;
#pragma unroll
    for (int k0 = 0; k0 < kPB; k0 += 4) {
      const int kk = k0 + lk;
      const S a = (ia < r && kk < pb) ? A[(int64_t)(p0 + kk) * lda + ia] : S(0.0);
      const int qb = qt + li;
      const S b = (qb < r && kk < pb) ? W[(int64_t)qb * kPB + kk] : S(0.0);
      acc.mma(a, b);
    }
    const int q = qt + li;
    if (q >= r || (q >= p0 && q < p0 + pb)) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + lk + 4 * v;
      if (i >= r) continue;
      const int us = ctl.ustep[i];
      const bool pivrow = us >= p0 && us < p0 + pb;
      S *pa = A + (int64_t)q * lda + i;
      *pa = (pivrow ? S(0.0) : *pa) + acc.get(v);
    }
  }
}

// G(a, b) = A(piv[a], ustep[b]), G column-major r x r.
template <class S>
__global__ __launch_bounds__(kThreads) void k_gj_wide_finish(const S *__restrict__ A, int lda,
                                                             int r, WideCtl ctl, S *__restrict__ G) {
  if (*ctl.fail) return;
  const int b = blockIdx.y;
  const int a = blockIdx.x * kThreads + threadIdx.x;
  if (a >= r) return;
  G[(int64_t)b * r + a] = A[(int64_t)ctl.ustep[b] * lda + ctl.piv[a]];
}

template <class S>
struct SweepOps {
  const S *T, *G, *E, *F;
  __device__ __forceinline__ explicit SweepOps(const SweepBox &B)
      : T(reinterpret_cast<const S *>(B.T)), G(reinterpret_cast<const S *>(B.G)),
        E(reinterpret_cast<const S *>(B.E)), F(reinterpret_cast<const S *>(B.F)) {}
};

// ---- FP64 MFMA sweeps (boxes with n <= the MFMA class limit) -----------------------
// Every 16 x 16 output tile is produced by one wave with the full K loop, so the
// arithmetic of a column does not depend on how many columns share the launch.
// acc += A(r0 + i, kk) * Bs(kk, c0 + j) over kk in [0, K); A(i, kk) = a(i, kk) for
// i < M (zero beyond), Bs row-major with leading dimension ldb (LDS).
template <class S, class AF>
__device__ __forceinline__ Acc<S> tile_gemm(AF a, const S *Bs, int ldb, int K, int M, int r0,
                                            int c0) {
  const int lane = threadIdx.x & 63, i = lane & 15, kq = lane >> 4;
  Acc<S> acc;
  const bool rowok = r0 + i < M;
  int k0 = 0;
  // four K steps' operands are loaded before their products (the same products in the
  // same order), so the operand loads are in flight together
  for (; k0 + 16 <= K; k0 += 16) {
    S av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = k0 + 4 * u + kq;
      av[u] = rowok ? a(r0 + i, kk) : S(0.0);
      bv[u] = Bs[kk * ldb + c0 + i];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc.mma(av[u], bv[u]);
  }
  for (; k0 < K; k0 += 4) {
    const int kk = k0 + kq;
    const bool kok = kk < K;
    const S av = (rowok && kok) ? a(r0 + i, kk) : S(0.0);
    const S bv = kok ? Bs[kk * ldb + c0 + i] : S(0.0);
    acc.mma(av, bv);
  }
  return acc;
}

// The box's rows of W (columns col0 .. col0 + nt, zero beyond) into LDS, row-major with
// NT columns; four elements per thread are loaded before they are stored.
template <class S, int NT>
__device__ __forceinline__ void sweep_gather(const S *__restrict__ W, int nrhs, int col0, int nt,
                                             const int32_t *idx, int rows, S *sh) {
  const int total = rows * NT;
  for (int e0 = threadIdx.x; e0 < total; e0 += 4 * kThreads) {
    S v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * kThreads;
      const int i = e / NT, c = e - i * NT;
      v[u] = (e < total && c < nt) ? W[(int64_t)idx[i] * nrhs + col0 + c] : S(0.0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * kThreads;
      if (e < total) sh[e] = v[u];
    }
  }
}

template <class S, int NT>
__device__ __forceinline__ void sweep_up_box_mfma(const SweepBox &B, S *__restrict__ W, int nrhs,
                                                  int col0, S *sh) {
  constexpr int TN = NT / 16;
  const int k = B.k, r = B.r;
  const int nt = min(NT, nrhs - col0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, kq = lane >> 4, cj = lane & 15;
  const SweepOps<S> O(B);
  S *bs = sh;              // k x NT
  S *t = sh + k * NT;      // r x NT
  const int32_t *idx = B.idx;
  sweep_gather<S, NT>(W, nrhs, col0, nt, idx, k + r, sh);
  __syncthreads();
  const S *T = O.T;
  const int tm_r = (r + 15) >> 4, tm_k = (k + 15) >> 4;
  if (k > 0) {   // t = b_r - T^T b_s
    for (int tile = wave; tile < tm_r * TN; tile += kWaves) {
      const int tm = tile / TN, tn = tile - tm * TN;
      const Acc<S> acc = tile_gemm<S>([&](int i, int kk) { return T[kk + (int64_t)k * i]; }, bs,
                                      NT, k, r, tm * 16, tn * 16);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = tm * 16 + kq + 4 * v;
        if (row < r) t[row * NT + tn * 16 + cj] -= acc.get(v);
      }
    }
    __syncthreads();
  }
  const S *G = O.G;
  for (int tile = wave; tile < tm_r * TN; tile += kWaves) {   // b_r <- G t
    const int tm = tile / TN, tn = tile - tm * TN;
    const Acc<S> acc = tile_gemm<S>([&](int i, int l) { return G[i + (int64_t)r * l]; }, t, NT,
                                    r, r, tm * 16, tn * 16);
    const int c = tn * 16 + cj;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = tm * 16 + kq + 4 * v;
      if (row < r && c < nt) W[(int64_t)idx[k + row] * nrhs + col0 + c] = acc.get(v);
    }
  }
  const S *E = O.E;
  for (int tile = wave; tile < tm_k * TN; tile += kWaves) {   // b_s <- b_s - E t
    const int tm = tile / TN, tn = tile - tm * TN;
    const Acc<S> acc = tile_gemm<S>([&](int i, int l) { return E[i + (int64_t)k * l]; }, t, NT,
                                    r, k, tm * 16, tn * 16);
    const int c = tn * 16 + cj;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = tm * 16 + kq + 4 * v;
      if (row < k && c < nt)
        W[(int64_t)idx[row] * nrhs + col0 + c] = bs[row * NT + c] - acc.get(v);
    }
  }
}

template <class S, int NT>
__device__ __forceinline__ void sweep_down_box_mfma(const SweepBox &B, S *__restrict__ W,
                                                    int nrhs, int col0, S *sh) {
  constexpr int TN = NT / 16;
  const int k = B.k, r = B.r;
  const int nt = min(NT, nrhs - col0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, kq = lane >> 4, cj = lane & 15;
  const SweepOps<S> O(B);
  S *z = sh;              // k x NT
  S *u = sh + k * NT;     // r x NT
  const int32_t *idx = B.idx;
  sweep_gather<S, NT>(W, nrhs, col0, nt, idx, k + r, sh);
  __syncthreads();
  const int tm_r = (r + 15) >> 4, tm_k = (k + 15) >> 4;
  const S *F = O.F;
  for (int tile = wave; tile < tm_r * TN; tile += kWaves) {   // u = y_r - F z
    const int tm = tile / TN, tn = tile - tm * TN;
    const Acc<S> acc = tile_gemm<S>([&](int j, int i) { return F[j + (int64_t)r * i]; }, z, NT,
                                    k, r, tm * 16, tn * 16);
    const int c = tn * 16 + cj;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = tm * 16 + kq + 4 * v;
      if (row < r) {
        const S val = u[row * NT + c] - acc.get(v);
        u[row * NT + c] = val;
        if (c < nt) W[(int64_t)idx[k + row] * nrhs + col0 + c] = val;
      }
    }
  }
  __syncthreads();
  const S *T = O.T;
  for (int tile = wave; tile < tm_k * TN; tile += kWaves) {   // x_s = z - T u
    const int tm = tile / TN, tn = tile - tm * TN;
    const Acc<S> acc = tile_gemm<S>([&](int i, int j) { return T[i + (int64_t)k * j]; }, u, NT,
                                    r, k, tm * 16, tn * 16);
    const int c = tn * 16 + cj;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = tm * 16 + kq + 4 * v;
      if (row < k && c < nt)
        W[(int64_t)idx[row] * nrhs + col0 + c] = z[row * NT + c] - acc.get(v);
    }
  }
}

template <class S, int NT>
__global__ __launch_bounds__(kThreads) void k_sweep_up_mfma(const SweepBox *__restrict__ boxes,
                                                            int first, S *__restrict__ W,
                                                            int nrhs) {
  extern __shared__ double sh_raw[];
  const SweepBox &B = boxes[first + blockIdx.x];
  if (B.r == 0) return;
  sweep_up_box_mfma<S, NT>(B, W, nrhs, blockIdx.y * NT, reinterpret_cast<S *>(sh_raw));
}

template <class S, int NT>
__global__ __launch_bounds__(kThreads) void k_sweep_down_mfma(const SweepBox *__restrict__ boxes,
                                                              int first, S *__restrict__ W,
                                                              int nrhs) {
  extern __shared__ double sh_raw[];
  const SweepBox &B = boxes[first + blockIdx.x];
  if (B.r == 0 || B.k == 0) return;
  sweep_down_box_mfma<S, NT>(B, W, nrhs, blockIdx.y * NT, reinterpret_cast<S *>(sh_raw));
}


// ---- wide boxes: row-tiled GEMMs over many workgroups ------------------------------
// A box above the MFMA sweep class is applied as a short chain of products, each spread
// over many workgroups: its rows of W are first gathered into a per-box scratch b
// (n x nrhs, row-major, skeleton rows first), then
//   up:   t = b_r - T^T b_s -> s1;  W_r <- G t;  W_s <- b_s - E t
//   down: u = b_r - F b_s -> s1 and W_r;  W_s <- b_s - T u
// Every output entry is one wave's full-length dot product in a fixed order, so results
// depend on the box alone, never on the launch.
enum WideStage { kWideUp1 = 0, kWideUp2, kWideUp3, kWideDn1, kWideDn2 };

template <class S>
__global__ void k_wide_gather(const SweepBox *__restrict__ boxes, const S *__restrict__ W,
                              int nrhs, S *__restrict__ s0, int64_t stride0) {
  const SweepBox bx = boxes[blockIdx.y];
  const int64_t total = (int64_t)(bx.k + bx.r) * nrhs;
  S *dst = s0 + blockIdx.y * stride0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / nrhs;
    const int c = (int)(e - i * nrhs);
    dst[e] = W[(int64_t)bx.idx[i] * nrhs + c];
  }
}

// blockIdx.x = box * rt + row tile (16 rows), blockIdx.y = column block (16 CT columns).
// The four waves of a workgroup take fixed quarters of the box's K range (a function of
// K alone), each accumulating its 16 x 16 CT partial tile in k order with FP64 MFMA; the
// partials meet in LDS and are summed in wave order.  A column's arithmetic is therefore
// the same for every CT, nrhs and launch.
template <class S, int STAGE, int CT>
__global__ __launch_bounds__(kThreads) void k_wide_gemm(const SweepBox *__restrict__ boxes, int rt,
                                                        S *__restrict__ W, int nrhs, S *s0,
                                                        int64_t stride0, S *s1, int64_t stride1) {
  constexpr int LD = 16 * CT + 1;                         // padded row of a partial tile
  __shared__ double part_raw[kWaves * 16 * LD * (sizeof(S) / 8)];
  S *part = reinterpret_cast<S *>(part_raw);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, ci = lane & 15, kq = lane >> 4;
  const int b = blockIdx.x / rt;
  const int r0 = (blockIdx.x - b * rt) * 16, cb = blockIdx.y * 16 * CT;
  const SweepBox bx = boxes[b];
  const int k = bx.k, r = bx.r;
  const int N = nrhs;
  S *bs = s0 + b * stride0;
  S *br = bs + (int64_t)k * N;
  S *sb1 = s1 + b * stride1;
  // out(i, c) = C0(i, c) - sum_l A(i, l) Bm(l, c)  (plain product for the G stage)
  int M, K;
  const S *A, *Bm, *C0;
  int64_t sa_i, sa_l;
  S *out_s = nullptr;
  const int32_t *oidx = nullptr;
  if (STAGE == kWideUp1) {
    if (k == 0) return;                                   // the G stage reads b_r directly
    M = r; K = k; A = reinterpret_cast<const S *>(bx.T); sa_i = k; sa_l = 1;
    Bm = bs; C0 = br; out_s = sb1;
  } else if (STAGE == kWideUp2) {
    M = r; K = r; A = reinterpret_cast<const S *>(bx.G); sa_i = 1; sa_l = r;
    Bm = k == 0 ? br : sb1; C0 = nullptr; oidx = bx.idx + k;
  } else if (STAGE == kWideUp3) {
    M = k; K = r; A = reinterpret_cast<const S *>(bx.E); sa_i = 1; sa_l = k;
    Bm = sb1; C0 = bs; oidx = bx.idx;
  } else if (STAGE == kWideDn1) {
    M = r; K = k; A = reinterpret_cast<const S *>(bx.F); sa_i = 1; sa_l = r;
    Bm = bs; C0 = br; out_s = sb1; oidx = bx.idx + k;
  } else {
    M = k; K = r; A = reinterpret_cast<const S *>(bx.T); sa_i = 1; sa_l = k;
    Bm = sb1; C0 = bs; oidx = bx.idx;
  }
  if (r0 >= M) return;                                    // uniform over the workgroup
  const int Kc = (K + 4 * kWaves - 1) / (4 * kWaves) * 4;
  const int kb = wave * Kc, ke = min(K, kb + Kc);
  const int i = r0 + ci;
  const bool iok = i < M;
  Acc<S> acc[CT];
  for (int k0 = kb; k0 < ke; k0 += 16) {
    S av[4], bv[4][CT];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = k0 + 4 * u + kq;
      const bool kok = kk < ke;
      av[u] = (iok && kok) ? A[i * sa_i + kk * sa_l] : S(0.0);
#pragma unroll
      for (int t = 0; t < CT; ++t) {
        const int c = cb + 16 * t + ci;
        bv[u][t] = (kok && c < N) ? Bm[(int64_t)kk * N + c] : S(0.0);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int t = 0; t < CT; ++t) acc[t].mma(av[u], bv[u][t]);
  }
  S *pw = part + wave * 16 * LD;
#pragma unroll
  for (int t = 0; t < CT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) pw[(kq + 4 * v) * LD + 16 * t + ci] = acc[t].get(v);
  __syncthreads();
  for (int e = threadIdx.x; e < 16 * 16 * CT; e += kThreads) {
    const int row = e / (16 * CT), col = e - row * (16 * CT);
    const int gi = r0 + row, c = cb + col;
    if (gi >= M || c >= N) continue;
    const int o = row * LD + col;
    S p = part[o];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) p = p + part[w * 16 * LD + o];
    const S val = C0 ? C0[(int64_t)gi * N + c] - p : p;
    if (out_s) out_s[(int64_t)gi * N + c] = val;
    if (oidx) W[(int64_t)oidx[gi] * N + c] = val;
  }
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

template <class S, int NT, bool UP>
__global__ __launch_bounds__(kThreads) void k_sweep_seg(const SweepSeg *__restrict__ segs,
                                                        int nseg) {
  extern __shared__ double sh_raw[];
  S *sh = reinterpret_cast<S *>(sh_raw);
  const SweepSeg &Sg = segs[find_seg(segs, nseg)];
  const SweepBox &B = Sg.boxes[blockIdx.x - Sg.block0];
  const int col0 = blockIdx.y * NT;
  if (B.r == 0 || (!UP && B.k == 0) || col0 >= Sg.nrhs) return;
  S *W = reinterpret_cast<S *>(Sg.W);
  if constexpr (UP) sweep_up_box_mfma<S, NT>(B, W, Sg.nrhs, col0, sh);
  else sweep_down_box_mfma<S, NT>(B, W, Sg.nrhs, col0, sh);
}

// Tiled caller <-> tree order permutation for wide right-hand-side blocks: a tile of
// 64 tree positions x 32 columns passes through LDS, so B (column-major, caller order)
// is read or written along tree positions -- caller indices perm[i], contiguous runs on
// curves and surfaces -- and W (row-major, tree order) along its columns.
constexpr int kPermTI = 64, kPermTC = 32;

template <class S, bool TO_TREE>
__device__ __forceinline__ void permute_tiles(S *__restrict__ Bm, int64_t ldb, S *__restrict__ W,
                                              const int64_t *__restrict__ perm, int64_t n,
                                              int nrhs, S (*tile)[kPermTI + 1]) {
  const int t = threadIdx.x;                       // 256 threads
  const int64_t tiles_i = (n + kPermTI - 1) / kPermTI;
  const int tiles_c = (nrhs + kPermTC - 1) / kPermTC;
  const int64_t ntiles = tiles_i * tiles_c;
  for (int64_t tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
    const int64_t i0 = (tl / tiles_c) * kPermTI;
    const int c0 = (int)(tl % tiles_c) * kPermTC;
    // B side: consecutive threads take consecutive tree positions
    const int il = t & (kPermTI - 1), cq = t >> 6;
    const int64_t i = i0 + il;
    const int64_t g = i < n ? perm[i] : 0;
    // W side: consecutive threads take consecutive columns
    const int cl = t & (kPermTC - 1), iq = t >> 5;
    if (TO_TREE) {
#pragma unroll
      for (int r = 0; r < kPermTC / 4; ++r) {
        const int c = cq + 4 * r;
        if (i < n && c0 + c < nrhs) tile[c][il] = Bm[g + ldb * (c0 + c)];
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kPermTI / 8; ++r) {
        const int ii = iq + 8 * r;
        if (i0 + ii < n && c0 + cl < nrhs) W[(i0 + ii) * nrhs + c0 + cl] = tile[cl][ii];
      }
    } else {
#pragma unroll
      for (int r = 0; r < kPermTI / 8; ++r) {
        const int ii = iq + 8 * r;
        if (i0 + ii < n && c0 + cl < nrhs) tile[cl][ii] = W[(i0 + ii) * nrhs + c0 + cl];
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kPermTC / 4; ++r) {
        const int c = cq + 4 * r;
        if (i < n && c0 + c < nrhs) Bm[g + ldb * (c0 + c)] = tile[c][il];
      }
    }
    __syncthreads();
  }
}

template <class S, bool TO_TREE>
__global__ __launch_bounds__(256) void k_permute_tiled(S *__restrict__ B, int64_t ldb,
                                                       S *__restrict__ W,
                                                       const int64_t *__restrict__ perm,
                                                       int64_t n, int nrhs) {
  __shared__ S tile[kPermTC][kPermTI + 1];
  permute_tiles<S, TO_TREE>(B, ldb, W, perm, n, nrhs, tile);
}

template <class S, bool TO_TREE>
__global__ __launch_bounds__(256) void k_permute_seg_tiled(const PermSeg *__restrict__ segs) {
  __shared__ S tile[kPermTC][kPermTI + 1];
  const PermSeg &Pg = segs[blockIdx.y];
  permute_tiles<S, TO_TREE>(reinterpret_cast<S *>(Pg.B), Pg.ldb, reinterpret_cast<S *>(Pg.W),
                            Pg.perm, Pg.n, Pg.nrhs, tile);
}

// Caller order <-> tree order for several right-hand-side blocks (grid.y = block).
template <class S>
__global__ void k_permute_seg(const PermSeg *__restrict__ segs, int to_tree) {
  const PermSeg &Pg = segs[blockIdx.y];
  const int64_t total = Pg.n * Pg.nrhs;
  S *Bm = reinterpret_cast<S *>(Pg.B);
  S *W = reinterpret_cast<S *>(Pg.W);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / Pg.nrhs;
    const int c = (int)(e - i * Pg.nrhs);
    if (to_tree) W[e] = Bm[Pg.perm[i] + Pg.ldb * c];
    else Bm[Pg.perm[i] + Pg.ldb * c] = W[e];
  }
}

template <class S>
__global__ void k_permute_in(const S *__restrict__ B, int64_t ldb, S *__restrict__ W,
                             const int64_t *__restrict__ perm, int64_t n, int nrhs) {
  const int64_t total = n * nrhs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / nrhs;
    const int c = (int)(e - i * nrhs);
    W[e] = B[perm[i] + ldb * c];
  }
}

template <class S>
__global__ void k_permute_out(S *__restrict__ B, int64_t ldb, const S *__restrict__ W,
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

constexpr size_t kMaxLds = 160 * 1024;

// Kernels using more than 64 KiB of dynamic LDS need the limit raised first; the call
// costs a runtime round trip, so the largest value set so far is remembered per device
// and kernel and the attribute is set again only when a launch needs more.
void allow_lds(const void *kern, size_t lds) {
  if (lds <= 64 * 1024) return;
  static std::mutex mu;
  static std::map<std::pair<int, const void *>, size_t> set;
  int dev = 0;
  RS_HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  size_t &cur = set[{dev, kern}];
  if (lds <= cur) return;
  RS_HIP_CHECK(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  cur = lds;
}
// Dynamic LDS requested per workgroup.
constexpr size_t kLdsLimit = 64 * 1024;

// Runs f with a value of the scalar type of the data (double or Cplx).
template <class F>
void with_scalar(bool cplx, F &&f) {
  if (cplx) f(Cplx{});
  else f(double{});
}

// MFMA sweeps: NT in {16, 32, 64} columns per workgroup, LDS within 64 KiB (the class
// limit guarantees NT = 16 fits).
int pick_nt_mfma(int nrhs, int max_n, int es) {
  const int tuned = tune_lookup(true, es, nrhs, max_n);
  if (tuned && sweep_nt_valid(true, tuned, max_n, es)) return tuned;
  int nt = nrhs <= 16 ? 16 : nrhs <= 32 ? 32 : 64;
  while (nt > 16 && (int64_t)max_n * nt * 8 * es > 65536) nt /= 2;
  return nt;
}

template <class S, int NT>
void sweep_mfma_nt(bool up, const SweepBox *boxes, int first, int count, double *W, int nrhs,
                   int max_n, hipStream_t st) {
  dim3 grid(count, (nrhs + NT - 1) / NT);
  const size_t lds = (size_t)max_n * NT * sizeof(S);
  S *Ws = reinterpret_cast<S *>(W);
  if (up)
    hipLaunchKernelGGL((k_sweep_up_mfma<S, NT>), grid, dim3(kThreads), lds, st, boxes, first, Ws,
                       nrhs);
  else
    hipLaunchKernelGGL((k_sweep_down_mfma<S, NT>), grid, dim3(kThreads), lds, st, boxes, first,
                       Ws, nrhs);
  check_launch("k_sweep_mfma");
}

template <class S, int NT>
void sweep_seg_nt(bool up, const SweepSeg *segs, int nseg, int nblocks, int max_nrhs, int max_n,
                  hipStream_t st) {
  dim3 grid(nblocks, (max_nrhs + NT - 1) / NT);
  const size_t lds = (size_t)max_n * NT * sizeof(S);
  if (up)
    hipLaunchKernelGGL((k_sweep_seg<S, NT, true>), grid, dim3(kThreads), lds, st, segs,
                       nseg);
  else
    hipLaunchKernelGGL((k_sweep_seg<S, NT, false>), grid, dim3(kThreads), lds, st, segs,
                       nseg);
  check_launch("k_sweep_seg");
}

constexpr int kVldsMaxRows = 8192;

size_t cpqr_lds_bytes_nt(int nth, int max_n, int max_m, int es) {
  const int nw = nth / 64;
  size_t b = (size_t)max_n * sizeof(double) + (size_t)2 * max_n * sizeof(int) +
             (size_t)nw * max_n * sizeof(double) * es;
  if (max_m <= kVldsMaxRows) b += (size_t)max_m * sizeof(double) * es;
  return b;
}

template <class S, int NTH, int RT, int CB, bool VLDS>
void cpqr_variant(const CompBox *boxes, int first, int count, const ProbDev *probs,
                  double *Marena, int32_t *order_pool, int32_t *ranks, size_t lds,
                  hipStream_t st) {
  auto kern = k_cpqr_id<S, NTH, RT, CB, VLDS>;
  allow_lds((const void *)kern, lds);
  hipLaunchKernelGGL(kern, dim3(count), dim3(NTH), lds, st, boxes, first, probs,
                     reinterpret_cast<S *>(Marena), order_pool, ranks);
  check_launch("k_cpqr_id");
}

template <class S, int NTH>
void cpqr_bucket(const CompBox *boxes, int first, int count, const ProbDev *probs,
                 double *Marena, int32_t *order_pool, int32_t *ranks, int max_n, int max_m,
                 hipStream_t st) {
  constexpr int es = sizeof(S) / sizeof(double);
  const size_t lds = cpqr_lds_bytes_nt(NTH, max_n, max_m, es);
  const size_t lds_nov = cpqr_lds_bytes_nt(NTH, max_n, kVldsMaxRows + 1, es);
  if (lds_nov > kMaxLds)
    throw DeviceError("k_cpqr_id: box too large for LDS", hipErrorInvalidValue);
  // size buckets: rows held per lane (RT) and columns per wave (CB); 1024-thread
  // workgroups have half the registers per lane, and complex entries twice the size,
  // so both hold fewer columns
  constexpr int CB4 = (NTH >= 1024 ? 2 : 4) / es;
  constexpr int CB8 = NTH >= 1024 ? 1 : 4 / es;
  constexpr int CB16 = (NTH >= 1024 || es == 2) ? 1 : 2;
  if (max_m <= 256 && lds <= kLdsLimit)
    cpqr_variant<S, NTH, 4, CB4, true>(boxes, first, count, probs, Marena, order_pool, ranks,
                                       lds, st);
  else if (max_m <= 512 && lds <= kLdsLimit)
    cpqr_variant<S, NTH, 8, CB8, true>(boxes, first, count, probs, Marena, order_pool, ranks,
                                       lds, st);
  else if (lds <= kLdsLimit)
    cpqr_variant<S, NTH, 16, CB16, true>(boxes, first, count, probs, Marena, order_pool, ranks,
                                         lds, st);
  else
    cpqr_variant<S, NTH, 16, CB16, false>(boxes, first, count, probs, Marena, order_pool, ranks,
                                          lds_nov, st);
}

template <class S, int NTH, bool INLDS>
void diag_factor_nt(const FacBox *boxes, int first, int count, const ProbDev *probs,
                    const int32_t *pool, const int32_t *order_pool, const int32_t *ranks,
                    double *work, int32_t *err, int err_base, size_t lds, hipStream_t st) {
  auto kern = k_diag_factor<S, NTH, INLDS>;
  allow_lds((const void *)kern, lds);
  hipLaunchKernelGGL(kern, dim3(count), dim3(NTH), lds, st, boxes, first, probs, pool,
                     order_pool, ranks, reinterpret_cast<S *>(work), err, err_base);
  check_launch("k_diag_factor");
}

}  // namespace

// ------------------------------------------------------------------ tuning table
namespace {
std::mutex g_tune_mu;
std::map<uint32_t, int> g_tune;   // bucket key -> tile width
}  // namespace

uint32_t tune_key(bool mfma, int es, int nrhs, int max_n) {
  int nb = 0;
  while ((1 << nb) < nrhs && nb < 20) ++nb;               // ceil(log2 nrhs)
  const int sb = std::min((max_n + 31) / 32, 255);        // box size in steps of 32
  return (uint32_t)(mfma ? 1 : 0) | (uint32_t)(es == 2 ? 2 : 0) | ((uint32_t)nb << 2) |
         ((uint32_t)sb << 8);
}

int tune_lookup(bool mfma, int es, int nrhs, int max_n) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_tune.empty()) return 0;
  auto it = g_tune.find(tune_key(mfma, es, nrhs, max_n));
  return it == g_tune.end() ? 0 : it->second;
}

void tune_set(uint32_t key, int nt) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = nt;
}

std::vector<std::pair<uint32_t, int>> tune_entries() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return std::vector<std::pair<uint32_t, int>>(g_tune.begin(), g_tune.end());
}

void tune_clear() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
}

bool sweep_nt_valid(bool mfma, int nt, int max_n, int es) {
  const bool allowed = mfma && (nt == 16 || nt == 32 || nt == 64);
  return allowed && (int64_t)max_n * nt * 8 * es <= 65536;
}

// ------------------------------------------------------------------ launchers

int mfma_max_n(bool cplx) { return cplx ? kMfmaMaxNComplex : kMfmaMaxN; }

int assemble_chunks(int max_n, int max_m) {
  const int64_t e = (int64_t)max_n * max_m;
  return (int)std::min<int64_t>(std::max<int64_t>((e + kThreads * 16 - 1) / (kThreads * 16), 1),
                                kAssembleMaxChunks);
}

void launch_assemble(bool cplx, const CompBox *boxes, int first, int count, const ProbDev *probs,
                     const int32_t *pool, double *Marena, int max_npx, int max_n, int max_m,
                     double *partials, hipStream_t st) {
  if (count <= 0) return;
  const int CH = assemble_chunks(max_n, max_m);
  with_scalar(cplx, [&](auto z) {
    using S = decltype(z);
    if (CH == 1) {
      hipLaunchKernelGGL(k_assemble<S>, dim3(count), dim3(kThreads),
                         (size_t)max_npx * 3 * sizeof(double), st, boxes, first, probs, pool,
                         reinterpret_cast<S *>(Marena));
      check_launch("k_assemble");
      return;
    }
    hipLaunchKernelGGL(k_assemble_chunks<S>, dim3(count * CH), dim3(kThreads),
                       (size_t)max_npx * 3 * sizeof(double), st, boxes, first, CH, probs, pool,
                       reinterpret_cast<S *>(Marena), partials);
    check_launch("k_assemble_chunks");
    hipLaunchKernelGGL(k_assemble_tail<S>, dim3(count), dim3(kThreads), 0, st, boxes, first, CH,
                       probs, pool, reinterpret_cast<S *>(Marena), partials);
    check_launch("k_assemble_tail");
  });
}

bool fused_class(bool cplx, int n, int m) { return !cplx && n <= kFusedMaxN && m <= kFusedMaxM; }

void launch_sketch(bool cplx, const CompBox *comp, const CompBox *comp_id, int first, int count,
                   const ProbDev *probs, double *Marena, int max_tiles, hipStream_t st) {
  if (count <= 0 || max_tiles <= 0) return;
  const int gy = std::min(256, (max_tiles + kWaves - 1) / kWaves);
  with_scalar(cplx, [&](auto z) {
    using S = decltype(z);
    hipLaunchKernelGGL(k_sketch<S>, dim3(count, gy), dim3(kThreads), 0, st, comp, comp_id,
                       first, probs, reinterpret_cast<S *>(Marena));
  });
  check_launch("k_sketch");
}

// Register-resident variants (threads, rows per lane, columns per wave), smallest first;
// a box takes the first whose column (NW * CPW) and row (64 RT) capacity covers it.
// Fewer waves per box mean less per-step overhead and more boxes resident per CU; the
// arithmetic of a box is the same in every variant.
bool fused_small(int n, int m) { return n <= 32 && m <= 512; }

int fused_variant_of(int n, int m) {
  if (n <= 24 && m <= 320) return 0;     // <256, 5, 6>
  if (n <= 32 && m <= 512) return 1;     // <256, 8, 8>
  if (n <= 48 && m <= 320) return 2;     // <512, 5, 6>
  if (n <= 64 && m <= 448) return 3;     // <512, 7, 8>
  return 4;                              // <512, 8, 10>
}

size_t fused_lds_bytes(int nth, int max_n, int max_m, int max_npx) {
  const int nw = nth / 64;
  const size_t max_nn = (size_t)max_m / 2;       // m >= 2 nn
  return sizeof(double) * ((size_t)3 * max_npx + max_n + max_m + (size_t)nw * max_n +
                           (size_t)fused_tile_doubles(nw, max_n, max_m) +
                           7 * ((size_t)max_n + max_nn)) +
         sizeof(int) * (size_t)3 * max_n;
}

template <int NTH, int RT, int CPW>
void fused_variant(const CompBox *boxes, int first, int count, const ProbDev *probs,
                   const int32_t *pool, int32_t *order_pool, int32_t *ranks,
                   int max_n, int max_m, int max_npx, hipStream_t st) {
  static_assert(CPW <= 32, "column mask");
  if (max_n > (NTH / 64) * CPW || max_m > 64 * RT)
    throw DeviceError("k_compress_fused: variant too small", hipErrorInvalidValue);
  const size_t lds = fused_lds_bytes(NTH, max_n, max_m, max_npx);
  if (lds > kMaxLds) throw DeviceError("k_compress_fused: LDS", hipErrorInvalidValue);
  auto kern = k_compress_fused<NTH, RT, CPW>;
  allow_lds((const void *)kern, lds);
  hipLaunchKernelGGL(kern, dim3(count), dim3(NTH), lds, st, boxes, first, probs, pool,
                     order_pool, ranks);
  check_launch("k_compress_fused");
}

void launch_compress_fused(const CompBox *boxes, int first, int count, const ProbDev *probs,
                           const int32_t *pool, int32_t *order_pool, int32_t *ranks, int max_n,
                           int max_m, int max_npx, hipStream_t st) {
  if (count <= 0) return;
  if (max_n > kFusedMaxN || max_m > kFusedMaxM)
    throw DeviceError("k_compress_fused: box outside the fused class", hipErrorInvalidValue);
  switch (fused_variant_of(max_n, max_m)) {
    case 0:
      fused_variant<256, 5, 6>(boxes, first, count, probs, pool, order_pool, ranks, max_n,
                               max_m, max_npx, st);
      break;
    case 1:
      fused_variant<256, 8, 8>(boxes, first, count, probs, pool, order_pool, ranks, max_n,
                               max_m, max_npx, st);
      break;
    case 2:
      fused_variant<512, 5, 6>(boxes, first, count, probs, pool, order_pool, ranks, max_n,
                               max_m, max_npx, st);
      break;
    case 3:
      fused_variant<512, 7, 8>(boxes, first, count, probs, pool, order_pool, ranks, max_n,
                               max_m, max_npx, st);
      break;
    default:
      fused_variant<512, 8, 10>(boxes, first, count, probs, pool, order_pool, ranks, max_n,
                                max_m, max_npx, st);
  }
}

namespace {
int g_coop_supported = -1;     // cooperative launches available on the device (-1: unknown)
}  // namespace

bool split_class(bool cplx, int n, int m) {
  return !cplx && !fused_class(cplx, n, m) && n <= kSplitMaxN && m <= 64 * kSplitRT;
}

size_t split_lds_bytes(int max_n, int max_m, int max_npx) {
  const int nw = kSplitThreads / 64;
  const size_t max_nn = (size_t)max_m / 2;
  const size_t kmax = (size_t)std::min(max_n, max_m);
  const size_t assemble = 7 * ((size_t)max_n + max_nn) + (size_t)nw * max_m;
  return sizeof(double) * (3 * (size_t)max_npx + std::max(assemble, kmax * kmax) +
                           (size_t)nw * kSplitCPW) +
         sizeof(int) * (3 * (size_t)max_n + kmax);
}

void launch_compress_split(const CompBox *boxes, int first, int count, const ProbDev *probs,
                           const int32_t *pool, int32_t *order_pool, int32_t *ranks, int max_n,
                           int max_m, int max_npx, hipStream_t st) {
  if (count <= 0) return;
  if (max_n > kSplitMaxN || max_m > 64 * kSplitRT)
    throw DeviceError("k_compress_split: box outside the split class", hipErrorInvalidValue);
  // at least enough workgroups for the columns; more (up to kSplitWideG) when the level
  // has few boxes -- a box's arithmetic does not depend on G
  const int G = std::max(split_groups(max_n), std::min(kSplitWideG, 256 / std::max(count, 1)));
  const size_t lds = split_lds_bytes(max_n, max_m, max_npx);
  if (lds > kMaxLds) throw DeviceError("k_compress_split: LDS", hipErrorInvalidValue);
  auto kern = k_compress_split<kSplitRT, kSplitCPW>;
  allow_lds((const void *)kern, lds);
  // boxes per launch: every workgroup of a launch resident at once (the occupancy and CU
  // count are queried once per device and LDS size)
  int per_cu = 0, dev = 0, ncu = 0;
  RS_HIP_CHECK(hipGetDevice(&dev));
  {
    static std::mutex mu;
    static std::map<std::pair<int, size_t>, std::pair<int, int>> known;
    std::lock_guard<std::mutex> lock(mu);
    auto it = known.find({dev, lds});
    if (it == known.end()) {
      RS_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern,
                                                                kSplitThreads, lds));
      RS_HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
      known[{dev, lds}] = {per_cu, ncu};
    } else {
      per_cu = it->second.first;
      ncu = it->second.second;
    }
  }
  const int chunk = std::max(1, (per_cu * ncu) / G);
  if (per_cu * ncu < G)
    throw DeviceError("k_compress_split: a box's workgroups cannot be resident together",
                      hipErrorInvalidValue);
  // exchange areas (step counts zeroed) and the abort flag
  const int per_launch = std::min(count, chunk);
  const size_t xbytes = (size_t)per_launch * (size_t)split_xarea(G) * sizeof(double);
  char *mem = nullptr;
  RS_HIP_CHECK(hipMallocAsync((void **)&mem, xbytes + 256, st));
  for (int b0 = 0; b0 < count; b0 += chunk) {
    const int nb = std::min(chunk, count - b0);
    RS_HIP_CHECK(hipMemsetAsync(mem, 0, xbytes + 256, st));
    double *xb = reinterpret_cast<double *>(mem);
    int *abort_flag = reinterpret_cast<int *>(mem + xbytes);
    int f = first + b0, gg = G;
    // A plain launch: every workgroup of it fits on the chip at once (the chunk above), so
    // the workgroups of a box are all placed as soon as the work of other streams leaves
    // room, and that work never waits for this kernel.  The waits are bounded, so a box
    // whose workgroups could not all be placed would end with its rank at -1, not hang.
    // (A cooperative launch adds 25-65 us of queue synchronization before the kernel,
    // on the critical path of the top levels.)
    hipLaunchKernelGGL(kern, dim3(nb * G), dim3(kSplitThreads), lds, st, boxes, f, gg, probs,
                       pool, order_pool, ranks, xb, abort_flag);
    check_launch("k_compress_split");
  }
  RS_HIP_CHECK(hipFreeAsync(mem, st));
}

size_t cpqr_lds_bytes(bool cplx, int max_n, int max_m) {
  return cpqr_lds_bytes_nt(256, max_n, max_m, cplx ? 2 : 1);
}

namespace {
// LDS of k_cpqr_coop: norms and flags of a workgroup's columns, the pivot list and sorted
// ranks, then the reflector (when it fits) or the T solves' column buffers.
size_t coop_lds_bytes(int max_n, int max_m, int G, int es, bool vlds) {
  const int kmax = std::min(max_n, max_m);
  const int nqmax = (max_n + G - 1) / G;
  // the kernel places the buffer at the 16-byte boundary after 12 nqmax + 8 kmax bytes
  const size_t head = ((size_t)nqmax * 12 + (size_t)kmax * 8 + 15) & ~size_t(15);
  const size_t vb = std::max<size_t>(vlds ? (size_t)max_m : 0, (size_t)4 * kmax) * 8 * es;
  return head + vb;
}

void launch_cpqr_coop(bool cplx, const CompBox *boxes, int first, int count, const ProbDev *probs,
                      double *Marena, int32_t *order_pool, int32_t *ranks, int max_n, int max_m,
                      hipStream_t st) {
  const int es = cplx ? 2 : 1;
  if (g_coop_supported < 0) {
    int dev = 0, v = 0;
    RS_HIP_CHECK(hipGetDevice(&dev));
    RS_HIP_CHECK(hipDeviceGetAttribute(&v, hipDeviceAttributeCooperativeLaunch, dev));
    g_coop_supported = v ? 1 : 0;
  }
  const int nbox_al = (count + 7) / 8 * 8;
  int G = std::min(kCoopMaxG, std::max(1, 256 / nbox_al));
  G = std::min(G, std::max(1, (max_n + 3) / 4));
  if (!g_coop_supported) G = 1;
  bool vlds = coop_lds_bytes(max_n, max_m, G, es, true) <= kMaxLds;
  size_t lds = coop_lds_bytes(max_n, max_m, G, es, vlds);
  if (lds > kMaxLds) throw DeviceError("k_cpqr_coop: box too large for LDS", hipErrorInvalidValue);
  // per box: barrier counter, offers (values, columns) of both step parities, conj(tau)
  const size_t off_val = 256;
  const size_t off_col = off_val + (size_t)count * 2 * kCoopMaxG * sizeof(double);
  const size_t off_tau = off_col + (size_t)count * 2 * kCoopMaxG * sizeof(int);
  const size_t off_abort = off_tau + (size_t)count * 2 * sizeof(double);
  const size_t bytes = off_abort + 256;
  char *sync = nullptr;
  RS_HIP_CHECK(hipMallocAsync((void **)&sync, bytes + (size_t)count * sizeof(unsigned), st));
  RS_HIP_CHECK(hipMemsetAsync(sync, 0, bytes + (size_t)count * sizeof(unsigned), st));
  unsigned *bar = reinterpret_cast<unsigned *>(sync + bytes);
  double *cval = reinterpret_cast<double *>(sync + off_val);
  int *ccol = reinterpret_cast<int *>(sync + off_col);
  double *ctau = reinterpret_cast<double *>(sync + off_tau);
  int *abort_flag = reinterpret_cast<int *>(sync + off_abort);
  with_scalar(cplx, [&](auto z) {
    using S = decltype(z);
    auto kern = k_cpqr_coop<S>;
    allow_lds((const void *)kern, lds);
    S *Mp = reinterpret_cast<S *>(Marena);
    int vl = vlds ? 1 : 0;
    const dim3 grid(nbox_al * G), block(kCoopThreads);
    if (G > 1) {
      void *args[] = {(void *)&boxes, (void *)&first, (void *)&count, (void *)&nbox_al,
                      (void *)&G, (void *)&probs, (void *)&Mp, (void *)&order_pool,
                      (void *)&ranks, (void *)&bar, (void *)&cval, (void *)&ccol,
                      (void *)&ctau, (void *)&abort_flag, (void *)&vl};
      RS_HIP_CHECK(hipLaunchCooperativeKernel((const void *)kern, grid, block, args,
                                              (unsigned)lds, st));
    } else {
      // one workgroup per box: its barriers complete on its own arrivals
      hipLaunchKernelGGL(kern, grid, block, lds, st, boxes, first, count, nbox_al, G, probs, Mp,
                         order_pool, ranks, bar, cval, ccol, ctau, abort_flag, vl);
    }
    check_launch("k_cpqr_coop");
  });
  RS_HIP_CHECK(hipFreeAsync(sync, st));
}
}  // namespace

void launch_cpqr_id(bool cplx, const CompBox *boxes, int first, int count, const ProbDev *probs,
                    double *Marena, int32_t *order_pool, int32_t *ranks, int max_n, int max_m,
                    hipStream_t st) {
  if (count <= 0) return;
  const int es = cplx ? 2 : 1;
  if (coop_class(max_m, max_n))
    launch_cpqr_coop(cplx, boxes, first, count, probs, Marena, order_pool, ranks, max_n, max_m,
                     st);
  with_scalar(cplx, [&](auto z) {
    using S = decltype(z);
    // Wide levels of small boxes: 256 threads, so several boxes share a CU; a few large
    // boxes: 1024 threads, so more trailing columns are updated at once.
    if (count >= 512 && max_n <= 96)
      cpqr_bucket<S, 256>(boxes, first, count, probs, Marena, order_pool, ranks, max_n, max_m,
                          st);
    else if (count <= 64 && max_m <= 512 &&
             cpqr_lds_bytes_nt(1024, max_n, kVldsMaxRows + 1, es) <= kLdsLimit)
      cpqr_bucket<S, 1024>(boxes, first, count, probs, Marena, order_pool, ranks, max_n, max_m,
                           st);
    else
      cpqr_bucket<S, 512>(boxes, first, count, probs, Marena, order_pool, ranks, max_n, max_m,
                          st);
  });
}

// Every box gets its own n x n workspace (plus a panel of the blocked inversion): the
// variant (LDS or global) is chosen per launch from the largest box, so the smaller
// boxes of a launch need one too.
size_t diag_work_elems(int n) { return (size_t)n * n + (size_t)kPB * n; }

void launch_root_wide(bool cplx, const FacBox *box, int n, const ProbDev *probs,
                      const int32_t *pool, double *work, int64_t work_off, double *G,
                      int32_t *err, int err_idx, hipStream_t st) {
  if (n < kWideRootMinN) throw DeviceError("launch_root_wide: root below the wide class",
                                           hipErrorInvalidValue);
  int *ctl_mem = nullptr;
  RS_HIP_CHECK(hipMallocAsync((void **)&ctl_mem, (size_t)(2 * n + 1) * sizeof(int), st));
  RS_HIP_CHECK(hipMemsetAsync(ctl_mem, 0xff, (size_t)(2 * n) * sizeof(int), st));
  RS_HIP_CHECK(hipMemsetAsync(ctl_mem + 2 * n, 0, sizeof(int), st));
  WideCtl ctl{ctl_mem, ctl_mem + n, ctl_mem + 2 * n};
  with_scalar(cplx, [&](auto z) {
    using S = decltype(z);
    S *wb = reinterpret_cast<S *>(work);
    S *A = wb + work_off;
    S *W = A + (int64_t)n * n;                   // kPB x n snapshot after the block
    hipLaunchKernelGGL(k_root_assemble<S>, dim3((n + 15) / 16), dim3(kThreads), 0, st, box,
                       probs, pool, wb);
    check_launch("k_root_assemble");
    const dim3 ug((n + 63) / 64, (n + 63) / 64);
    for (int p0 = 0; p0 < n; p0 += kPB) {
      const int pb = std::min(kPB, n - p0);
      hipLaunchKernelGGL(k_gj_wide_panel<S>, dim3(1), dim3(kWidePanelThreads), 0, st, A, n, n,
                         p0, pb, ctl, W, err, err_idx);
      check_launch("k_gj_wide_panel");
      hipLaunchKernelGGL(k_gj_wide_update<S>, ug, dim3(kThreads), 0, st, A, n, n, p0, pb, ctl,
                         (const S *)W);
      check_launch("k_gj_wide_update");
    }
    hipLaunchKernelGGL(k_gj_wide_finish<S>, dim3((n + kThreads - 1) / kThreads, n), dim3(kThreads),
                       0, st, (const S *)A, n, n, ctl, reinterpret_cast<S *>(G));
    check_launch("k_gj_wide_finish");
  });
  RS_HIP_CHECK(hipFreeAsync(ctl_mem, st));
}

void launch_root_regs(const FacBox *box, int n, const ProbDev *probs, const int32_t *pool,
                      double *work, int64_t work_off, double *G, int32_t *err, int err_idx,
                      hipStream_t st) {
  if (!root_in_regs(false, n))
    throw DeviceError("launch_root_regs: root outside the register class", hipErrorInvalidValue);
  hipLaunchKernelGGL(k_root_assemble<double>, dim3((n + 15) / 16), dim3(kThreads), 0, st, box,
                     probs, pool, work);
  check_launch("k_root_assemble");
  constexpr int kRS = (kGjRegRootMax + 63) / 64, kCPL = (kGjRegRootMax + 7) / 8;
  const size_t lds = gj_regs_lds(kRS, 8, kCPL, n);
  hipLaunchKernelGGL((k_root_regs<kRS, kCPL>), dim3(1), dim3(512), lds, st, work + work_off, n,
                     G, err, err_idx);
  check_launch("k_root_regs");
}

void launch_diag_factor(bool cplx, const FacBox *boxes, int first, int count,
                        const ProbDev *probs, const int32_t *pool, const int32_t *order_pool,
                        const int32_t *ranks, double *work, int32_t *err, int err_base,
                        int max_n, hipStream_t st) {
  if (count <= 0) return;
  const size_t es = cplx ? 2 : 1;
  with_scalar(cplx, [&](auto z) {
    using S = decltype(z);
    // The whole block in LDS when n^2 scalars plus the inversion's buffers fit: up to
    // 64 KiB with 256 threads (several workgroups per CU), beyond that one 1024-thread
    // workgroup.  The arithmetic of a box is the same in every variant.
    auto lds_in = [&](int nth) {
      return (size_t)max_n * max_n * 8 * es + gj_blocked_lds<S>(max_n, nth / 64, true);
    };
    if (lds_in(256) <= kLdsLimit) {
      diag_factor_nt<S, 256, true>(boxes, first, count, probs, pool, order_pool, ranks, work,
                                   err, err_base, lds_in(256), st);
      return;
    }
    if (lds_in(1024) <= kMaxLds) {
      diag_factor_nt<S, 1024, true>(boxes, first, count, probs, pool, order_pool, ranks, work,
                                    err, err_base, lds_in(1024), st);
      return;
    }
    // Few large boxes (the root): one 1024-thread workgroup each; otherwise 256 threads.
    const int nth = count <= 64 ? 1024 : 256;
    const size_t lds = gj_blocked_lds<S>(max_n, nth / 64, false);
    if (lds > kMaxLds) throw DeviceError("k_diag_factor: box too large", hipErrorInvalidValue);
    if (nth == 1024)
      diag_factor_nt<S, 1024, false>(boxes, first, count, probs, pool, order_pool, ranks, work,
                                     err, err_base, lds, st);
    else
      diag_factor_nt<S, 256, false>(boxes, first, count, probs, pool, order_pool, ranks, work,
                                    err, err_base, lds, st);
  });
}

// Right-hand-side blocks at least this wide use the LDS-tiled permutation.
constexpr int kPermTiledMinNrhs = 8;

int perm_tiled_blocks(int64_t n, int nrhs) {
  const int64_t tiles = ((n + kPermTI - 1) / kPermTI) * ((nrhs + kPermTC - 1) / kPermTC);
  return (int)std::min<int64_t>(tiles, 4096);
}

void launch_permute_in(bool cplx, const double *B, int64_t ldb, double *W, const int64_t *perm,
                       int64_t n, int nrhs, hipStream_t st) {
  const int64_t total = n * nrhs;
  if (total == 0) return;
  if (nrhs >= kPermTiledMinNrhs) {
    with_scalar(cplx, [&](auto z) {
      using S = decltype(z);
      hipLaunchKernelGGL((k_permute_tiled<S, true>), dim3(perm_tiled_blocks(n, nrhs)), dim3(256),
                         0, st, reinterpret_cast<S *>(const_cast<double *>(B)), ldb,
                         reinterpret_cast<S *>(W), perm, n, nrhs);
    });
    check_launch("k_permute_tiled");
    return;
  }
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
  with_scalar(cplx, [&](auto z) {
    using S = decltype(z);
    hipLaunchKernelGGL(k_permute_in<S>, dim3(blocks), dim3(256), 0, st,
                       reinterpret_cast<const S *>(B), ldb, reinterpret_cast<S *>(W), perm, n,
                       nrhs);
  });
  check_launch("k_permute_in");
}

void launch_permute_out(bool cplx, double *B, int64_t ldb, const double *W, const int64_t *perm,
                        int64_t n, int nrhs, hipStream_t st) {
  const int64_t total = n * nrhs;
  if (total == 0) return;
  if (nrhs >= kPermTiledMinNrhs) {
    with_scalar(cplx, [&](auto z) {
      using S = decltype(z);
      hipLaunchKernelGGL((k_permute_tiled<S, false>), dim3(perm_tiled_blocks(n, nrhs)),
                         dim3(256), 0, st, reinterpret_cast<S *>(B), ldb,
                         reinterpret_cast<S *>(const_cast<double *>(W)), perm, n, nrhs);
    });
    check_launch("k_permute_tiled");
    return;
  }
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
  with_scalar(cplx, [&](auto z) {
    using S = decltype(z);
    hipLaunchKernelGGL(k_permute_out<S>, dim3(blocks), dim3(256), 0, st,
                       reinterpret_cast<S *>(B), ldb, reinterpret_cast<const S *>(W), perm, n,
                       nrhs);
  });
  check_launch("k_permute_out");
}

void launch_permute_seg(bool cplx, const PermSeg *segs, int nseg, int64_t max_elems,
                        int max_nrhs, bool to_tree, hipStream_t st) {
  if (nseg <= 0 || max_elems <= 0) return;
  if (max_nrhs >= kPermTiledMinNrhs) {
    const int blocks = (int)std::min<int64_t>((max_elems + kPermTI * kPermTC - 1) /
                                              (kPermTI * kPermTC), 2048);
    with_scalar(cplx, [&](auto z) {
      using S = decltype(z);
      if (to_tree)
        hipLaunchKernelGGL((k_permute_seg_tiled<S, true>), dim3(blocks, nseg), dim3(256), 0, st,
                           segs);
      else
        hipLaunchKernelGGL((k_permute_seg_tiled<S, false>), dim3(blocks, nseg), dim3(256), 0,
                           st, segs);
    });
    check_launch("k_permute_seg_tiled");
    return;
  }
  const int blocks = (int)std::min<int64_t>((max_elems + 255) / 256, 2048);
  with_scalar(cplx, [&](auto z) {
    using S = decltype(z);
    hipLaunchKernelGGL(k_permute_seg<S>, dim3(blocks, nseg), dim3(256), 0, st, segs,
                       to_tree ? 1 : 0);
  });
  check_launch("k_permute_seg");
}


int64_t wide_scratch_doubles(int count, int max_n, int max_r, int nrhs, bool cplx) {
  return (int64_t)count * ((int64_t)max_n + max_r) * nrhs * (cplx ? 2 : 1);
}

void launch_wide_level(bool cplx, bool up, const SweepBox *boxes, int count, int max_n,
                       int max_k, int max_r, double *W, int nrhs, double *scratch,
                       int64_t scratch_doubles, hipStream_t st) {
  if (count <= 0 || nrhs <= 0 || max_r <= 0) return;
  const int64_t per_box = wide_scratch_doubles(1, max_n, max_r, nrhs, cplx);
  if (scratch_doubles < per_box) throw std::runtime_error("wide sweep: scratch too small");
  const int chunk = (int)std::min<int64_t>(count, scratch_doubles / per_box);
  with_scalar(cplx, [&](auto z) {
    using S = decltype(z);
    S *Ws = reinterpret_cast<S *>(W);
    const int64_t stride0 = (int64_t)max_n * nrhs, stride1 = (int64_t)max_r * nrhs;
    for (int first = 0; first < count; first += chunk) {
      const int cnt = std::min(chunk, count - first);
      const SweepBox *bx = boxes + first;
      S *s0 = reinterpret_cast<S *>(scratch);
      S *s1 = s0 + (int64_t)cnt * stride0;
      const int gx = (int)std::min<int64_t>((stride0 + 255) / 256, 1024);
      hipLaunchKernelGGL(k_wide_gather<S>, dim3(gx, cnt), dim3(256), 0, st, bx,
                         reinterpret_cast<const S *>(Ws), nrhs, s0, stride0);
      check_launch("k_wide_gather");
      const int ct = nrhs <= 16 ? 1 : nrhs <= 32 ? 2 : 4;   // column tiles per wave
      auto stage = [&](auto tag, int max_m) {
        constexpr int ST = decltype(tag)::value;
        if (max_m <= 0) return;
        const int rt = (max_m + 15) / 16;
        const dim3 grid(rt * cnt, (nrhs + 16 * ct - 1) / (16 * ct));
        if (ct == 1)
          hipLaunchKernelGGL((k_wide_gemm<S, ST, 1>), grid, dim3(kThreads), 0, st, bx, rt, Ws,
                             nrhs, s0, stride0, s1, stride1);
        else if (ct == 2)
          hipLaunchKernelGGL((k_wide_gemm<S, ST, 2>), grid, dim3(kThreads), 0, st, bx, rt, Ws,
                             nrhs, s0, stride0, s1, stride1);
        else
          hipLaunchKernelGGL((k_wide_gemm<S, ST, 4>), grid, dim3(kThreads), 0, st, bx, rt, Ws,
                             nrhs, s0, stride0, s1, stride1);
        check_launch("k_wide_gemm");
      };
      if (up) {
        if (max_k > 0) stage(std::integral_constant<int, kWideUp1>{}, max_r);
        stage(std::integral_constant<int, kWideUp2>{}, max_r);
        stage(std::integral_constant<int, kWideUp3>{}, max_k);
      } else {
        stage(std::integral_constant<int, kWideDn1>{}, max_r);
        stage(std::integral_constant<int, kWideDn2>{}, max_k);
      }
    }
  });
}

void launch_sweep_mfma(bool cplx, bool up, const SweepBox *boxes, int first, int count,
                       double *W, int nrhs, int max_n, hipStream_t st, int nt) {
  if (count <= 0 || nrhs <= 0) return;
  if (max_n > mfma_max_n(cplx))
    throw DeviceError("k_sweep_mfma: box too large", hipErrorInvalidValue);
  with_scalar(cplx, [&](auto z) {
    using S = decltype(z);
    if (nt && !sweep_nt_valid(true, nt, max_n, sizeof(S) / 8))
      throw DeviceError("k_sweep_mfma: invalid tile width", hipErrorInvalidValue);
    switch (nt ? nt : pick_nt_mfma(nrhs, max_n, sizeof(S) / 8)) {
      case 16: sweep_mfma_nt<S, 16>(up, boxes, first, count, W, nrhs, max_n, st); break;
      case 32: sweep_mfma_nt<S, 32>(up, boxes, first, count, W, nrhs, max_n, st); break;
      default: sweep_mfma_nt<S, 64>(up, boxes, first, count, W, nrhs, max_n, st); break;
    }
  });
}

void launch_sweep_seg(bool cplx, bool up, const SweepSeg *segs, int nseg, int nblocks,
                      int max_nrhs, int max_n, hipStream_t st) {
  if (nseg <= 0 || nblocks <= 0 || max_nrhs <= 0) return;
  if (max_n > mfma_max_n(cplx))
    throw DeviceError("k_sweep_seg: box too large for the MFMA class", hipErrorInvalidValue);
  with_scalar(cplx, [&](auto z) {
    using S = decltype(z);
    constexpr int es = sizeof(S) / 8;
    switch (pick_nt_mfma(max_nrhs, max_n, es)) {
      case 16: sweep_seg_nt<S, 16>(up, segs, nseg, nblocks, max_nrhs, max_n, st); break;
      case 32: sweep_seg_nt<S, 32>(up, segs, nseg, nblocks, max_nrhs, max_n, st); break;
      default: sweep_seg_nt<S, 64>(up, segs, nseg, nblocks, max_nrhs, max_n, st); break;
    }
  });
}

// ---------------------------------------------------------------------------------
// Compressed forward operator A_eps x (Section 3.3, the two passes of the compressed
// matrix-vector product; used as a generalized FMM in Section 6.1).  Upward, finest
// level first, every box replaces its skeleton values by x_s + T x_r (the
// interpolation R_B) after keeping the level's x_s; at the root and on the way down
// every box lifts its skeleton results to its redundant DOFs (y_r = T^T y_s, the
// interpolation L_B) and adds its diagonal block of the level's matrix times the level's
// values.  The diagonal blocks are evaluated from the kernel: A(J_B, J_B) with the
// diagonal rule at a leaf; above the leaves the entries between different children
// only (a child's own block belongs to the finer level).
constexpr int kMvCols = 16;        // right-hand-side columns per workgroup

template <class S>
__global__ __launch_bounds__(kThreads) void k_mv_up(const MvBox *__restrict__ boxes,
                                                    S *__restrict__ W, int nrhs,
                                                    S *__restrict__ save) {
  const MvBox &B = boxes[blockIdx.x];
  const int k = B.k, r = B.r;
  const int a = blockIdx.y * kThreads + threadIdx.x;      // skeleton row of the box
  const int c0 = blockIdx.z * kMvCols;
  if (a >= k) return;
  const int nc = min(kMvCols, nrhs - c0);
  const S *T = reinterpret_cast<const S *>(B.T);
  const int32_t *idx = B.idx;
  S *Wa = W + (int64_t)idx[a] * nrhs + c0;
  S *sv = save + (B.save_off + a) * (int64_t)nrhs + c0;
  S acc[kMvCols];
#pragma unroll
  for (int c = 0; c < kMvCols; ++c) acc[c] = c < nc ? Wa[c] : S(0.0);
#pragma unroll
  for (int c = 0; c < kMvCols; ++c)
    if (c < nc) sv[c] = acc[c];
  for (int q = 0; q < r; ++q) {
    const S t = T[a + (int64_t)k * q];
    const S *Wq = W + (int64_t)idx[k + q] * nrhs + c0;
#pragma unroll
    for (int c = 0; c < kMvCols; ++c)
      if (c < nc) acc[c] += t * Wq[c];
  }
#pragma unroll
  for (int c = 0; c < kMvCols; ++c)
    if (c < nc) Wa[c] = acc[c];
}

template <class S>
__global__ __launch_bounds__(kThreads) void k_mv_lift(const MvBox *__restrict__ boxes,
                                                      S *__restrict__ Y, int nrhs) {
  const MvBox &B = boxes[blockIdx.x];
  const int k = B.k, r = B.r;
  const int q = blockIdx.y * kThreads + threadIdx.x;      // redundant row of the box
  const int c0 = blockIdx.z * kMvCols;
  if (q >= r) return;
  const int nc = min(kMvCols, nrhs - c0);
  const S *T = reinterpret_cast<const S *>(B.T);
  const int32_t *idx = B.idx;
  S acc[kMvCols];
#pragma unroll
  for (int c = 0; c < kMvCols; ++c) acc[c] = S(0.0);
  for (int a = 0; a < k; ++a) {
    const S t = T[a + (int64_t)k * q];
    const S *Ya = Y + (int64_t)idx[a] * nrhs + c0;
#pragma unroll
    for (int c = 0; c < kMvCols; ++c)
      if (c < nc) acc[c] += t * Ya[c];
  }
  S *Yq = Y + (int64_t)idx[k + q] * nrhs + c0;
#pragma unroll
  for (int c = 0; c < kMvCols; ++c)
    if (c < nc) Yq[c] = acc[c];
}

__device__ __forceinline__ int mv_child_of(const MvBox &B, int64_t g) {
  int c = 0;
  for (int q = 1; q < B.nchild; ++q) c += g >= B.child_begin[q];
  return c;
}

template <class S>
__global__ __launch_bounds__(kThreads) void k_mv_diag(const MvBox *__restrict__ boxes,
                                                      const ProbDev *__restrict__ probs,
                                                      const S *__restrict__ W,
                                                      const S *__restrict__ save,
                                                      S *__restrict__ Y, int nrhs) {
  const MvBox &B = boxes[blockIdx.x];
  const ProbDev &P = probs[B.prob];
  const int k = B.k, n = B.k + B.r;
  const int i = blockIdx.y * kThreads + threadIdx.x;      // local row (s, then r)
  const int c0 = blockIdx.z * kMvCols;
  if (i >= n) return;
  const int nc = min(kMvCols, nrhs - c0);
  const int32_t *idx = B.idx;
  const int gi = idx[i];
  const int ci = B.leaf ? 0 : mv_child_of(B, gi);
  double ti[3];
  load_pt(P, gi, ti);
  S acc[kMvCols];
#pragma unroll
  for (int c = 0; c < kMvCols; ++c) acc[c] = S(0.0);
  for (int j = 0; j < n; ++j) {
    const int gj = idx[j];
    if (!B.leaf && mv_child_of(B, gj) == ci) continue;
    S d;
    if (gj == gi) {
      d = diag_entry<S>(P, gi);
    } else {
      double sj[3], nj[3];
      load_pt(P, gj, sj);
      load_nrm(P, gj, nj);
      d = kernel_val<S>(P, ti, sj, nj) * P.w[gj];
    }
    const S *xj = j < k ? save + (B.save_off + j) * (int64_t)nrhs + c0
                        : W + (int64_t)gj * nrhs + c0;
#pragma unroll
    for (int c = 0; c < kMvCols; ++c)
      if (c < nc) acc[c] += d * xj[c];
  }
  S *Yi = Y + (int64_t)gi * nrhs + c0;
#pragma unroll
  for (int c = 0; c < kMvCols; ++c)
    if (c < nc) Yi[c] += acc[c];
}

namespace {
dim3 mv_grid(int count, int rows, int nrhs) {
  return dim3(count, (rows + kThreads - 1) / kThreads, (nrhs + kMvCols - 1) / kMvCols);
}
}  // namespace

void launch_mv_up(bool cplx, const MvBox *boxes, int count, int max_k, double *W, int nrhs,
                  double *save, hipStream_t st) {
  if (count <= 0 || max_k <= 0 || nrhs <= 0) return;
  with_scalar(cplx, [&](auto z) {
    using S = decltype(z);
    hipLaunchKernelGGL(k_mv_up<S>, mv_grid(count, max_k, nrhs), dim3(kThreads), 0, st, boxes,
                       reinterpret_cast<S *>(W), nrhs, reinterpret_cast<S *>(save));
  });
  check_launch("k_mv_up");
}

void launch_mv_lift(bool cplx, const MvBox *boxes, int count, int max_r, double *Y, int nrhs,
                    hipStream_t st) {
  if (count <= 0 || max_r <= 0 || nrhs <= 0) return;
  with_scalar(cplx, [&](auto z) {
    using S = decltype(z);
    hipLaunchKernelGGL(k_mv_lift<S>, mv_grid(count, max_r, nrhs), dim3(kThreads), 0, st, boxes,
                       reinterpret_cast<S *>(Y), nrhs);
  });
  check_launch("k_mv_lift");
}

void launch_mv_diag(bool cplx, const MvBox *boxes, int count, int max_n, const ProbDev *probs,
                    const double *W, const double *save, double *Y, int nrhs, hipStream_t st) {
  if (count <= 0 || max_n <= 0 || nrhs <= 0) return;
  with_scalar(cplx, [&](auto z) {
    using S = decltype(z);
    hipLaunchKernelGGL(k_mv_diag<S>, mv_grid(count, max_n, nrhs), dim3(kThreads), 0, st, boxes,
                       probs, reinterpret_cast<const S *>(W), reinterpret_cast<const S *>(save),
                       reinterpret_cast<S *>(Y), nrhs);
  });
  check_launch("k_mv_diag");
}

// ------------------------------------------------------ allocation-free solve scratch
// Device scratch of the allocation-free solve entry point: the tree-ordered workspace
// and the wide-box staging of one solve, 64 MiB per device (every device the library
// runs on holds its own copy until the process ends).  Host code never passes the
// array's name to a kernel (on the host it is a stand-in, not a device address): the
// device address comes from hipGetSymbolAddress, looked up once per device with that
// device current, and only that pointer is used afterwards.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace {
std::mutex g_scratch_mu;
std::vector<double *> g_scratch_ptr;     // per device id
}  // namespace

size_t noalloc_scratch_bytes() { return kNoAllocScratchBytes; }

double *noalloc_scratch() {
  int dev = 0;
  RS_HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    RS_HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw DeviceError("hipGetSymbolAddress returned no address for the scratch array",
                                hipErrorInvalidSymbol);
    g_scratch_ptr[dev] = static_cast<double *>(ptr);
  }
  return g_scratch_ptr[dev];
}

}  // namespace rs
