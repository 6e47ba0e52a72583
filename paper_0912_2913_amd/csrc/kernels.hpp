// Kernels of the RLB step for gfx950 (MI355X).
//
// One thread updates one cell; a 64-lane wavefront covers 64 consecutive cells
// of the x-fastest linear index, so each of the 38 pulls of a wavefront is one
// contiguous 64-element read shifted by the streaming offset, and each of the
// 38 stores is one contiguous 64-element write (SoA [pop][q][cell]).  The
// update is a streaming, bandwidth-bound stencil (about 0.5 flop per byte in
// FP64): it is not a dense contraction, so no MFMA is used.  Workgroups are
// remapped so that each XCD (own L2) works on one contiguous slab of cells,
// which keeps the cache lines shared by neighbouring workgroups (the +-1 x
// shifts) inside one L2.
//
// Physics (eqs. lbe1/lbe2, equil1s/equil2as/equil2bs, the macroscopic
// constraints closed by e = 3P), in the form evaluated here:
//   E = sum g_i, M = c_l sum g_i e_i, N = sum f_i;
//   D = sqrt(4E^2 - 3|M|^2), e = D - E, W = (e+P) gamma^2 = (2E + D)/3,
//   beta = M / W   (the rest-continuous root of 3W^2 - 4EW + |M|^2 = 0);
//   with b_i = e_i.beta / c_l and s = (3/2)|beta|^2 / c_l^2:
//   g_i^eq = w_i [ e / c_l^2 + W (3 b_i + (9/2) b_i^2 - s) ]          (i > 0)
//   g_0^eq = w_0 [ e (3 - 2/c_l^2) + W (3 |beta|^2 - s) ]
//   f_i^eq = w_i N (1 + 3 b_i)
//   S' = pre + (1/tau)(eq - pre).
// These equal the paper's equilibria on the physical manifold
// (W = (4/3) e gamma^2, e gamma^2 / (gamma^2 c_l^2) = e / c_l^2, and
// 3W - 4e = 3 W |beta|^2), without the 1/(1 - beta^2) division.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "codec.hpp"
#include "lattice.hpp"

namespace rlb {

constexpr int BLOCK = 256;
// Cell word (one uint32 per cell, when an obstacle exists): bit 0 solid,
// bit 1 near (some resolved neighbour is solid), bit CLS_BOUNCE + q set when
// the resolved pull source of direction q is solid (half-way bounce-back).
constexpr uint32_t CLS_SOLID = 1u;
constexpr uint32_t CLS_NEAR = 2u;
constexpr int CLS_BOUNCE = 8;

// Division by a runtime constant via multiply-high (valid for n < 2^31).
struct FastDiv {
  uint32_t d, m, s;
};

__device__ __forceinline__ uint32_t fdiv(const FastDiv &f, uint32_t n) {
  return (__umulhi(n, f.m) + n) >> f.s;
}

struct Geom {
  int n[3];  // nx, ny, nz
  int batch;
  int per;  // cells per instance
  int nblk_per, nblk;
  long long qs;  // elements per direction slice (cells rounded up to 64)
  FastDiv div_x, div_y, div_blk;
  int periodic[3];
  int inflow_lo[3], inflow_hi[3];
  int any_inflow;
  int off[Q];  // interior pull offsets: source = cell - off[q]
  // Index corrections of a pull that leaves the domain through the low face
  // (cell on coordinate 0, e_a = +1) or the high face (coordinate n-1,
  // e_a = -1): +-n*stride wraps a periodic axis, +-stride clamps an outflow
  // axis onto the face (zero-gradient copy), 0 on a periodic axis of one cell.
  int corr_lo[3], corr_hi[3];
};

// Values the inflow plane holds (f then g, storage format), passed by value
// so that they are read from kernel-argument memory through the scalar unit.
template <class El>
struct HeldEq {
  El v[2 * Q];
};

// Population block layout: bricks of 64 consecutive cells, each holding its
// 19 directions one after another, so element (q, cell i) lives at
//   (i / 64) * 19 * 64 + q * 64 + i % 64.
// A wavefront's 19 reads or writes of one population then fall in one
// 19 * 64-element span (for unshifted directions) instead of 19 slices one
// population-plane apart, which keeps HBM page locality; the f block is
// followed by the g block (offset 19 * qs).  qs = cells rounded up to 64.
constexpr int BRICK = 64;

// Cell indices are 32-bit (a lattice holds at most 2^31 - 64 cells); only the
// element offset is widened, by one 32 x 32 -> 64-bit multiply-add.
__device__ __forceinline__ size_t at(int q, int i) {
  return (size_t)((unsigned)i >> 6) * (unsigned)(Q * BRICK) +
         (unsigned)(q * BRICK + (i & (BRICK - 1)));
}

struct Phys {
  double c, inv_c, inv_c2, k0;  // k0 = 3 - 6 kappa / c_l^2 (3 - 2/c_l^2 for e = 3P)
  double ad_c;                  // 3 kappa / c_l^2 (1/c_l^2 for e = 3P)
  double wfac;                  // W = wfac e gamma^2, wfac = 1 + kappa
  double kappa;                 // P = kappa e
  int gen_eos;                  // kappa != 1/3
  double eos_A, eos_B, eos_C, eos_H, eos_F, eos_G;  // inversion constants (see invert)
  double n_ref, e_ref;          // zero unless the storage holds deviations
  const double *omega;          // [batch] 1/tau
  const uint32_t *cls;          // [cells] cell words, or null (no obstacle)
  const double *omega_cell;     // [cells] 1/tau(x) of a per-cell tau field, or null
  double *dtau_cell;            // [cells] reverse-sweep dL/dtau(x) accumulator, or null
  double eta_s, d_G;            // eta_s > 0: tau from the local state holds eta/s
};

// Relaxation rate of cell c from the per-cell field or its instance.
__device__ __forceinline__ double omega_of(const Phys &ph, int b, int idx) {
  return ph.omega_cell ? ph.omega_cell[idx] : ph.omega[b];
}

// Transport quantities of the shock-tube section from the fields of a cell:
// T = e / (3n), n_eq = d_G T^3 / pi^2, lambda = n / n_eq,
// s = 4n - n ln(lambda); and the viscosity relation of the equilibrium
// section, eta = (4/9) gamma^2 e (tau - dt/2) c_l^2 with tau in units of
// dt = dx / c_l, i.e. eta = (4/9) gamma^2 e c_l (tau - 1/2).
struct Transport {
  double T, s, gamma2;
};

__device__ __forceinline__ Transport transport_of(double n, double e, double b2, double d_G) {
  Transport t;
  t.T = e / (3.0 * n);
  const double n_eq = d_G * t.T * t.T * t.T * (1.0 / (M_PI * M_PI));
  t.s = n * (4.0 - log(n / n_eq));
  t.gamma2 = 1.0 / (1.0 - b2);
  return t;
}

// 1/tau holding eta/s = eta_s at (n, e, beta): the viscosity relation solved
// for tau with eta = eta_s * s.
__device__ __forceinline__ double omega_for_eta_s(const Phys &ph, double n, double e, double b2) {
  const Transport t = transport_of(n, e, b2, ph.d_G);
  const double tau = 0.5 + (9.0 / 4.0) * ph.eta_s * t.s / (t.gamma2 * e * ph.c);
  return 1.0 / tau;
}

// Inflow state for the adjoint of the held face (e_in, beta_in).
struct InflowState {
  double e, bx, by, bz;
};

struct Cell {
  int b, x, y, z, local, L;
  int idx;
  bool active;
};

// Blocks are dispatched round-robin over the 8 XCDs; give XCD k the k-th
// contiguous range of logical blocks.
__device__ __forceinline__ int xcd_remap(int B, int nblk) {
  int per = nblk >> 3, rem = nblk & 7;
  int k = B & 7, i = B >> 3;
  return k * per + min(k, rem) + i;
}

__device__ __forceinline__ Cell decode_cell(const Geom &g, int B = -1) {
  Cell c;
  c.L = xcd_remap(B < 0 ? (int)blockIdx.x : B, g.nblk);
  c.b = (int)fdiv(g.div_blk, (uint32_t)c.L);
  c.local = (c.L - c.b * g.nblk_per) * BLOCK + (int)threadIdx.x;
  c.active = c.local < g.per;
  uint32_t t = fdiv(g.div_x, (uint32_t)c.local);
  c.x = c.local - (int)t * g.n[0];
  uint32_t z = fdiv(g.div_y, t);
  c.y = (int)t - (int)z * g.n[1];
  c.z = (int)z;
  c.idx = c.b * g.per + c.local;
  return c;
}

__device__ __forceinline__ bool is_inflow(const Geom &g, int x, int y, int z) {
  if (!g.any_inflow) return false;
  return (g.inflow_lo[0] && x == 0) || (g.inflow_hi[0] && x == g.n[0] - 1) ||
         (g.inflow_lo[1] && y == 0) || (g.inflow_hi[1] && y == g.n[1] - 1) ||
         (g.inflow_lo[2] && z == 0) || (g.inflow_hi[2] && z == g.n[2] - 1);
}

// Branch-free pull sources of a cell with no solid neighbour: the per-lane
// face corrections are selected once, then each direction adds the ones its
// velocity components call for (compile-time after unrolling).
struct FaceCorr {
  int lx, hx, ly, hy, lz, hz;
};

__device__ __forceinline__ FaceCorr face_corr(const Geom &g, const Cell &c) {
  FaceCorr f;
  f.lx = c.x == 0 ? g.corr_lo[0] : 0;
  f.hx = c.x == g.n[0] - 1 ? g.corr_hi[0] : 0;
  f.ly = c.y == 0 ? g.corr_lo[1] : 0;
  f.hy = c.y == g.n[1] - 1 ? g.corr_hi[1] : 0;
  f.lz = c.z == 0 ? g.corr_lo[2] : 0;
  f.hz = c.z == g.n[2] - 1 ? g.corr_hi[2] : 0;
  return f;
}

__device__ __forceinline__ int src_fast(const Geom &g, const Cell &c, const FaceCorr &f, int q) {
  int s = c.idx - g.off[q];
  if (EX[q] == 1) s += f.lx;
  if (EX[q] == -1) s += f.hx;
  if (EY[q] == 1) s += f.ly;
  if (EY[q] == -1) s += f.hy;
  if (EZ[q] == 1) s += f.lz;
  if (EZ[q] == -1) s += f.hz;
  return s;
}

// Pull-source coordinate on one axis: wrap (periodic) or clamp (outflow).
__device__ __forceinline__ int resolve(const Geom &g, int a, int r, bool &clamped) {
  const int n = g.n[a];
  if (g.periodic[a]) {
    if (r < 0) r += n;
    if (r >= n) r -= n;
    return r;
  }
  if (r < 0) {
    clamped = true;
    return 0;
  }
  if (r >= n) {
    clamped = true;
    return n - 1;
  }
  return r;
}

__device__ __forceinline__ int cell_index(const Geom &g, int b, int x, int y, int z) {
  return b * g.per + (z * g.n[1] + y) * g.n[0] + x;
}

__device__ __forceinline__ bool solid_at(const Phys &ph, int i) {
  return ph.cls != nullptr && (ph.cls[i] & CLS_SOLID);
}

// General pull of direction q at cell c: source cell and direction
// (bounce-back off a solid source returns the cell's own opposite population).
struct Pull {
  int idx;
  int q;
  bool clamped;  // source clamped into the domain on some axis
  bool bounce;
};

__device__ __forceinline__ Pull pull_general(const Geom &g, const Phys &ph, const Cell &c, int q) {
  Pull p;
  p.clamped = false;
  int sx = resolve(g, 0, c.x - EX[q], p.clamped);
  int sy = resolve(g, 1, c.y - EY[q], p.clamped);
  int sz = resolve(g, 2, c.z - EZ[q], p.clamped);
  int s = cell_index(g, c.b, sx, sy, sz);
  p.bounce = solid_at(ph, s);
  if (p.bounce) {
    p.idx = c.idx;
    p.q = OPP[q];
  } else {
    p.idx = s;
    p.q = q;
  }
  return p;
}

// Momentum sum_i e_i v_i over mirror pairs: each direction with e_a = +1 is
// differenced with its mirror image across the plane normal to axis a before
// anything else is added.  A state symmetric under that mirror then gives
// exactly zero momentum along a.  A sequential sum over i leaves a
// rounding residual (~1e-17) whenever mirror pairs hold values of opposite
// sign.  At high shock strengths the scheme is unstable to transverse
// perturbations (1-D shock tubes at e_L/e_R = 16 amplify them ~20x per 10
// steps), so that residual alone would seed a transverse blow-up of an
// otherwise one-dimensional flow.
//
// Contraction is off here: if v_i is a product (as in the reverse step),
// fusing it into the difference would compute exact(v_i) - rounded(v_j) and
// leave that rounding error as a residual, the same seed as above.
template <class T>
__device__ __forceinline__ void mirror_sums(const T (&v)[Q], T &mx, T &my, T &mz) {
#pragma clang fp contract(off)
  mx = ((v[1] - v[2]) + (v[7] - v[10])) + ((v[9] - v[8]) + (v[11] - v[14])) + (v[13] - v[12]);
  my = ((v[3] - v[4]) + (v[7] - v[9])) + ((v[10] - v[8]) + (v[15] - v[18])) + (v[17] - v[16]);
  mz = ((v[5] - v[6]) + (v[11] - v[13])) + ((v[14] - v[12]) + (v[15] - v[17])) + (v[18] - v[16]);
}

// E = sum v_i and the mirror-pair momentum sums of v, accumulated in Sm (the
// codec's sum type: the compute type, or FP64 over FP32 values).
template <class Sm, class T>
__device__ __forceinline__ void moment_sums(const T (&v)[Q], Sm &E, Sm &mx, Sm &my, Sm &mz) {
  Sm w[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) w[q] = (Sm)v[q];
  E = (Sm)0;
#pragma unroll
  for (int q = 0; q < Q; ++q) E += w[q];
  mirror_sums(w, mx, my, mz);
}

// Result of the moment inversion (FP64).
struct Inv {
  double E, Mx, My, Mz, D, eps, W, bx, by, bz;
  bool bad;
};

__device__ __forceinline__ Inv invert(const Phys &ph, double E, double Mx, double My, double Mz) {
  Inv r;
  r.E = E;
  r.Mx = Mx;
  r.My = My;
  r.Mz = Mz;
  // W^2 - (1 + kappa) E W + kappa |M|^2 = 0 (from E = W - P, |M| = W |beta|,
  // P = kappa e), rest-continuous root, as D^2 = A E^2 - B |M|^2,
  // W = (C E + D) H, e = (D - F E) G.  For kappa = 1/3 the constants are
  // (4, 3, 2, 1/3, 1, 1): D = sqrt(4E^2 - 3|M|^2), W = (2E + D)/3, e = D - E;
  // otherwise ((1+kappa)^2, 4 kappa, 1 + kappa, 1/2, 1 - kappa, 1/(2 kappa)).
  const double D2 = ph.eos_A * E * E - ph.eos_B * (Mx * Mx + My * My + Mz * Mz);
  r.D = sqrt(D2);
  r.eps = (r.D - ph.eos_F * E) * ph.eos_G;
  r.W = (ph.eos_C * E + r.D) * ph.eos_H;
  double iW = 1.0 / r.W;
  r.bx = Mx * iW;
  r.by = My * iW;
  r.bz = Mz * iW;
  double b2 = r.bx * r.bx + r.by * r.by + r.bz * r.bz;
  r.bad = !(D2 > 0.0) || !(r.eps > 0.0) || !(b2 < 1.0);
  return r;
}

// Equilibrium coefficients of one cell in the compute type T; eq() returns
// the equilibrium minus the rest reference R (R = 0 for non-deviation
// storage).
template <class T>
struct EqCoef {
  T W, Ad, A0, bx, by, bz, s, N, Nd;
};

template <class T>
__device__ __forceinline__ EqCoef<T> eq_coef(const Phys &ph, double N, double eps, double W,
                                             double bx, double by, double bz) {
  EqCoef<T> k;
  double b2 = bx * bx + by * by + bz * bz;
  double s = 1.5 * b2 * ph.inv_c2;
  k.W = (T)W;
  k.Ad = (T)((eps - ph.e_ref) * ph.ad_c);
  k.A0 = (T)((eps - ph.e_ref) * ph.k0 + W * (3.0 * b2 - s));
  k.bx = (T)(bx * ph.inv_c);
  k.by = (T)(by * ph.inv_c);
  k.bz = (T)(bz * ph.inv_c);
  k.s = (T)s;
  k.N = (T)N;
  k.Nd = (T)(N - ph.n_ref);
  return k;
}

template <class T>
__device__ __forceinline__ T dot_e(const EqCoef<T> &k, int q) {
  // e_q . beta / c_l with e_q in {-1, 0, 1}^3 (folds to adds after unrolling)
  T r = (T)0;
  if (EX[q] == 1) r += k.bx;
  if (EX[q] == -1) r -= k.bx;
  if (EY[q] == 1) r += k.by;
  if (EY[q] == -1) r -= k.by;
  if (EZ[q] == 1) r += k.bz;
  if (EZ[q] == -1) r -= k.bz;
  return r;
}

template <class T>
__device__ __forceinline__ T geq_dev(const EqCoef<T> &k, int q) {
  if (q == 0) return (T)W0 * k.A0;
  T b = dot_e(k, q);
  return (T)WQ[q] * (k.Ad + k.W * (b * ((T)3 + (T)4.5 * b) - k.s));
}

template <class T>
__device__ __forceinline__ T feq_dev(const EqCoef<T> &k, int q) {
  if (q == 0) return (T)W0 * k.Nd;
  T b = dot_e(k, q);
  return (T)WQ[q] * (k.Nd + (T)3 * k.N * b);
}

// Moment correction of an equilibrium evaluated in a lower precision than its
// moments (the codec's sum type is FP64, its compute type FP32): the FP32
// coefficients round the equilibrium's moments away from the pre-collision
// ones by an amount that repeats step after step for a slowly varying state,
// so the relaxation would drift the conserved sums.  With the equilibrium's
// moments summed in FP64, adding w_q (dE + 3 e_q . dm) restores them
// (sum_q w_q = 1, sum_q w_q e_q = 0, sum_q w_q e_q e_q = I/3).
struct EqFix {
  float dE, dx, dy, dz;
};

template <class Sm, class T>
__device__ __forceinline__ EqFix eq_fix(const EqCoef<T> &k, Sm sE, Sm sx, Sm sy, Sm sz) {
  Sm t[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) t[q] = (Sm)geq_dev(k, q);
  Sm E = (Sm)0, mx, my, mz;
#pragma unroll
  for (int q = 0; q < Q; ++q) E += t[q];
  mirror_sums(t, mx, my, mz);
  return {(float)(sE - E), (float)(sx - mx), (float)(sy - my), (float)(sz - mz)};
}

template <class T>
__device__ __forceinline__ T geq_fixed(const EqCoef<T> &k, const EqFix &f, int q) {
  T d = (T)f.dE;
  if (EX[q] == 1) d += (T)3 * (T)f.dx;
  if (EX[q] == -1) d -= (T)3 * (T)f.dx;
  if (EY[q] == 1) d += (T)3 * (T)f.dy;
  if (EY[q] == -1) d -= (T)3 * (T)f.dy;
  if (EZ[q] == 1) d += (T)3 * (T)f.dz;
  if (EZ[q] == -1) d -= (T)3 * (T)f.dz;
  return geq_dev(k, q) + (T)WQ[q] * d;
}

// Rest reference R_q (deviation storage) in FP64.
__device__ __forceinline__ double rest_g(const Phys &ph, int q) {
  return q == 0 ? W0 * ph.e_ref * ph.k0 : WQ[q] * ph.e_ref * ph.ad_c;
}
__device__ __forceinline__ double rest_f(const Phys &ph, int q) { return WQ[q] * ph.n_ref; }

// f^eq_i >= 0 needs 1 + 3 b_i > 0 for every i (the discussion section's
// positivity bound); the largest |b_i| is on a diagonal: |b_x| + |b_y|,
// |b_x| + |b_z| or |b_y| + |b_z| (over c_l).  True when the bound is broken
// (or beta is NaN).
__device__ __forceinline__ bool feq_nonpositive(double bx, double by, double bz, double inv_c) {
  const double ax = fabs(bx), ay = fabs(by), az = fabs(bz);
  const double mb = fmax(ax + ay, fmax(ax + az, ay + az)) * inv_c;
  return !(3.0 * mb < 1.0);
}

// Event counters: NSLOT slots per counter, one 128-byte line each, picked by
// workgroup, so that a state where every wave reports (a NaN-filled lattice)
// does not serialise on one address.  Counter k, slot i lives at
// ctr[(k * NSLOT + i) * CSTRIDE]; the host sums the slots.
constexpr int NSLOT = 256;
constexpr int CSTRIDE = 16;

// Wave-level ballot counter.
__device__ __forceinline__ void count_lanes(bool flag, unsigned long long *ctr, int k) {
  unsigned long long m = __ballot(flag);
  if (m != 0ull) {
    int lane = (int)(threadIdx.x & 63u);
    if (lane == __ffsll((long long)m) - 1)
      atomicAdd(&ctr[(k * NSLOT + (int)(blockIdx.x & (NSLOT - 1))) * CSTRIDE],
                (unsigned long long)__popcll(m));
  }
}

// Deterministic sum of K doubles over the workgroup; thread 0 gets the result.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double *out) {
  __shared__ double red[BLOCK / 64][K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double x = v[k];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    v[k] = x;
  }
  const int wave = (int)threadIdx.x >> 6;
  if ((threadIdx.x & 63u) == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[wave][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = red[0][k];
      for (int w = 1; w < BLOCK / 64; ++w) s += red[w][k];
      out[k] = s;
    }
  }
}

// Element offset of the pull of direction q for cell c: the resolved source
// (wrap / clamp by the branch-free face corrections), or, when the cell word
// `cls` (0 without an obstacle) marks that source solid, the cell's own
// opposite population (half-way bounce-back).  Both candidates have
// compile-time directions after unrolling, and the choice needs no load
// beyond the cell's own word.
__device__ __forceinline__ size_t pull_at(const Geom &g, const Cell &c, const FaceCorr &fc,
                                          uint32_t cls, int q) {
  // selects, not a branch: one offset per direction
  const bool bounce = (cls >> (CLS_BOUNCE + q)) & 1u;
  const int src = bounce ? c.idx : src_fast(g, c, fc, q);
  return at(bounce ? OPP[q] : q, src);
}

// A wave holds a cell with a solid pull source (the cell word's near bit).
// Such waves are few (the cells next to an obstacle).  For 4- and 8-byte
// populations the gathers below are written as plain pulls followed, in those
// waves only, by pulls with the bounce-back offsets: this compiles to one
// branch per wave on the near bit, and the other waves pull without the
// per-direction offset selects.  (Issuing the plain pulls before the cell
// word arrives, with per-lane bounce-back loads after it, measured slower:
// those loads wait inside their branches.)  The 16-bit forms are issue-bound
// and keep the offsets selected from the cell word in every wave.
__device__ __forceinline__ bool wave_near_solid(uint32_t cls) {
  return __builtin_amdgcn_ballot_w64((cls & CLS_NEAR) != 0u) != 0u;
}

// Pull the 19 values of one population for cell c (decoded to the compute
// type).  HELD = false: no cell word (lattice without solid cells).
template <class Cd, bool HELD>
__device__ __forceinline__ void gather(const Geom &g, const Cell &c, uint32_t cls,
                                       const typename Cd::elem *__restrict__ P,
                                       typename Cd::calc (&v)[Q]) {
  constexpr bool early = sizeof(typename Cd::elem) >= 4;
  const FaceCorr fc = face_corr(g, c);
#pragma unroll
  for (int q = 0; q < Q; ++q)
    v[q] = Cd::dec(P[early ? at(q, src_fast(g, c, fc, q)) : pull_at(g, c, fc, cls, q)]);
  if (early && HELD && wave_near_solid(cls)) {
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = Cd::dec(P[pull_at(g, c, fc, cls, q)]);
  }
}

// Both populations of cell c, pulled in one pass (same sources for f and g).
template <class Cd, bool HELD>
__device__ __forceinline__ void gather2(const Geom &g, const Cell &c, uint32_t cls,
                                        const typename Cd::elem *__restrict__ G,
                                        const typename Cd::elem *__restrict__ F,
                                        typename Cd::calc (&vg)[Q], typename Cd::calc (&vf)[Q]) {
  constexpr bool early = sizeof(typename Cd::elem) >= 4;
  const FaceCorr fc = face_corr(g, c);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const size_t o = early ? at(q, src_fast(g, c, fc, q)) : pull_at(g, c, fc, cls, q);
    vg[q] = Cd::dec(G[o]);
    vf[q] = Cd::dec(F[o]);
  }
  if (early && HELD && wave_near_solid(cls)) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const size_t o = pull_at(g, c, fc, cls, q);
      vg[q] = Cd::dec(G[o]);
      vf[q] = Cd::dec(F[o]);
    }
  }
}

// The step's outputs are read once, by the next step: stream them past the
// caches (non-temporal store).
template <class El>
__device__ __forceinline__ void stream_store(El *p, El v) {
  __builtin_nontemporal_store(v, p);
}

// ---------------------------------------------------------------------------
// Forward stream-collide step.  DO_F = false updates the g population only
// (src/dst then address g blocks).  HELD = false is the instantiation for
// lattices with neither solid cells nor an inflow plane: the held-value
// selection and the bounce-back test compile away (the 16-bit forms are
// issue-bound, so those instructions cost time there).  ETA_S (f+g steps
// only) sets each update's tau from its pre-collision moments to hold eta/s.
template <int ST, class TC, bool DO_F, bool HELD, bool ETA_S = false>
__global__ __launch_bounds__(BLOCK) void k_step(const Geom g, const Phys ph,
                                                const typename Codec<ST, TC>::elem *__restrict__ src,
                                                typename Codec<ST, TC>::elem *__restrict__ dst,
                                                const HeldEq<typename Codec<ST, TC>::elem> in_eq,
                                                unsigned long long *__restrict__ counters) {
  using Cd = Codec<ST, TC>;
  using T = typename Cd::calc;
  using El = typename Cd::elem;
  const Cell c = decode_cell(g);
  if (!c.active) return;
  const uint32_t cls = (HELD && ph.cls) ? ph.cls[c.idx] : 0u;
  // Solid cells keep their (zero) entries and inflow-plane cells the inflow
  // equilibrium; both still run the common path (their pulls stay in the
  // domain) so that every lane joins the same full-wavefront stores, with the
  // held value selected per lane.
  const bool solid = HELD && (cls & CLS_SOLID);
  const bool held = HELD && (solid || is_inflow(g, c.x, c.y, c.z));
  const size_t qs = (size_t)g.qs;
  const El *__restrict__ gs = DO_F ? src + Q * qs : src;
  El *__restrict__ gd = DO_F ? dst + Q * qs : dst;
  // All 38 pulls are issued before any arithmetic (both populations in
  // flight per wave); g then f are relaxed and streamed out.
  T pg[Q], pf[Q];
  if (DO_F)
    gather2<Cd, HELD>(g, c, cls, gs, src, pg, pf);
  else
    gather<Cd, HELD>(g, c, cls, gs, pg);
  using Sm = typename Cd::sum;
  Sm sE, sx, sy, sz;
  moment_sums(pg, sE, sx, sy, sz);
  const Inv iv = invert(ph, ph.e_ref + (double)sE, ph.c * (double)sx, ph.c * (double)sy,
                        ph.c * (double)sz);
  EqCoef<T> k = eq_coef<T>(ph, 0.0, iv.eps, iv.W, iv.bx, iv.by, iv.bz);
  double omd = omega_of(ph, c.b, c.idx);
  bool bad = iv.bad;
  double N = 0.0;
  if (DO_F) {
    Sm sN = (Sm)0;
#pragma unroll
    for (int q = 0; q < Q; ++q) sN += (Sm)pf[q];
    N = ph.n_ref + (double)sN;
    if (ETA_S) {
      // tau from the pre-collision moments of this update (n = N / gamma)
      const double b2 = iv.bx * iv.bx + iv.by * iv.by + iv.bz * iv.bz;
      omd = omega_for_eta_s(ph, N * sqrt(1.0 - b2), iv.eps, b2);
      bad = bad || !(omd > 0.0 && omd < 2.0);  // needs tau > 1/2
    }
  }
  const T om = (T)omd;
  const El zero = Cd::enc((T)0);
  constexpr bool fix = !std::is_same<Sm, T>::value;  // FP32 equilibrium, FP64 moments
  const EqFix ef = fix ? eq_fix(k, sE, sx, sy, sz) : EqFix{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const T eq = fix ? geq_fixed(k, ef, q) : geq_dev(k, q);
    const El v = Cd::enc(pg[q] + om * (eq - pg[q]));
    stream_store(&gd[at(q, c.idx)], held ? (solid ? zero : in_eq.v[Q + q]) : v);
  }
  count_lanes(bad && !held, counters, 0);
  if (DO_F) {
    k.N = (T)N;
    k.Nd = (T)(N - ph.n_ref);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const El v = Cd::enc(pf[q] + om * (feq_dev(k, q) - pf[q]));
      stream_store(&dst[at(q, c.idx)], held ? (solid ? zero : in_eq.v[q]) : v);
    }
    count_lanes(feq_nonpositive(iv.bx, iv.by, iv.bz, ph.inv_c) && !held, counters, 1);
  }
}

// ---------------------------------------------------------------------------
// Forward step with two cells per lane: cells 2t and 2t+1 of one x row, for
// lattices with an even x extent and no held cells (no solid, no inflow
// plane; constant or per-cell tau, not the eta/s rule), in FP64 storage or
// FP32 storage with FP64 collision.  The two cells' sources of a pull with no
// x component are adjacent cells of one row with the same wrap corrections,
// starting on an even cell: one aligned load of two elements reads both.
// Pulls with an x component read the two sources apart.  Every store writes
// an aligned pair.  g is pulled, relaxed and stored before f is pulled, so
// that two cells' state of one population is live at a time.  With held
// cells, 2-byte storage or FP32 collision k_step is kept (measured faster, or
// the moment correction of the FP32 collision is not part of this kernel).
template <class El>
struct Pair2 {
  typedef El type __attribute__((ext_vector_type(2)));
};

template <class Cd>
__device__ __forceinline__ void gather_pairs(const Geom &g, const Cell &c0, const Cell &c1,
                                             const FaceCorr &f0, const FaceCorr &f1,
                                             const typename Cd::elem *__restrict__ P,
                                             typename Cd::calc (&v0)[Q],
                                             typename Cd::calc (&v1)[Q]) {
  using P2 = typename Pair2<typename Cd::elem>::type;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if (EX[q] == 0) {
      const P2 pr = *reinterpret_cast<const P2 *>(&P[at(q, src_fast(g, c0, f0, q))]);
      v0[q] = Cd::dec(pr.x);
      v1[q] = Cd::dec(pr.y);
    } else {
      v0[q] = Cd::dec(P[at(q, src_fast(g, c0, f0, q))]);
      v1[q] = Cd::dec(P[at(q, src_fast(g, c1, f1, q))]);
    }
  }
}

// Both cells' flags counted in one atomic per wave.
__device__ __forceinline__ void count_pairs(bool f0, bool f1, unsigned long long *ctr, int k) {
  const unsigned long long m0 = __ballot(f0), m1 = __ballot(f1);
  if ((m0 | m1) != 0ull) {
    const int lane = (int)(threadIdx.x & 63u);
    if (lane == __ffsll((long long)(m0 | m1)) - 1)
      atomicAdd(&ctr[(k * NSLOT + (int)(blockIdx.x & (NSLOT - 1))) * CSTRIDE],
                (unsigned long long)(__popcll(m0) + __popcll(m1)));
  }
}

// npb = workgroups per instance (each covers 2 * BLOCK cells).
template <int ST, class TC>
__global__ __launch_bounds__(BLOCK) void k_step_pairs(const Geom g, const Phys ph, int npb,
                                                      const typename Codec<ST, TC>::elem *__restrict__ src,
                                                      typename Codec<ST, TC>::elem *__restrict__ dst,
                                                      unsigned long long *__restrict__ counters) {
  using Cd = Codec<ST, TC>;
  using T = typename Cd::calc;
  using El = typename Cd::elem;
  using Sm = typename Cd::sum;
  using P2 = typename Pair2<El>::type;
  Cell c0, c1;
  c0.L = c1.L = xcd_remap((int)blockIdx.x, npb * g.batch);
  c0.b = c1.b = c0.L / npb;
  c0.local = 2 * ((c0.L - c0.b * npb) * BLOCK + (int)threadIdx.x);
  if (c0.local >= g.per) return;  // the cell count per instance is even
  c1.local = c0.local + 1;
  const uint32_t t = fdiv(g.div_x, (uint32_t)c0.local);
  c0.x = c0.local - (int)t * g.n[0];
  c1.x = c0.x + 1;
  const uint32_t z = fdiv(g.div_y, t);
  c0.y = c1.y = (int)t - (int)z * g.n[1];
  c0.z = c1.z = (int)z;
  c0.idx = c0.b * g.per + c0.local;
  c1.idx = c0.idx + 1;
  c0.active = c1.active = true;
  const FaceCorr f0 = face_corr(g, c0), f1 = face_corr(g, c1);
  const El *__restrict__ gs = src + (size_t)Q * g.qs;
  El *__restrict__ gd = dst + (size_t)Q * g.qs;
  T p0[Q], p1[Q];
  gather_pairs<Cd>(g, c0, c1, f0, f1, gs, p0, p1);
  Sm e0, x0, y0, z0, e1, x1, y1, z1;
  moment_sums(p0, e0, x0, y0, z0);
  moment_sums(p1, e1, x1, y1, z1);
  const Inv i0 = invert(ph, ph.e_ref + (double)e0, ph.c * (double)x0, ph.c * (double)y0,
                        ph.c * (double)z0);
  const Inv i1 = invert(ph, ph.e_ref + (double)e1, ph.c * (double)x1, ph.c * (double)y1,
                        ph.c * (double)z1);
  EqCoef<T> k0 = eq_coef<T>(ph, 0.0, i0.eps, i0.W, i0.bx, i0.by, i0.bz);
  EqCoef<T> k1 = eq_coef<T>(ph, 0.0, i1.eps, i1.W, i1.bx, i1.by, i1.bz);
  const T om0 = (T)omega_of(ph, c0.b, c0.idx), om1 = (T)omega_of(ph, c1.b, c1.idx);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    P2 o;
    o.x = Cd::enc(p0[q] + om0 * (geq_dev(k0, q) - p0[q]));
    o.y = Cd::enc(p1[q] + om1 * (geq_dev(k1, q) - p1[q]));
    __builtin_nontemporal_store(o, reinterpret_cast<P2 *>(&gd[at(q, c0.idx)]));
  }
  count_pairs(i0.bad, i1.bad, counters, 0);
  asm volatile("" ::: "memory");  // compiler barrier: f is pulled after g is stored
  T q0[Q], q1[Q];
  gather_pairs<Cd>(g, c0, c1, f0, f1, src, q0, q1);
  Sm n0 = (Sm)0, n1 = (Sm)0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    n0 += (Sm)q0[q];
    n1 += (Sm)q1[q];
  }
  const double N0 = ph.n_ref + (double)n0, N1 = ph.n_ref + (double)n1;
  k0.N = (T)N0;
  k0.Nd = (T)(N0 - ph.n_ref);
  k1.N = (T)N1;
  k1.Nd = (T)(N1 - ph.n_ref);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    P2 o;
    o.x = Cd::enc(q0[q] + om0 * (feq_dev(k0, q) - q0[q]));
    o.y = Cd::enc(q1[q] + om1 * (feq_dev(k1, q) - q1[q]));
    __builtin_nontemporal_store(o, reinterpret_cast<P2 *>(&dst[at(q, c0.idx)]));
  }
  count_pairs(feq_nonpositive(i0.bx, i0.by, i0.bz, ph.inv_c),
              feq_nonpositive(i1.bx, i1.by, i1.bz, ph.inv_c), counters, 1);
}

// The 16-bit storages' encoder on n FP32 values (the conversion the step's
// stores apply); grid-stride.
template <int ST>
__global__ __launch_bounds__(BLOCK) void k_encode16(const float *__restrict__ src,
                                                    typename Format<ST>::elem *__restrict__ dst,
                                                    long long n) {
  const long long stride = (long long)gridDim.x * BLOCK;
  for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride)
    dst[i] = Format<ST>::enc(src[i]);
}

// ---------------------------------------------------------------------------
// Initial state: equilibria of (n0, e0, beta0); inflow cells take the inflow
// equilibrium; solid cells hold zeros in both buffers.
template <int ST, class TC>
__global__ __launch_bounds__(BLOCK) void k_init(const Geom g, const Phys ph,
                                                const double *__restrict__ n0,
                                                const double *__restrict__ e0,
                                                const double *__restrict__ beta0,
                                                typename Codec<ST, TC>::elem *__restrict__ pa,
                                                typename Codec<ST, TC>::elem *__restrict__ pb,
                                                const typename Codec<ST, TC>::elem *__restrict__ in_eq) {
  using Cd = Codec<ST, TC>;
  using T = typename Cd::calc;
  const Cell c = decode_cell(g);
  if (!c.active) return;
  const size_t qs = (size_t)g.qs;
  const size_t cells = (size_t)g.batch * g.per;
  if (solid_at(ph, c.idx)) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      pa[at(q, c.idx)] = Cd::enc((T)0);
      pb[at(q, c.idx)] = Cd::enc((T)0);
      pa[Q * qs + at(q, c.idx)] = Cd::enc((T)0);
      pb[Q * qs + at(q, c.idx)] = Cd::enc((T)0);
    }
    return;
  }
  if (is_inflow(g, c.x, c.y, c.z)) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      pa[at(q, c.idx)] = in_eq[q];
      pa[Q * qs + at(q, c.idx)] = in_eq[Q + q];
    }
    return;
  }
  const double bx = beta0[c.idx], by = beta0[cells + c.idx], bz = beta0[2 * cells + c.idx];
  const double g2 = 1.0 / (1.0 - (bx * bx + by * by + bz * bz));
  const double e = e0[c.idx];
  const double N = n0[c.idx] * sqrt(g2);
  const EqCoef<T> k = eq_coef<T>(ph, N, e, ph.wfac * e * g2, bx, by, bz);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    pa[at(q, c.idx)] = Cd::enc(feq_dev(k, q));
    pa[Q * qs + at(q, c.idx)] = Cd::enc(geq_dev(k, q));
  }
}

// Inflow equilibrium (38 values in storage format), one thread.
template <int ST, class TC>
__global__ void k_inflow_eq(const Phys ph, double n, double e, double bx, double by, double bz,
                            typename Codec<ST, TC>::elem *__restrict__ out) {
  using Cd = Codec<ST, TC>;
  using T = typename Cd::calc;
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double g2 = 1.0 / (1.0 - (bx * bx + by * by + bz * bz));
  const EqCoef<T> k = eq_coef<T>(ph, n * sqrt(g2), e, ph.wfac * e * g2, bx, by, bz);
  for (int q = 0; q < Q; ++q) {
    out[q] = Cd::enc(feq_dev(k, q));
    out[Q + q] = Cd::enc(geq_dev(k, q));
  }
}

// ---------------------------------------------------------------------------
// Fields and per-block conservation partials of a stored state.
// Sf may be null (g block only: n is not computed and the f sum is zero).
template <int ST, class TC>
__global__ __launch_bounds__(BLOCK) void k_moments(const Geom g, const Phys ph,
                                                   const typename Codec<ST, TC>::elem *__restrict__ Sf,
                                                   const typename Codec<ST, TC>::elem *__restrict__ Sg,
                                                   double *__restrict__ n, double *__restrict__ e,
                                                   double *__restrict__ beta,
                                                   double *__restrict__ part, int swap) {
  using Cd = Codec<ST, TC>;
  const Cell c = decode_cell(g);
  const size_t cells = (size_t)g.batch * g.per;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (c.active) {
    if (solid_at(ph, c.idx)) {
      if (n) n[c.idx] = 0.0;
      if (e) e[c.idx] = 0.0;
      if (beta) beta[c.idx] = beta[cells + c.idx] = beta[2 * cells + c.idx] = 0.0;
    } else {
      double N = 0.0, Eg = 0.0, sx, sy, sz, gv[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int sq = swap ? OPP[q] : q;  // in-place layout: S_q at slot opp(q)
        if (Sf) N += (double)Cd::dec(Sf[at(sq, c.idx)]);
        gv[q] = (double)Cd::dec(Sg[at(sq, c.idx)]);
        Eg += gv[q];
      }
      mirror_sums(gv, sx, sy, sz);
      if (Sf) N += ph.n_ref;  // the rest parts sum to (n_ref, e_ref, 0)
      Eg += ph.e_ref;
      const Inv iv = invert(ph, Eg, ph.c * sx, ph.c * sy, ph.c * sz);
      if (n && Sf) n[c.idx] = N * sqrt(1.0 - (iv.bx * iv.bx + iv.by * iv.by + iv.bz * iv.bz));
      if (e) e[c.idx] = iv.eps;
      if (beta) {
        beta[c.idx] = iv.bx;
        beta[cells + c.idx] = iv.by;
        beta[2 * cells + c.idx] = iv.bz;
      }
      acc[0] = N;
      acc[1] = Eg;
      acc[2] = iv.Mx;
      acc[3] = iv.My;
      acc[4] = iv.Mz;
    }
  }
  if (part) {
    double out[5];
    block_sum<5>(acc, out);
    if (threadIdx.x == 0)
      for (int k = 0; k < 5; ++k) part[(size_t)c.L * 5 + k] = out[k];
  }
}

// Transport quantities of a stored f+g state per cell (zeros on solid
// cells): temperature, entropy density, shear viscosity and eta/s, each cell
// with its relaxation time (per-cell field, instance, or the eta/s rule at
// the cell's fields).  Any output may be null.
template <int ST, class TC>
__global__ __launch_bounds__(BLOCK) void k_transport(const Geom g, const Phys ph,
                                                     const typename Codec<ST, TC>::elem *__restrict__ Sf,
                                                     const typename Codec<ST, TC>::elem *__restrict__ Sg,
                                                     double *__restrict__ temp, double *__restrict__ ent,
                                                     double *__restrict__ eta, double *__restrict__ eos,
                                                     int swap) {
  using Cd = Codec<ST, TC>;
  const Cell c = decode_cell(g);
  if (!c.active) return;
  double vT = 0.0, vs = 0.0, veta = 0.0, veos = 0.0;
  if (!solid_at(ph, c.idx)) {
    double N = ph.n_ref, Eg = ph.e_ref, sx, sy, sz, gv[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int sq = swap ? OPP[q] : q;
      N += (double)Cd::dec(Sf[at(sq, c.idx)]);
      gv[q] = (double)Cd::dec(Sg[at(sq, c.idx)]);
      Eg += gv[q];
    }
    mirror_sums(gv, sx, sy, sz);
    const Inv iv = invert(ph, Eg, ph.c * sx, ph.c * sy, ph.c * sz);
    const double b2 = iv.bx * iv.bx + iv.by * iv.by + iv.bz * iv.bz;
    const double n = N * sqrt(1.0 - b2);
    const double om = ph.eta_s > 0.0 ? omega_for_eta_s(ph, n, iv.eps, b2) : omega_of(ph, c.b, c.idx);
    const Transport t = transport_of(n, iv.eps, b2, ph.d_G);
    vT = t.T;
    vs = t.s;
    veta = (4.0 / 9.0) * t.gamma2 * iv.eps * ph.c * (1.0 / om - 0.5);
    veos = veta / vs;
  }
  if (temp) temp[c.idx] = vT;
  if (ent) ent[c.idx] = vs;
  if (eta) eta[c.idx] = veta;
  if (eos) eos[c.idx] = veos;
}

// omega(x) = 1/tau(x) of a per-cell tau field; counts (into *bad) the
// non-solid cells whose tau is not > 1/2 (or NaN).
__global__ __launch_bounds__(BLOCK) void k_set_omega_cell(const Geom g, const Phys ph,
                                                          const double *__restrict__ tau,
                                                          double *__restrict__ omega,
                                                          unsigned long long *__restrict__ bad) {
  const Cell c = decode_cell(g);
  bool flag = false;
  if (c.active) {
    const double t = tau[c.idx];
    const bool solid = solid_at(ph, c.idx);
    flag = !solid && !(t > 0.5);
    omega[c.idx] = solid ? 0.0 : 1.0 / t;
  }
  const unsigned long long m = __ballot(flag);
  if (m != 0ull && (threadIdx.x & 63u) == (unsigned)(__ffsll((long long)m) - 1))
    atomicAdd(bad, (unsigned long long)__popcll(m));
}

// out[i] += acc[i]; acc[i] = 0 over the cells (hand the per-cell gradient over).
__global__ __launch_bounds__(BLOCK) void k_take_cell_grad(long long cells, double *__restrict__ acc,
                                                          double *__restrict__ out) {
  const long long i = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= cells) return;
  out[i] += acc[i];
  acc[i] = 0.0;
}

// Per-instance, fixed-order reduction of per-workgroup [5] partials: one
// workgroup per instance b (gridDim.x = batch).  Instance b owns workgroups
// [b*nblk_per, (b+1)*nblk_per) of `part` and, when part2 is given, workgroups
// [start2[b], start2[b+1]) of `part2`.
//   res  != null: res[b][k] = the instance's sums (k = 0..4);
//   dtau != null: dtau[b] += component 0;
//   inst != null: inst[b][0..3] = components 1..4 (inflow partials, summed over
//                 instances in order by k_finish_inflow).
__global__ __launch_bounds__(BLOCK) void k_finish(const double *__restrict__ part, int nblk_per,
                                                  const double *__restrict__ part2,
                                                  const int *__restrict__ start2,
                                                  double *__restrict__ res,
                                                  double *__restrict__ dtau,
                                                  double *__restrict__ inst) {
  const int b = (int)blockIdx.x;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int j = (int)threadIdx.x; j < nblk_per; j += BLOCK)
    for (int k = 0; k < 5; ++k) v[k] += part[((size_t)b * nblk_per + j) * 5 + k];
  if (part2)
    for (int j = start2[b] + (int)threadIdx.x; j < start2[b + 1]; j += BLOCK)
      for (int k = 0; k < 5; ++k) v[k] += part2[(size_t)j * 5 + k];
  double out[5];
  block_sum<5>(v, out);
  if (threadIdx.x == 0) {
    if (res)
      for (int k = 0; k < 5; ++k) res[b * 5 + k] = out[k];
    if (dtau) dtau[b] += out[0];
    if (inst)
      for (int k = 0; k < 4; ++k) inst[b * 4 + k] = out[1 + k];
  }
}

// v[0..n) = 0 (a kernel, not a memset, so that it may sit in captured graphs).
__global__ __launch_bounds__(BLOCK) void k_zero(double *__restrict__ v, long long n) {
  const long long i = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) v[i] = 0.0;
}

// de_in[0] += sum_b inst[b][0]; dbeta_in[k] += sum_b inst[b][1 + k] (in order).
__global__ void k_finish_inflow(const double *__restrict__ inst, int batch,
                                double *__restrict__ de_in, double *__restrict__ dbeta_in) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = 0; b < batch; ++b)
    for (int k = 0; k < 4; ++k) t[k] += inst[b * 4 + k];
  if (de_in) de_in[0] += t[0];
  if (dbeta_in)
    for (int k = 0; k < 3; ++k) dbeta_in[k] += t[1 + k];
}

// ---------------------------------------------------------------------------
// Reverse mode.
//
// Eqs. (equil2a)/(equil2b) with P = kappa e and W = (e + P) gamma^2 read
// g^eq_i = w_i [A_i e + W P_i(beta)] with A_i = a = 3 kappa / c_l^2,
// P_i = 3b_i + (9/2) b_i^2 - s for i > 0 and A_0 = -a (2 + c_l^2),
// P_0 = 3 - s (e = 3P: a = 1/c_l^2).  The contraction of lambda with the
// equilibrium's partials is
//   Le = sum l_i w_i A_i = a (sum l_i w_i - (3 + c_l^2) l_0 w_0),
//   LW = sum l_i w_i P_i,
//   Lb_a = (W / c_l) [sum_{i>0} l_i w_i e_ia (3 + 9 b_i) - 3 (beta_a / c_l) sum l_i w_i],
// and the inversion's partials (D^2 = A E^2 - B|M|^2, e = (D - F E) G,
// W = (C E + D) H, beta = M/W; see invert) carry it to the moments:
//   K = LW - Lb.beta / W,
//   dL/dE = Le (A E/D - F) G + K (C + A E/D) H,
//   dL/dM_a = -(M_a / D) B (G Le + H K) + Lb_a / W,
// which for e = 3P is Le (4E/D - 1) + K (2 + 4E/D) / 3 and
// -(M_a / D)(3 Le + K) + Lb_a / W.
template <class T>
struct LamSums {
  T Slw, SW, Vx, Vy, Vz, lw0;
};

// With pre != null also dt = sum_q lam_q (pre_q - g^eq_q) (same order as a
// separate loop), so that pre is dead after this single pass.
template <class T>
__device__ __forceinline__ LamSums<T> lam_sums(const T (&lam)[Q], const EqCoef<T> &k,
                                               const T *pre = nullptr, T *dt = nullptr) {
  LamSums<T> r;
  r.Slw = r.SW = (T)0;
  T u[Q];
  u[0] = (T)0;
  T d = (T)0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const T lw = lam[q] * (T)WQ[q];
    r.Slw += lw;
    if (q == 0) {
      r.lw0 = lw;
      r.SW += lw * ((T)3 - k.s);
    } else {
      const T b = dot_e(k, q);
      r.SW += lw * (b * ((T)3 + (T)4.5 * b) - k.s);
      u[q] = lw * ((T)3 + (T)9 * b);
    }
    if (pre) d += lam[q] * (pre[q] - geq_dev(k, q));
  }
  mirror_sums(u, r.Vx, r.Vy, r.Vz);
  if (dt) *dt = d;
  return r;
}

struct LamEq {
  double Le, LW, Lbx, Lby, Lbz;
};

template <class T>
__device__ __forceinline__ LamEq lam_eq(const LamSums<T> &s, const Phys &ph, double W, double bx,
                                        double by, double bz) {
  LamEq r;
  const double Slw = (double)s.Slw;
  r.Le = Slw * ph.ad_c - (double)s.lw0 * (3.0 + ph.c * ph.c) * ph.ad_c;
  r.LW = (double)s.SW;
  const double f = W * ph.inv_c;
  r.Lbx = f * ((double)s.Vx - 3.0 * bx * ph.inv_c * Slw);
  r.Lby = f * ((double)s.Vy - 3.0 * by * ph.inv_c * Slw);
  r.Lbz = f * ((double)s.Vz - 3.0 * bz * ph.inv_c * Slw);
  return r;
}

// (dL/dE, dL/dM) from contractions with respect to (e, W, beta).
struct GradEM {
  double gE, gx, gy, gz;
};

__device__ __forceinline__ GradEM chain_moments(const Phys &ph, const Inv &iv, double Le, double LW,
                                                double Lbx, double Lby, double Lbz) {
  GradEM r;
  const double iW = 1.0 / iv.W, iD = 1.0 / iv.D;
  const double K = LW - (Lbx * iv.bx + Lby * iv.by + Lbz * iv.bz) * iW;
  const double rr = ph.eos_A * iv.E * iD;
  r.gE = Le * (rr - ph.eos_F) * ph.eos_G + K * (ph.eos_C + rr) * ph.eos_H;
  const double h = (ph.eos_B * ph.eos_G * Le + ph.eos_B * ph.eos_H * K) * iD;
  r.gx = -iv.Mx * h + Lbx * iW;
  r.gy = -iv.My * h + Lby * iW;
  r.gz = -iv.Mz * h + Lbz * iW;
  return r;
}

// d/d(e, beta) of w_i [A_i e + W P_i] at W = (1 + kappa) e gamma^2, contracted with lambda.
__device__ __forceinline__ void eq_param_grad(const Phys &ph, const LamEq &L, double e, double bx,
                                              double by, double bz, double out[4]) {
  const double g2 = 1.0 / (1.0 - (bx * bx + by * by + bz * bz));
  const double W = ph.wfac * e * g2;
  out[0] = L.Le + ph.wfac * g2 * L.LW;
  const double t = 2.0 * W * g2 * L.LW;
  out[1] = L.Lbx + t * bx;
  out[2] = L.Lby + t * by;
  out[3] = L.Lbz + t * bz;
}

// Cell of a linear index (general paths).
__device__ __forceinline__ Cell cell_at(const Geom &g, int idx) {
  Cell c;
  c.idx = idx;
  c.b = (int)(idx / g.per);
  c.local = idx - c.b * g.per;
  c.active = true;
  const uint32_t t = fdiv(g.div_x, (uint32_t)c.local);
  c.x = c.local - (int)t * g.n[0];
  const uint32_t z = fdiv(g.div_y, t);
  c.y = (int)t - (int)z * g.n[1];
  c.z = (int)z;
  c.L = 0;
  return c;
}

// Local reverse update of one updated cell: from the pulled populations pre
// and lambda_{t+1}(x), the contributions mu_q to lambda_t (one per pulled
// population) and lambda . d post / d tau.
struct LocalAdjoint {
  double om1, aE, ax, ay, az, dtau;
};

template <class T>
__device__ __forceinline__ LocalAdjoint adjoint_local(const Phys &ph, double om, const T (&pre)[Q],
                                                      const T (&lam)[Q]) {
  T sE = (T)0, sx, sy, sz;
#pragma unroll
  for (int q = 0; q < Q; ++q) sE += pre[q];
  mirror_sums(pre, sx, sy, sz);
  const Inv iv = invert(ph, ph.e_ref + (double)sE, ph.c * (double)sx, ph.c * (double)sy,
                        ph.c * (double)sz);
  const EqCoef<T> k = eq_coef<T>(ph, 0.0, iv.eps, iv.W, iv.bx, iv.by, iv.bz);
  T dt;
  const LamEq L = lam_eq(lam_sums(lam, k, pre, &dt), ph, iv.W, iv.bx, iv.by, iv.bz);
  const GradEM gm = chain_moments(ph, iv, L.Le, L.LW, L.Lbx, L.Lby, L.Lbz);
  LocalAdjoint r;
  r.om1 = 1.0 - om;
  r.aE = om * gm.gE;
  r.ax = om * ph.c * gm.gx;
  r.ay = om * ph.c * gm.gy;
  r.az = om * ph.c * gm.gz;
  r.dtau = om * om * (double)dt;
  return r;
}

// mu_q = (1 - omega) lambda_q + omega (dL/dE + c_l e_q . dL/dM)
__device__ __forceinline__ double adjoint_mu(const LocalAdjoint &a, double lam, int q) {
  double mu = a.om1 * lam + a.aE;
  if (EX[q] == 1) mu += a.ax;
  if (EX[q] == -1) mu -= a.ax;
  if (EY[q] == 1) mu += a.ay;
  if (EY[q] == -1) mu -= a.ay;
  if (EZ[q] == 1) mu += a.az;
  if (EZ[q] == -1) mu -= a.az;
  return mu;
}

// Reverse step in reader form.
//
// The transpose of the pull map sends each update's contribution mu_q(r)
// (from its pull of direction q) to the stored population that pull read.
// Stored there directly, a wavefront's 64 contributions of one direction land
// at a shifted address, with a partially written cache line at either end.
// Instead every update stores its contributions at its own cell, aligned, in
// the "reader form"
//     R_t(r)_q = mu_q(r)      (zero for solid and inflow cells: they pull nothing),
// and lambda_t is gathered from it with the shifted reads of a forward pull:
//     lambda_t(x)_p = R_t(x)_opp(p)   if x's pull of opp(p) bounces off a solid
//                   + R_t(x + e_p)_p  otherwise, when x + e_p lies in the domain
//                   + R_t(r)_p        for every r whose pull of p is clamped onto x.
// The readers of a clamped pull of p onto x: along each axis k of a clamp
// pattern m, r_k = x_k with x on the face that e_p points out of (x_k = 0 for
// e_pk = +1, n - 1 for e_pk = -1); along the other axes r_k = x_k + e_pk.

// Faces of non-periodic axes that a cell lies on.
struct FaceFlags {
  bool lo[3], hi[3];
  bool any;
};

__device__ __forceinline__ FaceFlags face_flags(const Geom &g, const Cell &c) {
  FaceFlags f;
  const int co[3] = {c.x, c.y, c.z};
  f.any = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    f.lo[a] = !g.periodic[a] && co[a] == 0;
    f.hi[a] = !g.periodic[a] && co[a] == g.n[a] - 1;
    f.any = f.any || f.lo[a] || f.hi[a];
  }
  return f;
}

// Component a of e_p (compile-time after unrolling).
__device__ __forceinline__ constexpr int ecomp(int p, int a) {
  return a == 0 ? EX[p] : (a == 1 ? EY[p] : EZ[p]);
}

// x + e_p leaves the domain along axis a (through a face of a non-periodic axis).
__device__ __forceinline__ bool leaves(const FaceFlags &f, int p, int a) {
  const int e = ecomp(p, a);
  return (e == 1 && f.hi[a]) || (e == -1 && f.lo[a]);
}

// A reader of p clamped along axis a onto this cell (the cell is on the face
// that e_p points out of).
__device__ __forceinline__ bool clamps_onto(const FaceFlags &f, int p, int a) {
  const int e = ecomp(p, a);
  return (e == 1 && f.lo[a]) || (e == -1 && f.hi[a]);
}

// Which face corrections a lattice needs in the reverse gather: none (every
// axis periodic), one non-periodic axis of extent > 1 (the axis is part of
// the kernel), or the general case.
enum : int { FACES_NONE = 0, FACES_X = 1, FACES_Y = 2, FACES_Z = 3, FACES_ANY = 4 };

// lambda_t(x)_p, p = 0 .. 18, gathered from the reader form R (see above).
// The 19 plain (or bounce-back) reads are issued together, like a forward
// pull; cells on a face of a non-periodic axis then drop the readers that lie
// outside the domain and add the readers of clamped pulls, in one branch that
// only waves holding such cells take.
//
// With one non-periodic axis A, a cell on its low face has a clamped reader
// for each of the five directions p with e_pA = +1 (and loses its reader for
// opp(p)), a cell on its high face for each opp(p) (and loses p); the reader
// is the plain one moved back onto the face along A.  One select-addressed
// load per pair serves both faces, all five issued together.  Several
// non-periodic axes take the general loop over clamp patterns.
template <int FACES>
__device__ __forceinline__ void lam_gather(const Geom &g, const Cell &c, const FaceCorr &fc,
                                           uint32_t cls, const LamT *__restrict__ R,
                                           double (&lam)[Q]) {
  // x + e_p is the source of x's pull of opp(p) (src_fast applies its wrap
  // corrections); bounce-back when that pull hits a solid (waves next to a
  // solid gather again, as the forward pulls do)
#pragma unroll
  for (int p = 0; p < Q; ++p) lam[p] = R[at(p, src_fast(g, c, fc, OPP[p]))];
  if (wave_near_solid(cls)) {
#pragma unroll
    for (int p = 0; p < Q; ++p) {
      const int q = OPP[p];
      const bool bounce = (cls >> (CLS_BOUNCE + q)) & 1u;
      const int src = bounce ? c.idx : src_fast(g, c, fc, q);
      lam[p] = R[at(bounce ? q : p, src)];
    }
  }
  if (FACES == FACES_NONE) return;
  if (FACES != FACES_ANY) {
    constexpr int A = FACES - 1;
    const int co = A == 0 ? c.x : (A == 1 ? c.y : c.z);
    const bool lo = co == 0, hi = co == g.n[A] - 1;
    if (!(lo || hi)) return;
    const int sA = A == 0 ? 1 : (A == 1 ? g.n[0] : g.n[0] * g.n[1]);
    double v[Q];
#pragma unroll
    for (int p = 0; p < Q; ++p) {
      if (ecomp(p, A) != 1) continue;  // compile-time after unrolling
      const int m = OPP[p];
      // low face: the reader of p, x + e_p moved back onto the face along A;
      // high face: the reader of m, x + e_m moved forward onto it
      const int r = lo ? src_fast(g, c, fc, m) - sA : src_fast(g, c, fc, p) + sA;
      v[p] = R[at(lo ? p : m, r)];
    }
#pragma unroll
    for (int p = 0; p < Q; ++p) {
      if (ecomp(p, A) != 1) continue;
      const int m = OPP[p];
      const bool bp = (cls >> (CLS_BOUNCE + m)) & 1u;  // x's pull of opp(p) bounces
      const bool bm = (cls >> (CLS_BOUNCE + p)) & 1u;  // x's pull of opp(m) bounces
      lam[p] = lo ? lam[p] + v[p] : (bp ? lam[p] : 0.0);
      lam[m] = hi ? lam[m] + v[p] : (bm ? lam[m] : 0.0);
    }
    return;
  }
  const FaceFlags ff = face_flags(g, c);
  if (!ff.any) return;
  const int stride[3] = {1, g.n[0], g.n[0] * g.n[1]};
#pragma unroll
  for (int p = 0; p < Q; ++p) {
    const int q = OPP[p];
    const bool bounce = (cls >> (CLS_BOUNCE + q)) & 1u;
    if (!bounce && (leaves(ff, p, 0) || leaves(ff, p, 1) || leaves(ff, p, 2))) lam[p] = 0.0;
    const int plain = src_fast(g, c, fc, q);
#pragma unroll
    for (int m = 1; m < 8; ++m) {
      bool possible = true;
#pragma unroll
      for (int a = 0; a < 3; ++a)
        if (((m >> a) & 1) && ecomp(p, a) == 0) possible = false;
      if (!possible) continue;  // compile-time after unrolling
      bool ok = true;
      int r = plain;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int e = ecomp(p, a);
        if (e == 0) continue;
        if ((m >> a) & 1) {
          ok = ok && clamps_onto(ff, p, a);
          r -= e * stride[a];
        } else {
          ok = ok && !leaves(ff, p, a);
        }
      }
      if (ok) lam[p] += R[at(p, r)];
    }
  }
}

// One reverse step of the g population (see rlb_adjoint_step) in reader form:
// lambda_{t+1} is read directly (NAT_IN) or gathered from the reader form of
// the previous reverse step; R_t is stored aligned.  Partials per workgroup,
// added to the previous step's when accum is set (a reverse sweep accumulates
// per workgroup in step order, then reduces once): part[L][5] = (dL/dtau,
// dL/de_in, dL/dbeta_in[3]).  Held cells (solid, inflow) run the common path
// and store zeros, so that every lane joins the same full-wavefront stores.
template <int ST, class TC, bool NAT_IN, int FACES>
__global__ __launch_bounds__(BLOCK) void k_adjoint(
    const Geom g, const Phys ph, const typename Codec<ST, TC>::elem *__restrict__ S,
    const LamT *__restrict__ lam_in, LamT *__restrict__ R_out, double *__restrict__ part,
    const InflowState in, int accum) {
  using Cd = Codec<ST, TC>;
  const Cell c = decode_cell(g);
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (c.active) {
    const uint32_t cls = ph.cls ? ph.cls[c.idx] : 0u;
    const bool solid = cls & CLS_SOLID;
    const bool inflow = is_inflow(g, c.x, c.y, c.z);
    const FaceCorr fc = face_corr(g, c);
    double pre[Q], lam[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) pre[q] = (double)Cd::dec(S[at(q, src_fast(g, c, fc, q))]);
    if (wave_near_solid(cls)) {
#pragma unroll
      for (int q = 0; q < Q; ++q) pre[q] = (double)Cd::dec(S[pull_at(g, c, fc, cls, q)]);
    }
    if (NAT_IN) {
#pragma unroll
      for (int p = 0; p < Q; ++p) lam[p] = lam_in[at(p, c.idx)];
    } else {
      lam_gather<FACES>(g, c, fc, cls, lam_in, lam);
    }
    if (inflow && !solid) {
      // the held face: lambda_{t+1} there is the gradient of the inflow state
      const double g2 = 1.0 / (1.0 - (in.bx * in.bx + in.by * in.by + in.bz * in.bz));
      const double W = ph.wfac * in.e * g2;
      const EqCoef<double> k = eq_coef<double>(ph, 0.0, in.e, W, in.bx, in.by, in.bz);
      const LamEq L = lam_eq(lam_sums(lam, k), ph, W, in.bx, in.by, in.bz);
      double gr[4];
      eq_param_grad(ph, L, in.e, in.bx, in.by, in.bz, gr);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) acc[1 + k2] = gr[k2];
    }
    const bool held = solid || inflow;
    const LocalAdjoint a = adjoint_local(ph, omega_of(ph, c.b, c.idx), pre, lam);
#pragma unroll
    for (int q = 0; q < Q; ++q)
      stream_store(&R_out[at(q, c.idx)], held ? 0.0 : adjoint_mu(a, lam[q], q));
    if (!held) {
      acc[0] = a.dtau;
      if (ph.dtau_cell) ph.dtau_cell[c.idx] += a.dtau;
    }
  }
  double out[5];
  block_sum<5>(acc, out);
  if (threadIdx.x == 0) {
    double *dst = part + (size_t)c.L * 5;
#pragma unroll
    for (int k2 = 0; k2 < 5; ++k2) dst[k2] = (accum ? dst[k2] : 0.0) + out[k2];
  }
}

// lambda (natural layout) from the reader form: lambda(x)_p as lam_gather
// gathers it; zeros on solid cells (their populations are never read).
template <int FACES>
__global__ __launch_bounds__(BLOCK) void k_lam_gather(const Geom g, const Phys ph,
                                                      const LamT *__restrict__ R,
                                                      LamT *__restrict__ lam) {
  const Cell c = decode_cell(g);
  if (!c.active) return;
  const uint32_t cls = ph.cls ? ph.cls[c.idx] : 0u;
  const bool solid = cls & CLS_SOLID;
  const FaceCorr fc = face_corr(g, c);
  double v[Q];
  lam_gather<FACES>(g, c, fc, cls, R, v);
#pragma unroll
  for (int p = 0; p < Q; ++p) stream_store(&lam[at(p, c.idx)], solid ? 0.0 : v[p]);
}

// Faces of non-periodic axes, flattened: face f = (axis, side) holds
// batch * (product of the other two extents) cells starting at start[f].
struct Faces {
  int count;
  int axis[6], side[6];
  long long start[7];
};

// lambda_T = (d(e, beta)/d S_T)^T (dL/de, dL/dbeta), cell-local.
template <int ST, class TC>
__global__ __launch_bounds__(BLOCK) void k_moments_adjoint(
    const Geom g, const Phys ph, const typename Codec<ST, TC>::elem *__restrict__ S,
    const double *__restrict__ dLde, const double *__restrict__ dLdb,
    typename Codec<ST, TC>::lam *__restrict__ lam) {
  using Cd = Codec<ST, TC>;
  using Lm = typename Cd::lam;
  const Cell c = decode_cell(g);
  if (!c.active) return;
  const size_t cells = (size_t)g.batch * g.per;
  if (solid_at(ph, c.idx)) {
#pragma unroll
    for (int q = 0; q < Q; ++q) lam[at(q, c.idx)] = (Lm)0;
    return;
  }
  double sE = 0.0, sx, sy, sz, gv[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    gv[q] = (double)Cd::dec(S[at(q, c.idx)]);
    sE += gv[q];
  }
  mirror_sums(gv, sx, sy, sz);
  const Inv iv = invert(ph, ph.e_ref + sE, ph.c * sx, ph.c * sy, ph.c * sz);
  const GradEM gm = chain_moments(ph, iv, dLde[c.idx], 0.0, dLdb[c.idx], dLdb[cells + c.idx],
                                  dLdb[2 * cells + c.idx]);
  const double ax = ph.c * gm.gx, ay = ph.c * gm.gy, az = ph.c * gm.gz;
#pragma unroll
  for (int q = 0; q < Q; ++q)
    lam[at(q, c.idx)] = (Lm)(gm.gE + EX[q] * ax + EY[q] * ay + EZ[q] * az);
}

// lambda_0 -> dL/de0, dL/dbeta0 (overwritten) and inflow partials.
template <int ST, class TC>
__global__ __launch_bounds__(BLOCK) void k_init_adjoint(
    const Geom g, const Phys ph, const double *__restrict__ e0, const double *__restrict__ beta0,
    const typename Codec<ST, TC>::lam *__restrict__ lam0, double *__restrict__ de0,
    double *__restrict__ db0, double *__restrict__ part, const InflowState in) {
  using T = double;  // reverse-mode arithmetic is FP64 for every storage
  const Cell c = decode_cell(g);
  const size_t cells = (size_t)g.batch * g.per;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (c.active) {
    de0[c.idx] = 0.0;
    db0[c.idx] = db0[cells + c.idx] = db0[2 * cells + c.idx] = 0.0;
    if (!solid_at(ph, c.idx)) {
      const bool inflow = is_inflow(g, c.x, c.y, c.z);
      T lam[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) lam[q] = (T)lam0[at(q, c.idx)];
      const double e = inflow ? in.e : e0[c.idx];
      const double bx = inflow ? in.bx : beta0[c.idx];
      const double by = inflow ? in.by : beta0[cells + c.idx];
      const double bz = inflow ? in.bz : beta0[2 * cells + c.idx];
      const double g2 = 1.0 / (1.0 - (bx * bx + by * by + bz * bz));
      const double W = ph.wfac * e * g2;
      const EqCoef<T> k = eq_coef<T>(ph, 0.0, e, W, bx, by, bz);
      const LamEq L = lam_eq(lam_sums(lam, k), ph, W, bx, by, bz);
      double gr[4];
      eq_param_grad(ph, L, e, bx, by, bz, gr);
      if (inflow) {
        for (int k2 = 0; k2 < 4; ++k2) acc[1 + k2] = gr[k2];
      } else {
        de0[c.idx] = gr[0];
        db0[c.idx] = gr[1];
        db0[cells + c.idx] = gr[2];
        db0[2 * cells + c.idx] = gr[3];
      }
    }
  }
  double out[5];
  block_sum<5>(acc, out);
  if (threadIdx.x == 0)
    for (int k2 = 0; k2 < 5; ++k2) part[(size_t)c.L * 5 + k2] = out[k2];
}

// Cell words: solid bit from the caller's mask; bounce bit q when the
// resolved pull source of direction q (wrapped or clamped) is solid; "near"
// when any of the 18 moving directions bounces.
__global__ __launch_bounds__(BLOCK) void k_classify(const Geom g, const uint8_t *__restrict__ solid,
                                                    uint32_t *__restrict__ cls) {
  const Cell c = decode_cell(g);
  if (!c.active) return;
  uint32_t v = solid[c.idx] ? CLS_SOLID : 0u;
  for (int q = 0; q < Q; ++q) {
    bool cl = false;
    const int sx = resolve(g, 0, c.x - EX[q], cl);
    const int sy = resolve(g, 1, c.y - EY[q], cl);
    const int sz = resolve(g, 2, c.z - EZ[q], cl);
    if (solid[cell_index(g, c.b, sx, sy, sz)]) {
      v |= 1u << (CLS_BOUNCE + q);
      if (q > 0) v |= CLS_NEAR;
    }
  }
  cls[c.idx] = v;
}

// ---------------------------------------------------------------------------
// In-place streaming (AA pattern): one state buffer A, two alternating
// kernels.  Representation "swapped": A holds S_t(x)_q at slot opp(q) of x
// itself; representation "streamed": A holds the pulled, pre-collision
// value P(x)_q = S(source_q(x)) at slot q of x.
//   k_aa_local  (streamed -> swapped): collide in place at the own cell.
//   k_aa_pull_all (swapped -> streamed): pull, collide, and push every
//     post-collision S(x)_q to each cell that will pull it: the plain
//     neighbour x + e_q, x itself (slot opp(q)) when x's pull of opp(q)
//     bounces off a solid, and the readers whose pull of q is clamped onto
//     x (enumerated per clamp pattern).  Each location of A is read and
//     written by the same cell only, so the kernel is race-free in place.
// A value needed by two readers, a face cell's S(x)_q pulled both by its
// plain neighbour and by a face reader whose pull is clamped onto x, is
// copied by k_aa_local into the face buffer Fb ([2][Q][face cells], one copy
// per non-periodic face the cell lies on); clamped pulls read it there.
struct FaceMap {
  int id[3][2];          // face index of (axis, side), -1 on a periodic axis
  long long start[7];    // first flattened position of each face
  long long nf;          // face cells in total
  int count;
};

__device__ __forceinline__ long long face_pos(const Geom &g, const FaceMap &fm, int f, int a,
                                              int b, int x, int y, int z) {
  const int co[3] = {x, y, z};
  const int u = a == 0 ? 1 : 0, v = a == 2 ? 1 : 2;
  return fm.start[f] + ((long long)b * g.n[v] + co[v]) * g.n[u] + co[u];
}

// Event flags of one update: unphysical moments (counter 0) and an f^eq
// with a non-positive component (counter 1).
constexpr uint32_t EV_UNPHYSICAL = 1u;
constexpr uint32_t EV_FNEG = 2u;

__device__ __forceinline__ void count_events(uint32_t ev, unsigned long long *ctr) {
  count_lanes((ev & EV_UNPHYSICAL) != 0u, ctr, 0);
  count_lanes((ev & EV_FNEG) != 0u, ctr, 1);
}

// Relax both populations of one update with the same arithmetic as k_step
// and hand each post-collision value to sg(q, v) / sf(q, v) as soon as it is
// formed (g first, then f), so that the pre-collision values die early;
// returns the update's event flags.
template <class Cd, class SG, class SF>
__device__ __forceinline__ uint32_t collide_emit(const Phys &ph, const Cell &c,
                                             const typename Cd::calc (&pg)[Q],
                                             const typename Cd::calc (&pf)[Q], const SG &sg,
                                             const SF &sf) {
  using T = typename Cd::calc;
  using Sm = typename Cd::sum;
  Sm sE, sx, sy, sz;
  moment_sums(pg, sE, sx, sy, sz);
  const Inv iv = invert(ph, ph.e_ref + (double)sE, ph.c * (double)sx, ph.c * (double)sy,
                        ph.c * (double)sz);
  EqCoef<T> k = eq_coef<T>(ph, 0.0, iv.eps, iv.W, iv.bx, iv.by, iv.bz);
  const T om = (T)omega_of(ph, c.b, c.idx);
  constexpr bool fix = !std::is_same<Sm, T>::value;  // FP32 equilibrium, FP64 moments
  const EqFix ef = fix ? eq_fix(k, sE, sx, sy, sz) : EqFix{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const T eq = fix ? geq_fixed(k, ef, q) : geq_dev(k, q);
    sg(q, Cd::enc(pg[q] + om * (eq - pg[q])));
  }
  Sm sN = (Sm)0;
#pragma unroll
  for (int q = 0; q < Q; ++q) sN += (Sm)pf[q];
  const double N = ph.n_ref + (double)sN;
  k.N = (T)N;
  k.Nd = (T)(N - ph.n_ref);
#pragma unroll
  for (int q = 0; q < Q; ++q) sf(q, Cd::enc(pf[q] + om * (feq_dev(k, q) - pf[q])));
  return (iv.bad ? EV_UNPHYSICAL : 0u) |
         (feq_nonpositive(iv.bx, iv.by, iv.bz, ph.inv_c) ? EV_FNEG : 0u);
}

// Relax both populations of one update in place (pre -> post) with the same
// arithmetic as k_step; returns the update's event flags.
template <class Cd>
__device__ __forceinline__ uint32_t collide_inplace(const Phys &ph, const Cell &c,
                                                    typename Cd::calc (&pg)[Q],
                                                    typename Cd::calc (&pf)[Q]) {
  using T = typename Cd::calc;
  using Sm = typename Cd::sum;
  Sm sE, sx, sy, sz;
  moment_sums(pg, sE, sx, sy, sz);
  const Inv iv = invert(ph, ph.e_ref + (double)sE, ph.c * (double)sx, ph.c * (double)sy,
                        ph.c * (double)sz);
  EqCoef<T> k = eq_coef<T>(ph, 0.0, iv.eps, iv.W, iv.bx, iv.by, iv.bz);
  const T om = (T)omega_of(ph, c.b, c.idx);
  Sm sN = (Sm)0;
#pragma unroll
  for (int q = 0; q < Q; ++q) sN += (Sm)pf[q];
  const double N = ph.n_ref + (double)sN;
  constexpr bool fix = !std::is_same<Sm, T>::value;  // FP32 equilibrium, FP64 moments
  const EqFix ef = fix ? eq_fix(k, sE, sx, sy, sz) : EqFix{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const T eq = fix ? geq_fixed(k, ef, q) : geq_dev(k, q);
    pg[q] = pg[q] + om * (eq - pg[q]);
  }
  k.N = (T)N;
  k.Nd = (T)(N - ph.n_ref);
#pragma unroll
  for (int q = 0; q < Q; ++q) pf[q] = pf[q] + om * (feq_dev(k, q) - pf[q]);
  return (iv.bad ? EV_UNPHYSICAL : 0u) |
         (feq_nonpositive(iv.bx, iv.by, iv.bz, ph.inv_c) ? EV_FNEG : 0u);
}

// Initial state into the in-place layout: a state written in the natural
// layout is permuted (slot q -> slot opp(q)) cell by cell, and face cells
// fill their copies in Fb.
template <int ST, class TC>
__global__ __launch_bounds__(BLOCK) void k_aa_swap(const Geom g, const Phys ph, const FaceMap fm,
                                                   typename Codec<ST, TC>::elem *__restrict__ A,
                                                   typename Codec<ST, TC>::elem *__restrict__ Fb) {
  using El = typename Codec<ST, TC>::elem;
  const Cell c = decode_cell(g);
  if (!c.active || solid_at(ph, c.idx)) return;
  const size_t qs = (size_t)g.qs;
  El v[2 * Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    v[q] = A[at(q, c.idx)];
    v[Q + q] = A[Q * qs + at(q, c.idx)];
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    A[at(OPP[q], c.idx)] = v[q];
    A[Q * qs + at(OPP[q], c.idx)] = v[Q + q];
  }
  const int co[3] = {c.x, c.y, c.z};
  for (int a = 0; a < 3; ++a) {
    if (g.periodic[a]) continue;
    const int sd = co[a] == 0 ? 0 : (co[a] == g.n[a] - 1 ? 1 : -1);
    if (sd < 0) continue;
    const long long t = face_pos(g, fm, fm.id[a][sd], a, c.b, c.x, c.y, c.z);
    for (int q = 0; q < 2 * Q; ++q) Fb[(size_t)q * fm.nf + t] = v[q];
  }
}

// Cells of the in-place pull kernel's fast path: no solid neighbour, not an
// inflow cell, and off every face of a non-periodic axis (pulls and pushes
// then reach plain neighbours only; pushes into an inflow cell's slots are
// overwritten by its held values at the next local step, so the layer next
// to an inflow plane is plain too).
__device__ __forceinline__ bool aa_plain(const Geom &g, const Phys &ph, const Cell &c) {
  const uint32_t cls = ph.cls ? ph.cls[c.idx] : 0u;
  if ((cls & (CLS_SOLID | CLS_NEAR)) || is_inflow(g, c.x, c.y, c.z)) return false;
  const int co[3] = {c.x, c.y, c.z};
  for (int a = 0; a < 3; ++a)
    if (!g.periodic[a] && (co[a] < 1 || co[a] > g.n[a] - 2)) return false;
  return true;
}

// flag[cell] = 1 for the non-solid cells off the fast path (the host lists them).
__global__ __launch_bounds__(BLOCK) void k_mark_aa(const Geom g, const Phys ph,
                                                   uint8_t *__restrict__ flag) {
  const Cell c = decode_cell(g);
  if (!c.active) return;
  flag[c.idx] = (!solid_at(ph, c.idx) && !aa_plain(g, ph, c)) ? (uint8_t)1 : (uint8_t)0;
}

// Face copies of one cell's post-collision values (one per non-periodic face
// the cell lies on).  Only the directions that a clamped pull reads are
// copied: a pull of q clamped onto the low face of axis a has e_qa = +1, onto
// the high face e_qa = -1 (five directions per face).
template <class El, class VF, class VG>
__device__ __forceinline__ void aa_face_copies(const Geom &g, const FaceMap &fm, const Cell &c,
                                               El *__restrict__ Fb, const VF &of, const VG &og) {
  const int co[3] = {c.x, c.y, c.z};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (g.periodic[a]) continue;
    const int sd = co[a] == 0 ? 0 : (co[a] == g.n[a] - 1 ? 1 : -1);
    if (sd < 0) continue;
    const long long t = face_pos(g, fm, fm.id[a][sd], a, c.b, c.x, c.y, c.z);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = a == 0 ? EX[q] : (a == 1 ? EY[q] : EZ[q]);  // compile-time
      if (e == 0 || (e == 1) != (sd == 0)) continue;
      Fb[(size_t)q * fm.nf + t] = of(q);
      Fb[(size_t)(Q + q) * fm.nf + t] = og(q);
    }
  }
}

template <int ST, class TC>
__global__ __launch_bounds__(BLOCK) void k_aa_local(const Geom g, const Phys ph, const FaceMap fm,
                                                    typename Codec<ST, TC>::elem *__restrict__ A,
                                                    typename Codec<ST, TC>::elem *__restrict__ Fb,
                                                    const HeldEq<typename Codec<ST, TC>::elem> in_eq,
                                                    unsigned long long *__restrict__ counters) {
  using Cd = Codec<ST, TC>;
  using T = typename Cd::calc;
  using El = typename Cd::elem;
  const Cell c = decode_cell(g);
  uint32_t ev = 0u;
  if (c.active && !solid_at(ph, c.idx)) {
    const size_t qs = (size_t)g.qs;
    El *__restrict__ Af = A;
    El *__restrict__ Ag = A + Q * qs;
    const bool face = fm.count > 0 && !aa_plain(g, ph, c);
    // Inflow cells run the common path and store their held values instead
    // of the collision's (no divergent branch in the waves that hold them).
    const bool inflow = is_inflow(g, c.x, c.y, c.z);
    T pf[Q], pg[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      pf[q] = Cd::dec(Af[at(q, c.idx)]);
      pg[q] = Cd::dec(Ag[at(q, c.idx)]);
    }
    ev = collide_emit<Cd>(
        ph, c, pg, pf, [&](int q, El v) { Ag[at(OPP[q], c.idx)] = inflow ? in_eq.v[Q + q] : v; },
        [&](int q, El v) { Af[at(OPP[q], c.idx)] = inflow ? in_eq.v[q] : v; });
    if (inflow) ev = 0u;
    // face cells copy what they just stored (same thread: reads see the writes)
    if (face)
      aa_face_copies(g, fm, c, Fb, [&](int q) { return Af[at(OPP[q], c.idx)]; },
                     [&](int q) { return Ag[at(OPP[q], c.idx)]; });
  }
  count_events(ev, counters);
}

// f(std::integral_constant<int, q>) for q = 0 .. Q-1, each a separate
// instance of the body.
template <class F, int... I>
__device__ __forceinline__ void static_for_q_(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <class F>
__device__ __forceinline__ void static_for_q(F &&f) {
  static_for_q_(f, std::make_integer_sequence<int, Q>{});
}

// Solid flags of the 27 cells around c (offsets -1..1 per axis, each
// resolved as a pull resolves its source: wrapped on periodic axes, clamped
// on the others), bit (dz+1)*9 + (dy+1)*3 + (dx+1).  All 27 loads are issued
// together, before the general path stores anything, so that none of its
// decisions waits on a load behind a store.
__device__ __forceinline__ unsigned solid_around(const Geom &g, const Phys &ph, const Cell &c) {
  if (!ph.cls) return 0u;
  unsigned m = 0u;
  bool cl = false;
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int i = cell_index(g, c.b, resolve(g, 0, c.x + dx, cl),
                                       resolve(g, 1, c.y + dy, cl), resolve(g, 2, c.z + dz, cl));
        if (ph.cls[i] & CLS_SOLID) m |= 1u << ((dz + 1) * 9 + (dy + 1) * 3 + (dx + 1));
      }
  return m;
}

__device__ __forceinline__ bool solid_off(unsigned m, int dx, int dy, int dz) {
  return (m >> ((dz + 1) * 9 + (dy + 1) * 3 + (dx + 1))) & 1u;
}

// In-place pull step of one updated cell on the general path (listed cells:
// near a solid, inflow, or on a face of a non-periodic axis).
template <class Cd>
__device__ __forceinline__ uint32_t aa_pull_general(const Geom &g, const Phys &ph, const FaceMap &fm,
                                                typename Cd::elem *__restrict__ A,
                                                const typename Cd::elem *__restrict__ Fb,
                                                const HeldEq<typename Cd::elem> &in_eq,
                                                const Cell &c) {
  using T = typename Cd::calc;
  using El = typename Cd::elem;
  const size_t qs = (size_t)g.qs;
  El *__restrict__ Af = A;
  El *__restrict__ Ag = A + Q * qs;
  const bool inflow = is_inflow(g, c.x, c.y, c.z);
  const int co[3] = {c.x, c.y, c.z};
  const unsigned sm = solid_around(g, ph, c);
  uint32_t ev = 0u;
  T pf[Q], pg[Q];
  if (inflow) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      pf[q] = Cd::dec(in_eq.v[q]);
      pg[q] = Cd::dec(in_eq.v[Q + q]);
    }
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      bool clamped = false;
      const int sx = resolve(g, 0, c.x - EX[q], clamped);
      const int sy = resolve(g, 1, c.y - EY[q], clamped);
      const int sz = resolve(g, 2, c.z - EZ[q], clamped);
      const bool bounce = solid_off(sm, -EX[q], -EY[q], -EZ[q]);
      // the first clamped axis names the face copy to read
      int a = -1, sd = 0;
#pragma unroll
      for (int k = 2; k >= 0; --k) {
        const int e = k == 0 ? EX[q] : (k == 1 ? EY[q] : EZ[q]);
        const int r = co[k] - e;
        if (!g.periodic[k] && (r < 0 || r >= g.n[k])) {
          a = k;
          sd = r < 0 ? 0 : 1;
        }
      }
      if (clamped && !bounce && a >= 0) {  // bounce-back takes precedence
        const long long t = face_pos(g, fm, fm.id[a][sd], a, c.b, sx, sy, sz);
        pf[q] = Cd::dec(Fb[(size_t)q * fm.nf + t]);
        pg[q] = Cd::dec(Fb[(size_t)(Q + q) * fm.nf + t]);
      } else {
        // plain source: S(src)_q sits at slot opp(q); bounce-back: S(x)_opp(q)
        // sits at slot q
        const size_t o = bounce ? at(q, c.idx) : at(OPP[q], cell_index(g, c.b, sx, sy, sz));
        pf[q] = Cd::dec(Af[o]);
        pg[q] = Cd::dec(Ag[o]);
      }
    }
    ev = collide_inplace<Cd>(ph, c, pg, pf);
  }
  // one instance of the body per direction (q a constant, so that pf[q] and
  // pg[q] stay in registers and impossible clamp patterns fold away)
  static_for_q([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int e[3] = {EX[q], EY[q], EZ[q]};
    const El vf = inflow ? in_eq.v[q] : Cd::enc(pf[q]);
    const El vg = inflow ? in_eq.v[Q + q] : Cd::enc(pg[q]);
    // Every reader whose pull of q resolves to this cell: along each axis in
    // the clamp pattern m it sits on this cell's face and its pull leaves the
    // domain there (clamped back onto this cell); along the other axes it is
    // the plain neighbour co + e.  m = 0 is the plain receiver x + e_q.
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      if ((m & 1) && e[0] == 0) continue;
      if ((m & 2) && e[1] == 0) continue;
      if ((m & 4) && e[2] == 0) continue;
      bool ok = true;
      int rc[3], off[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int n = g.n[d];
        if ((m >> d) & 1) {
          ok = ok && !g.periodic[d] &&
               ((e[d] == 1 && co[d] == 0) || (e[d] == -1 && co[d] == n - 1));
          rc[d] = co[d];
          off[d] = 0;
        } else {
          int r = co[d] + e[d];
          if (g.periodic[d]) {
            if (r < 0) r += n;
            if (r >= n) r -= n;
          } else {
            ok = ok && r >= 0 && r < n;
          }
          rc[d] = r;
          off[d] = e[d];
        }
      }
      if (ok && !solid_off(sm, off[0], off[1], off[2]) && !is_inflow(g, rc[0], rc[1], rc[2])) {
        const size_t o = at(q, cell_index(g, c.b, rc[0], rc[1], rc[2]));
        Af[o] = vf;
        Ag[o] = vg;
      }
    }
    // bounce-back receiver: this cell, when its pull of opp(q) hits a solid
    if (!inflow && solid_off(sm, e[0], e[1], e[2])) {
      Af[at(OPP[q], c.idx)] = vf;
      Ag[at(OPP[q], c.idx)] = vg;
    }
  });
  return ev;
}

// In-place pull step in one launch: the first nlist workgroups (a multiple
// of 8, so that the rest keep their XCD placement) take the listed cells on
// the general path, the others the fast path; the two sets of cells touch
// disjoint locations of A, and the latency-bound listed work overlaps the
// streaming work.
template <int ST, class TC>
__global__ __launch_bounds__(BLOCK) void k_aa_pull_all(const Geom g, const Phys ph,
                                                       const FaceMap fm, int nlist,
                                                       const int *__restrict__ list,
                                                       typename Codec<ST, TC>::elem *__restrict__ A,
                                                       const typename Codec<ST, TC>::elem *__restrict__ Fb,
                                                       const HeldEq<typename Codec<ST, TC>::elem> in_eq,
                                                       unsigned long long *__restrict__ counters) {
  using Cd = Codec<ST, TC>;
  using T = typename Cd::calc;
  using El = typename Cd::elem;
  uint32_t ev = 0u;
  if ((int)blockIdx.x < nlist) {
    const int li = list[(size_t)blockIdx.x * BLOCK + threadIdx.x];
    if (li >= 0) ev = aa_pull_general<Cd>(g, ph, fm, A, Fb, in_eq, cell_at(g, li));
  } else {
    const Cell c = decode_cell(g, (int)blockIdx.x - nlist);
    if (c.active && aa_plain(g, ph, c)) {
      const size_t qs = (size_t)g.qs;
      El *__restrict__ Af = A;
      El *__restrict__ Ag = A + Q * qs;
      const FaceCorr fc = face_corr(g, c);
      T pf[Q], pg[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const size_t o = at(OPP[q], src_fast(g, c, fc, q));
        pf[q] = Cd::dec(Af[o]);
        pg[q] = Cd::dec(Ag[o]);
      }
      ev = collide_emit<Cd>(
          ph, c, pg, pf, [&](int q, El v) { Ag[at(q, src_fast(g, c, fc, OPP[q]))] = v; },
          [&](int q, El v) { Af[at(q, src_fast(g, c, fc, OPP[q]))] = v; });
    }
  }
  count_events(ev, counters);
}

}  // namespace rlb
