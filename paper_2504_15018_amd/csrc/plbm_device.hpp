// Device-side definitions shared by every kernel translation unit of libplbm:
// lattice traits, storage codecs, the pseudo-potential and the kernel
// parameter block.  gfx950 (CDNA4), wave64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace plbm {

// ---------------------------------------------------------------------------
// Lattice traits.  Kernel axes are (x, y, z) with x fastest in memory and z the
// marching axis.  D2Q9 runs as a lattice of extent 1 in y: its second
// component maps to the marching axis z, so a 2-D lattice (nx, ny) is held as
// (nx, 1, ny) with the same memory layout f[q][y][x].
//
// D2Q9 order is eq. (VelocitySet) of the paper; D3Q19 order: rest, the six
// axis directions as opposite pairs, the twelve edge directions as pairs.

struct D2Q9L {
  static constexpr int Q = 9, D = 2, HY = 0;
  static constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static constexpr int cy[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr int cz[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  static constexpr double w[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                                  1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
  // physical component a (0: x, 1: y of the 2-D lattice)
  static constexpr int c(int i, int a) { return a == 0 ? cx[i] : cz[i]; }
  // opposite pairs (pa[p], pb[p]) with c_pb = -c_pa
  static constexpr int P = 4;
  static constexpr int pa[4] = {1, 2, 5, 6};
  static constexpr int pb[4] = {3, 4, 7, 8};
};

struct D3Q19L {
  static constexpr int Q = 19, D = 3, HY = 1;
  static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
  static constexpr double w[19] = {1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                                   1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                   1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                   1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
  static constexpr int c(int i, int a) { return a == 0 ? cx[i] : (a == 1 ? cy[i] : cz[i]); }
  static constexpr int P = 9;
  static constexpr int pa[9] = {1, 3, 5, 7, 9, 11, 13, 15, 17};
  static constexpr int pb[9] = {2, 4, 6, 8, 10, 12, 14, 16, 18};
};

// MRT extension: the non-hydrodynamic moments whose rate differs from the
// stress rate 1/tau(rho).  The collision is written as BGK at omega = 1/tau
// plus a correction on these moments only:
//   f* = f + Fhat - omega v - sum_k (s_k - omega) P_k(c_i) (sum_j P_k(c_j) v_j) / |P_k|^2,
//   v  = f - f_eq + Fhat/2,
// which equals m* = m - S(m - m_eq) + (I - S/2) M Fhat, f* = M^-1 m* for an
// orthogonal basis in which the stress moments relax at omega (the mass and
// momentum rows of M v vanish identically).
// Moment polynomials (|c|^2 = c2):
//   D2Q9  (Lallemand-Luo): e = 3c2-4, eps = (9c2^2-21c2+8)/2, q_a = (3c2-5)c_a
//   D3Q19 (d'Humieres):    e = 19c2-30, eps = (21c2^2-53c2+24)/2, q_a = (5c2-9)c_a,
//                          m_x = (cy^2-cz^2)cx, m_y = (cz^2-cx^2)cy, m_z = (cx^2-cy^2)cz
template <class L>
struct MrtCorr;

template <>
struct MrtCorr<D2Q9L> {
  static constexpr int K = 4;  // e, eps, q_x, q_y
  static constexpr int rate_class[4] = {0, 1, 2, 2};  // index into {s_e, s_eps, s_q, s_m}
  static constexpr double P(int k, int i) {
    double cx = D2Q9L::c(i, 0), cy = D2Q9L::c(i, 1), c2 = cx * cx + cy * cy;
    return k == 0 ? 3 * c2 - 4 : k == 1 ? (9 * c2 * c2 - 21 * c2 + 8) / 2 : k == 2 ? (3 * c2 - 5) * cx : (3 * c2 - 5) * cy;
  }
};

template <>
struct MrtCorr<D3Q19L> {
  static constexpr int K = 8;  // e, eps, q_x, q_y, q_z, m_x, m_y, m_z
  static constexpr int rate_class[8] = {0, 1, 2, 2, 2, 3, 3, 3};
  static constexpr double P(int k, int i) {
    double cx = D3Q19L::c(i, 0), cy = D3Q19L::c(i, 1), cz = D3Q19L::c(i, 2);
    double c2 = cx * cx + cy * cy + cz * cz;
    switch (k) {
      case 0: return 19 * c2 - 30;
      case 1: return (21 * c2 * c2 - 53 * c2 + 24) / 2;
      case 2: return (5 * c2 - 9) * cx;
      case 3: return (5 * c2 - 9) * cy;
      case 4: return (5 * c2 - 9) * cz;
      case 5: return (cy * cy - cz * cz) * cx;
      case 6: return (cz * cz - cx * cx) * cy;
      default: return (cx * cx - cy * cy) * cz;
    }
  }
};

// 1 / |P_k|^2 as a compile-time table (folded into the unrolled kernels).
template <class L>
struct MrtInvNorm {
  struct Tab {
    double v[MrtCorr<L>::K];
  };
  static constexpr Tab make() {
    Tab t{};
    for (int k = 0; k < MrtCorr<L>::K; ++k) {
      double s = 0;
      for (int i = 0; i < L::Q; ++i) s += MrtCorr<L>::P(k, i) * MrtCorr<L>::P(k, i);
      t.v[k] = 1.0 / s;
    }
    return t;
  }
  static constexpr Tab tab = make();
};

// ---------------------------------------------------------------------------
// Storage codecs.  Shifted storage keeps f_i - w_i rho0 (one global rho0) so
// that half-precision formats spend their bits on the deviation from the
// reference state.  Locally shifted storage (local = true) keeps
// f_i - w_i rho_ref(x) instead, with rho_ref(x) a per-node reference density
// held in its own 16-bit array: the node's density at the previous step,
// rounded to half precision.  The population f_i(x) is encoded with the
// reference of the node x that will decode it, so encoder and decoder always
// use the same value and its precision does not matter.

// dec/enc work in the arithmetic type C; dec64/enc64 are the float64 forms
// used by initialisation and population I/O.
struct StF64 {
  using T = double;
  using C = double;  // arithmetic type
  static constexpr bool shifted = false;
  static constexpr bool local = false;
  static __device__ __forceinline__ C dec(T v, C) { return v; }
  static __device__ __forceinline__ T enc(C f, C) { return f; }
  static __device__ __forceinline__ double dec64(T v, double) { return v; }
  static __device__ __forceinline__ T enc64(double f, double) { return f; }
};

struct StF32 {
  using T = float;
  using C = float;
  static constexpr bool shifted = false;
  static constexpr bool local = false;
  static __device__ __forceinline__ C dec(T v, C) { return v; }
  static __device__ __forceinline__ T enc(C f, C) { return f; }
  static __device__ __forceinline__ double dec64(T v, double) { return (double)v; }
  static __device__ __forceinline__ T enc64(double f, double) { return (float)f; }
};

// The shift is added and subtracted without contraction: with a per-node
// reference the shift is a product w_i rho_ref, and a multiply fused into the
// encoder's subtraction but not into the decoder's addition (or the reverse)
// leaves a systematic difference of one rounding of that product per
// population and step, which a uniform region accumulates as mass drift.
struct StF16S {
  using T = _Float16;
  using C = float;
  static constexpr bool shifted = true;
  static constexpr bool local = false;
  static __device__ __forceinline__ C dec(T v, C shift) {
#pragma clang fp contract(off)
    return (float)v + shift;
  }
  static __device__ __forceinline__ T enc(C f, C shift) {  // RNE
#pragma clang fp contract(off)
    return (_Float16)(f - shift);
  }
  // float64 forms: plain operation order, no fused multiply-add with the shift
  static __device__ __forceinline__ double dec64(T v, double shift) {
#pragma clang fp contract(off)
    return (double)(float)v + shift;
  }
  static __device__ __forceinline__ T enc64(double f, double shift) {
#pragma clang fp contract(off)
    return (_Float16)(float)(f - shift);
  }
};

struct StBF16S {
  using T = uint16_t;  // bfloat16 bit pattern
  using C = float;
  static constexpr bool shifted = true;
  static constexpr bool local = false;
  static __device__ __forceinline__ C dec(T v, C shift) {
#pragma clang fp contract(off)
    return __uint_as_float(((uint32_t)v) << 16) + shift;
  }
  // round to nearest even in hardware (v_cvt_pk_bf16_f32); NaN stays a quiet NaN
  static __device__ __forceinline__ T enc(C f, C shift) {
#pragma clang fp contract(off)
    return __builtin_bit_cast(uint16_t, (__bf16)(f - shift));
  }
  static __device__ __forceinline__ double dec64(T v, double shift) {
#pragma clang fp contract(off)
    return (double)__uint_as_float(((uint32_t)v) << 16) + shift;
  }
  static __device__ __forceinline__ T enc64(double f, double shift) {
#pragma clang fp contract(off)
    return enc((float)(f - shift), 0.0f);
  }
};

struct StF16R : StF16S {
  static constexpr bool local = true;
};

struct StBF16R : StBF16S {
  static constexpr bool local = true;
};

// Reference density code of locally shifted storage: IEEE half bits.
using RefT = _Float16;

// ---------------------------------------------------------------------------
// Kernel parameter block: one per lattice, resident in device memory (the
// batch launch reads one per slot).

enum : int32_t { EOS_PAPER = 0, EOS_PR = 1 };

struct KParams {
  void* pop[2];       // A-B population arrays, each Q*N entries (in-place pattern: both the one array)
  void* ref[2];       // locally shifted storage: A-B reference densities, N + 256 half values
  void* psi;          // in-place pattern: psi of every node at the current time (arithmetic type)
  double* aux;        // float64 staging, 4*N
  float* uprev;       // previous velocity for the residual, D*N
  double* red;        // reduction partials
  int64_t N;          // nodes
  int32_t nx, ny, nz; // kernel axes (2-D lattices: ny = 1)
  int32_t bb_z;       // half-way bounce-back walls on the marching axis
  int32_t tiles_x, tiles_y, tiles_z, cz;  // tiling: tiles per axis, planes per z chunk
  // z partition in two classes: items [0, ntl) split the first ncl tile
  // columns into chunks of cz planes, the other items the remaining columns
  // into chunks of cz2 (ncl = ntl = 0: one uniform class of cz2)
  int32_t cz2, ncl, ntl;
  int32_t ntiles;
  int32_t eos;
  // paper EOS: p = K [2 r^3 + (rv - 2 rl) r^2 + sqrt(rv) sqrt(r) (-3 r^2 + 2 rl r + rl^2)]
  double K, e_rv, e_rl, e_sqrt_rv;
  // Peng-Robinson: p = r R T / (1 - b r) - a alpha r^2 / (1 + 2 b r - b^2 r^2)
  double pr_RT, pr_b, pr_aalpha;
  double eps, kappa, G;
  double tau_v, tau_slope, rho_v;  // tau(rho) = tau_v + (rho - rho_v) tau_slope
  double Fg[3];
  double rates[4];                 // s_e, s_eps, s_q, s_m
  double rho0_shift;
  int32_t parity;  // batch slots: phase offset of this lattice (its time parity)
  int32_t aa;      // in-place (AA) pattern
  double rho_wall[2];  // wall densities below / above (wetting walls); <= 0: mirror psi ghost
  int32_t nxb;     // x blocks of one 128-byte line per row (storage layout)
  int64_t zblock;  // bytes of one z plane of stored populations (node data + trash)
  int64_t zdata;   // bytes of the node data of one z plane
  // well-balanced scheme: chemical-potential force and constant-pressure equilibrium
  int32_t wb;
  double wb_k, wb_rho0;
  void* wb_mu;  // chemical potential of every node at the current time (arithmetic type)
};

// Stored population layout: A[z][y][x / XB][q][x % XB] with XB = 128 bytes /
// sizeof(T) nodes (16 for float64, 32 for float32, 64 for 16-bit storage), so
// that the innermost unit, one direction of XB nodes, is one 128-byte line in
// every format (16-bit blocks of 32 nodes, half a line per direction, ran the
// update 11 % slower).  A block holds QS >= Q direction slots, so every block
// starts on a line and a tile row of a multiple of XB nodes covers whole
// lines that no other tile touches.  All directions of a node sit at a common
// offset plus q * QB bytes.
#ifndef PLBM_XB
#define PLBM_XB 64
#endif
template <class T>
struct Lines {
  static constexpr int XB = (128 / (int)sizeof(T)) < PLBM_XB ? (128 / (int)sizeof(T)) : PLBM_XB;
  static constexpr int QB = XB * (int)sizeof(T);
  template <int Q>
  static constexpr int slots() {
    return (Q * QB + 127) / 128 * 128 / QB;
  }
};

// Equation-of-state constants held in scalar registers by the kernels.
struct EosK {
  int32_t kind;
  double K, c2, sv, rl, rl2;  // paper EOS: p = K [2 r^3 + c2 r^2 + sv sqrt(r) (-3 r^2 + 2 rl r + rl2)]
  double RT, b, aa;           // Peng-Robinson: p = r RT / (1 - b r) - aa r^2 / (1 + 2 b r - b^2 r^2)
};

__device__ __forceinline__ EosK load_eos(const KParams* __restrict__ kp) {
  EosK e;
  e.kind = kp->eos;
  e.K = kp->K;
  e.c2 = kp->e_rv - 2.0 * kp->e_rl;
  e.sv = kp->e_sqrt_rv;
  e.rl = kp->e_rl;
  e.rl2 = kp->e_rl * kp->e_rl;
  e.RT = kp->pr_RT;
  e.b = kp->pr_b;
  e.aa = kp->pr_aalpha;
  return e;
}

// psi(rho) of eq. (Interaction_Potential), G = -1, lattice units, float64.
// The two Peng-Robinson fractions share one division.  Returns the clamped
// value; *neg is set when the radicand was negative.
__device__ __forceinline__ double psi_radicand(const EosK& e, double rho) {
  double pe;
  const double r2 = rho * rho;
  if (e.kind == EOS_PAPER) {
    const double s = sqrt(rho);
    pe = e.K * (2.0 * r2 * rho + e.c2 * r2 + e.sv * s * (-3.0 * r2 + 2.0 * e.rl * rho + e.rl2));
  } else {
    const double d1 = 1.0 - e.b * rho;
    const double d2 = 1.0 + 2.0 * e.b * rho - e.b * e.b * r2;
    pe = (rho * e.RT * d2 - e.aa * r2 * d1) / (d1 * d2);
  }
  return 2.0 * (rho * (1.0 / 3.0) - pe);
}

// psi in the arithmetic type C: the radicand (where p_EOS and rho/3 cancel)
// is always float64; a float32 result takes the square root in float32.
template <class C>
__device__ __forceinline__ C psi_eval(const EosK& e, double rho, bool* neg);
template <>
__device__ __forceinline__ double psi_eval<double>(const EosK& e, double rho, bool* neg) {
  const double rad = psi_radicand(e, rho);
  *neg = !(rad >= 0.0);
  return sqrt(rad > 0.0 ? rad : 0.0);
}
template <>
__device__ __forceinline__ float psi_eval<float>(const EosK& e, double rho, bool* neg) {
  const double rad = psi_radicand(e, rho);
  *neg = !(rad >= 0.0);
  return sqrtf(rad > 0.0 ? (float)rad : 0.0f);
}

// Bulk chemical potential per unit mass of the equation of state, float64, up
// to an additive constant: mu_b = int p / rho^2 d rho + p / rho, so that
// d mu_b / d rho = p'(rho) / rho (the well-balanced scheme's force).
__device__ __forceinline__ double mu_bulk(const EosK& e, double rho) {
  if (e.kind == EOS_PAPER) {
    // p = K [2 r^3 + c2 r^2 - 3 sv r^2.5 + 2 sv rl r^1.5 + sv rl^2 r^0.5]
    const double s = sqrt(rho);
    return e.K * (3.0 * rho * rho + 2.0 * e.c2 * rho - 5.0 * e.sv * rho * s + 6.0 * e.sv * e.rl * s -
                  e.sv * e.rl2 / s);
  }
  // Peng-Robinson: p = r RT / (1 - b r) - aa r^2 / (1 + 2 b r - b^2 r^2)
  const double r2 = 1.4142135623730951;
  const double d1 = 1.0 - e.b * rho;
  const double d2 = 1.0 + 2.0 * e.b * rho - e.b * e.b * rho * rho;
  return e.RT * log(rho / d1) - e.aa / (2.0 * r2 * e.b) * log((r2 - 1.0 + e.b * rho) / (r2 + 1.0 - e.b * rho)) +
         e.RT / d1 - e.aa * rho / d2;
}

// Reciprocal: IEEE division in float64; the hardware reciprocal (1 ulp) in float32.
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

}  // namespace plbm
