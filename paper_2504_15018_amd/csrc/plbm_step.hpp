// The fused P-LBM step kernel (and its moment / reduction read-out modes).
//
// One workgroup owns a TX x TY tile of (x, y) columns and marches through a
// chunk of z planes.  Populations are stored post-collision ("pull" A-B
// pattern): the state at time t is f_i(x, t) = A_i(x - c_i), and a step writes
// B_i(x) = f*_i(x).  For every plane the workgroup
//   A. pulls the populations of plane z+1 for its tile (kept in registers for
//      the next iteration) and for a one-node halo ring, sums rho and writes
//      psi(rho) (float64 evaluation) into a 4-plane LDS ring;
//   B. after one barrier, evaluates the psi stencil of plane z from LDS, the
//      interaction force, u, tau(rho) and the collision of plane z, and stores
//      the Q post-collision populations with coalesced writes.
// HBM traffic is the algorithmic 2 Q S bytes per node; the halo ring and the
// two extra planes per chunk are re-read from L2 / the Infinity Cache.
//
// The same march carries the well-balanced scheme (SCH_WB), whose force is
// F = -rho grad_d mu + F_g with the chemical potential
// mu = mu_b(rho) - k lap_d rho (mu_b: float64 bulk chemical potential of the
// EOS), lap_d g = 6 sum_i w_i (g(x + c_i) - g(x)), grad_d g = 3 sum_i w_i c_i
// g(x + c_i), and whose equilibrium carries a constant reference density rho0
// on the moving populations at rest.  mu needs rho one node out and the force
// needs mu one node out, so a step is two launches:
//   MODE_MU  the LDS ring holds rho of the pulled populations (tile and halo);
//            phase B evaluates mu of the plane and stores it per node;
//   update   the ring holds mu loaded from that array (the halo waves load one
//            value per node instead of pulling Q populations); phase B forms
//            the force and collides with the well-balanced equilibrium.
// Beyond a half-way bounce-back wall rho and mu mirror the wall-adjacent
// plane (the clamped plane index).
#pragma once

#include <type_traits>
#include <utility>

#include "plbm_device.hpp"

namespace plbm {

#ifndef PLBM_HALO_SPLIT
#define PLBM_HALO_SPLIT 1  // the halo ring is carried by extra waves of its own
#endif
#ifndef PLBM_PREFETCH
#define PLBM_PREFETCH 2  // plane iterations between issuing a plane's loads and summing it
#endif
#ifndef PLBM_MIN_WAVES
#define PLBM_MIN_WAVES 2  // waves per SIMD the register allocation must allow
#endif
#ifndef PLBM_MU_PREFETCH
#define PLBM_MU_PREFETCH 3  // plane loads in flight per wave in the chemical-potential pass
#endif
#ifndef PLBM_HALO_PREFETCH
#define PLBM_HALO_PREFETCH PLBM_PREFETCH  // plane loads in flight per halo wave
#endif
#ifndef PLBM_HALO_PRIO
#define PLBM_HALO_PRIO 1  // wave issue priority of the halo waves (0: that of the tile waves)
#endif

enum : int { COLL_BGK = 0, COLL_MRT = 1 };
enum : int { MODE_STEP = 0, MODE_MOMENTS = 1, MODE_REDUCE = 2, MODE_MU = 3 };
enum : int { SCH_PP = 0, SCH_WB = 1 };  // pseudopotential force / well-balanced scheme

struct WorkItem {
  int32_t slot;
  int32_t tile;
};

// Per-block reduction record (REDUCE mode), float64.
struct RedRec {
  double mass_s, mass_c;  // Neumaier sum and its compensation
  double mom[3];
  double max_u, max_du;
  double flags;  // bit pattern stored as an exact small integer
};

__device__ __forceinline__ void neumaier_add(double& s, double& c, double v) {
  double t = s + v;
  if (fabs(s) >= fabs(v))
    c += (s - t) + v;
  else
    c += (v - t) + s;
  s = t;
}

// Combine two reduction records: compensated mass, summed momentum, maxima,
// or-ed flags.
__device__ __forceinline__ void red_combine(RedRec& o, const RedRec& q) {
  neumaier_add(o.mass_s, o.mass_c, q.mass_s);
  o.mass_c += q.mass_c;
  for (int a = 0; a < 3; ++a) o.mom[a] += q.mom[a];
  o.max_u = fmax(o.max_u, q.max_u);
  o.max_du = fmax(o.max_du, q.max_du);
  o.flags = (double)((int)o.flags | (int)q.flags);
}

// Workgroup reduction of one record per thread, in a fixed order (the result
// is the same on every run): a butterfly over the 64 lanes of each wave with
// cross-lane shuffles, then the per-wave results in wave order by one thread,
// which stores the workgroup's record at *dst.  wl holds NT / 64 records of
// LDS.  Every thread of the workgroup must call it.
template <int NT>
__device__ __forceinline__ void block_reduce_store(RedRec r, RedRec* wl, RedRec* dst) {
  static_assert(NT % 64 == 0, "whole waves");
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    RedRec q;
    q.mass_s = __shfl_xor(r.mass_s, off, 64);
    q.mass_c = __shfl_xor(r.mass_c, off, 64);
#pragma unroll
    for (int a = 0; a < 3; ++a) q.mom[a] = __shfl_xor(r.mom[a], off, 64);
    q.max_u = __shfl_xor(r.max_u, off, 64);
    q.max_du = __shfl_xor(r.max_du, off, 64);
    q.flags = __shfl_xor(r.flags, off, 64);
    red_combine(r, q);
  }
  const int t = threadIdx.x;
  if ((t & 63) == 0) wl[t >> 6] = r;
  __syncthreads();
  if (t == 0) {
    RedRec o = wl[0];
    for (int w = 1; w < NT / 64; ++w) red_combine(o, wl[w]);
    *dst = o;
  }
}

// Map a launch index so that consecutive logical tiles share an XCD (the
// hardware dispatches workgroups round-robin over the 8 XCDs, each with its
// own L2); halo re-reads of neighbouring tiles then hit the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int nfull = nb - (nb & 7);
  if (b >= nfull) return b;
  return (b & 7) * (nfull >> 3) + (b >> 3);
}

// Launch index -> work item of a single-lattice launch whose first ntl items
// (the long chunks of the two-class z partition) must start first: each class
// is XCD-remapped within itself, so the first ntl launch indices stay in the
// long class.
__device__ __forceinline__ int class_remap(int b, int nb, int ntl) {
  if (ntl <= 0 || ntl >= nb) return xcd_remap(b, nb);
  return b < ntl ? xcd_remap(b, ntl) : ntl + xcd_remap(b - ntl, nb - ntl);
}

// Tile column and z range of work item `tile` of a lattice.
__device__ __forceinline__ void tile_extent(const KParams* __restrict__ kp, int tile, int* txi, int* tyi, int* z0,
                                            int* z1) {
  const int tiles_x = kp->tiles_x, ncl = kp->ncl, ntl = kp->ntl;
  int col, cz;
  if (tile < ntl) {
    col = tile % ncl;
    cz = kp->cz;
    *z0 = (tile / ncl) * cz;
  } else {
    const int r = tile - ntl, nc = tiles_x * kp->tiles_y - ncl;
    col = ncl + r % nc;
    cz = kp->cz2;
    *z0 = (r / nc) * cz;
  }
  *txi = col % tiles_x;
  *tyi = col / tiles_x;
  *z1 = min(*z0 + cz, kp->nz);
}

// Loads and stores through a scalar (wave-uniform) base pointer in the global
// address space plus a 32-bit byte offset: global_load/store with an SGPR
// base.  The library keeps every per-direction array below 4 GiB.
template <class T>
__device__ __forceinline__ T gld(const void* base, uint32_t byte_off) {
  typedef const __attribute__((address_space(1))) char gchar;
  typedef const __attribute__((address_space(1))) T gT;
  return *(gT*)((gchar*)base + byte_off);
}

// Element access to a per-node array (psi, reference densities) through a
// global-address-space pointer: global_load/store rather than flat, whose
// completion the LDS counter also waits for.
template <class T>
__device__ __forceinline__ T gld_at(const void* base, uint32_t idx) {
  typedef const __attribute__((address_space(1))) T gT;
  return ((gT*)base)[idx];
}
template <class T>
__device__ __forceinline__ void gst_at(void* base, uint32_t idx, T v) {
  typedef __attribute__((address_space(1))) T gT;
  ((gT*)base)[idx] = v;
}

#ifndef PLBM_NT_STORE
#define PLBM_NT_STORE 1  // populations stored with the non-temporal hint (read again only next step)
#endif
template <class T>
__device__ __forceinline__ void gst(void* base, uint32_t byte_off, T v) {
  typedef __attribute__((address_space(1))) char gchar;
  typedef __attribute__((address_space(1))) T gT;
#if PLBM_NT_STORE
  __builtin_nontemporal_store(v, (gT*)((gchar*)base + byte_off));
#else
  *(gT*)((gchar*)base + byte_off) = v;
#endif
}

// psi stencil and interaction force at one node (Sec. II):
//   M1_a = 3 sum_i w_i psi_i c_ia,  M2_ab = 9 sum_i w_i psi_i c_ia c_ib - 3 delta_ab sum_i w_i psi_i,
//   F = cA psi M1 + cB (M1.M2) + cC M1 tr(M2) + F_g,
// summed over opposite pairs: psi_a + psi_b carries the even moments,
// psi_a - psi_b the odd ones.
template <class L, class C, int W2>
__device__ __forceinline__ void stencil_force(const C* s_m, const C* s_0, const C* s_p, int il, C cA, C cB, C cC,
                                              const C* Fg, C* F) {
  constexpr int D = L::D;
  auto psi_at = [&](int i) {
    const int cz = L::cz[i];
    const C* sl = cz > 0 ? s_p : (cz < 0 ? s_m : s_0);
    return sl[il + L::cy[i] * W2 + L::cx[i]];
  };
  const C psi_c = s_0[il];
  C S0 = (C)L::w[0] * psi_c, S1[D], S2[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    S1[a] = 0;
#pragma unroll
    for (int b = 0; b < D; ++b) S2[a][b] = 0;
  }
#pragma unroll
  for (int p = 0; p < L::P; ++p) {
    const int ia = L::pa[p];
    const C pa = psi_at(ia), pb = psi_at(L::pb[p]);
    const C sum = pa + pb, dif = pa - pb;
    const C w = (C)L::w[ia];
    S0 += w * sum;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int ca = L::c(ia, a);
      if (ca != 0) S1[a] += (C)(ca)*w * dif;
#pragma unroll
      for (int b = a; b < D; ++b) {
        const int cc = ca * L::c(ia, b);
        if (cc != 0) S2[a][b] += (C)(cc)*w * sum;
      }
    }
  }
  C M1[D], M2[D][D], tr = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    M1[a] = (C)3 * S1[a];
#pragma unroll
    for (int b = a; b < D; ++b) {
      M2[a][b] = (C)9 * S2[a][b] - (a == b ? (C)3 * S0 : (C)0);
      M2[b][a] = M2[a][b];
    }
    tr += M2[a][a];
  }
#pragma unroll
  for (int a = 0; a < D; ++a) {
    C m1m2 = 0;
#pragma unroll
    for (int b = 0; b < D; ++b) m1m2 += M1[b] * M2[a][b];
    F[a] = cA * psi_c * M1[a] + cB * m1m2 + cC * M1[a] * tr + Fg[a];
  }
}

// Value of a 3-plane LDS ring (planes z-1, z, z+1; rows of W2) at x + c_i.
template <class L, class C, int W2>
__device__ __forceinline__ C ring_at(const C* s_m, const C* s_0, const C* s_p, int il, int i) {
  const int cz = L::cz[i];
  return (cz > 0 ? s_p : (cz < 0 ? s_m : s_0))[il + L::cy[i] * W2 + L::cx[i]];
}

// Well-balanced scheme: chemical potential of a node from the density ring,
// mu = mu_b(rho) - k 6 sum_i w_i (rho(x + c_i) - rho(x)), in float64.
template <class L, class C, int W2>
__device__ __forceinline__ double wb_mu_node(const EosK& eos, const C* s_m, const C* s_0, const C* s_p, int il,
                                             double k) {
  const double r0 = (double)s_0[il];
  double lap = 0.0;
#pragma unroll
  for (int i = 1; i < L::Q; ++i) lap += L::w[i] * ((double)ring_at<L, C, W2>(s_m, s_0, s_p, il, i) - r0);
  return mu_bulk(eos, r0) - k * 6.0 * lap;
}

// Well-balanced scheme: F = -rho grad_d mu + F_g from the chemical-potential
// ring, grad_d mu = 3 sum_i w_i c_i mu(x + c_i).
template <class L, class C, int W2>
__device__ __forceinline__ void wb_force(const C* s_m, const C* s_0, const C* s_p, int il, C rho, const C* Fg,
                                         C* F) {
  constexpr int D = L::D;
  C g[D];
#pragma unroll
  for (int a = 0; a < D; ++a) g[a] = 0;
#pragma unroll
  for (int i = 1; i < L::Q; ++i) {
    const C mi = ring_at<L, C, W2>(s_m, s_0, s_p, il, i);
#pragma unroll
    for (int a = 0; a < D; ++a)
      if (L::c(i, a) != 0) g[a] += (C)(3.0 * L::w[i] * L::c(i, a)) * mi;
  }
#pragma unroll
  for (int a = 0; a < D; ++a) F[a] = -rho * g[a] + Fg[a];
}

// BGK collision with Guo forcing (eqs. LBE, Single_Phase_EDF,
// Guo_Forcing_Scheme), dt = 1:  f* = (1 - omega) f + omega f_eq + (1 - omega/2) Fhat,
// written per opposite pair (a, b = opp a) through even and odd parts:
//   f_eq = E +- O,  E = w rho (1 - 1.5 u.u + 4.5 (c.u)^2),  O = 3 w rho (c.u)
//   Fhat = hE +- hO, hE = w (9 (c.u)(c.F) - 3 u.F),      hO = 3 w (c.F).
// MRT adds  - sum_k (s_k - omega) P_k(c_i) (sum_j P_k(c_j) v_j) / |P_k|^2 with
// v = f - f_eq + Fhat/2 over the non-hydrodynamic moments of MrtCorr<L>; the
// moment sums read v_a + v_b (even P_k) or v_a - v_b (odd P_k).
// dp[p] = f_a - f_b is shared with the momentum sum.
// WB: the equilibrium of the well-balanced scheme, whose moving populations
// carry the constant rho0 at rest: f_eq = w rho0 + w rho (-1.5 u.u + 4.5 (c.u)^2)
// +- O, and f_eq,0 = rho - (1 - w_0) rho0 + w_0 rho (-1.5 u.u).
// The collision conserves mass (the equilibrium holds the node's density, the
// forcing and the MRT corrections carry none).  In float32 arithmetic the rest
// population is therefore written as the node's mass less its moving
// populations, f*_0 = f_0 + sum_{i>0} (f_i - f*_i): the same value in exact
// arithmetic, but (1 - omega) f_0 + omega f_eq,0 inherits the rounding of the
// density sum every step, the same way at neighbouring nodes, a mass drift
// that grows linearly (1e-5 to 2e-5 of a settling droplet's mass per 1000
// steps); the differences are exact near equilibrium and vanish where the
// moving populations do not change.  float64 keeps the definition's form (its
// drift is ~2e-13 in 4000 steps, and it stays on the oracle's rounding path).
template <class L, class C, int COLL, bool WB = false>
__device__ __forceinline__ void collide(const C* f, const C* dp, C rho, const C* u, const C* F, C omega,
                                        const C* rate, C* fs, C rho0 = (C)0) {
  constexpr int D = L::D;
  using MC = MrtCorr<L>;
  constexpr int K = (COLL == COLL_MRT) ? MC::K : 1;
  C usq = 0, uF = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    usq += u[a] * u[a];
    uF += u[a] * F[a];
  }
  const C A = (C)1 - (C)1.5 * usq;
  const C om1 = (C)1 - omega;
  const C omh = (C)1 - (C)0.5 * omega;
  const C w0 = (C)L::w[0];
  const C E0 = WB ? (rho - (C)(1.0 - L::w[0]) * rho0) + w0 * rho * ((C)-1.5 * usq) : w0 * rho * A;
  const C h0 = -(C)3 * w0 * uF;
  constexpr bool BALANCE = std::is_same<C, float>::value;
  C B0 = omega * E0 + omh * h0;
  C BE[L::P], BO[L::P];
  C mk[K];
  if (COLL == COLL_MRT) {
    const C v0 = f[0] - E0 + (C)0.5 * h0;
#pragma unroll
    for (int k = 0; k < K; ++k) mk[k] = (MC::P(k, 0) != 0.0) ? (C)MC::P(k, 0) * v0 : (C)0;
  }
#pragma unroll
  for (int p = 0; p < L::P; ++p) {
    const int ia = L::pa[p], ib = L::pb[p];
    C cu = 0, cF = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      if (L::c(ia, a) > 0) {
        cu += u[a];
        cF += F[a];
      }
      if (L::c(ia, a) < 0) {
        cu -= u[a];
        cF -= F[a];
      }
    }
    const C w = (C)L::w[ia];
    const C E = WB ? w * rho0 + (w * rho) * ((C)-1.5 * usq + (C)4.5 * cu * cu) : (w * rho) * (A + (C)4.5 * cu * cu);
    const C O = ((C)3 * w * rho) * cu;
    const C hE = (C)9 * w * (cu * cF) - (C)3 * w * uF;
    const C hO = ((C)3 * w) * cF;
    const C be = omega * E + omh * hE;
    const C bo = omega * O + omh * hO;
    if (COLL == COLL_MRT) {
      BE[p] = be;
      BO[p] = bo;
      const C vs = (f[ia] + f[ib]) - (C)2 * E + hE;  // v_a + v_b
      const C vd = dp[p] - (C)2 * O + hO;             // v_a - v_b
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double ca = MC::P(k, ia), cb = MC::P(k, ib);
        if (ca != 0.0) mk[k] += (C)ca * (ca == cb ? vs : vd);
      }
    } else {
      fs[ia] = om1 * f[ia] + (be + bo);
      fs[ib] = om1 * f[ib] + (be - bo);
    }
  }
  if (COLL == COLL_MRT) {
    C coef[K];
#pragma unroll
    for (int k = 0; k < K; ++k) coef[k] = (rate[MC::rate_class[k]] - omega) * ((C)MrtInvNorm<L>::tab.v[k] * mk[k]);
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (!BALANCE && MC::P(k, 0) != 0.0) B0 -= (C)MC::P(k, 0) * coef[k];
#pragma unroll
    for (int p = 0; p < L::P; ++p) {
      C be = BE[p], bo = BO[p];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double ca = MC::P(k, L::pa[p]), cb = MC::P(k, L::pb[p]);
        if (ca == cb) {
          if (ca != 0.0) be -= (C)ca * coef[k];
        } else {
          bo -= (C)ca * coef[k];
        }
      }
      fs[L::pa[p]] = om1 * f[L::pa[p]] + (be + bo);
      fs[L::pb[p]] = om1 * f[L::pb[p]] + (be - bo);
    }
  }
  if constexpr (BALANCE) {
    C d = f[1] - fs[1];
#pragma unroll
    for (int i = 2; i < L::Q; ++i) d += f[i] - fs[i];
    fs[0] = f[0] + d;
  } else {
    fs[0] = om1 * f[0] + B0;
  }
}

template <bool B>
struct BoolC {
  static constexpr bool value = B;
};
template <int K>
struct IntC {
  static constexpr int value = K;
};
// f(IntC<0>{}), ..., f(IntC<N-1>{}), in order
template <int N, class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(IntC<I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl<N>(f, std::make_integer_sequence<int, N>{});
}

template <class L, class St, int COLL, int MODE, int TX, int TY, int NT, bool WALLS, int SCH>
__global__ __launch_bounds__(NT, PLBM_MIN_WAVES) void k_step(const KParams* __restrict__ P,
                                                             const WorkItem* __restrict__ work, int32_t nwork,
                                                             int32_t phase, double* __restrict__ out_rho,
                                                             double* __restrict__ out_u,
                                                             RedRec* __restrict__ red_out) {
  using T = typename St::T;
  using C = typename St::C;
  constexpr int Q = L::Q, D = L::D, HY = L::HY;
  constexpr int NI = TX * TY;             // tile nodes: one per interior thread per plane
  constexpr int W2 = TX + 2;
  constexpr int PL = W2 * (TY + 2 * HY);  // LDS plane (tile + halo)
  constexpr int H = PL - NI;              // halo nodes per plane
  constexpr int HW = (H + 63) / 64;       // waves that carry the halo ring
  constexpr bool SPLIT = PLBM_HALO_SPLIT != 0;
  static_assert(NT == (SPLIT ? NI + 64 * HW : NI), "thread count of the tile shape");
  static_assert(NI % 64 == 0 && H <= NI, "whole interior waves; halo fits");
  constexpr uint32_t TS = sizeof(T);
  constexpr int XB = Lines<T>::XB;
  constexpr int QB = Lines<T>::QB;
  constexpr int QS = Lines<T>::template slots<Q>();
  // 16-bit storage: populations stay in their stored form in registers until
  // they are used, so that the loads of a plane overlap the collision of the
  // previous one; they are decoded where they are summed and collided.
  constexpr bool RAW = St::shifted;
  constexpr bool LOC = St::local;  // per-node reference densities
  using R = typename std::conditional<RAW, T, C>::type;
  // well-balanced scheme: the chemical-potential pass (ring: rho) or the
  // update and its read-outs (ring: mu)
  constexpr bool WB = SCH == SCH_WB;
  constexpr bool WBMU = WB && MODE == MODE_MU;
  constexpr bool WBLD = WB && MODE != MODE_MU;
  static_assert(!WB || (!RAW && !LOC), "well-balanced scheme: float64 or float32 storage");
  static_assert(WB || MODE != MODE_MU, "MODE_MU belongs to the well-balanced scheme");
  // per-node value carried with a plane's populations through the march: the
  // reference density (locally shifted storage) or the chemical potential
  // (well-balanced update)
  using QT = typename std::conditional<WBLD, C, RefT>::type;
  // plane iterations between issuing a plane's loads and summing it
  constexpr int PF = PLBM_PREFETCH;

  __shared__ C lds_psi[4 * PL + 64];  // 4-plane psi ring + a slot per lane for idle halo lanes
  __shared__ C lds_ref[LOC ? 4 * PL + 64 : 1];  // reference densities, same ring
  __shared__ RedRec red_lds[(MODE == MODE_REDUCE) ? NT / 64 : 1];  // one record per wave

  int wid = work != nullptr ? xcd_remap(blockIdx.x, gridDim.x) : class_remap(blockIdx.x, gridDim.x, P->ntl);
  int slot = 0, tile = wid;
  if (work != nullptr) {
    if (wid >= nwork) return;
    slot = work[wid].slot;
    tile = work[wid].tile;
  }
  const KParams* __restrict__ kp = P + slot;
  if (tile >= kp->ntiles) return;

  const int nx = kp->nx, ny = kp->ny, nz = kp->nz;
  const uint32_t N = (uint32_t)kp->N;
  const int nxb = kp->nxb;
  const uint64_t zblock = (uint64_t)kp->zblock;  // bytes of one z plane of stored populations
  const uint32_t zdata = (uint32_t)kp->zdata;    // bytes of its node data (a trash area follows)
  int txi, tyi, z0, z1;
  tile_extent(kp, tile, &txi, &tyi, &z0, &z1);
  const int x0 = txi * TX, y0 = tyi * TY;
  const int par = (phase + kp->parity) & 1;
  char* const pop0 = reinterpret_cast<char*>(kp->pop[0]);
  char* const pop1 = reinterpret_cast<char*>(kp->pop[1]);
  const char* const src = par ? pop1 : pop0;
  char* const dst = par ? pop0 : pop1;
  const int plane = nx * ny;
  const EosK eos = load_eos(kp);
  const double rho0_shift = kp->rho0_shift;

  C shift[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) shift[i] = (C)(L::w[i] * rho0_shift);
  // psi of the ghost planes beyond the walls: the mirror of the wall-adjacent
  // plane, or psi(rho_w) of a wall density (wetting walls)
  const bool wet_lo = WALLS && kp->rho_wall[0] > 0.0, wet_hi = WALLS && kp->rho_wall[1] > 0.0;
  C psw_lo = 0, psw_hi = 0;
  if (wet_lo) {
    bool d_;
    psw_lo = psi_eval<C>(eos, kp->rho_wall[0], &d_);
  }
  if (wet_hi) {
    bool d_;
    psw_hi = psi_eval<C>(eos, kp->rho_wall[1], &d_);
  }
  auto ghost_psi = [&](int zl, C ps) -> C {
    if constexpr (WALLS) {
      if (zl < 0 && wet_lo) return psw_lo;
      if (zl >= nz && wet_hi) return psw_hi;
    }
    return ps;
  };

  // ---- node offsets of this thread, fixed for the whole z march ----
  // oxy[(cx+1) + 3 (cy+1)] = byte offset, within a z plane of stored
  // populations, of direction 0 of the pull source (x - cx, y - cy);
  // direction q adds q * QB bytes.
  const int t = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(t) >> 6;
  // with SPLIT, threads t >= NI carry only the halo ring (halo node t - NI);
  // otherwise the first HW waves carry it besides their tile nodes
  const bool halo_thread = SPLIT && wave >= NI / 64;
  const int ti = halo_thread ? 0 : t;
  const int th = SPLIT ? (halo_thread ? t - NI : H) : t;
  auto node_off = [&](int x, int y) -> uint32_t {
    return (uint32_t)((((y * nxb + x / XB) * QS) * XB + x % XB) * (int)TS);
  };
  uint32_t ioxy[9], hoxy[9];
  uint32_t soff;  // store offset: own node, or the trash area for ragged-tile lanes
  int ilds, hlds, own, hown;
  bool ivalid;
  {
    const int lx = ti % TX, ly = ti / TX;
    int gx = x0 + lx, gy = y0 + ly;
    ivalid = (gx < nx) && (gy < ny) && !halo_thread;
    gx = gx < nx ? gx : gx % nx;  // ragged tile: a wrapped duplicate, never stored
    gy = gy < ny ? gy : gy % ny;
    const int xm = gx == 0 ? nx - 1 : gx - 1, xp = gx == nx - 1 ? 0 : gx + 1;
    const int ym = gy == 0 ? ny - 1 : gy - 1, yp = gy == ny - 1 ? 0 : gy + 1;
#pragma unroll
    for (int cy = -1; cy <= 1; ++cy)
#pragma unroll
      for (int cx = -1; cx <= 1; ++cx)
        ioxy[(cx + 1) + 3 * (cy + 1)] =
            node_off(cx > 0 ? xm : (cx < 0 ? xp : gx), cy > 0 ? ym : (cy < 0 ? yp : gy));
    ilds = (ly + HY) * W2 + (lx + 1);
    own = gy * nx + gx;
    soff = ivalid ? ioxy[4] : zdata + (uint32_t)((((ti / XB) * QS) * XB + ti % XB) * (int)TS);
  }
  {
    // halo node h of the ring around the tile; lanes h >= H of the halo
    // waves repeat their own node and write psi to a spare LDS slot
    const int h = th;
    const bool hact = h < H;
    int lx, ly;
    if (HY) {
      if (h < W2) {
        lx = h - 1;
        ly = -1;
      } else if (h < 2 * W2) {
        lx = h - W2 - 1;
        ly = TY;
      } else {
        const int r = h - 2 * W2;
        lx = (r & 1) ? TX : -1;
        ly = r >> 1;
      }
    } else {
      lx = (h & 1) ? TX : -1;
      ly = 0;
    }
    if (hact) {
      const int gx = ((x0 + lx) % nx + nx) % nx;  // periodic in x and y
      const int gy = ((y0 + ly) % ny + ny) % ny;
      const int xm = gx == 0 ? nx - 1 : gx - 1, xp = gx == nx - 1 ? 0 : gx + 1;
      const int ym = gy == 0 ? ny - 1 : gy - 1, yp = gy == ny - 1 ? 0 : gy + 1;
#pragma unroll
      for (int cy = -1; cy <= 1; ++cy)
#pragma unroll
        for (int cx = -1; cx <= 1; ++cx)
          hoxy[(cx + 1) + 3 * (cy + 1)] =
              node_off(cx > 0 ? xm : (cx < 0 ? xp : gx), cy > 0 ? ym : (cy < 0 ? yp : gy));
      hlds = (ly + HY) * W2 + (lx + 1);
      hown = gy * nx + gx;
    } else {
#pragma unroll
      for (int c = 0; c < 9; ++c) hoxy[c] = ioxy[c];
      hlds = 4 * PL + (t & 63);
      hown = own;
    }
  }

  // logical plane zl -> stored plane in [0, nz).  The march loads planes
  // z0 - 1 <= zl <= z1 + n, n the planes it keeps in flight (one or two for
  // the update, NM for the chemical-potential pass): up to n past the last
  // plane the collision needs, whose values are never used (loading them
  // unconditionally keeps the unrolled register rotation free of branches).
  // A periodic axis may be shorter than that window (nz = 1, 2, ...), so it
  // wraps as often as needed; walls clamp.
  auto wrapz = [&](int zl) {
    if constexpr (WALLS) {
      return zl < 0 ? 0 : (zl >= nz ? nz - 1 : zl);
    } else {
      while (zl < 0) zl += nz;
      while (zl >= nz) zl -= nz;
      return zl;
    }
  };

  // Pull the Q populations of one node of stored plane pz; bm, b0, bp are
  // the population blocks of the planes pz-1, pz, pz+1.  With walls on the
  // marching axis, a population whose source lies beyond the wall is the
  // opposite population of the same node (half-way bounce-back); the choice
  // is wave-uniform and made by selects, keeping the loop free of branches.
  // A bounced population is decoded with its own shift: opposite directions
  // have equal weights.
  auto pull = [&](const uint32_t* oxy, const char* bm, const char* b0, const char* bp, bool lo, bool hi, R* f) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int cx = L::cx[i], cy = L::cy[i], cz = L::cz[i];
      const char* b = (cz > 0 ? bm : (cz < 0 ? bp : b0)) + i * QB;
      const uint32_t off = oxy[(cx + 1) + 3 * (cy + 1)];
      if (WALLS && cz != 0) {
        const bool bounce = cz > 0 ? lo : hi;
        const int o = L::opp[i];
        f[i] = (R)gld<T>(bounce ? b0 + o * QB : b, bounce ? oxy[4] : off);
      } else {
        f[i] = (R)gld<T>(b, off);
      }
    }
  };
  // decoded population i of a node whose reference density is ref (LOC)
  auto decode = [&](const R* f, int i, C ref) -> C {
    if constexpr (RAW) return St::dec(f[i], LOC ? (C)L::w[i] * ref : shift[i]);
    else return f[i];
  };

  auto density = [&](const R* f, C ref) {
    C r = decode(f, 0, ref);
#pragma unroll
    for (int i = 1; i < Q; ++i) r += decode(f, i, ref);
    return r;
  };
  const void* const ref_src = LOC ? kp->ref[par] : nullptr;
  void* const ref_dst = LOC ? kp->ref[par ^ 1] : nullptr;
  auto ref_ld = [&](uint32_t n) -> RefT { return gld_at<RefT>(ref_src, n); };
  // well-balanced scheme: the per-node chemical potential (read by the update, written by MODE_MU)
  void* const mu_arr = WB ? kp->wb_mu : nullptr;
  auto mu_ld = [&](uint32_t n) -> C { return gld_at<C>(mu_arr, n); };

  bool psi_neg = false;

  // Phase A, split in two so that a plane's loads are in flight while the
  // previous plane is collided: issue() pulls the populations of logical
  // plane zl (tile node into fo, halo node into ho); finish() sums rho and
  // writes psi of the tile and the halo ring into the LDS ring.
  auto issue = [&](auto halo_c, int zl, R* fo, R* ho, QT& qo, QT& qh) {
    constexpr bool HALO = decltype(halo_c)::value;
    const int pz = wrapz(zl);
    const int zm = pz == 0 ? (WALLS ? 0 : nz - 1) : pz - 1;
    const int zp = pz == nz - 1 ? (WALLS ? nz - 1 : 0) : pz + 1;
    const char* b0 = src + (uint64_t)pz * zblock;
    const char* bm = src + (uint64_t)zm * zblock;
    const char* bp = src + (uint64_t)zp * zblock;
    const bool lo = WALLS && pz == 0;
    const bool hi = WALLS && pz == nz - 1;
    pull(ioxy, bm, b0, bp, lo, hi, fo);
    if constexpr (WBLD) {
      qo = mu_ld((uint32_t)(pz * plane + own));
      if constexpr (HALO) qh = mu_ld((uint32_t)(pz * plane + hown));
    } else if constexpr (HALO) {
      pull(hoxy, bm, b0, bp, lo, hi, ho);
    }
    if constexpr (LOC) {
      qo = ref_ld((uint32_t)(pz * plane + own));
      if constexpr (HALO) qh = ref_ld((uint32_t)(pz * plane + hown));
    }
  };
  auto as_ref = [&](QT v) -> C {
    if constexpr (LOC) return (C)v;
    else return (C)0;
  };
  auto finish = [&](auto halo_c, int zl, bool keep, const R* fo, C& ro, QT qo, const R* ho, QT qh) {
    constexpr bool HALO = decltype(halo_c)::value;
    C* sl = lds_psi + ((zl - z0 + 1) & 3) * PL;
    const C r = density(fo, as_ref(qo));
    ro = r;
    if constexpr (WB) {
      sl[ilds] = WBLD ? (C)qo : r;
      if constexpr (HALO) (hlds < 4 * PL ? sl : lds_psi)[hlds] = WBLD ? (C)qh : density(ho, as_ref(qh));
      return;
    }
    bool ng;
    sl[ilds] = ghost_psi(zl, psi_eval<C>(eos, (double)r, &ng));
    psi_neg |= ng && ivalid && keep;
    if constexpr (LOC) lds_ref[((zl - z0 + 1) & 3) * PL + ilds] = (C)(RefT)r;
    if constexpr (HALO) {
      bool hng;
      const C rh = density(ho, as_ref(qh));
      const C ph = ghost_psi(zl, psi_eval<C>(eos, (double)rh, &hng));
      // the spare slots of idle lanes sit past the ring
      (hlds < 4 * PL ? sl : lds_psi)[hlds] = ph;
      if constexpr (LOC) (hlds < 4 * PL ? lds_ref + ((zl - z0 + 1) & 3) * PL : lds_ref)[hlds] = (C)(RefT)rh;
    }
  };

  // force coefficients: F = cA psi M1 + cB (M1.M2) + cC M1 tr(M2) + Fg
  const double G = kp->G, eps_ = kp->eps, kap = kp->kappa;
  const C cA = (C)(-G);
  const C cB = (C)(G / 4.0 * eps_ - G / 6.0 * (kap - 1.0));
  const C cC = (C)(G / 6.0 * (kap - 1.0));
  C Fg[D];
#pragma unroll
  for (int a = 0; a < D; ++a) Fg[a] = (C)kp->Fg[a];
  const C tau_v = (C)kp->tau_v, tau_slope = (C)kp->tau_slope, rho_v = (C)kp->rho_v;
  C rate[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) rate[k] = (C)kp->rates[k];
  typedef __attribute__((address_space(1))) float gfloat;  // global_load/store, not flat
  gfloat* const uprev = (gfloat*)kp->uprev;

  // reduction accumulators
  double acc_ms = 0.0, acc_mc = 0.0, acc_mom[3] = {0.0, 0.0, 0.0}, acc_umax = 0.0, acc_dumax = 0.0;
  int acc_flags = 0;

  // Phase B for output plane z with the populations f / rho of that plane.
  const C wb_rho0 = WB ? (C)kp->wb_rho0 : (C)0;
  const double wb_k = WB ? kp->wb_k : 0.0;
  auto phaseB = [&](int z, const R* fr, C rho, QT qr) {
    if constexpr (WBMU) {
      if (ivalid)
        gst_at<C>(mu_arr, (uint32_t)(z * plane + own),
                  (C)wb_mu_node<L, C, W2>(eos, lds_psi + ((z - z0) & 3) * PL, lds_psi + ((z - z0 + 1) & 3) * PL,
                                          lds_psi + ((z - z0 + 2) & 3) * PL, ilds, wb_k));
      return;
    }
    C f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = decode(fr, i, as_ref(qr));
    const C* s_m = lds_psi + ((z - z0) & 3) * PL;
    const C* s_0 = lds_psi + ((z - z0 + 1) & 3) * PL;
    const C* s_p = lds_psi + ((z - z0 + 2) & 3) * PL;
    C F[D], u[D];
    if constexpr (WB)
      wb_force<L, C, W2>(s_m, s_0, s_p, ilds, rho, Fg, F);
    else
      stencil_force<L, C, W2>(s_m, s_0, s_p, ilds, cA, cB, cC, Fg, F);
    // j_a = sum_i f_i c_ia over opposite pairs
    C dp[L::P];
#pragma unroll
    for (int p = 0; p < L::P; ++p) dp[p] = f[L::pa[p]] - f[L::pb[p]];
    const C inv_rho = recip(rho);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      C ja = 0;
#pragma unroll
      for (int p = 0; p < L::P; ++p) {
        if (L::c(L::pa[p], a) > 0) ja += dp[p];
        if (L::c(L::pa[p], a) < 0) ja -= dp[p];
      }
      u[a] = (ja + (C)0.5 * F[a]) * inv_rho;
    }
    const uint32_t nid = (uint32_t)(z * plane + own);  // canonical node index
    if (MODE == MODE_STEP) {
      const C omega = recip(tau_v + (rho - rho_v) * tau_slope);
      C fs[Q];
      collide<L, C, COLL, WB>(f, dp, rho, u, F, omega, rate, fs, wb_rho0);
      char* dz = dst + (uint64_t)z * zblock;
      if constexpr (LOC) {
        // f*_i(x) is decoded next step by x + c_i (by x itself when it
        // bounces off a wall), with that node's reference density, which is
        // its density now, rounded to half precision
        const C* r_m = lds_ref + ((z - z0) & 3) * PL;
        const C* r_0 = lds_ref + ((z - z0 + 1) & 3) * PL;
        const C* r_p = lds_ref + ((z - z0 + 2) & 3) * PL;
        const bool zlo = WALLS && z == 0, zhi = WALLS && z == nz - 1;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const int cz = L::cz[i];
          const C* rr = cz < 0 ? r_m : (cz > 0 ? r_p : r_0);
          C rd = rr[ilds + L::cx[i] + L::cy[i] * W2];
          if (WALLS && cz != 0) rd = (cz > 0 ? zhi : zlo) ? r_0[ilds] : rd;
          gst<T>(dz + i * QB, soff, St::enc(fs[i], (C)L::w[i] * rd));
        }
        // ragged-tile lanes write one of the 256 spare slots after the N
        // nodes (never read; a tile has up to 1024 threads)
        const uint32_t ridx = ivalid ? nid : (uint32_t)N + ((uint32_t)t & 255u);
        gst_at<RefT>(ref_dst, ridx, (RefT)rho);
      } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) gst<T>(dz + i * QB, soff, St::enc(fs[i], shift[i]));
      }
    } else if (MODE == MODE_MOMENTS) {
      if (ivalid) {
        out_rho[nid] = (double)rho;
#pragma unroll
        for (int a = 0; a < D; ++a) out_u[(size_t)a * N + nid] = (double)u[a];
      }
    } else {  // MODE_REDUCE
      if (ivalid) {
        const double dr = (double)rho;
        neumaier_add(acc_ms, acc_mc, dr);
        double usq = 0.0, dsq = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const double ua = (double)u[a];
          acc_mom[a] += dr * ua;
          usq += ua * ua;
          gfloat* up = uprev + (size_t)a * N + nid;
          const double dd = ua - (double)*up;
          dsq += dd * dd;
          *up = (float)ua;
        }
        acc_umax = fmax(acc_umax, sqrt(usq));
        acc_dumax = fmax(acc_dumax, sqrt(dsq));
        if (!(dr == dr) || !(usq == usq)) acc_flags |= 1;
        if (!(dr > 0.0)) acc_flags |= 2;
      }
    }
  };

  // The march, specialised per wave (the waves holding the halo ring and the
  // others run separate branch-free loops with the same barriers).  Three
  // population register sets rotate roles (unrolled by three, no copies):
  // plane z is collided while plane z+1 waits with its psi in LDS and the
  // loads of plane z+2 are in flight.
  auto march1 = [&](auto halo_c) {
    R f0[Q], f1[Q], f2[Q], hb[Q];
    C r0, r1, r2;      // densities
    QT q0 = 0, q1 = 0, q2 = 0, qh = 0;  // reference densities (LOC) or mu (well-balanced update)
    issue(halo_c, z0 - 1, f0, hb, q0, qh);
    finish(halo_c, z0 - 1, false, f0, r0, q0, hb, qh);
    issue(halo_c, z0, f0, hb, q0, qh);
    finish(halo_c, z0, true, f0, r0, q0, hb, qh);
    issue(halo_c, z0 + 1, f1, hb, q1, qh);
    finish(halo_c, z0 + 1, true, f1, r1, q1, hb, qh);
    // loads of z+2 into pf, barrier, collide z, psi of z+2
    auto stepz = [&](int z, R* cur, C rc, QT qc, R* pf, C& rp, QT& qp) {
      issue(halo_c, z + 2, pf, hb, qp, qh);
      __syncthreads();
      phaseB(z, cur, rc, qc);
      finish(halo_c, z + 2, true, pf, rp, qp, hb, qh);
    };
    int z = z0;
    for (; z + 2 < z1; z += 3) {
      stepz(z, f0, r0, q0, f2, r2, q2);
      stepz(z + 1, f1, r1, q1, f0, r0, q0);
      stepz(z + 2, f2, r2, q2, f1, r1, q1);
    }
    if (z < z1) {
      stepz(z, f0, r0, q0, f2, r2, q2);
      ++z;
    }
    if (z < z1) stepz(z, f1, r1, q1, f0, r0, q0);
  };
  // Loads run a full plane iteration ahead of their use: iteration z issues
  // plane z+3, collides plane z and sums the density and psi of plane z+2,
  // whose loads were issued one iteration earlier.  Four population register
  // sets and two halo sets rotate (unrolled by four, no copies).
  auto march2 = [&](auto halo_c) {
    R fa[Q], fb[Q], fc[Q], fd[Q], ha[Q], hb[Q];
    C ra, rb, rc, rd;
    QT qa = 0, qb = 0, qc = 0, qd = 0, qha = 0, qhb = 0;  // reference densities (LOC) or mu
    issue(halo_c, z0 - 1, fa, ha, qa, qha);
    finish(halo_c, z0 - 1, false, fa, ra, qa, ha, qha);
    issue(halo_c, z0, fa, ha, qa, qha);
    finish(halo_c, z0, true, fa, ra, qa, ha, qha);
    issue(halo_c, z0 + 1, fb, ha, qb, qha);
    finish(halo_c, z0 + 1, true, fb, rb, qb, ha, qha);
    issue(halo_c, z0 + 2, fc, ha, qc, qha);
    auto stepz = [&](int z, R* cur, C rcur, QT qcur, R* f2, C& r2, QT& q2, R* h2, QT& qh2, R* pf, QT& qp,
                     R* hp, QT& qhp) {
      issue(halo_c, z + 3, pf, hp, qp, qhp);
      __syncthreads();
      phaseB(z, cur, rcur, qcur);
      finish(halo_c, z + 2, true, f2, r2, q2, h2, qh2);
    };
    int z = z0;
    for (; z + 3 < z1; z += 4) {
      stepz(z, fa, ra, qa, fc, rc, qc, ha, qha, fd, qd, hb, qhb);
      stepz(z + 1, fb, rb, qb, fd, rd, qd, hb, qhb, fa, qa, ha, qha);
      stepz(z + 2, fc, rc, qc, fa, ra, qa, ha, qha, fb, qb, hb, qhb);
      stepz(z + 3, fd, rd, qd, fb, rb, qb, hb, qhb, fc, qc, ha, qha);
    }
    if (z < z1) {
      stepz(z, fa, ra, qa, fc, rc, qc, ha, qha, fd, qd, hb, qhb);
      ++z;
    }
    if (z < z1) {
      stepz(z, fb, rb, qb, fd, rd, qd, hb, qhb, fa, qa, ha, qha);
      ++z;
    }
    if (z < z1) stepz(z, fc, rc, qc, fa, ra, qa, ha, qha, fb, qb, hb, qhb);
  };
  auto march = [&](auto halo_c) {
    if constexpr (PF == 1)
      march1(halo_c);
    else
      march2(halo_c);
  };
  // The chemical-potential pass has no collision to hide a plane's loads
  // behind, and needs a plane's populations only to sum its density, so it
  // keeps NM planes of loads in flight in NM register sets: iteration z issues
  // plane z+1+NM, evaluates mu of plane z and sums plane z+2 (issued NM-1
  // iterations earlier).  Plane z0+2+j uses set j mod NM; the loop is unrolled
  // by NM so that every set index is a constant.
  constexpr int NM = PLBM_MU_PREFETCH;
  static_assert(NM >= 1, "at least one plane in flight");
  auto march_mu = [&](auto halo_c) {
    R fs[NM][Q], hs[NM][Q];
    QT qs[NM] = {}, qhs[NM] = {};
    C rd;
    for (int zl = z0 - 1; zl <= z0 + 1; ++zl) {
      issue(halo_c, zl, fs[0], hs[0], qs[0], qhs[0]);
      finish(halo_c, zl, true, fs[0], rd, qs[0], hs[0], qhs[0]);
    }
#pragma unroll
    for (int j = 0; j + 1 < NM; ++j) issue(halo_c, z0 + 2 + j, fs[j], hs[j], qs[j], qhs[j]);
    auto stepmu = [&](int z, auto u_c) {
      constexpr int u = decltype(u_c)::value, ui = (u + NM - 1) % NM;
      issue(halo_c, z + 1 + NM, fs[ui], hs[ui], qs[ui], qhs[ui]);
      __syncthreads();
      phaseB(z, fs[u], rd, qs[u]);
      finish(halo_c, z + 2, true, fs[u], rd, qs[u], hs[u], qhs[u]);
    };
    int z = z0;
    for (; z + NM - 1 < z1; z += NM)
      static_for<NM>([&](auto u_c) { stepmu(z + decltype(u_c)::value, u_c); });
    static_for<NM - 1>([&](auto u_c) {
      if (z + decltype(u_c)::value < z1) stepmu(z + decltype(u_c)::value, u_c);
    });
  };
  // Halo waves (SPLIT): pull the ring nodes of a plane, sum their density and
  // write their psi (or, in the well-balanced scheme, their density or the
  // loaded mu), with the same barriers as the tile waves.  They keep NH planes
  // of loads in flight in NH register sets (plane z0+2+j in set j mod NH,
  // unrolled by NH): iteration z issues plane z+1+NH and writes plane z+2.
  // The ring a plane barrier waits for is the halo waves' work, so their loads
  // may run further ahead than the tile waves'.
  constexpr int NH = WBMU ? NM : PLBM_HALO_PREFETCH;
  static_assert(NH >= 1, "at least one plane in flight");
  auto march_halo = [&]() {
    R hs[NH][Q];
    QT qhs[NH] = {};
    auto hissue = [&](int zl, R* ho, QT& qh) {
      const int pz = wrapz(zl);
      if constexpr (WBLD) {
        qh = mu_ld((uint32_t)(pz * plane + hown));
        return;
      }
      const int zm = pz == 0 ? (WALLS ? 0 : nz - 1) : pz - 1;
      const int zp = pz == nz - 1 ? (WALLS ? nz - 1 : 0) : pz + 1;
      pull(hoxy, src + (uint64_t)zm * zblock, src + (uint64_t)pz * zblock, src + (uint64_t)zp * zblock,
           WALLS && pz == 0, WALLS && pz == nz - 1, ho);
      if constexpr (LOC) qh = ref_ld((uint32_t)(pz * plane + hown));
    };
    auto hfinish = [&](int zl, const R* ho, QT qh) {
      const int slot = ((zl - z0 + 1) & 3) * PL;
      if constexpr (WB) {
        (hlds < 4 * PL ? lds_psi + slot : lds_psi)[hlds] = WBLD ? (C)qh : density(ho, as_ref(qh));
        return;
      }
      const C rh = density(ho, as_ref(qh));
      bool hng;
      const C ph = ghost_psi(zl, psi_eval<C>(eos, (double)rh, &hng));
      (hlds < 4 * PL ? lds_psi + slot : lds_psi)[hlds] = ph;
      if constexpr (LOC) (hlds < 4 * PL ? lds_ref + slot : lds_ref)[hlds] = (C)(RefT)rh;
    };
    for (int zl = z0 - 1; zl <= z0 + 1; ++zl) {
      hissue(zl, hs[0], qhs[0]);
      hfinish(zl, hs[0], qhs[0]);
    }
#pragma unroll
    for (int j = 0; j + 1 < NH; ++j) hissue(z0 + 2 + j, hs[j], qhs[j]);
    auto hstep = [&](int z, auto u_c) {
      constexpr int u = decltype(u_c)::value, ui = (u + NH - 1) % NH;
      hissue(z + 1 + NH, hs[ui], qhs[ui]);
      __syncthreads();
      hfinish(z + 2, hs[u], qhs[u]);
    };
    int z = z0;
    for (; z + NH - 1 < z1; z += NH)
      static_for<NH>([&](auto u_c) { hstep(z + decltype(u_c)::value, u_c); });
    static_for<NH - 1>([&](auto u_c) {
      if (z + decltype(u_c)::value < z1) hstep(z + decltype(u_c)::value, u_c);
    });
  };
  if constexpr (WBMU) {
    if constexpr (SPLIT) {
      if (PLBM_HALO_PRIO > 0 && halo_thread) __builtin_amdgcn_s_setprio(PLBM_HALO_PRIO);
      if (halo_thread)
        march_halo();
      else
        march_mu(BoolC<false>{});
    } else {
      if (wave < HW)
        march_mu(BoolC<true>{});
      else
        march_mu(BoolC<false>{});
    }
  } else if constexpr (SPLIT) {
    // Every tile wave waits at the plane barrier for the psi ring the halo
    // waves produce; issue priority for the halo waves shortens that wait.
    if (PLBM_HALO_PRIO > 0 && halo_thread) __builtin_amdgcn_s_setprio(PLBM_HALO_PRIO);
    if (halo_thread)
      march_halo();
    else
      march(BoolC<false>{});
  } else {
    if (wave < HW)
      march(BoolC<true>{});
    else
      march(BoolC<false>{});
  }

  if (MODE == MODE_REDUCE) {
    if (psi_neg) acc_flags |= 4;
    RedRec r;
    r.mass_s = acc_ms;
    r.mass_c = acc_mc;
    r.mom[0] = acc_mom[0];
    r.mom[1] = acc_mom[1];
    r.mom[2] = acc_mom[2];
    r.max_u = acc_umax;
    r.max_du = acc_dumax;
    r.flags = (double)acc_flags;
    // the lattice's own tile records, or a caller-given record array (single-lattice launches only)
    block_reduce_store<NT>(r, red_lds, (red_out != nullptr ? red_out : reinterpret_cast<RedRec*>(kp->red)) + tile);
  }
}

}  // namespace plbm
