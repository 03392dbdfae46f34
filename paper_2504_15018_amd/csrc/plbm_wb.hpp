// The well-balanced discretisation of the two-phase force (A-B pattern):
//
//   mu(x) = mu_b(rho(x)) - k lap_d rho(x),   F(x) = -rho(x) grad_d mu(x) + F_g,
//   grad_d g = sum_i w_i c_i g(x + c_i) / cs^2,  lap_d g = 2 sum_i w_i (g(x + c_i) - g(x)) / cs^2,
//
// with mu_b the bulk chemical potential of the equation of state
// (d mu_b / d rho = p'(rho) / rho) and an equilibrium whose moving populations
// carry the constant rho0 at rest.  A fluid at rest with uniform mu is an
// exact steady state.  The force needs mu of the neighbours, and mu needs rho
// of theirs, so a step is three passes over the nodes, one thread per node:
//   k_wb_rho  rho = sum_i f_i of every node, in direction order  -> wb_rho
//   k_wb_mu   mu from the rho stencil (float64 mu_b)             -> wb_mu
//   k_wb_step pull, rho (the same sum), mu stencil, force, u, tau(rho),
//             collision with the well-balanced equilibrium, store (or the
//             moments / reductions of the current state).
// Neighbour values beyond a half-way bounce-back wall mirror the wall-adjacent
// node.
#pragma once

#include "plbm_aux.hpp"

namespace plbm {

// Bulk chemical potential per unit mass, float64 (up to an additive constant):
// mu_b = int p / rho^2 d rho + p / rho.
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

// Linear index of the neighbour x + (cx, cy, cz) of node (x, y, z): periodic
// in x and y, periodic or mirrored (clamped) on the marching axis.
__device__ __forceinline__ int64_t wb_neighbour(const KParams& p, int x, int y, int z, int cx, int cy, int cz) {
  int xn = x + cx, yn = y + cy, zn = z + cz;
  xn = xn < 0 ? xn + p.nx : (xn >= p.nx ? xn - p.nx : xn);
  yn = yn < 0 ? yn + p.ny : (yn >= p.ny ? yn - p.ny : yn);
  if (p.bb_z)
    zn = zn < 0 ? 0 : (zn >= p.nz ? p.nz - 1 : zn);
  else
    zn = zn < 0 ? zn + p.nz : (zn >= p.nz ? zn - p.nz : zn);
  return ((int64_t)zn * p.ny + yn) * p.nx + xn;
}

// Element index of slot i of node (x, y, z) in a population array (the
// post-collision store of the A-B pattern: B_i(x) = f*_i(x)).
template <class L, class T>
__device__ __forceinline__ int64_t own_index(const KParams& p, int i, int x, int y, int z) {
  constexpr int XB = Lines<T>::XB;
  constexpr int QS = Lines<T>::template slots<L::Q>();
  return (int64_t)z * (p.zblock / (int64_t)sizeof(T)) + (((int64_t)y * p.nxb + x / XB) * QS + i) * XB + x % XB;
}

template <class L, class St>
__device__ __forceinline__ void wb_pull(const KParams& p, int par, int x, int y, int z, typename St::C* f) {
  const typename St::T* A = reinterpret_cast<const typename St::T*>(p.pop[par]);
#pragma unroll
  for (int i = 0; i < L::Q; ++i) f[i] = St::dec(A[storage_index<L, typename St::T>(p, par, i, x, y, z)], 0);
}

template <class L, class St>
__global__ __launch_bounds__(256) void k_wb_rho(const KParams* __restrict__ P, int32_t phase) {
  using C = typename St::C;
  const KParams p = *P;
  const int par = (phase + p.parity) & 1;
  C* R = reinterpret_cast<C*>(p.wb_rho);
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < p.N; n += (int64_t)gridDim.x * blockDim.x) {
    int x, y, z;
    node_xyz(p, n, &x, &y, &z);
    C f[L::Q];
    wb_pull<L, St>(p, par, x, y, z, f);
    C r = f[0];
#pragma unroll
    for (int i = 1; i < L::Q; ++i) r += f[i];
    R[n] = r;
  }
}

template <class L, class St>
__global__ __launch_bounds__(256) void k_wb_mu(const KParams* __restrict__ P) {
  using C = typename St::C;
  const KParams p = *P;
  const EosK eos = load_eos(&p);
  const C* R = reinterpret_cast<const C*>(p.wb_rho);
  C* M = reinterpret_cast<C*>(p.wb_mu);
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < p.N; n += (int64_t)gridDim.x * blockDim.x) {
    int x, y, z;
    node_xyz(p, n, &x, &y, &z);
    const double r0 = (double)R[n];
    double lap = 0.0;
#pragma unroll
    for (int i = 1; i < L::Q; ++i)
      lap += L::w[i] * ((double)R[wb_neighbour(p, x, y, z, L::cx[i], L::cy[i], L::cz[i])] - r0);
    M[n] = (C)(mu_bulk(eos, r0) - p.wb_k * 6.0 * lap);  // 2 / cs^2 = 6
  }
}

template <class L, class St, int COLL, int MODE>
__global__ __launch_bounds__(256) void k_wb_step(const KParams* __restrict__ P, int32_t phase,
                                                 double* __restrict__ out_rho, double* __restrict__ out_u,
                                                 RedRec* __restrict__ red_out) {
  using C = typename St::C;
  using T = typename St::T;
  constexpr int Q = L::Q, D = L::D;
  __shared__ RedRec red_lds[(MODE == MODE_REDUCE) ? 256 / 64 : 1];
  const KParams p = *P;
  const int par = (phase + p.parity) & 1;
  T* const dst = reinterpret_cast<T*>(p.pop[par ^ 1]);
  const C* M = reinterpret_cast<const C*>(p.wb_mu);
  C Fg[D];
#pragma unroll
  for (int a = 0; a < D; ++a) Fg[a] = (C)p.Fg[a];
  const C tau_v = (C)p.tau_v, tau_slope = (C)p.tau_slope, rho_v = (C)p.rho_v, rho0 = (C)p.wb_rho0;
  C rate[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) rate[k] = (C)p.rates[k];
  typedef __attribute__((address_space(1))) float gfloat;
  gfloat* const uprev = (gfloat*)p.uprev;
  double acc_ms = 0.0, acc_mc = 0.0, acc_mom[3] = {0.0, 0.0, 0.0}, acc_umax = 0.0, acc_dumax = 0.0;
  int acc_flags = 0;
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < p.N; n += (int64_t)gridDim.x * blockDim.x) {
    int x, y, z;
    node_xyz(p, n, &x, &y, &z);
    C f[Q];
    wb_pull<L, St>(p, par, x, y, z, f);
    C rho = f[0];
#pragma unroll
    for (int i = 1; i < Q; ++i) rho += f[i];
    // grad_d mu over the moving directions (3 = 1 / cs^2)
    C g[D];
#pragma unroll
    for (int a = 0; a < D; ++a) g[a] = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const C mi = M[wb_neighbour(p, x, y, z, L::cx[i], L::cy[i], L::cz[i])];
#pragma unroll
      for (int a = 0; a < D; ++a)
        if (L::c(i, a) != 0) g[a] += (C)(3.0 * L::w[i] * L::c(i, a)) * mi;
    }
    C F[D], u[D], dp[L::P];
#pragma unroll
    for (int a = 0; a < D; ++a) F[a] = -rho * g[a] + Fg[a];
#pragma unroll
    for (int q = 0; q < L::P; ++q) dp[q] = f[L::pa[q]] - f[L::pb[q]];
    const C inv_rho = recip(rho);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      C ja = 0;
#pragma unroll
      for (int q = 0; q < L::P; ++q) {
        if (L::c(L::pa[q], a) > 0) ja += dp[q];
        if (L::c(L::pa[q], a) < 0) ja -= dp[q];
      }
      u[a] = (ja + (C)0.5 * F[a]) * inv_rho;
    }
    if (MODE == MODE_STEP) {
      const C omega = recip(tau_v + (rho - rho_v) * tau_slope);
      C fs[Q];
      collide<L, C, COLL, true>(f, dp, rho, u, F, omega, rate, fs, rho0);
#pragma unroll
      for (int i = 0; i < Q; ++i) dst[own_index<L, T>(p, i, x, y, z)] = St::enc(fs[i], 0);
    } else if (MODE == MODE_MOMENTS) {
      out_rho[n] = (double)rho;
#pragma unroll
      for (int a = 0; a < D; ++a) out_u[(size_t)a * p.N + n] = (double)u[a];
    } else {
      const double dr = (double)rho;
      neumaier_add(acc_ms, acc_mc, dr);
      double usq = 0.0, dsq = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const double ua = (double)u[a];
        acc_mom[a] += dr * ua;
        usq += ua * ua;
        gfloat* up = uprev + (size_t)a * p.N + n;
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
  if (MODE == MODE_REDUCE) {
    RedRec r;
    r.mass_s = acc_ms;
    r.mass_c = acc_mc;
    r.mom[0] = acc_mom[0];
    r.mom[1] = acc_mom[1];
    r.mom[2] = acc_mom[2];
    r.max_u = acc_umax;
    r.max_du = acc_dumax;
    r.flags = (double)acc_flags;
    block_reduce_store<256>(r, red_lds, (red_out != nullptr ? red_out : reinterpret_cast<RedRec*>(p.red)) + blockIdx.x);
  }
}

}  // namespace plbm
