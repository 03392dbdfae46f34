// Auxiliary kernels: initialisation to equilibrium, population read/write in
// the canonical post-streaming form, and the fixed-order final reduction.
#pragma once

#include "plbm_step.hpp"

namespace plbm {

// Storage index (in elements of T) of f_i(x) of the post-streaming state at
// time parity par.  A-B pattern: populations are kept post-collision, f_i(x)
// lives at A_i(x - c_i), or at A_opp(i)(x) when x - c_i lies beyond a
// half-way bounce-back wall.  In-place pattern: at even time f_i(x) lives at
// A_i(x); at odd time at A_opp(i)(x - c_i), or at A_i(x) beyond a wall.
template <class L, class T>
__device__ __forceinline__ int64_t storage_index(const KParams& p, int par, int i, int x, int y, int z) {
  constexpr int XB = Lines<T>::XB;
  constexpr int QS = Lines<T>::template slots<L::Q>();
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  int sz = z - L::cz[i], sx = x - L::cx[i], sy = y - L::cy[i], q = i;
  const bool wall = p.bb_z && (sz < 0 || sz >= nz);
  if (p.aa) {
    if (par == 0 || wall) {
      sx = x;
      sy = y;
      sz = z;
    } else {
      q = L::opp[i];
    }
  } else if (wall) {
    sx = x;
    sy = y;
    sz = z;
    q = L::opp[i];
  }
  sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
  sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
  sz = sz < 0 ? sz + nz : (sz >= nz ? sz - nz : sz);
  // z planes are zblock bytes apart (node data followed by a trash area)
  return (int64_t)sz * (p.zblock / (int64_t)sizeof(T)) + (((int64_t)sy * p.nxb + sx / XB) * QS + q) * XB + sx % XB;
}

// Direction whose storage slot holds f_i(x) (the weight of the shift of a
// shifted storage; opposite directions have equal weights).
template <class L>
__device__ __forceinline__ int storage_dir(const KParams& p, int par, int i, int z) {
  const int sz = z - L::cz[i];
  const bool wall = p.bb_z && (sz < 0 || sz >= p.nz);
  if (p.aa) return (par == 0 || wall) ? i : L::opp[i];
  return wall ? L::opp[i] : i;
}

// Second-order equilibrium of eq. (Single_Phase_EDF), float64.
template <class L>
__device__ __forceinline__ double feq64(int i, double rho, const double* u) {
  double cu = 0.0, usq = 0.0;
#pragma unroll
  for (int a = 0; a < L::D; ++a) {
    cu += (double)L::c(i, a) * u[a];
    usq += u[a] * u[a];
  }
  return L::w[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
}

// Density whose multiples w_i rho shift the stored populations of node n:
// the global rho0, or the node's reference density (locally shifted storage).
template <class St>
__device__ __forceinline__ double shift_density(const KParams& p, int par, int64_t n) {
  if constexpr (St::local) return (double)reinterpret_cast<const RefT*>(p.ref[par])[n];
  else return p.rho0_shift;
}

// Equilibrium of the well-balanced scheme, float64: the moving populations
// carry the constant rho0 at rest, the rest population the remainder.
template <class L>
__device__ __forceinline__ double feq64_wb(int i, double rho, const double* u, double rho0) {
  double cu = 0.0, usq = 0.0;
#pragma unroll
  for (int a = 0; a < L::D; ++a) {
    cu += (double)L::c(i, a) * u[a];
    usq += u[a] * u[a];
  }
  const double base = i == 0 ? rho - (1.0 - L::w[0]) * rho0 : L::w[i] * rho0;
  return base + L::w[i] * rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
}

template <class L, class St>
__device__ __forceinline__ void write_equilibrium(const KParams& p, int par, int64_t n, int x, int y, int z,
                                                  double rho, const double* u) {
  typename St::T* A = reinterpret_cast<typename St::T*>(p.pop[par]);
  if constexpr (St::local) reinterpret_cast<RefT*>(p.ref[par])[n] = (RefT)(float)rho;
  const double rs = shift_density<St>(p, par, n);
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const int dir = storage_dir<L>(p, par, i, z);
    const double fe = p.wb ? feq64_wb<L>(i, rho, u, p.wb_rho0) : feq64<L>(i, rho, u);
    A[storage_index<L, typename St::T>(p, par, i, x, y, z)] = St::enc64(fe, L::w[dir] * rs);
  }
}

__device__ __forceinline__ void node_xyz(const KParams& p, int64_t n, int* x, int* y, int* z) {
  *x = (int)(n % p.nx);
  int64_t r = n / p.nx;
  *y = (int)(r % p.ny);
  *z = (int)(r / p.ny);
}

// f = f_eq(rho, u) from float64 fields rho[N], u[D][N] (u may be null).
template <class L, class St>
__global__ __launch_bounds__(256) void k_init_fields(const KParams* __restrict__ P, int par,
                                                     const double* __restrict__ rho, const double* __restrict__ u) {
  const KParams p = *P;
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < p.N; n += (int64_t)gridDim.x * blockDim.x) {
    int x, y, z;
    node_xyz(p, n, &x, &y, &z);
    double uu[3] = {0.0, 0.0, 0.0};
    if (u != nullptr)
      for (int a = 0; a < L::D; ++a) uu[a] = u[(size_t)a * (size_t)p.N + n];
    write_equilibrium<L, St>(p, par, n, x, y, z, rho[n], uu);
  }
}

// Shape description mirrored from plbm_shape (plbm.h).
struct ShapeK {
  int32_t kind, axis;
  double rho_in, rho_out, W, R;
  double centre[3];
  double level;
  double u0[3];
};

// f = f_eq of a tanh-interface density shape; physical coordinates are
// (x, y) in 2-D (kernel z is the 2-D y) and (x, y, z) in 3-D.
template <class L, class St>
__global__ __launch_bounds__(256) void k_init_shape(const KParams* __restrict__ P, int par, ShapeK sh) {
  const KParams p = *P;
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < p.N; n += (int64_t)gridDim.x * blockDim.x) {
    int x, y, z;
    node_xyz(p, n, &x, &y, &z);
    double pc[3] = {(double)x, L::D == 2 ? (double)z : (double)y, (double)z};
    int dims[3] = {p.nx, L::D == 2 ? p.nz : p.ny, p.nz};
    double rho;
    const double dl = sh.rho_in - sh.rho_out;
    if (sh.kind == 0) {  // slab: liquid in the central half of `axis`
      double c = pc[sh.axis], nn = dims[sh.axis];
      rho = sh.rho_out + 0.5 * dl * (tanh(2.0 * (c - nn / 4.0) / sh.W) - tanh(2.0 * (c - 3.0 * nn / 4.0) / sh.W));
    } else if (sh.kind == 1) {  // droplet
      double r2 = 0.0;
      for (int a = 0; a < L::D; ++a) r2 += (pc[a] - sh.centre[a]) * (pc[a] - sh.centre[a]);
      rho = 0.5 * (sh.rho_in + sh.rho_out) - 0.5 * dl * tanh(2.0 * (sqrt(r2) - sh.R) / sh.W);
    } else {  // layers: liquid below `level` along `axis`
      rho = 0.5 * (sh.rho_in + sh.rho_out) - 0.5 * dl * tanh(2.0 * (pc[sh.axis] - sh.level) / sh.W);
    }
    write_equilibrium<L, St>(p, par, n, x, y, z, rho, sh.u0);
  }
}

// out[n] = f_dir(x_n, t), decoded to float64.
template <class L, class St>
__global__ __launch_bounds__(256) void k_read_pop(const KParams* __restrict__ P, int par, int dirq,
                                                  double* __restrict__ out) {
  const KParams p = *P;
  const typename St::T* A = reinterpret_cast<const typename St::T*>(p.pop[par]);
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < p.N; n += (int64_t)gridDim.x * blockDim.x) {
    int x, y, z;
    node_xyz(p, n, &x, &y, &z);
    const int dir = storage_dir<L>(p, par, dirq, z);
    out[n] = St::dec64(A[storage_index<L, typename St::T>(p, par, dirq, x, y, z)], L::w[dir] * shift_density<St>(p, par, n));
  }
}

// Inverse of k_read_pop: f_dir(x_n, t) = in[n].
template <class L, class St>
__global__ __launch_bounds__(256) void k_write_pop(const KParams* __restrict__ P, int par, int dirq,
                                                   const double* __restrict__ in) {
  const KParams p = *P;
  typename St::T* A = reinterpret_cast<typename St::T*>(p.pop[par]);
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < p.N; n += (int64_t)gridDim.x * blockDim.x) {
    int x, y, z;
    node_xyz(p, n, &x, &y, &z);
    const int dir = storage_dir<L>(p, par, dirq, z);
    A[storage_index<L, typename St::T>(p, par, dirq, x, y, z)] = St::enc64(in[n], L::w[dir] * shift_density<St>(p, par, n));
  }
}

}  // namespace plbm
