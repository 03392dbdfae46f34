// In-place (AA-pattern) population storage: one population array instead of
// the two of the A-B pattern.
//
// At even time t the state is f_i(x, t) = A_i(x): an even step reads the
// node's own Q slots, collides, and writes f*_i(x) into the opposite slot
// A_opp(i)(x).  At odd time f_i(x, t) = A_opp(i)(x - c_i): an odd step reads
// those slots, collides, and writes f*_i(x) into A_i(x + c_i), where the next
// even step finds it as f_i(x + c_i, t + 1).  Each node reads exactly the
// slots it then writes and no two nodes share a slot, so the update needs no
// second array and no synchronisation between workgroups.  At a half-way
// bounce-back wall a link whose neighbour lies beyond the wall stays on the
// node: an odd step reads f_i(x) from A_i(x) and writes f*_i(x) to A_opp(i)(x).
//
// The interaction force needs psi of the neighbours at time t, and a tile
// cannot read a neighbour's populations once that neighbour may have been
// updated in place.  psi is therefore evaluated for every node by a first
// kernel (k_aa_psi) into a psi array in the arithmetic type, and the update
// kernel (k_aa_step) takes the stencil from that array through an LDS ring.
// HBM traffic per node and step: Q S + sizeof(C) (psi pass) plus
// 2 Q S + sizeof(C) (update), against 2 Q S for the fused A-B update; the
// population memory halves.
//
// Both kernels use the same density sum, psi evaluation, force and collision
// code as the A-B kernel, so the two patterns give identical results.
#pragma once

#include "plbm_aux.hpp"

namespace plbm {

// Tile indices of a workgroup (shared by both kernels; the tiling is that of
// the A-B kernel).
struct AaTile {
  const KParams* kp;
  int x0, y0, z0, z1, tile;
};

__device__ __forceinline__ bool aa_tile(int wid, const KParams* __restrict__ P, const WorkItem* __restrict__ work,
                                        int32_t nwork, int TX, int TY, AaTile* o) {
  int slot = 0, tile = wid;
  if (work != nullptr) {
    if (wid >= nwork) return false;
    slot = work[wid].slot;
    tile = work[wid].tile;
  }
  const KParams* __restrict__ kp = P + slot;
  if (tile >= kp->ntiles) return false;
  int txi, tyi;
  tile_extent(kp, tile, &txi, &tyi, &o->z0, &o->z1);
  o->kp = kp;
  o->tile = tile;
  o->x0 = txi * TX;
  o->y0 = tyi * TY;
  return true;
}

template <class L, class T>
__device__ __forceinline__ uint32_t aa_node_off(int x, int y, int nxb) {
  constexpr int XB = Lines<T>::XB;
  constexpr int QS = Lines<T>::template slots<L::Q>();
  return (uint32_t)((((y * nxb + x / XB) * QS) * XB + x % XB) * (int)sizeof(T));
}

// Byte offsets, within a z plane of stored populations, of direction 0 of
// the nine nodes (x - cx, y - cy): oxy[(cx + 1) + 3 (cy + 1)] (periodic).
template <class L, class T>
__device__ __forceinline__ void aa_neighbour_offsets(int gx, int gy, int nx, int ny, int nxb, uint32_t* oxy) {
  const int xm = gx == 0 ? nx - 1 : gx - 1, xp = gx == nx - 1 ? 0 : gx + 1;
  const int ym = gy == 0 ? ny - 1 : gy - 1, yp = gy == ny - 1 ? 0 : gy + 1;
#pragma unroll
  for (int cy = -1; cy <= 1; ++cy)
#pragma unroll
    for (int cx = -1; cx <= 1; ++cx)
      oxy[(cx + 1) + 3 * (cy + 1)] =
          aa_node_off<L, T>(cx > 0 ? xm : (cx < 0 ? xp : gx), cy > 0 ? ym : (cy < 0 ? yp : gy), nxb);
}

// Load the Q stored values of f_i(x, t) of one node of plane z at parity par
// (0: own slots; 1: opposite slots of the upstream neighbours, own slot at a
// wall).  bm, b0, bp are the population planes z - 1, z, z + 1.
template <class L, class St, bool WALLS>
__device__ __forceinline__ void aa_load(const uint32_t* oxy, const char* bm, const char* b0, const char* bp, int par,
                                        bool lo, bool hi, typename St::T* v) {
  using T = typename St::T;
  constexpr int QB = Lines<T>::QB;
  if (par == 0) {
#pragma unroll
    for (int i = 0; i < L::Q; ++i) v[i] = gld<T>(b0 + i * QB, oxy[4]);
  } else {
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
      const int cx = L::cx[i], cy = L::cy[i], cz = L::cz[i];
      const char* b = (cz > 0 ? bm : (cz < 0 ? bp : b0)) + L::opp[i] * QB;
      const uint32_t off = oxy[(cx + 1) + 3 * (cy + 1)];
      if (WALLS && cz != 0) {
        const bool bounce = cz > 0 ? lo : hi;
        v[i] = gld<T>(bounce ? b0 + i * QB : b, bounce ? oxy[4] : off);
      } else {
        v[i] = gld<T>(b, off);
      }
    }
  }
}

template <class St>
__device__ __forceinline__ typename St::C aa_dec(typename St::T v, typename St::C shift) {
  if constexpr (St::shifted) return St::dec(v, shift);
  else return (typename St::C)v;
}

// psi(rho(x, t)) of every node of a tile's z chunk into kp->psi.  The chunk
// is split over `split` workgroups (the update's tiling gives about one
// workgroup per CU, too few for a pass that only streams populations in).
template <class L, class St, int TX, int TY, bool WALLS>
__global__ __launch_bounds__(TX* TY) void k_aa_psi(const KParams* __restrict__ P, const WorkItem* __restrict__ work,
                                                   int32_t nwork, int32_t phase, int32_t split) {
  using T = typename St::T;
  using C = typename St::C;
  constexpr int Q = L::Q;
  // consecutive (tile, sub-chunk) items share an XCD, as in the update
  const int item =
      work != nullptr ? xcd_remap(blockIdx.x, gridDim.x) : class_remap(blockIdx.x, gridDim.x, P->ntl * split);
  AaTile tl;
  if (!aa_tile(item / split, P, work, nwork, TX, TY, &tl)) return;
  const KParams* __restrict__ kp = tl.kp;
  const int nx = kp->nx, ny = kp->ny, nz = kp->nz;
  {
    const int sub = item % split, len = tl.z1 - tl.z0;
    tl.z1 = tl.z0 + len * (sub + 1) / split;
    tl.z0 = tl.z0 + len * sub / split;
  }
  const int t = threadIdx.x;
  const int gx = tl.x0 + t % TX, gy = tl.y0 + t / TX;
  if (gx >= nx || gy >= ny) return;  // no barriers in this kernel
  const int par = (phase + kp->parity) & 1;
  const char* const A = reinterpret_cast<const char*>(kp->pop[0]);
  const uint64_t zblock = (uint64_t)kp->zblock;
  const EosK eos = load_eos(kp);
  C shift[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) shift[i] = (C)(L::w[i] * kp->rho0_shift);
  uint32_t oxy[9];
  aa_neighbour_offsets<L, T>(gx, gy, nx, ny, kp->nxb, oxy);
  void* const psi = kp->psi;
  const uint32_t own = (uint32_t)(gy * nx + gx), plane = (uint32_t)(nx * ny);
  // locally shifted storage: a node's populations are decoded with its own
  // reference density (its density one step earlier); the new one is written
  // for the update's encoder and the next step's decoder
  constexpr bool LOC = St::local;
  const void* const ref_src = LOC ? kp->ref[par] : nullptr;
  void* const ref_dst = LOC ? kp->ref[par ^ 1] : nullptr;
  auto load = [&](int z, T* v) {
    const int zm = z == 0 ? (WALLS ? 0 : nz - 1) : z - 1;
    const int zp = z == nz - 1 ? (WALLS ? nz - 1 : 0) : z + 1;
    aa_load<L, St, WALLS>(oxy, A + (uint64_t)zm * zblock, A + (uint64_t)z * zblock, A + (uint64_t)zp * zblock, par,
                          WALLS && z == 0, WALLS && z == nz - 1, v);
  };
  auto store = [&](int z, const T* v) {
    const uint32_t n = (uint32_t)z * plane + own;
    C rs = 0;
    if constexpr (LOC) rs = (C)gld_at<RefT>(ref_src, n);
    auto dsh = [&](int i) -> C {
      if constexpr (LOC) return (C)L::w[i] * rs;
      else return shift[i];
    };
    C r = aa_dec<St>(v[0], dsh(0));
#pragma unroll
    for (int i = 1; i < Q; ++i) r += aa_dec<St>(v[i], dsh(i));
    bool ng;
    gst_at<C>(psi, n, psi_eval<C>(eos, (double)r, &ng));
    if constexpr (LOC) gst_at<RefT>(ref_dst, n, (RefT)r);
  };
  for (int z = tl.z0; z < tl.z1; ++z) {
    T v[Q];
    load(z, v);
    store(z, v);
  }
}

// The in-place update (MODE_STEP), or the moments / reductions of the
// current state, of one tile's z chunk; psi comes from kp->psi.
template <class L, class St, int COLL, int MODE, int TX, int TY, bool WALLS>
__global__ __launch_bounds__(TX* TY, PLBM_MIN_WAVES) void k_aa_step(const KParams* __restrict__ P,
                                                                    const WorkItem* __restrict__ work,
                                                                    int32_t nwork, int32_t phase,
                                                                    double* __restrict__ out_rho,
                                                                    double* __restrict__ out_u,
                                                                    RedRec* __restrict__ red_out) {
  using T = typename St::T;
  using C = typename St::C;
  constexpr int Q = L::Q, D = L::D, HY = L::HY;
  constexpr int NT = TX * TY;
  constexpr int W2 = TX + 2;
  constexpr int PL = W2 * (TY + 2 * HY);
  static_assert(PL <= 2 * NT, "two psi loads per thread cover a plane with its halo");
  constexpr int QB = Lines<T>::QB;
  constexpr int XB = Lines<T>::XB;
  constexpr int QS = Lines<T>::template slots<Q>();
  constexpr uint32_t TS = sizeof(T);

  constexpr bool LOC = St::local;
  __shared__ C lds_psi[4 * PL];                 // 4-plane psi ring
  __shared__ C lds_ref[LOC ? 4 * PL : 1];       // reference densities (locally shifted storage), same ring
  __shared__ RedRec red_lds[(MODE == MODE_REDUCE) ? NT / 64 : 1];  // one record per wave

  AaTile tl;
  const int wid = work != nullptr ? xcd_remap(blockIdx.x, gridDim.x) : class_remap(blockIdx.x, gridDim.x, P->ntl);
  if (!aa_tile(wid, P, work, nwork, TX, TY, &tl)) return;  // whole workgroup
  const KParams* __restrict__ kp = tl.kp;
  const int nx = kp->nx, ny = kp->ny, nz = kp->nz;
  const int x0 = tl.x0, y0 = tl.y0, z0 = tl.z0, z1 = tl.z1;
  const uint32_t N = (uint32_t)kp->N;
  const uint32_t plane = (uint32_t)(nx * ny);
  const uint64_t zblock = (uint64_t)kp->zblock;
  const uint32_t zdata = (uint32_t)kp->zdata;
  const int par = (phase + kp->parity) & 1;
  char* const A = reinterpret_cast<char*>(kp->pop[0]);
  const void* const psi = kp->psi;
  const EosK eos = load_eos(kp);
  C shift[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) shift[i] = (C)(L::w[i] * kp->rho0_shift);

  const int t = threadIdx.x;
  const int lx = t % TX, ly = t / TX;
  const int gx = x0 + lx, gy = y0 + ly;
  const bool ivalid = gx < nx && gy < ny;
  const int ilds = (ly + HY) * W2 + (lx + 1);
  const uint32_t own = (uint32_t)(gy * nx + gx);
  // node offsets; a ragged-tile lane reads and writes a trash slot of its own
  // after each plane, whatever the direction
  uint32_t oxy[9];
  if (ivalid) {
    aa_neighbour_offsets<L, T>(gx, gy, nx, ny, kp->nxb, oxy);
  } else {
    const uint32_t tr = zdata + (uint32_t)((((t / XB) * QS) * XB + t % XB) * (int)TS);
#pragma unroll
    for (int c = 0; c < 9; ++c) oxy[c] = tr;
  }
  // the (at most two) psi values of each plane this thread stages into LDS
  uint32_t po[2];
  bool pact[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int j = t + k * NT;
    pact[k] = j < PL;
    const int jx = j % W2 - 1, jy = j / W2 - HY;
    const int hx = ((x0 + jx) % nx + nx) % nx, hy = ((y0 + jy) % ny + ny) % ny;  // periodic in x and y
    po[k] = (uint32_t)(hy * nx + hx);
  }
  // ring planes zl in [z0 - 1, z1 + 1]; a periodic axis may be shorter than
  // that window (nz = 1), so it wraps as often as needed; walls clamp (the
  // mirror psi ghost)
  auto wrapz = [&](int zl) {
    if constexpr (WALLS) {
      return zl < 0 ? 0 : (zl >= nz ? nz - 1 : zl);
    } else {
      while (zl < 0) zl += nz;
      while (zl >= nz) zl -= nz;
      return zl;
    }
  };
  // wetting walls: psi(rho_w) on the ghost plane instead of the mirror
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
  // locally shifted storage: own populations decode with the node's previous
  // density (ref_src); f*_i(x) encodes with the new density of the node that
  // decodes it next step, x + c_i (x itself where it bounces off a wall),
  // written by the psi pass (ref_dst) and staged into LDS with psi
  const void* const ref_src = LOC ? kp->ref[par] : nullptr;
  const void* const ref_dst = LOC ? kp->ref[par ^ 1] : nullptr;
  // psi (and reference densities) of ring plane zl: loaded into registers a
  // plane iteration before they are written to the LDS ring, so that the
  // loads are in flight across a whole update
  auto psi_issue = [&](int zl, C* pv, RefT* rv) {
    const uint32_t pz = (uint32_t)wrapz(zl) * plane;
#pragma unroll
    for (int k = 0; k < 2; ++k)
      if (pact[k]) pv[k] = gld_at<C>(psi, pz + po[k]);
    if constexpr (LOC) {
#pragma unroll
      for (int k = 0; k < 2; ++k)
        if (pact[k]) rv[k] = gld_at<RefT>(ref_dst, pz + po[k]);
    }
  };
  auto psi_commit = [&](int zl, const C* pv, const RefT* rv) {
    C* sl = lds_psi + ((zl - z0 + 1) & 3) * PL;
    const bool ghost = WALLS && ((zl < 0 && wet_lo) || (zl >= nz && wet_hi));
    const C gv = zl < 0 ? psw_lo : psw_hi;
#pragma unroll
    for (int k = 0; k < 2; ++k)
      if (pact[k]) sl[t + k * NT] = ghost ? gv : pv[k];
    if constexpr (LOC) {
      C* rl = lds_ref + ((zl - z0 + 1) & 3) * PL;
#pragma unroll
      for (int k = 0; k < 2; ++k)
        if (pact[k]) rl[t + k * NT] = (C)rv[k];
    }
  };
  auto load = [&](int z, T* v) {
    const int zm = z == 0 ? (WALLS ? 0 : nz - 1) : z - 1;
    const int zp = z == nz - 1 ? (WALLS ? nz - 1 : 0) : z + 1;
    aa_load<L, St, WALLS>(oxy, A + (uint64_t)zm * zblock, A + (uint64_t)z * zblock, A + (uint64_t)zp * zblock, par,
                          WALLS && z == 0, WALLS && z == nz - 1, v);
  };

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

  double acc_ms = 0.0, acc_mc = 0.0, acc_mom[3] = {0.0, 0.0, 0.0}, acc_umax = 0.0, acc_dumax = 0.0;
  int acc_flags = 0;

  auto update = [&](int z, const T* v) {
    C f[Q];
    C rs = 0;  // a ragged-tile lane reads a spare reference slot
    if constexpr (LOC) rs = (C)gld_at<RefT>(ref_src, ivalid ? (uint32_t)z * plane + own : (uint32_t)N + ((uint32_t)t & 255u));
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = aa_dec<St>(v[i], LOC ? (C)L::w[i] * rs : shift[i]);
    C rho = f[0];
#pragma unroll
    for (int i = 1; i < Q; ++i) rho += f[i];
    const C* s_m = lds_psi + ((z - z0) & 3) * PL;
    const C* s_0 = lds_psi + ((z - z0 + 1) & 3) * PL;
    const C* s_p = lds_psi + ((z - z0 + 2) & 3) * PL;
    C F[D], u[D];
    stencil_force<L, C, W2>(s_m, s_0, s_p, ilds, cA, cB, cC, Fg, F);
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
    const uint32_t nid = (uint32_t)z * plane + own;
    if (MODE == MODE_STEP) {
      const C omega = recip(tau_v + (rho - rho_v) * tau_slope);
      C fs[Q];
      collide<L, C, COLL>(f, dp, rho, u, F, omega, rate, fs);
      const int zm = z == 0 ? (WALLS ? 0 : nz - 1) : z - 1;
      const int zp = z == nz - 1 ? (WALLS ? nz - 1 : 0) : z + 1;
      char* b0 = A + (uint64_t)z * zblock;
      char* bm = A + (uint64_t)zm * zblock;
      char* bp = A + (uint64_t)zp * zblock;
      const bool lo = WALLS && z == 0, hi = WALLS && z == nz - 1;
      // encoding shift of f*_i(x)
      const C* r_m = lds_ref + ((z - z0) & 3) * PL;
      const C* r_0 = lds_ref + ((z - z0 + 1) & 3) * PL;
      const C* r_p = lds_ref + ((z - z0 + 2) & 3) * PL;
      auto esh = [&](int i) -> C {
        if constexpr (LOC) {
          const int cz = L::cz[i];
          const C* rr = cz < 0 ? r_m : (cz > 0 ? r_p : r_0);
          C rd = rr[ilds + L::cx[i] + L::cy[i] * W2];
          if (WALLS && cz != 0) rd = (cz > 0 ? hi : lo) ? r_0[ilds] : rd;
          return (C)L::w[i] * rd;
        } else {
          return shift[i];
        }
      };
      if (par == 0) {
#pragma unroll
        for (int i = 0; i < Q; ++i) gst<T>(b0 + L::opp[i] * QB, oxy[4], St::enc(fs[i], esh(i)));
      } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          // f*_i(x) goes downstream to A_i(x + c_i), i.e. offset index (-cx, -cy)
          const int cx = L::cx[i], cy = L::cy[i], cz = L::cz[i];
          char* b = (cz > 0 ? bp : (cz < 0 ? bm : b0)) + i * QB;
          const uint32_t off = oxy[(1 - cx) + 3 * (1 - cy)];
          const T e = St::enc(fs[i], esh(i));
          if (WALLS && cz != 0) {
            const bool bounce = cz > 0 ? hi : lo;
            gst<T>(bounce ? b0 + L::opp[i] * QB : b, bounce ? oxy[4] : off, e);
          } else {
            gst<T>(b, off, e);
          }
        }
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
        bool ng;
        (void)psi_eval<C>(eos, dr, &ng);
        if (ng) acc_flags |= 4;
      }
    }
  };

  // One barrier per plane: psi of plane z + 1 (loaded during the previous
  // plane) goes into the slot last read two planes ago, the psi loads of plane
  // z + 2 and the populations of plane z + 1 are issued (a node's slots are
  // disjoint from every other node's, so reading them before plane z is
  // written back is safe), then plane z is updated.  Two register sets of
  // each rotate (unrolled by two).  The psi loads of plane z1 + 1 after the
  // last plane are never used.
  T va[Q], vb[Q];
  C pa[2] = {}, pb[2] = {};
  RefT ra[2] = {}, rb[2] = {};
  psi_issue(z0 - 1, pa, ra);
  psi_commit(z0 - 1, pa, ra);
  psi_issue(z0, pa, ra);
  psi_commit(z0, pa, ra);
  psi_issue(z0 + 1, pa, ra);
  load(z0, va);
  auto plane_step = [&](int z, const T* cur, T* nxt, const C* pc, const RefT* rc, C* pn, RefT* rn) {
    psi_commit(z + 1, pc, rc);
    psi_issue(z + 2, pn, rn);
    if (z + 1 < z1) load(z + 1, nxt);
    __syncthreads();
    update(z, cur);
  };
  int z = z0;
  for (; z + 1 < z1; z += 2) {
    plane_step(z, va, vb, pa, ra, pb, rb);
    plane_step(z + 1, vb, va, pb, rb, pa, ra);
  }
  if (z < z1) plane_step(z, va, vb, pa, ra, pb, rb);

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
    block_reduce_store<NT>(r, red_lds, (red_out != nullptr ? red_out : reinterpret_cast<RedRec*>(kp->red)) + tl.tile);
  }
}

}  // namespace plbm
