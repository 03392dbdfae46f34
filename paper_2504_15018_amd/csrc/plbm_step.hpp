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
#pragma once

#include "plbm_device.hpp"

namespace plbm {

enum : int { COLL_BGK = 0, COLL_MRT = 1 };
enum : int { MODE_STEP = 0, MODE_MOMENTS = 1, MODE_REDUCE = 2 };

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

// Map a launch index so that consecutive logical tiles share an XCD (the
// hardware dispatches workgroups round-robin over the 8 XCDs, each with its
// own L2); halo re-reads of neighbouring tiles then hit the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int nfull = nb - (nb & 7);
  if (b >= nfull) return b;
  return (b & 7) * (nfull >> 3) + (b >> 3);
}

template <class L, class St, int COLL, int MODE, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_step(const KParams* __restrict__ P, const WorkItem* __restrict__ work,
                                             int32_t nwork, int32_t phase, double* __restrict__ out_rho,
                                             double* __restrict__ out_u) {
  using T = typename St::T;
  using C = typename St::C;
  constexpr int Q = L::Q, D = L::D, HY = L::HY;
  constexpr int S = (TX * TY) / NT;  // interior nodes per thread per plane
  static_assert(S * NT == TX * TY, "tile must be a multiple of the block");
  constexpr int W2 = TX + 2;
  constexpr int PL = W2 * (TY + 2 * HY);  // LDS plane (tile + halo)
  constexpr int H = PL - TX * TY;         // halo nodes per plane
  constexpr int HPT = (H + NT - 1) / NT;  // halo nodes per thread (upper bound)

  __shared__ C lds_psi[4 * PL];
  __shared__ RedRec red_lds[(MODE == MODE_REDUCE) ? NT : 1];

  int wid = xcd_remap(blockIdx.x, gridDim.x);
  int slot = 0, tile = wid;
  if (work != nullptr) {
    if (wid >= nwork) return;
    slot = work[wid].slot;
    tile = work[wid].tile;
  }
  const KParams p = P[slot];
  if (tile >= p.ntiles) return;

  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int64_t N = p.N;
  const int txi = tile % p.tiles_x;
  const int tyi = (tile / p.tiles_x) % p.tiles_y;
  const int tzi = tile / (p.tiles_x * p.tiles_y);
  const int x0 = txi * TX, y0 = tyi * TY, z0 = tzi * p.cz;
  const int z1 = min(z0 + p.cz, nz);
  const int par = (phase + p.parity) & 1;
  const T* __restrict__ src = reinterpret_cast<const T*>(p.pop[par]);
  T* __restrict__ dst = reinterpret_cast<T*>(p.pop[par ^ 1]);
  const int plane = nx * ny;
  const bool bbz = p.bb_z != 0;

  C shift[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) shift[i] = (C)(L::w[i] * p.rho0_shift);

  // ---- per-thread node coordinates (fixed for the whole z march) ----
  const int t = threadIdx.x;
  int ix[S], ixm[S], ixp[S], iyo[S], iyom[S], iyop[S], ilds[S];
  bool ivalid[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    int flat = t + s * NT;
    int lx = flat % TX, ly = flat / TX;
    int gx = x0 + lx, gy = y0 + ly;
    ivalid[s] = (gx < nx) && (gy < ny);
    gx = gx % nx;  // ragged tile: wrapped duplicate, never stored
    gy = gy % ny;
    ix[s] = gx;
    ixm[s] = gx == 0 ? nx - 1 : gx - 1;
    ixp[s] = gx == nx - 1 ? 0 : gx + 1;
    iyo[s] = gy * nx;
    iyom[s] = (gy == 0 ? ny - 1 : gy - 1) * nx;
    iyop[s] = (gy == ny - 1 ? 0 : gy + 1) * nx;
    ilds[s] = (ly + HY) * W2 + (lx + 1);
  }
  int hx[HPT], hxm[HPT], hxp[HPT], hyo[HPT], hyom[HPT], hyop[HPT], hlds[HPT];
  bool hact[HPT];
#pragma unroll
  for (int k = 0; k < HPT; ++k) {
    int h = t + k * NT;
    hact[k] = h < H;
    int lx, ly;
    if (HY) {
      if (h < W2) {
        lx = h - 1;
        ly = -1;
      } else if (h < 2 * W2) {
        lx = h - W2 - 1;
        ly = TY;
      } else {
        int r = h - 2 * W2;
        lx = (r & 1) ? TX : -1;
        ly = r >> 1;
      }
    } else {
      lx = (h & 1) ? TX : -1;
      ly = 0;
    }
    if (!hact[k]) {
      lx = 0;
      ly = 0;
    }
    int gx = ((x0 + lx) % nx + nx) % nx;  // periodic in x and y
    int gy = ((y0 + ly) % ny + ny) % ny;
    hx[k] = gx;
    hxm[k] = gx == 0 ? nx - 1 : gx - 1;
    hxp[k] = gx == nx - 1 ? 0 : gx + 1;
    hyo[k] = gy * nx;
    hyom[k] = (gy == 0 ? ny - 1 : gy - 1) * nx;
    hyop[k] = (gy == ny - 1 ? 0 : gy + 1) * nx;
    hlds[k] = (ly + HY) * W2 + (lx + 1);
  }

  // Pull the populations of one node of plane pz (pz already in [0, nz)).
  auto pull = [&](int x, int xm, int xp, int yo, int yom, int yop, int zo, int zom, int zop, bool lo, bool hi,
                  C* f) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int cx = L::cx[i], cy = L::cy[i], cz = L::cz[i];
      const bool bounce = (cz > 0 && lo) || (cz < 0 && hi);
      if (bounce) {
        const T* b = src + (size_t)L::opp[i] * (size_t)N;
        f[i] = St::dec(b[zo + yo + x], shift[L::opp[i]]);
      } else {
        const int sx = cx > 0 ? xm : (cx < 0 ? xp : x);
        const int sy = cy > 0 ? yom : (cy < 0 ? yop : yo);
        const int sz = cz > 0 ? zom : (cz < 0 ? zop : zo);
        const T* b = src + (size_t)i * (size_t)N;
        f[i] = St::dec(b[sz + sy + sx], shift[i]);
      }
    }
  };

  auto density = [&](const C* f) {
    C r = f[0];
#pragma unroll
    for (int i = 1; i < Q; ++i) r += f[i];
    return r;
  };

  // plane index helpers: logical plane zl (may be -1 or nz) -> stored plane
  auto wrapz = [&](int zl) {
    if (zl < 0) return bbz ? 0 : zl + nz;
    if (zl >= nz) return bbz ? nz - 1 : zl - nz;
    return zl;
  };

  bool psi_neg = false;

  // Phase A for logical plane zl: psi of tile + halo into LDS slot; interior
  // populations into fout (when keep) and rho into rout.
  auto phaseA = [&](int zl, bool keep, C (*fout)[Q], C* rout) {
    const int pz = wrapz(zl);
    const int zo = pz * plane;
    const int zom = (pz == 0 ? (bbz ? 0 : nz - 1) : pz - 1) * plane;
    const int zop = (pz == nz - 1 ? (bbz ? nz - 1 : 0) : pz + 1) * plane;
    const bool lo = bbz && pz == 0;
    const bool hi = bbz && pz == nz - 1;
    C* sl = lds_psi + ((zl - z0 + 1) & 3) * PL;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      C f[Q];
      pull(ix[s], ixm[s], ixp[s], iyo[s], iyom[s], iyop[s], zo, zom, zop, lo, hi, f);
      C r = density(f);
      bool ng;
      double ps = psi_of_rho(p, (double)r, &ng);
      psi_neg |= ng && ivalid[s] && keep;
      sl[ilds[s]] = (C)ps;
      if (keep) {
#pragma unroll
        for (int i = 0; i < Q; ++i) fout[s][i] = f[i];
        rout[s] = r;
      }
    }
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
      if (hact[k]) {
        C f[Q];
        pull(hx[k], hxm[k], hxp[k], hyo[k], hyom[k], hyop[k], zo, zom, zop, lo, hi, f);
        bool ng;
        sl[hlds[k]] = (C)psi_of_rho(p, (double)density(f), &ng);
      }
    }
  };

  // force coefficients: F = cA psi M1 + cB (M1.M2) + cC M1 tr(M2) + Fg
  const C cA = (C)(-p.G);
  const C cB = (C)(p.G / 4.0 * p.eps - p.G / 6.0 * (p.kappa - 1.0));
  const C cC = (C)(p.G / 6.0 * (p.kappa - 1.0));
  C Fg[D];
#pragma unroll
  for (int a = 0; a < D; ++a) Fg[a] = (C)p.Fg[a];
  const C tau_v = (C)p.tau_v, tau_slope = (C)p.tau_slope, rho_v = (C)p.rho_v;
  C rate[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) rate[k] = (C)p.rates[k];

  // reduction accumulators
  double acc_ms = 0.0, acc_mc = 0.0, acc_mom[3] = {0.0, 0.0, 0.0}, acc_umax = 0.0, acc_dumax = 0.0;
  int acc_flags = 0;

  C fc[S][Q], fn[S][Q];
  C rc[S], rn[S];

  phaseA(z0 - 1, false, fn, rn);
  phaseA(z0, true, fc, rc);

  for (int z = z0; z < z1; ++z) {
    phaseA(z + 1, true, fn, rn);
    __syncthreads();
    const C* s_m = lds_psi + ((z - z0) & 3) * PL;
    const C* s_0 = lds_psi + ((z - z0 + 1) & 3) * PL;
    const C* s_p = lds_psi + ((z - z0 + 2) & 3) * PL;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const C rho = rc[s];
      const C* f = fc[s];
      // psi stencil: S0 = sum w psi, S1_a = sum w psi c_a, S2_ab = sum w psi c_a c_b
      C S0 = 0, S1[D], S2[D][D];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        S1[a] = 0;
#pragma unroll
        for (int b = 0; b < D; ++b) S2[a][b] = 0;
      }
      C psi_c = s_0[ilds[s]];
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int cz = L::cz[i];
        const C* sl = cz > 0 ? s_p : (cz < 0 ? s_m : s_0);
        const C ps = sl[ilds[s] + L::cy[i] * W2 + L::cx[i]];
        const C wp = (C)L::w[i] * ps;
        S0 += wp;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          if (L::c(i, a) != 0) S1[a] += (C)L::c(i, a) * wp;
#pragma unroll
          for (int b = 0; b < D; ++b)
            if (L::c(i, a) * L::c(i, b) != 0) S2[a][b] += (C)(L::c(i, a) * L::c(i, b)) * wp;
        }
      }
      C M1[D], M2[D][D], tr = 0;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        M1[a] = (C)3 * S1[a];
#pragma unroll
        for (int b = 0; b < D; ++b) M2[a][b] = (C)9 * S2[a][b] - (a == b ? (C)3 * S0 : (C)0);
        tr += M2[a][a];
      }
      C F[D], j[D], u[D];
      const C inv_rho = (C)1 / rho;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        C m1m2 = 0;
#pragma unroll
        for (int b = 0; b < D; ++b) m1m2 += M1[b] * M2[a][b];
        F[a] = cA * psi_c * M1[a] + cB * m1m2 + cC * M1[a] * tr + Fg[a];
        C ja = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          if (L::c(i, a) > 0) ja += f[i];
          if (L::c(i, a) < 0) ja -= f[i];
        }
        j[a] = ja;
        u[a] = (ja + (C)0.5 * F[a]) * inv_rho;
      }

      const int own = z * plane + iyo[s] + ix[s];
      if (MODE == MODE_STEP) {
        const C tau = tau_v + (rho - rho_v) * tau_slope;
        const C omega = (C)1 / tau;
        C usq = 0, uF = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          usq += u[a] * u[a];
          uF += u[a] * F[a];
        }
        C fs[Q], v[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          C cu = 0, cF = 0;
#pragma unroll
          for (int a = 0; a < D; ++a) {
            if (L::c(i, a) > 0) {
              cu += u[a];
              cF += F[a];
            }
            if (L::c(i, a) < 0) {
              cu -= u[a];
              cF -= F[a];
            }
          }
          const C wi = (C)L::w[i];
          const C feq = wi * rho * ((C)1 + (C)3 * cu + (C)4.5 * cu * cu - (C)1.5 * usq);
          const C fh = wi * ((C)3 * cF + (C)9 * cu * cF - (C)3 * uF);
          v[i] = f[i] - feq + (C)0.5 * fh;
          fs[i] = f[i] + fh - omega * v[i];
        }
        if (COLL == COLL_MRT) {
          using MC = MrtCorr<L>;
#pragma unroll
          for (int k = 0; k < MC::K; ++k) {
            C mk = 0;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
              if (MC::P(k, i) != 0.0) mk += (C)MC::P(k, i) * v[i];
            }
            const C coef = (rate[MC::rate_class[k]] - omega) * (C)(1.0 / mrt_norm<L>(k)) * mk;
#pragma unroll
            for (int i = 0; i < Q; ++i)
              if (MC::P(k, i) != 0.0) fs[i] -= (C)MC::P(k, i) * coef;
          }
        }
        if (ivalid[s]) {
#pragma unroll
          for (int i = 0; i < Q; ++i) dst[(size_t)i * (size_t)N + own] = St::enc(fs[i], shift[i]);
        }
      } else if (MODE == MODE_MOMENTS) {
        if (ivalid[s]) {
          out_rho[own] = (double)rho;
#pragma unroll
          for (int a = 0; a < D; ++a) out_u[(size_t)a * (size_t)N + own] = (double)u[a];
        }
      } else {  // MODE_REDUCE
        if (ivalid[s]) {
          const double dr = (double)rho;
          neumaier_add(acc_ms, acc_mc, dr);
          double usq = 0.0, dsq = 0.0;
#pragma unroll
          for (int a = 0; a < D; ++a) {
            const double ua = (double)u[a];
            acc_mom[a] += dr * ua;
            usq += ua * ua;
            float* up = p.uprev + (size_t)a * (size_t)N + own;
            const double d = ua - (double)*up;
            dsq += d * d;
            *up = (float)ua;
          }
          acc_umax = fmax(acc_umax, sqrt(usq));
          acc_dumax = fmax(acc_dumax, sqrt(dsq));
          if (!(dr == dr) || !(usq == usq)) acc_flags |= 1;
          if (!(dr > 0.0)) acc_flags |= 2;
        }
      }
    }
    // rotate the register pipeline: plane z+1 becomes the current plane
#pragma unroll
    for (int s = 0; s < S; ++s) {
      rc[s] = rn[s];
#pragma unroll
      for (int i = 0; i < Q; ++i) fc[s][i] = fn[s][i];
    }
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
    red_lds[t] = r;
    __syncthreads();
    if (t == 0) {
      RedRec o = red_lds[0];
      for (int k = 1; k < NT; ++k) {  // fixed order: deterministic
        const RedRec& q = red_lds[k];
        neumaier_add(o.mass_s, o.mass_c, q.mass_s);
        o.mass_c += q.mass_c;
        for (int a = 0; a < 3; ++a) o.mom[a] += q.mom[a];
        o.max_u = fmax(o.max_u, q.max_u);
        o.max_du = fmax(o.max_du, q.max_du);
        o.flags = (double)((int)o.flags | (int)q.flags);
      }
      reinterpret_cast<RedRec*>(p.red)[tile] = o;
    }
  }
}

}  // namespace plbm
