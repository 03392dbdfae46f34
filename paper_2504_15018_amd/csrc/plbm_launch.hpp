// Host-visible launch entry points of the kernel translation units.  Each
// population storage type is compiled in its own translation unit (the
// float64 one without floating-point contraction, so that its rounding follows
// the plain operation order).
#pragma once

#include <hip/hip_runtime.h>

#include "plbm_device.hpp"

#ifndef PLBM_HALO_SPLIT
#define PLBM_HALO_SPLIT 1
#endif

namespace plbm {

struct WorkItem;
struct ShapeK;

// Compile-time tile shapes (one node per thread per plane): D3Q19 TX x TY
// nodes, set per storage translation unit (default 32 x 8); D2Q9 rows of 256
// nodes.
template <class L>
struct TileShape;
#ifndef PLBM_D3_TX
#define PLBM_D3_TX 32
#endif
#ifndef PLBM_D3_TY
#define PLBM_D3_TY 8
#endif
// With PLBM_HALO_SPLIT the workgroup adds whole waves for the halo ring
// (D3Q19: (TX+2)(TY+2) - TX TY nodes; D2Q9: the two row ends of 256-node rows).
template <>
struct TileShape<D3Q19L> {
  static constexpr int TX = PLBM_D3_TX, TY = PLBM_D3_TY;
  static constexpr int H = (TX + 2) * (TY + 2) - TX * TY;
  static constexpr int NT = TX * TY + (PLBM_HALO_SPLIT ? 64 * ((H + 63) / 64) : 0);
};
#ifndef PLBM_D2_TX
#define PLBM_D2_TX 256
#endif
template <>
struct TileShape<D2Q9L> {
  static constexpr int TX = PLBM_D2_TX, TY = 1;
  static constexpr int NT = TX * TY + (PLBM_HALO_SPLIT ? 64 : 0);
};

// Tile shape of the in-place pattern's kernels (no halo waves: the psi
// stencil comes from the psi array), set per storage translation unit; the
// default is the A-B shape.
#ifndef PLBM_AA_TX
#define PLBM_AA_TX PLBM_D3_TX
#endif
#ifndef PLBM_AA_TY
#define PLBM_AA_TY PLBM_D3_TY
#endif
template <class L>
struct AaTileShape;
template <>
struct AaTileShape<D3Q19L> {
  static constexpr int TX = PLBM_AA_TX, TY = PLBM_AA_TY;
};
template <>
struct AaTileShape<D2Q9L> {
  static constexpr int TX = TileShape<D2Q9L>::TX, TY = 1;
};

struct StepLaunch {
  int lattice;  // 0 D2Q9, 1 D3Q19
  int coll;     // 0 BGK, 1 MRT
  int mode;     // 0 step, 1 moments, 2 reduce
  int walls;    // half-way bounce-back on the marching axis
  int aa;       // in-place pattern: psi pass, then the in-place update
  int psplit;   // in-place pattern: workgroups per tile chunk of the psi pass (>= 1)
  int nblocks;
  hipStream_t stream;
  const KParams* P;
  const WorkItem* work;
  int nwork;
  int phase;
  double* out_rho;
  double* out_u;
  void* red;  // reduce mode: tile records go here instead of the lattice's own (single-lattice launches)
  int wb;     // well-balanced scheme: chemical-potential pass, then the update
};

enum : int { AUX_INIT_FIELDS = 0, AUX_INIT_SHAPE = 1, AUX_READ_POP = 2, AUX_WRITE_POP = 3 };

struct AuxLaunch {
  int lattice;
  int what;
  int nblocks;
  hipStream_t stream;
  const KParams* P;
  int par;
  int dir;
  const double* in0;
  const double* in1;
  double* out;
  const ShapeK* shape;
};

hipError_t launch_step_f64(const StepLaunch&);
hipError_t launch_step_f32(const StepLaunch&);
hipError_t launch_step_f16s(const StepLaunch&);
hipError_t launch_step_bf16s(const StepLaunch&);
hipError_t launch_aux_f64(const AuxLaunch&);
hipError_t launch_aux_f32(const AuxLaunch&);
hipError_t launch_aux_f16s(const AuxLaunch&);
hipError_t launch_aux_bf16s(const AuxLaunch&);
hipError_t launch_step_f16r(const StepLaunch&);
hipError_t launch_step_bf16r(const StepLaunch&);
hipError_t launch_aux_f16r(const AuxLaunch&);
hipError_t launch_aux_bf16r(const AuxLaunch&);
// D3Q19 tile shape (x nodes, y rows) of each storage's kernels (compiled per
// storage translation unit)
// (aa: the in-place pattern's shape)
void tile_shape_f64(int aa, int* tx, int* ty);
void tile_shape_f32(int aa, int* tx, int* ty);
void tile_shape_f16s(int aa, int* tx, int* ty);
void tile_shape_bf16s(int aa, int* tx, int* ty);
void tile_shape_f16r(int aa, int* tx, int* ty);
void tile_shape_bf16r(int aa, int* tx, int* ty);
// resident workgroups per CU of the update kernel (hipOccupancy...)
hipError_t occupancy_step_f64(int lattice, int coll, int walls, int aa, int* blocks);
hipError_t occupancy_step_f32(int lattice, int coll, int walls, int aa, int* blocks);
hipError_t occupancy_step_f16s(int lattice, int coll, int walls, int aa, int* blocks);
hipError_t occupancy_step_bf16s(int lattice, int coll, int walls, int aa, int* blocks);
hipError_t occupancy_step_f16r(int lattice, int coll, int walls, int aa, int* blocks);
hipError_t occupancy_step_bf16r(int lattice, int coll, int walls, int aa, int* blocks);
hipError_t launch_accum(hipStream_t st, int nblocks, int64_t N, int first, const double* in, double* acc);
hipError_t launch_set_ref(hipStream_t st, int nblocks, const KParams* P, int par, const double* acc);
// recs: the tile records to combine (nullptr: the lattice's own)
hipError_t launch_reduce_final(hipStream_t st, const KParams* P, int ntiles, void* out, const void* recs);
hipError_t launch_reduce_final_batch(hipStream_t st, const KParams* P, int nslots, void* out);

}  // namespace plbm
