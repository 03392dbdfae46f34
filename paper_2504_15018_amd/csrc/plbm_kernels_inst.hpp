// Instantiation of every kernel for one storage type.  Included by the
// per-storage translation units with PLBM_ST (codec) and PLBM_SUFFIX defined.
#include <type_traits>

#include "plbm_aa.hpp"
#include "plbm_aux.hpp"
#include "plbm_launch.hpp"

#define PLBM_CAT2(a, b) a##b
#define PLBM_CAT(a, b) PLBM_CAT2(a, b)

namespace plbm {

#ifndef PLBM_LDS_PAD
#define PLBM_LDS_PAD 0  // extra LDS bytes per workgroup (limits workgroups per CU)
#endif

// In-place pattern: the psi pass, then the update.
template <class L, int COLL, int MODE, bool WALLS>
static hipError_t go_aa(const StepLaunch& a) {
  using TS = AaTileShape<L>;
  hipLaunchKernelGGL((k_aa_psi<L, PLBM_ST, TS::TX, TS::TY, WALLS>), dim3((uint32_t)a.nblocks * (uint32_t)a.psplit),
                     dim3(TS::TX * TS::TY), 0, a.stream, a.P, a.work, a.nwork, a.phase, a.psplit);
  hipLaunchKernelGGL((k_aa_step<L, PLBM_ST, COLL, MODE, TS::TX, TS::TY, WALLS>), dim3(a.nblocks),
                     dim3(TS::TX * TS::TY), 0, a.stream, a.P, a.work, a.nwork, a.phase, a.out_rho, a.out_u,
                     reinterpret_cast<RedRec*>(a.red));
  return hipGetLastError();
}

// Well-balanced scheme (float64 and float32 storage): the chemical-potential
// pass, then the update (or its read-outs), both on the A-B tiling.
template <class L, int COLL, int MODE, bool WALLS>
static hipError_t go_wb(const StepLaunch& a) {
  if constexpr (std::is_same<PLBM_ST, StF64>::value || std::is_same<PLBM_ST, StF32>::value) {
    using TS = TileShape<L>;
    hipLaunchKernelGGL((k_step<L, PLBM_ST, COLL_BGK, MODE_MU, TS::TX, TS::TY, TS::NT, WALLS, SCH_WB>),
                       dim3(a.nblocks), dim3(TS::NT), PLBM_LDS_PAD, a.stream, a.P, a.work, a.nwork, a.phase, nullptr,
                       nullptr, nullptr);
    hipLaunchKernelGGL((k_step<L, PLBM_ST, COLL, MODE, TS::TX, TS::TY, TS::NT, WALLS, SCH_WB>), dim3(a.nblocks),
                       dim3(TS::NT), PLBM_LDS_PAD, a.stream, a.P, a.work, a.nwork, a.phase, a.out_rho, a.out_u,
                       reinterpret_cast<RedRec*>(a.red));
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <class L, int COLL, int MODE>
static hipError_t go_step(const StepLaunch& a) {
  using TS = TileShape<L>;
  if (a.wb) return a.walls ? go_wb<L, COLL, MODE, true>(a) : go_wb<L, COLL, MODE, false>(a);
  if (a.aa) return a.walls ? go_aa<L, COLL, MODE, true>(a) : go_aa<L, COLL, MODE, false>(a);
  if (a.walls)
    hipLaunchKernelGGL((k_step<L, PLBM_ST, COLL, MODE, TS::TX, TS::TY, TS::NT, true, SCH_PP>), dim3(a.nblocks), dim3(TS::NT),
                       PLBM_LDS_PAD, a.stream, a.P, a.work, a.nwork, a.phase, a.out_rho, a.out_u,
                       reinterpret_cast<RedRec*>(a.red));
  else
    hipLaunchKernelGGL((k_step<L, PLBM_ST, COLL, MODE, TS::TX, TS::TY, TS::NT, false, SCH_PP>), dim3(a.nblocks),
                       dim3(TS::NT), PLBM_LDS_PAD, a.stream, a.P, a.work, a.nwork, a.phase, a.out_rho, a.out_u,
                       reinterpret_cast<RedRec*>(a.red));
  return hipGetLastError();
}

template <class L>
static hipError_t step_for(const StepLaunch& a) {
  if (a.mode == MODE_STEP) return a.coll == COLL_MRT ? go_step<L, COLL_MRT, MODE_STEP>(a) : go_step<L, COLL_BGK, MODE_STEP>(a);
  if (a.mode == MODE_MOMENTS) return go_step<L, COLL_BGK, MODE_MOMENTS>(a);
  return go_step<L, COLL_BGK, MODE_REDUCE>(a);
}

hipError_t PLBM_CAT(launch_step_, PLBM_SUFFIX)(const StepLaunch& a) {
  return a.lattice == 1 ? step_for<D3Q19L>(a) : step_for<D2Q9L>(a);
}

template <class L, int COLL, bool WALLS>
static hipError_t occ_go(int aa, int* blocks) {
  using TS = TileShape<L>;
  using AS = AaTileShape<L>;
  if (aa)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks, k_aa_step<L, PLBM_ST, COLL, MODE_STEP, AS::TX, AS::TY, WALLS>, AS::TX * AS::TY, 0);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      blocks, k_step<L, PLBM_ST, COLL, MODE_STEP, TS::TX, TS::TY, TS::NT, WALLS, SCH_PP>, TS::NT, PLBM_LDS_PAD);
}

template <class L>
static hipError_t occ_for(int coll, int walls, int aa, int* blocks) {
  if (coll == COLL_MRT) return walls ? occ_go<L, COLL_MRT, true>(aa, blocks) : occ_go<L, COLL_MRT, false>(aa, blocks);
  return walls ? occ_go<L, COLL_BGK, true>(aa, blocks) : occ_go<L, COLL_BGK, false>(aa, blocks);
}

void PLBM_CAT(tile_shape_, PLBM_SUFFIX)(int aa, int* tx, int* ty) {
  *tx = aa ? AaTileShape<D3Q19L>::TX : TileShape<D3Q19L>::TX;
  *ty = aa ? AaTileShape<D3Q19L>::TY : TileShape<D3Q19L>::TY;
}

hipError_t PLBM_CAT(occupancy_step_, PLBM_SUFFIX)(int lattice, int coll, int walls, int aa, int* blocks) {
  return lattice == 1 ? occ_for<D3Q19L>(coll, walls, aa, blocks) : occ_for<D2Q9L>(coll, walls, aa, blocks);
}

template <class L>
static hipError_t aux_for(const AuxLaunch& a) {
  dim3 g(a.nblocks), b(256);
  switch (a.what) {
    case AUX_INIT_FIELDS:
      hipLaunchKernelGGL((k_init_fields<L, PLBM_ST>), g, b, 0, a.stream, a.P, a.par, a.in0, a.in1);
      break;
    case AUX_INIT_SHAPE:
      hipLaunchKernelGGL((k_init_shape<L, PLBM_ST>), g, b, 0, a.stream, a.P, a.par, *a.shape);
      break;
    case AUX_READ_POP:
      hipLaunchKernelGGL((k_read_pop<L, PLBM_ST>), g, b, 0, a.stream, a.P, a.par, a.dir, a.out);
      break;
    default:
      hipLaunchKernelGGL((k_write_pop<L, PLBM_ST>), g, b, 0, a.stream, a.P, a.par, a.dir, a.in0);
      break;
  }
  return hipGetLastError();
}

hipError_t PLBM_CAT(launch_aux_, PLBM_SUFFIX)(const AuxLaunch& a) {
  return a.lattice == 1 ? aux_for<D3Q19L>(a) : aux_for<D2Q9L>(a);
}

}  // namespace plbm
