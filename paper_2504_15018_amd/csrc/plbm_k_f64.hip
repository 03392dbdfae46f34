// Kernels for population storage StF64.
#define PLBM_ST plbm::StF64
#define PLBM_SUFFIX f64
#include "plbm_kernels_inst.hpp"

namespace plbm {

// Sum the per-tile reduction records of one lattice in tile order (one
// thread: deterministic, independent of the launch configuration).
__global__ void k_reduce_final(const KParams* __restrict__ P, int ntiles, RedRec* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const RedRec* r = reinterpret_cast<const RedRec*>(P->red);
  RedRec o = r[0];
  for (int k = 1; k < ntiles; ++k) {
    neumaier_add(o.mass_s, o.mass_c, r[k].mass_s);
    o.mass_c += r[k].mass_c;
    for (int a = 0; a < 3; ++a) o.mom[a] += r[k].mom[a];
    o.max_u = fmax(o.max_u, r[k].max_u);
    o.max_du = fmax(o.max_du, r[k].max_du);
    o.flags = (double)((int)o.flags | (int)r[k].flags);
  }
  *out = o;
}


hipError_t launch_reduce_final(hipStream_t st, const KParams* P, int ntiles, void* out) {
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(64), 0, st, P, ntiles, reinterpret_cast<RedRec*>(out));
  return hipGetLastError();
}
}  // namespace plbm
