// Kernels for population storage StF64.
#define PLBM_ST plbm::StF64
#define PLBM_SUFFIX f64
#include "plbm_kernels_inst.hpp"

namespace plbm {

// Combine the per-tile reduction records of one lattice: thread k folds
// tiles k, k + 256, ... in order, then the workgroup's fixed-order wave
// reduction.  The order depends only on the tile count, so the result is
// deterministic.
__device__ __forceinline__ void reduce_tiles(const RedRec* __restrict__ r, int ntiles, RedRec* __restrict__ out) {
  __shared__ RedRec wl[256 / 64];
  RedRec o;
  o.mass_s = o.mass_c = 0.0;
  o.mom[0] = o.mom[1] = o.mom[2] = 0.0;
  o.max_u = o.max_du = 0.0;
  o.flags = 0.0;
  for (int k = threadIdx.x; k < ntiles; k += 256) red_combine(o, r[k]);
  block_reduce_store<256>(o, wl, out);
}

__global__ __launch_bounds__(256) void k_reduce_final(const KParams* __restrict__ P, int ntiles,
                                                      RedRec* __restrict__ out, const RedRec* __restrict__ recs) {
  reduce_tiles(recs != nullptr ? recs : reinterpret_cast<const RedRec*>(P->red), ntiles, out);
}

// One workgroup per batch slot: the same fixed-order combination for every
// attached lattice at once (slots without a lattice have ntiles = 0 and give
// a zero record).
__global__ __launch_bounds__(256) void k_reduce_final_batch(const KParams* __restrict__ P,
                                                            RedRec* __restrict__ out) {
  const KParams* kp = P + blockIdx.x;
  reduce_tiles(reinterpret_cast<const RedRec*>(kp->red), kp->ntiles, out + blockIdx.x);
}

hipError_t launch_reduce_final(hipStream_t st, const KParams* P, int ntiles, void* out, const void* recs) {
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, st, P, ntiles, reinterpret_cast<RedRec*>(out),
                     reinterpret_cast<const RedRec*>(recs));
  return hipGetLastError();
}

hipError_t launch_reduce_final_batch(hipStream_t st, const KParams* P, int nslots, void* out) {
  hipLaunchKernelGGL(k_reduce_final_batch, dim3(nslots), dim3(256), 0, st, P, reinterpret_cast<RedRec*>(out));
  return hipGetLastError();
}

// Locally shifted storage, before k_write_pop: acc[n] (+)= in[n] over the
// directions (first = 1 starts the sum), then the reference densities
// ref[n] = acc[n] rounded to float32, then to half precision.
__global__ __launch_bounds__(256) void k_accum(int64_t N, int first, const double* __restrict__ in,
                                               double* __restrict__ acc) {
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x)
    acc[n] = (first ? 0.0 : acc[n]) + in[n];
}

__global__ __launch_bounds__(256) void k_set_ref(const KParams* __restrict__ P, int par, const double* __restrict__ acc) {
  const KParams p = *P;
  RefT* ref = reinterpret_cast<RefT*>(p.ref[par]);
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < p.N; n += (int64_t)gridDim.x * blockDim.x)
    ref[n] = (RefT)(float)acc[n];
}

hipError_t launch_accum(hipStream_t st, int nblocks, int64_t N, int first, const double* in, double* acc) {
  hipLaunchKernelGGL(k_accum, dim3(nblocks), dim3(256), 0, st, N, first, in, acc);
  return hipGetLastError();
}

hipError_t launch_set_ref(hipStream_t st, int nblocks, const KParams* P, int par, const double* acc) {
  hipLaunchKernelGGL(k_set_ref, dim3(nblocks), dim3(256), 0, st, P, par, acc);
  return hipGetLastError();
}

}  // namespace plbm
