// Bandwidth probes for the population access pattern, built into their own
// library (libplbm_probe.so) for the benchmark's reference points; not part of
// the method or of libplbm.
//
// k_probe_stream19: 19 float32 arrays in the blocked population layout
// (blocks of 32 nodes, the 19 directions of a block contiguous, 128 bytes per
// direction) read and written once, one node per thread, one add per value,
// stores with the non-temporal hint as in the update kernel.  It moves the
// update's algorithmic bytes with none of its halo, stencil or collision, so
// its rate bounds what the update can reach in this layout.
// k_probe_copy4: a plain float4 copy, one vector per thread.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kQ = 19;
constexpr int kXB = 32;

__global__ __launch_bounds__(256) void k_probe_stream19(const float* __restrict__ src, float* __restrict__ dst,
                                                        uint32_t nodes) {
  const uint32_t n = blockIdx.x * 256u + threadIdx.x;
  if (n >= nodes) return;
  const uint64_t at = (uint64_t)(n / kXB) * (kQ * kXB) + (n % kXB);
  float v[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) v[q] = src[at + (uint64_t)q * kXB];
#pragma unroll
  for (int q = 0; q < kQ; ++q) __builtin_nontemporal_store(v[q] + 1.0f, dst + at + (uint64_t)q * kXB);
}

__global__ __launch_bounds__(256) void k_probe_copy4(const float4* __restrict__ src, float4* __restrict__ dst,
                                                     uint64_t n) {
  const uint64_t i = blockIdx.x * 256ull + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace

extern "C" {

// src and dst hold 19 * 32 * ceil(nodes / 32) floats each; returns a hipError_t.
int plbm_probe_stream19(const void* src, void* dst, uint32_t nodes, void* stream) {
  if (nodes == 0) return 0;
  hipLaunchKernelGGL(k_probe_stream19, dim3((nodes + 255u) / 256u), dim3(256), 0, (hipStream_t)stream,
                     (const float*)src, (float*)dst, nodes);
  return (int)hipGetLastError();
}

// bytes must be a multiple of 16 and below 2^43; returns a hipError_t.
int plbm_probe_copy4(const void* src, void* dst, uint64_t bytes, void* stream) {
  const uint64_t n = bytes / 16;
  if (n == 0) return 0;
  if ((n + 255) / 256 > 0x7fffffffull) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_probe_copy4, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     (const float4*)src, (float4*)dst, n);
  return (int)hipGetLastError();
}

}  // extern "C"
