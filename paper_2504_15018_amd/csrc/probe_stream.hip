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
// k_probe_stream19v<V>: the same bytes and layout with V = 2 or 4 consecutive
// nodes per thread (8- or 16-byte accesses per direction).
// k_probe_stream19x<XB, V>: the same bytes in blocks of XB = 32, 64 or 128
// nodes (128, 256 or 512 bytes per direction), V = 1, 2 or 4 nodes per thread
// (4: XB = 128 only, a wave's access one contiguous 1 KiB per direction),
// optionally with unused dynamic LDS capping the workgroups per CU.
// k_probe_stream19s<NT, ORDER>: blocks of 32 nodes, one node per thread, with
// plain (NT = 0) or non-temporal stores, all loads before the stores
// (ORDER = 0) or each direction stored right after its load (ORDER = 1).
// k_probe_copy4nt: the float4 copy with non-temporal stores.
// k_probe_read19<ORDER>: the 19 arrays read once, their sum written once per
// node (a read-mostly pass), on a cube of side 256: ORDER 0 one node per
// thread in memory order; ORDER 1 a 64 x 8 tile of one plane per workgroup
// (the tiles of a plane consecutive); ORDER 2 a 64 x 8 tile column per
// workgroup marching through 256 / SPLIT planes (SPLIT chunks per column).
// k_probe_stream19h<V>: 19 arrays of 16-bit values in blocks of 64 nodes (128
// bytes per direction), V = 1, 2 or 4 consecutive nodes per thread (2-, 4- or
// 8-byte accesses), non-temporal stores: the 16-bit update's bytes.
// k_probe_pingpong<NT>: the 19-array stream of k_probe_stream19 (NT = 1) or
// with plain stores (NT = 0), its workgroups taking the blocks in memory order
// or (rev) in reverse, for ping-pong pairs (a to b, then b to a) in which the
// second pass starts where the first ended.
// k_probe_copy4: a plain float4 copy, one vector per thread;
// k_probe_copy4u: the same with four vectors per thread (a block-stride loop).
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

template <int NT>
__global__ __launch_bounds__(256) void k_probe_pingpong(const float* __restrict__ src, float* __restrict__ dst,
                                                        uint32_t nodes, int rev) {
  const uint32_t blk = rev ? gridDim.x - 1u - blockIdx.x : blockIdx.x;
  const uint32_t n = blk * 256u + threadIdx.x;
  if (n >= nodes) return;
  const uint64_t at = (uint64_t)(n / kXB) * (kQ * kXB) + (n % kXB);
  float v[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) v[q] = src[at + (uint64_t)q * kXB];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    if constexpr (NT) __builtin_nontemporal_store(v[q] + 1.0f, dst + at + (uint64_t)q * kXB);
    else dst[at + (uint64_t)q * kXB] = v[q] + 1.0f;
  }
}

template <int V>
__global__ __launch_bounds__(256) void k_probe_stream19v(const float* __restrict__ src, float* __restrict__ dst,
                                                         uint32_t nodes) {
  typedef float vec __attribute__((ext_vector_type(V)));
  const uint32_t n = (blockIdx.x * 256u + threadIdx.x) * V;  // first of V nodes, in one block of 32
  if (n >= nodes) return;
  const uint64_t at = (uint64_t)(n / kXB) * (kQ * kXB) + (n % kXB);
  vec v[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) v[q] = *reinterpret_cast<const vec*>(src + at + (uint64_t)q * kXB);
#pragma unroll
  for (int q = 0; q < kQ; ++q)
    __builtin_nontemporal_store(v[q] + 1.0f, reinterpret_cast<vec*>(dst + at + (uint64_t)q * kXB));
}

template <int XB, int V>
__global__ __launch_bounds__(256) void k_probe_stream19x(const float* __restrict__ src, float* __restrict__ dst,
                                                         uint32_t nodes) {
  typedef float vec __attribute__((ext_vector_type(V)));
  const uint32_t n = (blockIdx.x * 256u + threadIdx.x) * V;
  if (n >= nodes) return;
  const uint64_t at = (uint64_t)(n / XB) * (kQ * XB) + (n % XB);
  vec v[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) v[q] = *reinterpret_cast<const vec*>(src + at + (uint64_t)q * XB);
#pragma unroll
  for (int q = 0; q < kQ; ++q)
    __builtin_nontemporal_store(v[q] + 1.0f, reinterpret_cast<vec*>(dst + at + (uint64_t)q * XB));
}

template <int NTS, int ORDER>
__global__ __launch_bounds__(256) void k_probe_stream19s(const float* __restrict__ src, float* __restrict__ dst,
                                                         uint32_t nodes) {
  const uint32_t n = blockIdx.x * 256u + threadIdx.x;
  if (n >= nodes) return;
  const uint64_t at = (uint64_t)(n / kXB) * (kQ * kXB) + (n % kXB);
  auto put = [&](int q, float v) {
    if constexpr (NTS) __builtin_nontemporal_store(v, dst + at + (uint64_t)q * kXB);
    else dst[at + (uint64_t)q * kXB] = v;
  };
  if constexpr (ORDER == 0) {
    float v[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) v[q] = src[at + (uint64_t)q * kXB];
#pragma unroll
    for (int q = 0; q < kQ; ++q) put(q, v[q] + 1.0f);
  } else {
#pragma unroll
    for (int q = 0; q < kQ; ++q) put(q, src[at + (uint64_t)q * kXB] + 1.0f);
  }
}

__global__ __launch_bounds__(256) void k_probe_copy4nt(const float* __restrict__ src, float* __restrict__ dst,
                                                       uint64_t n) {
  typedef float vec __attribute__((ext_vector_type(4)));
  const uint64_t i = blockIdx.x * 256ull + threadIdx.x;
  if (i < n) __builtin_nontemporal_store(reinterpret_cast<const vec*>(src)[i], reinterpret_cast<vec*>(dst) + i);
}

template <int V>
__global__ __launch_bounds__(256) void k_probe_stream19h(const uint16_t* __restrict__ src, uint16_t* __restrict__ dst,
                                                         uint32_t nodes) {
  constexpr int XB = 64;
  typedef uint16_t vec __attribute__((ext_vector_type(V)));
  const uint32_t n = (blockIdx.x * 256u + threadIdx.x) * V;
  if (n >= nodes) return;
  const uint64_t at = (uint64_t)(n / XB) * (kQ * XB) + (n % XB);
  vec v[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) v[q] = *reinterpret_cast<const vec*>(src + at + (uint64_t)q * XB);
#pragma unroll
  for (int q = 0; q < kQ; ++q)
    __builtin_nontemporal_store(v[q] + (uint16_t)1, reinterpret_cast<vec*>(dst + at + (uint64_t)q * XB));
}

template <int ORDER, int SPLIT>
__global__ __launch_bounds__(512) void k_probe_read19(const float* __restrict__ src, float* __restrict__ dst) {
  constexpr uint32_t S = 256;  // cube side
  auto node = [&](uint32_t n) {
    const uint64_t at = (uint64_t)(n / kXB) * (kQ * kXB) + (n % kXB);
    float r = 0.0f;
#pragma unroll
    for (int q = 0; q < kQ; ++q) r += src[at + (uint64_t)q * kXB];
    __builtin_nontemporal_store(r, dst + n);
  };
  const uint32_t t = threadIdx.x;
  if constexpr (ORDER == 0) {
    node(blockIdx.x * 512u + t);
  } else {
    const uint32_t tile = blockIdx.x % 128u;  // 4 x 32 tiles of 64 x 8 per plane
    const uint32_t x = (tile % 4u) * 64u + t % 64u, y = (tile / 4u) * 8u + t / 64u;
    if constexpr (ORDER == 1) {
      node((blockIdx.x / 128u * S + y) * S + x);
    } else {
      const uint32_t z0 = blockIdx.x / 128u * (S / SPLIT);
      for (uint32_t z = z0; z < z0 + S / SPLIT; ++z) node((z * S + y) * S + x);
    }
  }
}

__global__ __launch_bounds__(256) void k_probe_copy4u(const float4* __restrict__ src, float4* __restrict__ dst,
                                                      uint64_t n) {
  const uint64_t base = blockIdx.x * 1024ull + threadIdx.x;
  float4 v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint64_t i = base + 256ull * k;
    if (i < n) v[k] = src[i];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint64_t i = base + 256ull * k;
    if (i < n) dst[i] = v[k];
  }
}

__global__ __launch_bounds__(256) void k_probe_copy4(const float4* __restrict__ src, float4* __restrict__ dst,
                                                     uint64_t n) {
  const uint64_t i = blockIdx.x * 256ull + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace

extern "C" {

// src and dst hold 19 * 32 * ceil(nodes / 32) floats each; returns a hipError_t.
// A ping-pong pair over 19 arrays of `nodes` floats in the blocked layout: a
// to b in memory order, then b to a in memory order (alternate = 0) or in
// reverse (alternate = 1); nt selects non-temporal stores.
int plbm_probe_pingpong(void* a, void* b, uint32_t nodes, int nt, int alternate, void* stream) {
  if (nodes == 0) return 0;
  const hipStream_t st = (hipStream_t)stream;
  const dim3 grid((nodes + 255u) / 256u);
  if (nt) {
    hipLaunchKernelGGL((k_probe_pingpong<1>), grid, dim3(256), 0, st, (const float*)a, (float*)b, nodes, 0);
    hipLaunchKernelGGL((k_probe_pingpong<1>), grid, dim3(256), 0, st, (const float*)b, (float*)a, nodes, alternate);
  } else {
    hipLaunchKernelGGL((k_probe_pingpong<0>), grid, dim3(256), 0, st, (const float*)a, (float*)b, nodes, 0);
    hipLaunchKernelGGL((k_probe_pingpong<0>), grid, dim3(256), 0, st, (const float*)b, (float*)a, nodes, alternate);
  }
  return (int)hipGetLastError();
}

// plbm_probe_stream19 with `lds` bytes of dynamic LDS per workgroup (unused),
// which caps the workgroups resident per CU (160 KiB of LDS per CU) and so
// the loads in flight; lds at most 65536.
int plbm_probe_stream19_lds(const void* src, void* dst, uint32_t nodes, uint32_t lds, void* stream) {
  if (nodes == 0) return 0;
  if (lds > 65536u) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_probe_stream19, dim3((nodes + 255u) / 256u), dim3(256), lds, (hipStream_t)stream,
                     (const float*)src, (float*)dst, nodes);
  return (int)hipGetLastError();
}

int plbm_probe_stream19(const void* src, void* dst, uint32_t nodes, void* stream) {
  if (nodes == 0) return 0;
  hipLaunchKernelGGL(k_probe_stream19, dim3((nodes + 255u) / 256u), dim3(256), 0, (hipStream_t)stream,
                     (const float*)src, (float*)dst, nodes);
  return (int)hipGetLastError();
}

// As plbm_probe_stream19 with vec = 2 or 4 nodes per thread; nodes must be a multiple of vec.
int plbm_probe_stream19v(const void* src, void* dst, uint32_t nodes, int vec, void* stream) {
  if (nodes == 0) return 0;
  if ((vec != 2 && vec != 4) || nodes % (uint32_t)vec) return (int)hipErrorInvalidValue;
  const uint32_t threads = nodes / (uint32_t)vec;
  if (vec == 2)
    hipLaunchKernelGGL(k_probe_stream19v<2>, dim3((threads + 255u) / 256u), dim3(256), 0, (hipStream_t)stream,
                       (const float*)src, (float*)dst, nodes);
  else
    hipLaunchKernelGGL(k_probe_stream19v<4>, dim3((threads + 255u) / 256u), dim3(256), 0, (hipStream_t)stream,
                       (const float*)src, (float*)dst, nodes);
  return (int)hipGetLastError();
}

// Blocks of xb = 32, 64 or 128 nodes, vec = 1 or 2 nodes per thread; nodes a
// multiple of xb; src and dst hold 19 * nodes floats each.
int plbm_probe_stream19x(const void* src, void* dst, uint32_t nodes, int xb, int vec, uint32_t lds, void* stream) {
  if (nodes == 0) return 0;
  if ((xb != 32 && xb != 64 && xb != 128) || (vec != 1 && vec != 2 && vec != 4) || (vec == 4 && xb != 128) ||
      nodes % (uint32_t)xb || lds > 65536u)
    return (int)hipErrorInvalidValue;
  const dim3 g((nodes / (uint32_t)vec + 255u) / 256u), b(256);
  const hipStream_t st = (hipStream_t)stream;
  const float* s = (const float*)src;
  float* d = (float*)dst;
  if (xb == 32 && vec == 1) hipLaunchKernelGGL((k_probe_stream19x<32, 1>), g, b, lds, st, s, d, nodes);
  if (xb == 32 && vec == 2) hipLaunchKernelGGL((k_probe_stream19x<32, 2>), g, b, lds, st, s, d, nodes);
  if (xb == 64 && vec == 1) hipLaunchKernelGGL((k_probe_stream19x<64, 1>), g, b, lds, st, s, d, nodes);
  if (xb == 64 && vec == 2) hipLaunchKernelGGL((k_probe_stream19x<64, 2>), g, b, lds, st, s, d, nodes);
  if (xb == 128 && vec == 1) hipLaunchKernelGGL((k_probe_stream19x<128, 1>), g, b, lds, st, s, d, nodes);
  if (xb == 128 && vec == 2) hipLaunchKernelGGL((k_probe_stream19x<128, 2>), g, b, lds, st, s, d, nodes);
  if (xb == 128 && vec == 4) hipLaunchKernelGGL((k_probe_stream19x<128, 4>), g, b, lds, st, s, d, nodes);
  return (int)hipGetLastError();
}

// Blocks of 32 nodes, one node per thread; nt: non-temporal stores; order 0:
// all loads, then the stores; order 1: each direction stored after its load.
int plbm_probe_stream19s(const void* src, void* dst, uint32_t nodes, int nt, int order, void* stream) {
  if (nodes == 0) return 0;
  const dim3 g((nodes + 255u) / 256u), b(256);
  const hipStream_t st = (hipStream_t)stream;
  const float* s = (const float*)src;
  float* d = (float*)dst;
  if (!nt && !order) hipLaunchKernelGGL((k_probe_stream19s<0, 0>), g, b, 0, st, s, d, nodes);
  if (!nt && order) hipLaunchKernelGGL((k_probe_stream19s<0, 1>), g, b, 0, st, s, d, nodes);
  if (nt && !order) hipLaunchKernelGGL((k_probe_stream19s<1, 0>), g, b, 0, st, s, d, nodes);
  if (nt && order) hipLaunchKernelGGL((k_probe_stream19s<1, 1>), g, b, 0, st, s, d, nodes);
  return (int)hipGetLastError();
}

// 16-bit populations in blocks of 64 nodes, vec = 1, 2 or 4 nodes per thread;
// nodes a multiple of 64; src and dst hold 19 * nodes 16-bit values each.
int plbm_probe_stream19h(const void* src, void* dst, uint32_t nodes, int vec, void* stream) {
  if (nodes == 0) return 0;
  if ((vec != 1 && vec != 2 && vec != 4) || nodes % 64u) return (int)hipErrorInvalidValue;
  const dim3 g((nodes / (uint32_t)vec + 255u) / 256u), b(256);
  const hipStream_t st = (hipStream_t)stream;
  const uint16_t* s = (const uint16_t*)src;
  uint16_t* d = (uint16_t*)dst;
  if (vec == 1) hipLaunchKernelGGL((k_probe_stream19h<1>), g, b, 0, st, s, d, nodes);
  if (vec == 2) hipLaunchKernelGGL((k_probe_stream19h<2>), g, b, 0, st, s, d, nodes);
  if (vec == 4) hipLaunchKernelGGL((k_probe_stream19h<4>), g, b, 0, st, s, d, nodes);
  return (int)hipGetLastError();
}

// Read-mostly pass over a 256^3 cube (src: 19 * 256^3 floats, dst: 256^3
// floats; nodes must be 256^3); order 0, 1 as k_probe_read19, 2 and 3 its tile
// columns in 2 and 16 chunks.
int plbm_probe_read19(const void* src, void* dst, uint32_t nodes, int order, void* stream) {
  if (nodes != 256u * 256u * 256u) return (int)hipErrorInvalidValue;
  const hipStream_t st = (hipStream_t)stream;
  const float* s = (const float*)src;
  float* d = (float*)dst;
  if (order == 0) hipLaunchKernelGGL((k_probe_read19<0, 1>), dim3(256u * 256u * 256u / 512u), dim3(512), 0, st, s, d);
  else if (order == 1) hipLaunchKernelGGL((k_probe_read19<1, 1>), dim3(128u * 256u), dim3(512), 0, st, s, d);
  else if (order == 2) hipLaunchKernelGGL((k_probe_read19<2, 2>), dim3(128u * 2u), dim3(512), 0, st, s, d);
  else if (order == 3) hipLaunchKernelGGL((k_probe_read19<2, 16>), dim3(128u * 16u), dim3(512), 0, st, s, d);
  else return (int)hipErrorInvalidValue;
  return (int)hipGetLastError();
}

// The float4 copy with non-temporal stores; bytes a multiple of 16 below 2^43.
int plbm_probe_copy4nt(const void* src, void* dst, uint64_t bytes, void* stream) {
  const uint64_t n = bytes / 16;
  if (n == 0) return 0;
  if ((n + 255) / 256 > 0x7fffffffull) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_probe_copy4nt, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     (const float*)src, (float*)dst, n);
  return (int)hipGetLastError();
}

// Four float4 per thread; bytes a multiple of 16 below 2^43.
int plbm_probe_copy4u(const void* src, void* dst, uint64_t bytes, void* stream) {
  const uint64_t n = bytes / 16;
  if (n == 0) return 0;
  if ((n + 1023) / 1024 > 0x7fffffffull) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_probe_copy4u, dim3((unsigned)((n + 1023) / 1024)), dim3(256), 0, (hipStream_t)stream,
                     (const float4*)src, (float4*)dst, n);
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
