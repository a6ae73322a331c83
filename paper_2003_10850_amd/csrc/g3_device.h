// Device-side helpers shared by the kernels of libg3.so.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace g3 {

// Order LDS traffic between the lanes of one wavefront (a compiler barrier
// with wavefront-scope release/acquire fences; LDS executes a wave's
// instructions in order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2). Renumber them so that XCD x runs one contiguous range of logical
// blocks: spatially adjacent groups then share tree nodes and candidates in
// the same L2. The map is a bijection of [0, nb).
__device__ __forceinline__ int64_t xcd_block() {
  constexpr unsigned kXcd = 8;
  const unsigned b = blockIdx.x, nb = gridDim.x;
  const unsigned x = b % kXcd, q = nb / kXcd, r = nb % kXcd;
  return (int64_t)x * q + (x < r ? x : r) + b / kXcd;
}

// Broadcast of a wave-uniform value into a scalar register.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Exact neighbour test quantity: dx = fl(b - a) per axis,
// r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx)); no contraction beyond that.
__device__ __forceinline__ float dist2_exact(float dx, float dy, float dz) {
#pragma clang fp contract(off)
  const float xx = dx * dx;
  return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, xx));
}

// fl(b - a) with no contraction into a neighbouring product.
__device__ __forceinline__ float sub_exact(float b, float a) {
#pragma clang fp contract(off)
  return b - a;
}

// Squared distance from x to the box [lo, hi] evaluated with the same
// rounding steps as dist2_exact; never larger than dist2_exact of any point
// inside the box (rounding is monotone), so it prunes exactly.
__device__ __forceinline__ float box_dist2(float3 x, float4 lo, float4 hi) {
#pragma clang fp contract(off)
  const float dx = fmaxf(fmaxf(lo.x - x.x, x.x - hi.x), 0.0f);
  const float dy = fmaxf(fmaxf(lo.y - x.y, x.y - hi.y), 0.0f);
  const float dz = fmaxf(fmaxf(lo.z - x.z, x.z - hi.z), 0.0f);
  return dist2_exact(dx, dy, dz);
}

// Neumaier's compensated addition: s + c tracks the sum of every x added
// with an error of a few ulp of the total, independent of the count. The
// kernels add plain FP32 per-tile partial sums through it.
__device__ __forceinline__ void neumaier_add(float &s, float &c, float x) {
#pragma clang fp contract(off)
  const float t = s + x;
  c += (fabsf(s) >= fabsf(x)) ? ((s - t) + x) : ((x - t) + s);
  s = t;
}

// fl(a * a) with no contraction (the squared search radius).
__device__ __forceinline__ float sq_exact(float a) {
#pragma clang fp contract(off)
  return a * a;
}

}  // namespace g3
