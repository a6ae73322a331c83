// Device-side helpers shared by the kernels of libg3.so.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "g3_internal.h"

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

// Wendland C6 in 3D with support radius h (Dehnen & Aly 2012): the
// normalisation C = 1365 / (64 pi), and the radial factor of
// F = (1/r) dW/dr = -22 C/h^5 (1-q)^7 (1 + 7q + 16q^2) as a function of
// q = r/h: wendland_f(q) = (1-q)^7 (1 + 7q + 16q^2), zero at and beyond the
// support.
constexpr float kWendlandC = 6.7889530412636603f;
constexpr float kWendlandF = -22.0f * 6.7889530412636603f;
__device__ __forceinline__ float wendland_f(float q) {
  const float t = fmaxf(1.0f - q, 0.0f);
  const float t2 = t * t, t4 = t2 * t2;
  return t4 * t2 * t * (1.0f + q * (7.0f + q * 16.0f));
}

}  // namespace g3

namespace g3 {

// Index k of the segment holding v, for a non-decreasing table
// off[0..n] with off[0] <= v < off[n]: the largest k with off[k] <= v (so
// empty segments are skipped).
template <typename T>
__device__ __forceinline__ int segment_of(const T *__restrict__ off, int n, int64_t v) {
  int lo = 0, hi = n;  // off[lo] <= v < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)off[mid] <= v) lo = mid;
    else hi = mid;
  }
  return lo;
}

struct Group {
  int t0, count;  // targets [t0, t0 + count), count in 1..64
  int snap;       // snapshot
  int root, end;  // the snapshot's nodes [root, end)
};

__device__ __forceinline__ Group group_at(const Groups &gs, int g) {
  Group G;
  const int k = segment_of(gs.gstart, *gs.nseg, g);
  const int t1 = gs.tstart[k + 1];
  G.t0 = gs.tstart[k] + (g - gs.gstart[k]) * 64;
  G.count = min(64, t1 - G.t0);
  G.snap = gs.seg_snap[k];
  G.root = gs.nroot[G.snap];
  G.end = gs.nroot[G.snap + 1];
  return G;
}

// Persistent launches: a wave takes groups one at a time from a queue until
// none is left. The groups are split into 8 contiguous ranges, one per XCD
// (workgroups are dispatched round-robin over the XCDs), so spatially close
// groups share an L2; a wave drains its own XCD's range first and then
// helps with the others. Returns the next group, or -1 when all are taken.
// `range` is the wave's state (0 before the first call). Every wave leaves
// after at most (its groups + 8) atomic increments.
__device__ __forceinline__ int next_group(const Groups &gs, int &range) {
  constexpr int kXcd = 8;
  const int total = gs.gstart[*gs.nseg];
  const int home = (int)(blockIdx.x % kXcd);
  while (range < kXcd) {
    const int r = (home + range) % kXcd;
    const int lo = (int)(((int64_t)total * r) / kXcd);
    const int hi = (int)(((int64_t)total * (r + 1)) / kXcd);
    unsigned got = 0u;
    if (lo < hi) {
      if ((threadIdx.x & 63u) == 0u) got = atomicAdd(&gs.queue[r], 1u);
      got = (unsigned)__builtin_amdgcn_readfirstlane((int)got);
      if ((int64_t)lo + got < (int64_t)hi) return lo + (int)got;
    }
    ++range;
  }
  return -1;
}

// Mixed precision: the FP64 centre of a wave's group of targets, the first
// target's FP64 position moved to the middle of the box of the targets'
// FP32-rounded offsets from it (any FP64 point serves; the middle halves the
// largest offset). Wave-uniform; invalid lanes take no part.
__device__ __forceinline__ double4 group_centre(double4 c0, double4 p, bool valid) {
  float3 a = make_float3((float)(p.x - c0.x), (float)(p.y - c0.y), (float)(p.z - c0.z));
  float3 lo = valid ? a : make_float3(INFINITY, INFINITY, INFINITY);
  float3 hi = valid ? a : make_float3(-INFINITY, -INFINITY, -INFINITY);
#pragma unroll
  for (int m = 1; m < kWave; m <<= 1) {
    lo.x = fminf(lo.x, __shfl_xor(lo.x, m));
    lo.y = fminf(lo.y, __shfl_xor(lo.y, m));
    lo.z = fminf(lo.z, __shfl_xor(lo.z, m));
    hi.x = fmaxf(hi.x, __shfl_xor(hi.x, m));
    hi.y = fmaxf(hi.y, __shfl_xor(hi.y, m));
    hi.z = fmaxf(hi.z, __shfl_xor(hi.z, m));
  }
  // held in scalar registers: every lane computed the same value
  auto su = [](double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo32 = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi32 = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi32 << 32) | lo32));
  };
  return make_double4(su(c0.x + (double)(0.5f * (lo.x + hi.x))),
                      su(c0.y + (double)(0.5f * (lo.y + hi.y))),
                      su(c0.z + (double)(0.5f * (lo.z + hi.z))), 0.0);
}

// o = fl32(x - c) and its residual l = fl32((x - c) - o).
__device__ __forceinline__ void two_float_offset(double4 x, double4 c, float3 &o, float3 &l) {
  const double dx = x.x - c.x, dy = x.y - c.y, dz = x.z - c.z;
  o = make_float3((float)dx, (float)dy, (float)dz);
  l = make_float3((float)(dx - (double)o.x), (float)(dy - (double)o.y), (float)(dz - (double)o.z));
}

// FP64 neighbour test on the stored FP64 positions, the same expression as
// the mixed-precision definition: ((dx dx + dy dy) + dz dz) < H H.
__device__ __forceinline__ bool within64(double4 a, double4 b, double H) {
#pragma clang fp contract(off)
  const double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
  return (dx * dx + dy * dy) + dz * dz < H * H;
}

// The opening test in FP64 on the stored FP64 positions and node centres:
// l l < (theta theta) ((dx dx + dy dy) + dz dz), no contraction.
__device__ __forceinline__ bool open_accept64(double l, double theta, double4 c, double4 x) {
#pragma clang fp contract(off)
  const double dx = c.x - x.x, dy = c.y - x.y, dz = c.z - x.z;
  return l * l < theta * theta * ((dx * dx + dy * dy) + dz * dz);
}

// FP64 positions: a walk radius for pruning on the FP32 copies (node boxes,
// group boxes, FP32 h). It covers the FP32 rounding of h (and of its
// square) with the factor 1 + 2^-22, and that of the coordinates with
// slack = 2^-20 max|x|, the pad the kernels take from the tree.
__device__ __forceinline__ float walk_radius64(float h, float slack) {
  return h * 1.0000002384185791f + slack;  // 1 + 2^-22
}

}  // namespace g3
