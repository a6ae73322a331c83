// Explicit interaction lists (g3_walk): the same wave-coherent walks as the
// density, hydro and gravity kernels, emitting the accepted entries instead
// of summing them. A counting pass sizes each row, a scan gives the CSR
// offsets, a filling pass writes the rows. On trees of FP64 positions
// (kF64) every neighbour and opening decision is the FP64 one, the one the
// mixed-precision kernels take; the walk's pruning on the FP32 copies is
// padded as theirs (walk_radius64).
#include "g3_device.h"
#include "g3_internal.h"

namespace g3 {

namespace {

constexpr int kBlock = 256;

template <bool kF64>
__global__ __launch_bounds__(kBlock) void k_walk_sph(
    const Node *__restrict__ nodes, const float4 *__restrict__ xm,
    const float4 *__restrict__ vh, const double4 *__restrict__ x64,
    const double *__restrict__ h64, const unsigned *__restrict__ absmax,
    const int32_t *__restrict__ perm, const Groups gs, const int32_t *__restrict__ rows,
    int symmetric, int32_t *__restrict__ counts, const int64_t *__restrict__ offsets,
    int32_t *__restrict__ list) {
  const int lane = lane_id();
  const float slack = kF64 ? ldexpf(__uint_as_float(*absmax), -20) : 0.0f;
  int range = 0;
  for (int g; (g = next_group(gs, range)) >= 0;) {
  const Group grp = group_at(gs, g);
  const int64_t t = grp.t0 + lane;
  const bool valid = lane < grp.count;
  const int s = valid ? (gs.targets ? gs.targets[t] : (int)t) : 0;
  // rows follow `active`; with every particle active they are caller ids
  const int64_t row = valid ? (rows ? (int64_t)rows[t] : (int64_t)perm[s]) : 0;
  const float4 me = xm[s];
  const float3 xi = make_float3(me.x, me.y, me.z);
  const float hi = valid ? vh[s].w : -1.0f;
  const float h2 = valid ? sq_exact(hi) : -1.0f;
  int64_t pos = (list && valid) ? offsets[row] : 0;
  int cnt = 0;
  int cur = grp.root;
  while (cur < grp.end) {
    const Node nd = nodes[cur];
    const float d2 = box_dist2(xi, nd.lo_h, nd.hi_l);
    const float hw = symmetric ? fmaxf(hi, nd.lo_h.w) : hi;
    const bool want = valid && d2 < (kF64 ? sq_exact(walk_radius64(hw, slack)) : sq_exact(hw));
    if (__ballot(want) == 0ull) {
      cur = nd.meta.x;
      continue;
    }
    if (!(nd.meta.w & kLeafBit)) {
      ++cur;
      continue;
    }
    for (int k = nd.meta.y; k < nd.meta.y + nd.meta.z; ++k) {
      bool take;
      if constexpr (kF64) {
        take = valid && (symmetric ? k != s && within64(x64[s], x64[k], fmax(h64[s], h64[k]))
                                   : within64(x64[s], x64[k], h64[s]));
      } else {
        const float4 q = xm[k];
        const float r2 = dist2_exact(sub_exact(q.x, xi.x), sub_exact(q.y, xi.y),
                                     sub_exact(q.z, xi.z));
        if (symmetric) take = valid && k != s && r2 < sq_exact(fmaxf(hi, vh[k].w));
        else take = valid && r2 < h2;
      }
      if (take) {
        if (list) list[pos++] = perm[k];
        ++cnt;
      }
    }
    cur = nd.meta.x;
  }
  if (valid && !list) counts[row] = cnt;
  }  // groups
}

__device__ __forceinline__ bool open_accept(float l, float theta2, float r2) {
#pragma clang fp contract(off)
  const float lhs = l * l;
  const float rhs = theta2 * r2;
  return lhs < rhs;
}

template <bool kF64>
__global__ __launch_bounds__(kBlock) void k_walk_grav(
    const Node *__restrict__ nodes, const float4 *__restrict__ xm,
    const double4 *__restrict__ x64, const double4 *__restrict__ c64n,
    const uint64_t *__restrict__ keys, const int32_t *__restrict__ perm, const Groups gs,
    const int32_t *__restrict__ rows, float theta2, double theta64, int inside_test,
    int32_t *__restrict__ counts, const int64_t *__restrict__ offsets,
    int32_t *__restrict__ list) {
  const int lane = lane_id();
  int range = 0;
  for (int g; (g = next_group(gs, range)) >= 0;) {
  const Group grp = group_at(gs, g);
  const int64_t t = grp.t0 + lane;
  const bool valid = lane < grp.count;
  const int s = valid ? (gs.targets ? gs.targets[t] : (int)t) : 0;
  // rows follow `active`; with every particle active they are caller ids
  const int64_t row = valid ? (rows ? (int64_t)rows[t] : (int64_t)perm[s]) : 0;
  const float4 me = xm[s];
  const float3 xi = make_float3(me.x, me.y, me.z);
  const uint64_t ki = keys[s];
  int64_t pos = (list && valid) ? offsets[row] : 0;
  int cnt = 0;
  int resume = valid ? grp.root : INT32_MAX;
  int cur = grp.root;
  while (cur < grp.end) {
    const Node nd = nodes[cur];
    const bool act = cur >= resume;
    bool accept;
    if constexpr (kF64) {
      // the cube side of the node's level, exact in FP64
      accept = act && open_accept64(ldexp(gs.sbox[grp.snap].w, -(nd.meta.w & 255)), theta64,
                                    c64n[cur], x64[s]);
    } else {
      const float r2 = dist2_exact(sub_exact(nd.com_m.x, xi.x), sub_exact(nd.com_m.y, xi.y),
                                   sub_exact(nd.com_m.z, xi.z));
      accept = act && open_accept(nd.hi_l.w, theta2, r2);
    }
    if (inside_test) {
      const int level = nd.meta.w & 255;
      const uint64_t nk = keys[nd.meta.y];
      accept = accept && (((ki ^ nk) >> (3 * (kMaxLevel - level))) != 0ull);
    }
    const bool open = act && !accept;
    if (accept) {
      resume = nd.meta.x;
      if (list) list[pos++] = -(cur + 1);
      ++cnt;
    }
    if (__ballot(open) == 0ull) {
      cur = nd.meta.x;
      continue;
    }
    if (!(nd.meta.w & kLeafBit)) {
      ++cur;
      continue;
    }
    for (int k = nd.meta.y; k < nd.meta.y + nd.meta.z; ++k) {
      if (open && k != s) {
        if (list) list[pos++] = perm[k];
        ++cnt;
      }
    }
    cur = nd.meta.x;
  }
  if (valid && !list) counts[row] = cnt;
  }  // groups
}

}  // namespace

hipError_t launch_walk(const Octree &o, int kind, const Groups &gs, const int32_t *rows,
                       int64_t max_groups, const GravParams &gp, const unsigned *absmax,
                       int32_t *counts, const int64_t *offsets, int32_t *list, hipStream_t s) {
  if (max_groups <= 0 || o.nnodes == 0) return hipSuccess;
  if (gp.f64 && (!o.x64 || (kind == G3_GRAVITY ? !o.c64 : (!o.h64 || !absmax))))
    return hipErrorInvalidValue;
  if (kind == G3_GRAVITY) {
    auto kern = gp.f64 ? k_walk_grav<true> : k_walk_grav<false>;
    kern<<<persistent_grid((const void *)kern, kBlock, max_groups), kBlock, 0, s>>>(
        o.nodes, o.xm, o.x64, o.c64, o.keys, o.perm, gs, rows, gp.theta2, gp.theta,
        gp.inside_test, counts, offsets, list);
  } else {
    auto kern = gp.f64 ? k_walk_sph<true> : k_walk_sph<false>;
    kern<<<persistent_grid((const void *)kern, kBlock, max_groups), kBlock, 0, s>>>(
        o.nodes, o.xm, o.vh, o.x64, o.h64, absmax, o.perm, gs, rows, kind == G3_SYMMETRIC,
        counts, offsets, list);
  }
  return hipGetLastError();
}

}  // namespace g3
