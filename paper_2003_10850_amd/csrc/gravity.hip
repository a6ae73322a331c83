// Barnes-Hut gravity with per-particle opening decisions, walked by a whole
// wavefront at a time.
//
// A wave serves 64 Morton-consecutive targets. It visits the all-particle
// octree in preorder with one scalar node load per step, and every lane
// takes the per-particle Barnes-Hut decision for that node (Barnes & Hut
// 1986): accept the monopole, open it, or skip it because an ancestor was
// already accepted (the lane then resumes at the ancestor's skip index).
// The wave descends while any lane opens. Accepted monopoles and the members
// of opened leaves become entries of a 64-entry interaction tile in LDS,
// each with the 64-bit mask of lanes that use it; the tile is then
// evaluated by all lanes with the mask applied to the inverse distance. This
// keeps the interaction step out of the walk's branches (the limitation the
// paper names for gravity, section 2.4) and reproduces the per-particle
// interaction list exactly.
#include "g3_device.h"
#include "g3_internal.h"

namespace g3 {

namespace {

constexpr int kBlock = 256;
constexpr int kWpb = kBlock / kWave;
constexpr int kTile = kWave;

struct __align__(16) Entry {
  float4 p;       // source position, mass
  int4 meta;      // source sorted index (-1: node), mask low, mask high, unused
};
// A lane's mask word is meta.y (lanes 0..31) or meta.z (lanes 32..63); the
// bit of a lane whose own target is the source is cleared when the entry is
// made, so the tile loop needs no self test.
constexpr int kMaskWord = 5;  // meta.y as the 32-bit word index within Entry

// The opening test, exact in FP32: fl(l * l) < fl(theta2 * r2).
__device__ __forceinline__ bool open_accept(float l, float theta2, float r2) {
#pragma clang fp contract(off)
  const float lhs = l * l;
  const float rhs = theta2 * r2;
  return lhs < rhs;
}


// Mixed precision (kF64): positions are stored in FP64 and the node centres
// of mass come from FP64 moments. Each term works on the FP32 difference of
// the source's and the target's FP32 offsets from the group's FP64 centre;
// the opening test on the FP32 rounding of the node's FP64 offset from the
// target, and near the threshold, where that test could disagree with the
// FP64 one, the FP64 test decides.
template <bool kF64, bool kInside>
__global__ __launch_bounds__(kBlock) void k_gravity(
    const GNode *__restrict__ nodes, const double4 *__restrict__ c64n,
    const float4 *__restrict__ xm, const double4 *__restrict__ x64,
    const uint64_t *__restrict__ keys, const int32_t *__restrict__ perm, const Groups gs,
    float theta2, float eps2, float G, int inside_test, double theta64,
    float *__restrict__ acc, float *__restrict__ pot, int32_t *__restrict__ nterms) {
  __shared__ Entry tiles[kWpb][kTile];
  // running totals (acc, pot) and their Neumaier compensations, and the term
  // count, one slot per lane: touched only at a flush, so the walk loop
  // carries no per-lane sums from one node to the next
  __shared__ float4 tot[kWpb][kTile], comp[kWpb][kTile];
  __shared__ int32_t nts[kWpb][kTile];
  const int w = (int)(threadIdx.x >> 6), lane = lane_id();
  int range = 0;
  for (int g; (g = next_group(gs, range)) >= 0;) {
  const Group grp = group_at(gs, g);
  const int64_t t = grp.t0 + lane;
  const bool valid = lane < grp.count;
  const int s = valid ? (gs.targets ? gs.targets[t] : (int)t) : 0;
  const double side = gs.sbox[grp.snap].w;  // root cube side
  // a node's level from its cube side: l = (float)side * 2^-level exactly
  const int root_exp = ilogbf((float)side);
  const float4 me = xm[s];
  const float3 xi = make_float3(me.x, me.y, me.z);
  // mixed precision: tile entries hold FP32 offsets from the group's FP64
  // centre and each term takes the FP32 difference of the source's and this
  // target's offsets; the opening test takes the FP32 rounding of the FP64
  // difference from this target (FP64 near the threshold)
  const double4 p64 = kF64 ? x64[s] : make_double4(0, 0, 0, 0);
  const double4 c64 = kF64 ? group_centre(x64[gs.targets ? gs.targets[grp.t0] : grp.t0], p64, valid)
                           : make_double4(0, 0, 0, 0);
  const float3 xo = kF64 ? make_float3((float)(p64.x - c64.x), (float)(p64.y - c64.y),
                                       (float)(p64.z - c64.z))
                         : xi;
  const uint64_t ki = keys[s];
  Entry *tile = tiles[w];

  tot[w][lane] = make_float4(0.f, 0.f, 0.f, 0.f);
  comp[w][lane] = make_float4(0.f, 0.f, 0.f, 0.f);
  nts[w][lane] = 0;
  int tc = 0;

  // this lane's bit in an entry's mask: word (low or high half) and offset
  const bool hiword = lane >= 32;
  const uint32_t bitpos = (uint32_t)lane & 31u;
  // this lane's mask word of entry k sits at word kMaskWord + hiword of it
  const uint32_t *maskw = (const uint32_t *)tile + kMaskWord + (hiword ? 1 : 0);
  auto flush = [&](int nc) {
    wave_sync();
    float px = 0.f, py = 0.f, pz = 0.f, pp = 0.f;
    int pn = 0;  // terms: entries whose mask holds this lane's bit
    for (int k = 0; k < nc; ++k) {
      const float4 ep = tile[k].p;
      // branch-free use: the signed extract of the lane's bit is 0 or all
      // ones, and masks the inverse distance
      const int32_t use = __builtin_amdgcn_sbfe((int32_t)maskw[k * (int)(sizeof(Entry) / 4)],
                                                bitpos, 1u);
      const float dx = ep.x - xo.x, dy = ep.y - xo.y, dz = ep.z - xo.z;
      const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
      // masked here (not the mass), so that an unused entry adds exact
      // zeros even at r2 = 0 (the own entry with zero softening)
      const float rinv = __int_as_float(__float_as_int(__builtin_amdgcn_rsqf(r2)) & use);
      const float mr = ep.w * rinv;
      const float mr3 = mr * rinv * rinv;
      px += mr3 * dx;
      py += mr3 * dy;
      pz += mr3 * dz;
      pp -= mr;
      pn -= use;
    }
    float4 t = tot[w][lane], c = comp[w][lane];
    neumaier_add(t.x, c.x, px);
    neumaier_add(t.y, c.y, py);
    neumaier_add(t.z, c.z, pz);
    neumaier_add(t.w, c.w, pp);
    tot[w][lane] = t;
    comp[w][lane] = c;
    nts[w][lane] += pn;
    wave_sync();
  };

  // the group's node range, wave-uniform (in scalar registers for the
  // FP32 walk; the mixed-precision walk measured faster without)
  const int groot = kF64 ? grp.root : __builtin_amdgcn_readfirstlane(grp.root);
  const int gend = kF64 ? grp.end : __builtin_amdgcn_readfirstlane(grp.end);
  int resume = valid ? groot : INT32_MAX;  // lanes idle while cur < resume
  int cur = groot;
  while (cur < gend) {
    const GNode nd = nodes[cur];
    const float l = __int_as_float(nd.meta.w);
    const bool act = cur >= resume;
    double4 cn = make_double4(0, 0, 0, 0);
    float r2;
    if constexpr (kF64) {
      cn = c64n[cur];
      r2 = dist2_exact((float)(cn.x - p64.x), (float)(cn.y - p64.y), (float)(cn.z - p64.z));
    } else {
      r2 = dist2_exact(sub_exact(nd.com_m.x, xi.x), sub_exact(nd.com_m.y, xi.y),
                       sub_exact(nd.com_m.z, xi.z));
    }
    bool accept, open;
    if constexpr (!kF64 && !kInside) {
      // one compare per decision: an idle lane compares with NaN, for which
      // both are false; otherwise the exact test fl(l l) < fl(theta2 r2)
      float t;
      {
#pragma clang fp contract(off)
        t = act ? theta2 * r2 : __builtin_nanf("");
      }
      const float lhs = sq_exact(l);
      accept = lhs < t;
      open = lhs >= t;
    } else {
      accept = act && open_accept(l, theta2, r2);
      if constexpr (kF64) {
        // the FP32 r2 of exact-to-2^-24 offsets is within about 2^-22 of the
        // FP64 value (relative); inside 2^-19 of the threshold FP64 decides
        const float lhs = l * l, rhs = theta2 * r2;
        if (act && fabsf(lhs - rhs) <= rhs * 1.9073486e-6f)
          accept = open_accept64(ldexp(side, -(root_exp - ilogbf(l))), theta64, cn, p64);
      }
      if (kInside || (kF64 && inside_test)) {
        const int level = root_exp - ilogbf(l);
        const uint64_t nk = keys[nd.meta.y];
        const bool inside = ((ki ^ nk) >> (3 * (kMaxLevel - level))) == 0ull;
        accept = accept && !inside;
      }
      open = act && !accept;
    }
    const uint64_t amask = __ballot(accept);
    const uint64_t omask = __ballot(open);
    if (accept) resume = nd.meta.x;
    if (amask) {
      if (tc == kTile) {
        flush(kTile);
        tc = 0;
      }
      if (lane == 0) {
        Entry e;
        e.p = nd.com_m;
        if constexpr (kF64)
          e.p = make_float4((float)(cn.x - c64.x), (float)(cn.y - c64.y), (float)(cn.z - c64.z),
                            nd.com_m.w);
        e.meta = make_int4(-1, (int)(uint32_t)amask, (int)(uint32_t)(amask >> 32), 0);
        tile[tc] = e;
      }
      ++tc;
    }
    if (omask == 0ull) {
      cur = nd.meta.x;
      continue;
    }
    if (nd.meta.z < 0) {  // internal
      ++cur;
      continue;
    }
    int st = nd.meta.y, c = nd.meta.z;
    while (c > 0) {
      if (tc == kTile) {
        flush(kTile);
        tc = 0;
      }
      const int take = min(c, kTile - tc);
      if (lane < take) {
        Entry e;
        if constexpr (kF64) {
          // the FP32 offset from the group centre; the fourth slot holds the
          // (FP32) mass exactly
          const double4 q = x64[st + lane];
          e.p = make_float4((float)(q.x - c64.x), (float)(q.y - c64.y), (float)(q.z - c64.z),
                            (float)q.w);
        } else {
          e.p = xm[st + lane];
        }
        e.meta = make_int4(st + lane, (int)(uint32_t)omask, (int)(uint32_t)(omask >> 32), 0);
        tile[tc + lane] = e;
      }
      wave_sync();
      // an opening lane whose own target is among these members clears its
      // bit in that member's entry (one lane per entry)
      const int rel = s - st;
      if (open && rel >= 0 && rel < take) {
        uint32_t *wd = (uint32_t *)&tile[tc + rel] + kMaskWord + (hiword ? 1 : 0);
        *wd &= ~(1u << bitpos);
      }
      tc += take;
      st += take;
      c -= take;
    }
    cur = nd.meta.x;
  }
  if (tc > 0) flush(tc);
  const float4 tt = tot[w][lane], tc4 = comp[w][lane];
  const float ax = tt.x + tc4.x, ay = tt.y + tc4.y, az = tt.z + tc4.z, ph = tt.w + tc4.w;
  const int nt = nts[w][lane];

  if (valid) {
    const int cid = perm[s];
    if (acc) {
      acc[3 * cid] = G * ax;
      acc[3 * cid + 1] = G * ay;
      acc[3 * cid + 2] = G * az;
    }
    if (pot) pot[cid] = G * ph;
    if (nterms) nterms[cid] = nt;
  }
  }  // groups
}

}  // namespace

hipError_t launch_gravity(const Octree &all, const Groups &gs, int64_t max_groups,
                          const GravParams &gp, float *acc, float *pot, int32_t *nterms,
                          hipStream_t s) {
  if (max_groups <= 0 || all.nnodes == 0) return hipSuccess;
  // FP32: the containment test is compiled in or out; FP64: a runtime flag
  auto kern = gp.f64 ? k_gravity<true, false>
                     : (gp.inside_test ? k_gravity<false, true> : k_gravity<false, false>);
  if (!all.gnodes) return hipErrorInvalidValue;
  kern<<<persistent_grid((const void *)kern, kBlock, max_groups), kBlock, 0, s>>>(
      all.gnodes, all.c64, all.xm, all.x64, all.keys, all.perm, gs, gp.theta2, gp.eps2, gp.G,
      gp.inside_test, gp.theta, acc, pot, nterms);
  return hipGetLastError();
}

}  // namespace g3
