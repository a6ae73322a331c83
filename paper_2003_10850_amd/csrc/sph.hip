// SPH density (with the smoothing-length solve) and hydro force.
//
// One wavefront serves a group of 64 Morton-consecutive target particles,
// one per lane, as in the paper's walk over groups of active particles
// (section 1). The wave walks the gas octree in preorder with one scalar
// node load per step; a node is opened when any lane's search sphere
// reaches its tight bounding box. Leaf members are appended to a 64-entry
// candidate tile in LDS (the paper's neighbour chunks, section 2.4, here one
// wave wide); every lane then scans the tile against its own target with the
// exact neighbour test, so walk and interaction sums are decoupled without a
// per-particle list in memory.
#include <type_traits>

#include "g3_device.h"
#include "g3_internal.h"

namespace g3 {

namespace {

constexpr int kBlock = 256;
constexpr int kWpb = kBlock / kWave;  // waves per block
constexpr int kTile = kWave;

// Wendland C6 in 3D, support radius h: W = C/h^3 w(q),
// w(q) = (1-q)^8 (1 + 8q + 25q^2 + 32q^3); h dW/dh = C/h^3 wh(q),
// wh(q) = (1-q)^7 (448q^4 + 133q^3 - 29q^2 - 21q - 3);
// F = (1/r) dW/dr = -22 C/h^5 (1-q)^7 (1 + 7q + 16q^2).
constexpr float kC = 6.7889530412636603f;        // 1365 / (64 pi)
constexpr float kNeffSelf = 28.4375f;            // (4 pi / 3) C = 1365 / 48

// With s = ln h and q = r/h: w(q), wh = -3 w - q w' (so that d(h^-3 w)/ds =
// h^-3 wh), and wss = q w' + q^2 w'' = d(-q w')/ds, the curvature term of
// the h solve.
__device__ __forceinline__ void wc6_w_wh(float q, float &w, float &wh, float &wss) {
  const float t = 1.0f - q;
  const float t2 = t * t, t4 = t2 * t2, t6 = t4 * t2, t7 = t6 * t;
  w = t7 * t * (1.0f + q * (8.0f + q * (25.0f + q * 32.0f)));
  wh = t7 * (-3.0f + q * (-21.0f + q * (-29.0f + q * (133.0f + q * 448.0f))));
  wss = (q * q) * t6 * (-44.0f + q * (-264.0f + q * (132.0f + q * 3872.0f)));
}

// First guess of h: descend from the root along target s while the child
// still holds at least `least` members, then take that node's mean mass
// density over its cube. (Against the converged h of clustered workloads,
// a quarter of N_ngb over the cube gives a median error near 10 % where the
// group-wide density of an N_ngb node gives 15 % with a heavier tail.)
__device__ float node_density_guess(const Node *__restrict__ nodes, int root, int s,
                                    float least) {
  int cur = root;
  for (;;) {
    const int4 meta = nodes[cur].meta;
    if (meta.w & kLeafBit) break;
    int c = cur + 1, found = -1;
    while (c < meta.x) {
      const int4 cm = nodes[c].meta;
      if (s >= cm.y && s < cm.y + cm.z) {
        found = c;
        break;
      }
      c = cm.x;
    }
    if (found < 0 || (float)nodes[found].meta.z < least) break;
    cur = found;
  }
  const Node nd = nodes[cur];
  const float l = nd.hi_l.w;
  return nd.com_m.w / (l * l * l);
}


// The mixed precision of the density and hydro kernels works on FP32 offsets
// from one FP64 centre per group (the position of its first target), each
// carried as two floats: o = fl32(x - c) and its residual l = fl32((x - c) - o)
// (the FP64 difference itself is exact to 2^-53 |x - c|). A candidate is
// first tested on the high parts: d = fl(o_j - o_i) differs from x_j - x_i
// by at most 2^-24 (|x_j - x_i| + 2E) per axis, E the largest offset
// component of the group's targets and candidates, so
// r2 = fmaf(dz,dz,fmaf(dy,dy,dx dx)) is within 2^-24 (5 r^2 + 7 E r) of the
// FP64 value, below 2^-20 (h^2 + E h) near the threshold (r ~ h). Only a
// candidate inside 2^-19 (h^2 + E h) of it or closer takes the low parts,
// d' = d + fl(l_j - l_i), exact to about 2^-23 |x_j - x_i| + 2^-47 E per
// axis whatever the group's extent; its r2 then stands within 2^-21 h^2 of
// the FP64 value near the threshold, and inside the band 2^-19 (h^2 +
// 2^-20 E h) the FP64 positions decide, which keeps every decision exact.
// The sums take r2 of d', so their accuracy does not depend on E either.
constexpr float kBandOff = 1.9073486e-6f;  // 2^-19

// A group whose targets' offsets stay within kFineExt times its smallest h
// skips the low parts (outside the FP64 band): there the high parts alone
// give r2 within 2^-22 (1.5 r^2 + 1.8 E r) + 2^-24 3 r^2 of the FP64 value,
// about 2^-20 h^2 near the threshold, of the order of the FP32 sums' own
// rounding; wider groups take the low parts for every pair near or inside
// the threshold.
constexpr float kFineExt = 1.0f;


// Candidate streams per wave (kQ > 1, FP32 path): the lanes are split into
// kQ quarters of 64/kQ targets, and a leaf or small subtree the walk accepts
// is queued only for the quarters that have a lane reaching its box. A round
// loads up to 64 queued candidates of every quarter into that quarter's
// tile and each lane scans its own quarter's tile, so a lane tests the union
// of its quarter's candidates instead of the whole wave's.
constexpr int kRing = 256;  // queued candidate indices per quarter

template <bool kF64, int kQ>
__global__ __launch_bounds__(kBlock) void k_density(
    const Node *__restrict__ nodes, const float4 *__restrict__ xm,
    const double4 *__restrict__ x64, const int32_t *__restrict__ perm, const Groups gs,
    float n_ngb, float tol, int solve, int max_iter, int walk_leaf,
    const unsigned *__restrict__ absmax,
    void *__restrict__ hptr, float *__restrict__ rho, float *__restrict__ drho_dh,
    float *__restrict__ omega, int32_t *__restrict__ nngb,
    unsigned long long *__restrict__ counters) {
  using HT = typename std::conditional<kF64, double, float>::type;
  HT *h = (HT *)hptr;
  static_assert(kQ == 1 || !kF64, "candidate streams are for the FP32 path");
  // FP64 positions: the walk's pad for the rounding of the FP32 copies
  const float slack = kF64 ? ldexpf(__uint_as_float(*absmax), -20) : 0.0f;
  __shared__ float4 tiles[kWpb][kQ > 1 ? 1 : kTile];
  // mixed precision: the low parts of the offsets, and the sorted index of
  // each entry as the fourth component
  __shared__ float4 tlos[kWpb][kF64 ? kTile : 1];
  __shared__ int32_t ring[kWpb][kQ > 1 ? kQ : 1][kQ > 1 ? kRing : 1];
  __shared__ float4 qtile[kWpb][kQ > 1 ? kQ : 1][kQ > 1 ? kTile : 1];
  const int w = (int)(threadIdx.x >> 6), lane = lane_id();
  int range = 0;
  for (int g; (g = next_group(gs, range)) >= 0;) {
  const Group grp = group_at(gs, g);
  const int64_t t = grp.t0 + lane;
  const bool valid = lane < grp.count;
  const int s = valid ? (gs.targets ? gs.targets[t] : (int)t) : 0;
  // h_hi is capped at twice the diagonal of the snapshot's box
  const float hcap = (float)(3.4641016151377544 * gs.sbox[grp.snap].w);
  const float4 me = xm[s];
  const float3 xi = make_float3(me.x, me.y, me.z);  // FP32 position (box tests)
  const int cid = perm[s];
  float4 *tile = tiles[w];
  float4 *tlo64 = tlos[w];
  // mixed precision: the group's FP64 centre (the middle of its targets'
  // box, wave-uniform), this target's two-float offset from it and the
  // group's largest offset component; the target's FP64 position is read
  // again by the rare FP64 decisions rather than held in registers
  double4 c64 = make_double4(0, 0, 0, 0);
  float3 xo = make_float3(0.f, 0.f, 0.f), xl = xo;
  float ext = 0.0f;
  if constexpr (kF64) {
    const double4 p64 = x64[s];
    c64 = group_centre(x64[gs.targets ? gs.targets[grp.t0] : grp.t0], p64, valid);
    two_float_offset(p64, c64, xo, xl);
    ext = valid ? fmaxf(fabsf(xo.x), fmaxf(fabsf(xo.y), fabsf(xo.z))) : 0.0f;
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) ext = fmaxf(ext, __shfl_xor(ext, m));
  }

  HT hcur = valid ? h[cid] : HT(1);
  if (solve) {
    if (valid && !(hcur > HT(0))) {
      const float rho_g = node_density_guess(nodes, grp.root, s, 0.25f * n_ngb);
      // started 10 % above the node estimate: on clustered inputs the
      // iteration then does less walk work in total (measured: 8 % less
      // time for about the same number of passes), on uniform ones the
      // same within 1 %
      const float guess = 1.1f * cbrtf(3.0f * n_ngb * me.w / (4.0f * 3.14159265f * rho_g));
      hcur = (HT)fminf(guess, hcap);
    }
  }
  HT lo = HT(0), hi = HT(INFINITY);
  // the previous evaluation of the solve: its h, f and f' (have_prev: set)
  HT h_prev = HT(0);
  float f_prev = 0.0f, g_prev = 0.0f;
  bool have_prev = false;
  bool done = !valid;
  // results of the accepted evaluation
  HT res_h = hcur;
  float res_sw = 0.0f, res_swh = 0.0f;
  int res_n = 0;
  bool failed = false;
  int passes = 0;

  for (int iter = 0;; ++iter) {
    const bool live = !done;
    const float hf = (float)hcur;
    // squared radius of the FP32 test: fl32(h^2) (of the FP64 h when mixed)
    const float h2 = !live ? -1.0f : (kF64 ? (float)((double)hcur * (double)hcur) : sq_exact(hf));
    // walk pruning radius: exact for FP32 positions, padded by the rounding
    // of FP32 absolute coordinates when the positions are FP64
    const float hw2 = !live ? -1.0f : (kF64 ? sq_exact(walk_radius64(hf, slack)) : h2);

    const float hinv = 1.0f / hf;
    // sums of m w, m wh and m wss: plain per tile, compensated across tiles
    float sw = 0.0f, swh = 0.0f, sss = 0.0f, csw = 0.0f, cswh = 0.0f, csss = 0.0f;
    int cnt = 0;
    int tc = 0, cand = 0;
    // the box of this pass's live targets and their largest squared radius:
    // a candidate whose box_dist2 to that box is not below it fails every
    // lane's neighbour test (box_dist2 never exceeds the r2 of a point in
    // the box), so it is dropped before the tile is scanned
    float4 tlo = make_float4(live ? xi.x : INFINITY, live ? xi.y : INFINITY,
                             live ? xi.z : INFINITY, 0.f);
    float4 thi = make_float4(live ? xi.x : -INFINITY, live ? xi.y : -INFINITY,
                             live ? xi.z : -INFINITY, 0.f);
    // (with FP64 positions: the FP32 copies and the walk's padded radius)
    float hmax2 = kF64 ? hw2 : h2;
    if constexpr (kQ == 1) {
#pragma unroll
      for (int m = 1; m < kWave; m <<= 1) {
        tlo.x = fminf(tlo.x, __shfl_xor(tlo.x, m));
        tlo.y = fminf(tlo.y, __shfl_xor(tlo.y, m));
        tlo.z = fminf(tlo.z, __shfl_xor(tlo.z, m));
        thi.x = fmaxf(thi.x, __shfl_xor(thi.x, m));
        thi.y = fmaxf(thi.y, __shfl_xor(thi.y, m));
        thi.z = fmaxf(thi.z, __shfl_xor(thi.z, m));
        hmax2 = fmaxf(hmax2, __shfl_xor(hmax2, m));
      }
      // wave-uniform now: held in scalar registers through the walk
      auto su = [](float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); };
      tlo = make_float4(su(tlo.x), su(tlo.y), su(tlo.z), 0.f);
      thi = make_float4(su(thi.x), su(thi.y), su(thi.z), 0.f);
      hmax2 = su(hmax2);
    }
    // mixed precision: the low parts are taken within 2^-19 (h^2 + E h) of
    // the threshold and the FP64 test decides within 2^-19 (h^2 + 2^-20 E h),
    // E bounding every offset component of this pass's targets and
    // candidates (the candidates lie within the walk's radius of a target)
    const float eh = kF64 ? (ext + sqrtf(fmaxf(hmax2, 0.0f))) * hf : 0.0f;
    const float band = kBandOff * (h2 + eh);
    const float band2 = kBandOff * (h2 + ldexpf(eh, -20));
    bool fine = false;  // mixed: this pass skips the low parts
    if constexpr (kF64) {
      float hmin = live ? hf : INFINITY;
#pragma unroll
      for (int m = 1; m < kWave; m <<= 1) hmin = fminf(hmin, __shfl_xor(hmin, m));
      fine = ext <= kFineExt * hmin;
    }
    auto flush = [&](int nc) {
      // unused slots sit at infinity and fail every neighbour test
      if constexpr (kF64) {
        float4 o = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
        float4 v = o, l = make_float4(0.f, 0.f, 0.f, 0.f);
        if (lane < nc) {
          const double4 v64 = x64[cand];
          v = xm[cand];
          o = make_float4((float)(v64.x - c64.x), (float)(v64.y - c64.y), (float)(v64.z - c64.z),
                          v.w);
          l = make_float4((float)((v64.x - c64.x) - (double)o.x),
                          (float)((v64.y - c64.y) - (double)o.y),
                          (float)((v64.z - c64.z) - (double)o.z), __int_as_float(cand));
        }
        const bool keep = lane < nc && box_dist2(make_float3(v.x, v.y, v.z), tlo, thi) < hmax2;
        const uint64_t km = __ballot(keep);
        const int slot = (int)__builtin_amdgcn_mbcnt_hi(
            (uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
        tile[lane] = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
        if (keep) {
          tile[slot] = o;
          tlo64[slot] = l;
        }
        nc = __popcll(km);
      } else if constexpr (kQ == 1) {
        const float4 v = (lane < nc) ? xm[cand] : make_float4(INFINITY, INFINITY, INFINITY, 0.f);
        const bool keep = lane < nc && box_dist2(make_float3(v.x, v.y, v.z), tlo, thi) < hmax2;
        const uint64_t km = __ballot(keep);
        const int slot = (int)__builtin_amdgcn_mbcnt_hi(
            (uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
        // kept candidates in their order at the front, infinity behind
        // (the two stores of one wave reach LDS in program order)
        tile[lane] = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
        if (keep) tile[slot] = v;
        nc = __popcll(km);
      } else {
        tile[lane] = (lane < nc) ? xm[cand] : make_float4(INFINITY, INFINITY, INFINITY, 0.f);
      }
      wave_sync();
      // every lane tests every entry (read by broadcast); the kernel sum runs
      // under the lanes that pass, and is skipped when none does. (Marking
      // each lane's entries first and then visiting only its own measured
      // slower: it costs occupancy and per-lane LDS addressing.)
      float pw = 0.0f, pwh = 0.0f, pss = 0.0f;
      auto pair = [&](float r2, float mj) {
        const float u = __builtin_amdgcn_sqrtf(r2) * hinv;
        float wv, whv, wsv;
        wc6_w_wh(u, wv, whv, wsv);
        pw += mj * wv;
        pwh += mj * whv;
        pss += mj * wsv;
        ++cnt;
      };
      if (kF64 && !fine) {
        for (int k = 0; k < nc; ++k) {
          // the FP32 difference of the high parts, then near the threshold
          // or inside the low parts too; close to it the FP64 positions decide
          const float4 q = tile[k];
          float dx = sub_exact(q.x, xo.x), dy = sub_exact(q.y, xo.y), dz = sub_exact(q.z, xo.z);
          if (dist2_exact(dx, dy, dz) < h2 + band) {
            const float4 l = tlo64[k];
            dx += sub_exact(l.x, xl.x);
            dy += sub_exact(l.y, xl.y);
            dz += sub_exact(l.z, xl.z);
            const float r2 = dist2_exact(dx, dy, dz);
            const bool in = fabsf(r2 - h2) <= band2
                                ? within64(x64[s], x64[__float_as_int(l.w)], (double)hcur)
                                : r2 < h2;
            if (in) pair(r2, q.w);
          }
        }
      } else if constexpr (kF64) {
        for (int k = 0; k < nc; ++k) {
          // a narrow group: the high parts; near the threshold the FP64
          // positions decide
          const float4 q = tile[k];
          const float r2 =
              dist2_exact(sub_exact(q.x, xo.x), sub_exact(q.y, xo.y), sub_exact(q.z, xo.z));
          if (r2 < h2 + band) {
            const bool in = r2 < h2 - band ||
                            within64(x64[s], x64[__float_as_int(tlo64[k].w)], (double)hcur);
            if (in) pair(r2, q.w);
          }
        }
      } else {
        // entries are read four at a time, one group ahead of their tests,
        // so the LDS latency overlaps the previous group's arithmetic (the
        // slots past nc hold infinity and fail every test)
        const int ngr = (nc + 3) >> 2;
        float4 a0 = tile[0], a1 = tile[1], a2 = tile[2], a3 = tile[3];
        for (int gq = 0; gq < ngr; ++gq) {
          const float4 q0 = a0, q1 = a1, q2 = a2, q3 = a3;
          const int nx = min(4 * gq + 4, kTile - 4);
          a0 = tile[nx];
          a1 = tile[nx + 1];
          a2 = tile[nx + 2];
          a3 = tile[nx + 3];
          const float4 qs[4] = {q0, q1, q2, q3};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float4 q = qs[e];
            const float r2 =
                dist2_exact(sub_exact(q.x, xi.x), sub_exact(q.y, xi.y), sub_exact(q.z, xi.z));
            if (r2 < h2) pair(r2, q.w);
          }
        }
      }
      neumaier_add(sw, csw, pw);
      neumaier_add(swh, cswh, pwh);
      neumaier_add(sss, csss, pss);
      wave_sync();
    };
    // candidate streams: queue positions (wave-uniform, monotone) and one
    // round of evaluation over up to 64 queued candidates of every quarter
    constexpr int kQl = kWave / kQ;
    constexpr uint64_t kQmask = kQ > 1 ? ((1ull << kQl) - 1ull) : ~0ull;
    int qhead[kQ], qtail[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) qhead[q] = qtail[q] = 0;
    auto qround = [&]() {
      if constexpr (kQ > 1) {
        wave_sync();  // the queued indices are visible
        int mx = 0;
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          const int nq = min(kTile, qtail[q] - qhead[q]);
          mx = max(mx, nq);
          float4 v = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
          if (lane < nq) v = xm[ring[w][q][(qhead[q] + lane) & (kRing - 1)]];
          qtile[w][q][lane] = v;
          qhead[q] += nq;
        }
        wave_sync();
        const float4 *tq = qtile[w][lane / kQl];
        float pw = 0.0f, pwh = 0.0f, pss = 0.0f;
        const int ngr = (mx + 3) >> 2;
        float4 a0 = tq[0], a1 = tq[1], a2 = tq[2], a3 = tq[3];
        for (int gq = 0; gq < ngr; ++gq) {
          const float4 q0 = a0, q1 = a1, q2 = a2, q3 = a3;
          const int nx = min(4 * gq + 4, kTile - 4);
          a0 = tq[nx];
          a1 = tq[nx + 1];
          a2 = tq[nx + 2];
          a3 = tq[nx + 3];
          const float4 qs[4] = {q0, q1, q2, q3};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float4 qq = qs[e];
            const float r2 = dist2_exact(sub_exact(qq.x, xi.x), sub_exact(qq.y, xi.y),
                                         sub_exact(qq.z, xi.z));
            if (r2 < h2) {
              const float u = __builtin_amdgcn_sqrtf(r2) * hinv;
              float wv, whv, wsv;
              wc6_w_wh(u, wv, whv, wsv);
              pw += qq.w * wv;
              pwh += qq.w * whv;
              pss += qq.w * wsv;
              ++cnt;
            }
          }
        }
        neumaier_add(sw, csw, pw);
        neumaier_add(swh, cswh, pwh);
        neumaier_add(sss, csss, pss);
        wave_sync();
      }
    };
    // The next node is either cur + 1 (descend) or the skip target: both
    // are loaded while the current one is tested, so the walk waits for one
    // load latency per step instead of a load after every decision.
    const int last = grp.end - 1;
    int cur = grp.root;
    Node nd = nodes[cur];
    while (cur < grp.end) {
      const int next_a = cur + 1, next_b = nd.meta.x;
      const Node nda = nodes[min(next_a, last)];
      const Node ndb = nodes[min(next_b, last)];
      const bool want = box_dist2(xi, nd.lo_h, nd.hi_l) < hw2;
      bool descend = false;
      const uint64_t wm = __ballot(want);
      if (wm != 0ull) {
        // a small subtree is taken whole: its members are one contiguous run
        if (!(nd.meta.w & kLeafBit) && nd.meta.z > walk_leaf) {
          descend = true;
        } else if constexpr (kQ > 1) {
          const int st = nd.meta.y, c = nd.meta.z;
#pragma unroll
          for (int q = 0; q < kQ; ++q) {
            if (((wm >> (q * kQl)) & kQmask) == 0ull) continue;
            // appended a tile at a time: a leaf of coincident particles can
            // hold more than the ring, and a round frees up to a tile
            for (int off = 0; off < c; off += kTile) {
              const int take = min(kTile, c - off);
              while (qtail[q] - qhead[q] + take > kRing) qround();
              if (lane < take) ring[w][q][(qtail[q] + lane) & (kRing - 1)] = st + off + lane;
              qtail[q] += take;
            }
          }
          // a round once every quarter has a full tile waiting
          for (;;) {
            bool full = true;
#pragma unroll
            for (int q = 0; q < kQ; ++q) full = full && qtail[q] - qhead[q] >= kTile;
            if (!full) break;
            qround();
          }
        } else {
          int st = nd.meta.y, c = nd.meta.z;
          while (c > 0) {
            const int take = min(c, kTile - tc);
            if (lane >= tc && lane < tc + take) cand = st + lane - tc;
            tc += take;
            st += take;
            c -= take;
            if (tc == kTile) {
              flush(kTile);
              tc = 0;
            }
          }
        }
      }
      cur = descend ? next_a : next_b;
      nd = descend ? nda : ndb;
    }
    if constexpr (kQ > 1) {
      for (;;) {  // drain
        bool any = false;
#pragma unroll
        for (int q = 0; q < kQ; ++q) any = any || qtail[q] > qhead[q];
        if (!any) break;
        qround();
      }
    } else if (tc > 0) {
      flush(tc);
    }
    sw += csw;
    swh += cswh;
    sss += csss;

    if (live) {
      if (!solve) {
        done = true;
        res_h = hcur; res_sw = sw; res_swh = swh; res_n = cnt;
      } else {
        // N_eff(h) = (4 pi/3) h^3 rho / m_i = (1365/48) sum_j (m_j / m_i) w(q_j).
        // With A = sum m w as a function of s = ln h: A' = sum m (-q w') =
        // 3 A + sum m wh and A'' = sum m wss, so ln N_eff has the slope
        // f' = 3 + sum m wh / A and the curvature f'' = sum m wss / A - f'^2.
        const float N = kNeffSelf * sw / me.w;
        const bool below = N < n_ngb;
        if (below) lo = lo > hcur ? lo : hcur;
        else hi = hi < hcur ? hi : hcur;
        const float slope = 3.0f + swh / sw;
        // Halley step on f(s) = ln(N_eff / N_ngb) (cubic convergence: about
        // one walk pass fewer than Newton from the node-density first
        // guess), in FP32; the log of the ratio (not a difference of logs;
        // log1p of the relative difference with FP64 h) keeps the step
        // accurate to a few 1e-8 near the root, well inside the convergence
        // test below. Far from the root, where the curvature factor leaves
        // [1/2, 2], it is a Newton step.
        HT hn, hstep;  // the Halley (or Newton) step, which decides convergence; the next h
        if (N == n_ngb) {
          hn = hstep = hcur;
          have_prev = false;
        } else if (slope > 0.05f) {
          const float f = kF64 ? log1pf((N - n_ngb) / n_ngb) : logf(N / n_ngb);
          const float curv = sss / sw - slope * slope;
          const float den = 1.0f - f * (curv / (2.0f * slope * slope));
          const bool halley = den > 0.5f && den < 2.0f;
          float d = -f / slope;
          if (halley) d /= den;
          // With the previous evaluation at distance D = ln(h_prev / h), the
          // quartic in t = ln h - ln h_now that matches f, f', f'' here and
          // f, f' there has a root that is more accurate than Halley's step by
          // about the factor D^2 / 20 (Hermite interpolation error): from a
          // far first guess it saves the solve's last walk. Newton on the
          // quartic from Halley's step; kept only if it stays close to it.
          float dq = d;
          if (halley && have_prev) {
            const float D = logf((float)(h_prev / hcur));
            if (fabsf(D) > 1e-4f && fabsf(D) < 1.5f) {
              const float R0 = f_prev - f - D * (slope + 0.5f * curv * D);
              const float R1 = g_prev - slope - curv * D;
              const float D2 = D * D, D3 = D2 * D;
              const float b4 = (R1 - 3.0f * R0 / D) / D3;
              const float a3 = (R0 - b4 * D3 * D) / D3;
              float t = d;
#pragma unroll
              for (int it = 0; it < 3; ++it) {
                const float pv = f + t * (slope + t * (0.5f * curv + t * (a3 + t * b4)));
                const float dp = slope + t * (curv + t * (3.0f * a3 + 4.0f * b4 * t));
                t -= pv / dp;
              }
              if (isfinite(t) && fabsf(t - d) <= 0.5f * fabsf(d)) dq = t;
            }
          }
          h_prev = hcur;
          f_prev = f;
          g_prev = slope;
          have_prev = true;
          if constexpr (kF64) {
            // FP64 h: steps in FP32 transcendentals, accurate to about 1e-7
            // of themselves (N is an FP32 sum; N - N_ngb is exact near the
            // root), applied in FP64 as h + h expm1(d); FP64 log and exp here
            // would set the kernel's register count
            hstep = hcur + hcur * (HT)expm1f(d);
            hn = hcur + hcur * (HT)expm1f(dq);
          } else {
            hstep = hcur * expf(d);
            hn = hcur * expf(dq);
          }
        } else {
          hn = hstep = below ? HT(2) * hcur : HT(0.5) * hcur;
          have_prev = false;
        }
        // converged when the Newton correction itself is below half the
        // tolerance (h then lies within it of the root), or the bracket has
        // closed; tested before any safeguard replaces the step
        const bool conv = fabs(hstep - hcur) <= HT(0.5) * (HT)tol * hcur ||
                          (hi < HT(INFINITY) && hi - lo <= (HT)tol * hi);
        hn = hn < HT(0.25) * hcur ? HT(0.25) * hcur : (hn > HT(4) * hcur ? HT(4) * hcur : hn);
        if (!(hn > lo && hn < hi)) {
          if (hi < HT(INFINITY) && lo > HT(0)) hn = HT(0.5) * (lo + hi);
          else if (hi < HT(INFINITY)) hn = HT(0.5) * hi;
          else hn = HT(2) * lo;
        }
        const bool capped = below && hcur >= (HT)hcap;
        if (conv || capped || iter + 1 >= max_iter) {
          done = true;
          failed = !conv;
          res_h = hcur; res_sw = sw; res_swh = swh; res_n = cnt;
        } else {
          hcur = hn < (HT)hcap ? hn : (HT)hcap;
        }
      }
    }
    if (__ballot(!done) == 0ull) {
      passes = iter + 1;
      break;
    }
  }
  // counters: [0] non-converged particles, [1] walk passes, [2] waves
  if (lane == 0) {
    atomicAdd(&counters[1], (unsigned long long)passes);
    atomicAdd(&counters[2], 1ull);
  }

  if (valid) {
    const float hinv = 1.0f / (float)res_h;
    const float r = kC * res_sw * hinv * hinv * hinv;
    if (solve) h[cid] = res_h;
    if (rho) rho[cid] = r;
    if (drho_dh) drho_dh[cid] = kC * res_swh * hinv * hinv * hinv * hinv;
    if (omega) omega[cid] = 1.0f + res_swh / (3.0f * res_sw);
    if (nngb) nngb[cid] = res_n;
    if (failed) atomicAdd(&counters[0], 1ull);
  }
  }  // groups
}

template <typename HT>
__global__ void k_hydro_prep(const int32_t *__restrict__ perm, int64_t m,
                             const float *__restrict__ vel, const float *__restrict__ u,
                             const HT *__restrict__ h, const float *__restrict__ rho,
                             const float *__restrict__ omega, float gamma,
                             float4 *__restrict__ vh, float4 *__restrict__ aux,
                             double *__restrict__ h64) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= m) return;
  const int j = perm[s];
  const float hj = (float)h[j];
  if (h64) h64[s] = (double)h[j];
  vh[s] = make_float4(vel ? vel[3 * j] : 0.f, vel ? vel[3 * j + 1] : 0.f,
                      vel ? vel[3 * j + 2] : 0.f, hj);
  if (aux) {
    const float uj = u[j], rj = rho[j];
    // A = P / (Omega rho^2) with P = (gamma - 1) rho u
    const float A = (gamma - 1.0f) * uj / (omega[j] * rj);
    aux[s] = make_float4(A, sqrtf(gamma * (gamma - 1.0f) * uj), rj, 1.0f / hj);
  }
}

// The improved-SPH switches' sorted inputs: ext[s] = (alpha, Balsara
// factor, u, rho) (alpha, balsara nullable: alpha0 and 1).
__global__ void k_hydro_ext_prep(const int32_t *__restrict__ perm, int64_t m,
                                 const float *__restrict__ u, const float *__restrict__ rho,
                                 const float *__restrict__ alpha,
                                 const float *__restrict__ balsara, float alpha0,
                                 float4 *__restrict__ ext) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= m) return;
  const int j = perm[s];
  ext[s] = make_float4(alpha ? alpha[j] : alpha0, balsara ? balsara[j] : 1.0f, u[j], rho[j]);
}

// rho_i u_i - rho_j u_j to a few ulp of itself: the second product split
// into its FP32 rounding and the exact error of that rounding (an FMA), so
// that nearly equal pressures do not cancel to the rounding of each.
__device__ __forceinline__ float rho_u_difference(float ri, float ui, float rj, float uj) {
  const float pj = rj * uj;
  const float ej = __builtin_fmaf(rj, uj, -pj);
  return __builtin_fmaf(ri, ui, -pj) - ej;
}

struct HydroTile {
  float4 xm[kWpb][kTile];
  float4 vh[kWpb][kTile];
  float4 aux[kWpb][kTile];
};

// The extra tile of the switches' inputs (a one-entry stand-in without them).
template <bool kExt>
struct ExtTile {
  float4 e[kWpb][kExt ? kTile : 1];
};

// kExt: the improved-SPH switches (per-particle viscosity strengths and
// Balsara factors, artificial conduction of strength alpha_u) from ext.
template <bool kF64, bool kExt>
__global__ __launch_bounds__(kBlock) void k_hydro(
    const Node *__restrict__ nodes, const float4 *__restrict__ xm,
    const double4 *__restrict__ x64, const double *__restrict__ h64,
    const float4 *__restrict__ vh, const float4 *__restrict__ aux,
    const float4 *__restrict__ ext, const int32_t *__restrict__ perm, const Groups gs,
    float alpha, float alpha_u, float gm1, int walk_leaf, const unsigned *__restrict__ absmax,
    float *__restrict__ acc,
    float *__restrict__ dudt, float *__restrict__ vsig, int32_t *__restrict__ npairs) {
  __shared__ HydroTile T;
  __shared__ ExtTile<kExt> E;
  // mixed precision: the low parts of the offsets, and the sorted index of
  // each entry as the fourth component
  __shared__ float4 tlos[kWpb][kF64 ? kTile : 1];
  const int w = (int)(threadIdx.x >> 6), lane = lane_id();
  // FP64 positions: the walk's pad for the rounding of the FP32 copies
  const float slack = kF64 ? ldexpf(__uint_as_float(*absmax), -20) : 0.0f;
  int range = 0;
  for (int g; (g = next_group(gs, range)) >= 0;) {
  const Group grp = group_at(gs, g);
  const int64_t t = grp.t0 + lane;
  const bool valid = lane < grp.count;
  const int s = valid ? (gs.targets ? gs.targets[t] : (int)t) : 0;
  const float4 me = xm[s], mv = vh[s], ma = aux[s];
  const float4 mx = kExt ? ext[s] : make_float4(0.f, 0.f, 0.f, 0.f);
  const float3 xi = make_float3(me.x, me.y, me.z);  // FP32 position (box tests)
  const double hi64 = kF64 ? h64[s] : 0.0;
  // mixed precision: two-float offsets from the group's FP64 centre, as in
  // the density; gext is the group's largest target offset component
  double4 c64 = make_double4(0, 0, 0, 0);
  float3 xo = make_float3(0.f, 0.f, 0.f), xl = xo;
  float gext = 0.0f, ext2 = 0.0f;
  if constexpr (kF64) {
    const double4 p64 = x64[s];
    c64 = group_centre(x64[gs.targets ? gs.targets[grp.t0] : grp.t0], p64, valid);
    two_float_offset(p64, c64, xo, xl);
    gext = valid ? fmaxf(fabsf(xo.x), fmaxf(fabsf(xo.y), fabsf(xo.z))) : 0.0f;
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) gext = fmaxf(gext, __shfl_xor(gext, m));
    ext2 = gext * gext;
  }
  bool fine = false;  // mixed: the group skips the low parts
  if constexpr (kF64) {
    float hmin = valid ? (float)hi64 : INFINITY;
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) hmin = fminf(hmin, __shfl_xor(hmin, m));
    fine = gext <= kFineExt * hmin;
  }
  const float hi = valid ? mv.w : -1.0f;  // invalid lanes never want anything
  const float hi2 = valid ? sq_exact(hi) : -1.0f;
  const float Ai = ma.x, ci = ma.y, rhoi = ma.z, hinvi = ma.w;
  const float ki = kWendlandF * (hinvi * hinvi) * (hinvi * hinvi) * hinvi;
  // totals with Neumaier compensation terms; per-tile partials are plain
  float ax = 0.f, ay = 0.f, az = 0.f, du = 0.f, vs = 0.f;
  float cax = 0.f, cay = 0.f, caz = 0.f, cdu = 0.f;
  int np = 0, tc = 0, cand = 0;
  // the box of the group's targets and their largest squared radius: a
  // candidate j whose box_dist2 to that box reaches both it and fl(h_j^2)
  // fails every lane's symmetric test (box_dist2 never exceeds the r2 of a
  // point in the box), so it is dropped before the tile is scanned
  float4 tlo = make_float4(valid ? xi.x : INFINITY, valid ? xi.y : INFINITY,
                           valid ? xi.z : INFINITY, 0.f);
  float4 thi = make_float4(valid ? xi.x : -INFINITY, valid ? xi.y : -INFINITY,
                           valid ? xi.z : -INFINITY, 0.f);
  // (with FP64 positions: the FP32 copies and radii padded as in the walk)
  float hmax2 = kF64 ? (valid ? sq_exact(walk_radius64(hi, slack)) : -1.0f) : hi2;
  {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) {
      tlo.x = fminf(tlo.x, __shfl_xor(tlo.x, m));
      tlo.y = fminf(tlo.y, __shfl_xor(tlo.y, m));
      tlo.z = fminf(tlo.z, __shfl_xor(tlo.z, m));
      thi.x = fmaxf(thi.x, __shfl_xor(thi.x, m));
      thi.y = fmaxf(thi.y, __shfl_xor(thi.y, m));
      thi.z = fmaxf(thi.z, __shfl_xor(thi.z, m));
      hmax2 = fmaxf(hmax2, __shfl_xor(hmax2, m));
    }
    // wave-uniform now: held in scalar registers through the walk
    auto su = [](float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); };
    tlo = make_float4(su(tlo.x), su(tlo.y), su(tlo.z), 0.f);
    thi = make_float4(su(thi.x), su(thi.y), su(thi.z), 0.f);
    hmax2 = su(hmax2);
  }

  auto flush = [&](int nc) {
    {
      float4 vx = make_float4(INFINITY, INFINITY, INFINITY, 0.f), vv = make_float4(0.f, 0.f, 0.f, 0.f);
      float4 va = vv, ve = vv;
      float4 vo = vx;  // the tile's position: the FP32 copy, or the offset (mixed)
      float4 vl = vv;  // mixed: the offset's low parts and the sorted index
      if (lane < nc) {
        vx = xm[cand];
        vv = vh[cand];
        va = aux[cand];
        if constexpr (kExt) ve = ext[cand];
        vo = vx;
        if constexpr (kF64) {
          const double4 v64 = x64[cand];
          vo = make_float4((float)(v64.x - c64.x), (float)(v64.y - c64.y),
                           (float)(v64.z - c64.z), vx.w);
          vl = make_float4((float)((v64.x - c64.x) - (double)vo.x),
                           (float)((v64.y - c64.y) - (double)vo.y),
                           (float)((v64.z - c64.z) - (double)vo.z), __int_as_float(cand));
        }
      }
      const float d2 = box_dist2(make_float3(vx.x, vx.y, vx.z), tlo, thi);
      const bool keep =
          lane < nc && (d2 < hmax2 || d2 < sq_exact(kF64 ? walk_radius64(vv.w, slack) : vv.w));
      const uint64_t km = __ballot(keep);
      const int slot = (int)__builtin_amdgcn_mbcnt_hi(
          (uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
      // kept candidates in their order at the front; the scan stops at nc
      if (keep) {
        T.xm[w][slot] = vo;
        T.vh[w][slot] = vv;
        T.aux[w][slot] = va;
        if constexpr (kExt) E.e[w][slot] = ve;
        if constexpr (kF64) tlos[w][slot] = vl;
      }
      nc = __popcll(km);
    }
    wave_sync();
    float px = 0.f, py = 0.f, pz = 0.f, pu = 0.f;
    // one pair (i, entry k) that passed the symmetric neighbour test; the
    // self pair (r = 0) passes too: it is counted and subtracted at the end,
    // and any pair at r = 0 adds nothing to the sums
    auto pair = [&](int k, const float4 &q, const float4 &qv, float dx, float dy, float dz,
                    float r2) {
      {
        const float4 qa = T.aux[w][k];
        if (r2 > 0.0f) {
          const float rinv = __builtin_amdgcn_rsqf(r2);
          const float r = r2 * rinv;
          const float hj5 = (qa.w * qa.w) * (qa.w * qa.w) * qa.w;
          const float gi = ki * wendland_f(r * hinvi);
          const float gj = kWendlandF * hj5 * wendland_f(r * qa.w);
          // x_ij = x_i - x_j = -(dx, dy, dz); v_ij = v_i - v_j
          const float vdx = (mv.x - qv.x) * dx + (mv.y - qv.y) * dy + (mv.z - qv.z) * dz;
          const float vx = -vdx;  // v_ij . x_ij
          const float wv = vx * rinv;
          const float wneg = fminf(wv, 0.0f);
          const float vsig_ij = ci + qa.y - 3.0f * wneg;
          vs = fmaxf(vs, vsig_ij);
          // the hardware reciprocal (1 ulp) in place of an IEEE division
          const float rsum_inv = __builtin_amdgcn_rcpf(rhoi + qa.z);
          float a_ij = alpha;
          if constexpr (kExt) {
            // (alpha_i + alpha_j)/2 times the mean Balsara factor
            const float4 qe = E.e[w][k];
            a_ij = 0.25f * (mx.x + qe.x) * (mx.y + qe.y);
          }
          const float Pi = a_ij * vsig_ij * (-wneg) * rsum_inv;
          const float gbar = 0.5f * (gi + gj);
          const float mj = q.w;
          const float coef = mj * (Ai * gi + qa.x * gj + Pi * gbar);  // a_i -= coef x_ij
          px += coef * dx;
          py += coef * dy;
          pz += coef * dz;
          pu += mj * (Ai * gi + 0.5f * Pi * gbar) * vx;
          if constexpr (kExt) {
            // artificial conduction: m_j alpha_u v_u (u_i - u_j) gbar r / rhobar,
            // v_u = sqrt(|P_i - P_j| / rhobar), rhobar = (rho_i + rho_j)/2
            const float4 qe = E.e[w][k];
            const float two_inv = 2.0f * rsum_inv;  // 1 / rhobar
            const float dP = gm1 * rho_u_difference(mx.w, mx.z, qe.w, qe.z);
            const float vu = __builtin_amdgcn_sqrtf(fabsf(dP) * two_inv);
            pu += mj * alpha_u * vu * (mx.z - qe.z) * gbar * r * two_inv;
          }
        }
      }
    };
    // every lane tests every entry (read by broadcast)
    auto scan = [&](auto refine_c) {
      constexpr bool kRefine = decltype(refine_c)::value;
      for (int k = 0; k < nc; ++k) {
        const float4 q = T.xm[w][k];
        const float4 qv = T.vh[w][k];
        // plain: the FP32 positions; mixed: the FP32 difference of the two
        // offsets from the group centre
        float dx = sub_exact(q.x, kF64 ? xo.x : xi.x);
        float dy = sub_exact(q.y, kF64 ? xo.y : xi.y);
        float dz = sub_exact(q.z, kF64 ? xo.z : xi.z);
        float r2 = dist2_exact(dx, dy, dz);
        // r2 < fl(max(h_i, h_j)^2) taken as r2 < fl(h_i^2) or r2 < fl(h_j^2)
        // (the same decision: rounding is monotone), without a max
        const float hj2 = sq_exact(qv.w);
        bool in = r2 < hi2 || r2 < hj2;
        if constexpr (kF64) {
          // the density's bands with E bounded by gext + H near the
          // threshold, E H <= 3 H^2 + gext^2: a narrow group decides on the
          // high parts outside 2^-19 (3 H^2 + gext^2) of it; a wide one
          // adds the low parts to every entry and decides on them outside
          // 2^-19 (H^2 + 2^-20 (3 H^2 + gext^2)); inside the band the FP64
          // test decides (rare: a wave-uniform branch)
          const float H2 = fmaxf(hi2, hj2);
          const float eb = 3.0f * H2 + ext2;
          float bd = kBandOff * eb;
          if constexpr (kRefine) {
            const float4 l = tlos[w][k];
            dx += sub_exact(l.x, xl.x);
            dy += sub_exact(l.y, xl.y);
            dz += sub_exact(l.z, xl.z);
            r2 = dist2_exact(dx, dy, dz);
            bd = kBandOff * (H2 + ldexpf(eb, -20));
          }
          in = r2 < H2;
          const bool near = valid && fabsf(r2 - H2) <= bd;
          if (__ballot(near) != 0ull && near) {
            const int j = __float_as_int(tlos[w][k].w);
            in = within64(x64[s], x64[j], fmax(hi64, h64[j]));
          }
        }
        if (in) {
          ++np;
          pair(k, q, qv, dx, dy, dz, r2);
        }
      }
    };
    if (kF64 && !fine)
      scan(std::true_type{});
    else
      scan(std::false_type{});
    neumaier_add(ax, cax, px);
    neumaier_add(ay, cay, py);
    neumaier_add(az, caz, pz);
    neumaier_add(du, cdu, pu);
    wave_sync();
  };

  int cur = grp.root;
  while (cur < grp.end) {
    const Node nd = nodes[cur];
    const float hm = kF64 ? walk_radius64(fmaxf(hi, nd.lo_h.w), slack) : fmaxf(hi, nd.lo_h.w);
    // one compare: a lane without a target (hi = 0) tests against -1, which
    // no squared distance is below
    const float lim = hi > 0.0f ? sq_exact(hm) : -1.0f;
    const bool want = box_dist2(xi, nd.lo_h, nd.hi_l) < lim;
    if (__ballot(want) == 0ull) {
      cur = nd.meta.x;
      continue;
    }
    // a small subtree is taken whole: its members are one contiguous run
    if (!(nd.meta.w & kLeafBit) && nd.meta.z > walk_leaf) {
      ++cur;
      continue;
    }
    int st = nd.meta.y, c = nd.meta.z;
    while (c > 0) {
      const int take = min(c, kTile - tc);
      if (lane >= tc && lane < tc + take) cand = st + lane - tc;
      tc += take;
      st += take;
      c -= take;
      if (tc == kTile) {
        flush(kTile);
        tc = 0;
      }
    }
    cur = nd.meta.x;
  }
  if (tc > 0) flush(tc);
  ax += cax;
  ay += cay;
  az += caz;
  du += cdu;

  if (valid) {
    const int cid = perm[s];
    if (acc) {
      acc[3 * cid] = ax;
      acc[3 * cid + 1] = ay;
      acc[3 * cid + 2] = az;
    }
    if (dudt) dudt[cid] = du;
    if (vsig) vsig[cid] = vs;
    if (npairs) npairs[cid] = np - 1;  // the self pair always passes the test
  }
  }  // groups
}

inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_density(const Octree &gas, const Groups &gs, int64_t max_groups,
                          const SphParams &sp, int solve_h, void *h, float *rho,
                          float *drho_dh, float *omega, int32_t *nngb,
                          unsigned long long *counters, hipStream_t s) {
  if (max_groups <= 0 || gas.nnodes == 0) return hipSuccess;
  auto kern = sp.f64 ? k_density<true, 1>
                     : (sp.streams == 4 ? k_density<false, 4> : k_density<false, 1>);
  kern<<<persistent_grid((const void *)kern, kBlock, max_groups), kBlock, 0, s>>>(
      gas.nodes, gas.xm, gas.x64, gas.perm, gs, sp.n_ngb, sp.h_tol, solve_h, sp.max_iter,
      sp.walk_leaf, sp.absmax, h, rho, drho_dh, omega, nngb, counters);
  return hipGetLastError();
}

hipError_t launch_hydro_prep(Octree &gas, const float *vel, const float *u, const void *h,
                             const float *rho, const float *omega, float gamma, int f64,
                             hipStream_t s) {
  if (gas.n == 0) return hipSuccess;
  if (f64) {
    // the FP64 h copy is sized by the caller (ensure_h64) before any launch
    if (!gas.h64 || gas.cap_h64 < gas.n) return hipErrorInvalidValue;
    k_hydro_prep<double><<<nblk(gas.n, 256), 256, 0, s>>>(
        gas.perm, gas.n, vel, u, (const double *)h, rho, omega, gamma, gas.vh,
        rho ? gas.aux : nullptr, gas.h64);
  } else {
    k_hydro_prep<float><<<nblk(gas.n, 256), 256, 0, s>>>(
        gas.perm, gas.n, vel, u, (const float *)h, rho, omega, gamma, gas.vh,
        rho ? gas.aux : nullptr, nullptr);
  }
  return hipGetLastError();
}

hipError_t launch_hydro(const Octree &gas, const Groups &gs, int64_t max_groups,
                        const SphParams &sp, float *acc, float *dudt, float *vsig,
                        int32_t *npairs, hipStream_t s, const float4 *ext, float alpha_u) {
  if (max_groups <= 0 || gas.nnodes == 0) return hipSuccess;
  auto kern = sp.f64 ? (ext ? k_hydro<true, true> : k_hydro<true, false>)
                     : (ext ? k_hydro<false, true> : k_hydro<false, false>);
  kern<<<persistent_grid((const void *)kern, kBlock, max_groups), kBlock, 0, s>>>(
      gas.nodes, gas.xm, gas.x64, gas.h64, gas.vh, gas.aux, ext, gas.perm, gs, sp.alpha,
      alpha_u, sp.gamma - 1.0f, sp.walk_leaf, sp.absmax, acc, dudt, vsig, npairs);
  return hipGetLastError();
}

hipError_t launch_hydro_ext_prep(Octree &gas, const float *u, const float *rho,
                                 const float *alpha, const float *balsara, float alpha0,
                                 float4 *ext, hipStream_t s) {
  if (gas.n == 0) return hipSuccess;
  k_hydro_ext_prep<<<nblk(gas.n, 256), 256, 0, s>>>(gas.perm, gas.n, u, rho, alpha, balsara,
                                                    alpha0, ext);
  return hipGetLastError();
}

}  // namespace g3
