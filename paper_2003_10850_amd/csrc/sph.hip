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
constexpr float kF = -22.0f * 6.7889530412636603f;

__device__ __forceinline__ void wc6_w_wh(float q, float &w, float &wh) {
  const float t = 1.0f - q;
  const float t2 = t * t, t4 = t2 * t2, t7 = t4 * t2 * t;
  w = t7 * t * (1.0f + q * (8.0f + q * (25.0f + q * 32.0f)));
  wh = t7 * (-3.0f + q * (-21.0f + q * (-29.0f + q * (133.0f + q * 448.0f))));
}

// (1-q)^7 (1 + 7q + 16q^2), zero at and beyond the support
__device__ __forceinline__ float wc6_f(float q) {
  const float t = fmaxf(1.0f - q, 0.0f);
  const float t2 = t * t, t4 = t2 * t2;
  return t4 * t2 * t * (1.0f + q * (7.0f + q * 16.0f));
}

// First guess of h for a group: descend from the root along the group's
// first member while the child still holds >= n_ngb members, then take the
// mean density of that node's bounding box (of its cube if the box is flat).
__device__ float group_density_guess(const Node *__restrict__ nodes, int s0, float n_ngb) {
  int cur = 0;
  for (;;) {
    const int4 meta = nodes[cur].meta;
    if (meta.w & kLeafBit) break;
    int c = cur + 1, found = -1;
    while (c < meta.x) {
      const int4 cm = nodes[c].meta;
      if (s0 >= cm.y && s0 < cm.y + cm.z) {
        found = c;
        break;
      }
      c = cm.x;
    }
    if (found < 0 || (float)nodes[found].meta.z < n_ngb) break;
    cur = found;
  }
  const Node nd = nodes[cur];
  const float l = nd.hi_l.w;
  float V = (nd.hi_l.x - nd.lo_h.x) * (nd.hi_l.y - nd.lo_h.y) * (nd.hi_l.z - nd.lo_h.z);
  if (!(V > 1e-3f * l * l * l)) V = l * l * l;
  return nd.com_m.w / V;  // mass density
}

__global__ __launch_bounds__(kBlock) void k_density(
    const Node *__restrict__ nodes, int nnodes, const float4 *__restrict__ xm,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ targets,
    const uint32_t *__restrict__ dcount, int64_t ntmax, float n_ngb, float tol,
    float hcap, int solve, int max_iter, int walk_leaf, float *__restrict__ h,
    float *__restrict__ rho,
    float *__restrict__ drho_dh, float *__restrict__ omega, int32_t *__restrict__ nngb,
    unsigned long long *__restrict__ counters) {
  __shared__ float4 tiles[kWpb][kTile];
  const int w = (int)(threadIdx.x >> 6), lane = lane_id();
  const int64_t ntarg = targets ? (int64_t)(*dcount) : ntmax;
  const int64_t g0 = (xcd_block() * kWpb + w) * kWave;
  if (g0 >= ntarg) return;
  const int64_t t = g0 + lane;
  const bool valid = t < ntarg;
  const int s = valid ? (targets ? targets[t] : (int)t) : 0;
  const float4 me = xm[s];
  const float3 xi = make_float3(me.x, me.y, me.z);
  const int cid = perm[s];
  float4 *tile = tiles[w];

  float hcur = valid ? h[cid] : 1.0f;
  if (solve) {
    const int s0 = uniform(targets ? targets[g0] : (int)g0);
    if (__ballot(valid && !(hcur > 0.0f))) {
      const float rho_g = group_density_guess(nodes, s0, n_ngb);
      const float guess = cbrtf(3.0f * n_ngb * me.w / (4.0f * 3.14159265f * rho_g));
      if (!(hcur > 0.0f)) hcur = fminf(guess, hcap);
    }
  }
  float lo = 0.0f, hi = INFINITY;
  bool done = !valid;
  // results of the accepted evaluation
  float res_h = hcur, res_sw = 0.0f, res_swh = 0.0f;
  int res_n = 0;
  bool failed = false;
  int passes = 0;

  for (int iter = 0;; ++iter) {
    const bool live = !done;
    const float h2 = live ? sq_exact(hcur) : -1.0f;
    const float hinv = 1.0f / hcur;
    // sums of m w and m wh: plain per tile, compensated across tiles
    float sw = 0.0f, swh = 0.0f, csw = 0.0f, cswh = 0.0f;
    int cnt = 0;
    int tc = 0, cand = 0;
    auto flush = [&](int nc) {
      // unused slots sit at infinity and fail every neighbour test
      tile[lane] = (lane < nc) ? xm[cand] : make_float4(INFINITY, INFINITY, INFINITY, 0.f);
      wave_sync();
      // every lane tests every entry (read by broadcast); the kernel sum runs
      // under the lanes that pass, and is skipped when none does. (Marking
      // each lane's entries first and then visiting only its own measured
      // slower: it costs occupancy and per-lane LDS addressing.)
      float pw = 0.0f, pwh = 0.0f;
      for (int k = 0; k < nc; ++k) {
        const float4 q = tile[k];
        const float r2 = dist2_exact(sub_exact(q.x, xi.x), sub_exact(q.y, xi.y),
                                     sub_exact(q.z, xi.z));
        if (r2 < h2) {
          const float u = __builtin_amdgcn_sqrtf(r2) * hinv;
          float wv, whv;
          wc6_w_wh(u, wv, whv);
          pw += q.w * wv;
          pwh += q.w * whv;
          ++cnt;
        }
      }
      neumaier_add(sw, csw, pw);
      neumaier_add(swh, cswh, pwh);
      wave_sync();
    };
    int cur = 0;
    while (cur < nnodes) {
      const Node nd = nodes[cur];
      const bool want = box_dist2(xi, nd.lo_h, nd.hi_l) < h2;
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
    sw += csw;
    swh += cswh;

    if (live) {
      if (!solve) {
        done = true;
        res_h = hcur; res_sw = sw; res_swh = swh; res_n = cnt;
      } else {
        // N_eff(h) = (4 pi/3) h^3 rho / m_i = (1365/48) sum_j (m_j / m_i) w(q_j);
        // its log-slope is 3 + h rho'/rho = 3 + sum m wh / sum m w.
        const float N = kNeffSelf * sw / me.w;
        const bool below = N < n_ngb;
        if (below) lo = fmaxf(lo, hcur);
        else hi = fminf(hi, hcur);
        const float slope = 3.0f + swh / sw;
        // Newton step on ln N_eff(ln h); the log of the ratio (not a
        // difference of logs) keeps the step accurate to a few 1e-8 near
        // the root, well inside the convergence test below
        float hn;
        if (N == n_ngb) hn = hcur;
        else if (slope > 0.05f) hn = hcur * expf(logf(n_ngb / N) / slope);
        else hn = below ? 2.0f * hcur : 0.5f * hcur;
        // converged when the Newton correction itself is below half the
        // tolerance (h then lies within it of the root), or the bracket has
        // closed; tested before any safeguard replaces the step
        const bool conv = fabsf(hn - hcur) <= 0.5f * tol * hcur ||
                          (hi < INFINITY && hi - lo <= tol * hi);
        hn = fminf(fmaxf(hn, 0.25f * hcur), 4.0f * hcur);
        if (!(hn > lo && hn < hi)) {
          if (hi < INFINITY && lo > 0.0f) hn = 0.5f * (lo + hi);
          else if (hi < INFINITY) hn = 0.5f * hi;
          else hn = 2.0f * lo;
        }
        const bool capped = below && hcur >= hcap;
        if (conv || capped || iter + 1 >= max_iter) {
          done = true;
          failed = !conv;
          res_h = hcur; res_sw = sw; res_swh = swh; res_n = cnt;
        } else {
          hcur = fminf(hn, hcap);
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
    const float hinv = 1.0f / res_h;
    const float r = kC * res_sw * hinv * hinv * hinv;
    if (solve) h[cid] = res_h;
    if (rho) rho[cid] = r;
    if (drho_dh) drho_dh[cid] = kC * res_swh * hinv * hinv * hinv * hinv;
    if (omega) omega[cid] = 1.0f + res_swh / (3.0f * res_sw);
    if (nngb) nngb[cid] = res_n;
    if (failed) atomicAdd(&counters[0], 1ull);
  }
}

__global__ void k_hydro_prep(const int32_t *__restrict__ perm, int64_t m,
                             const float *__restrict__ vel, const float *__restrict__ u,
                             const float *__restrict__ h, const float *__restrict__ rho,
                             const float *__restrict__ omega, float gamma,
                             float4 *__restrict__ vh, float4 *__restrict__ aux) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= m) return;
  const int j = perm[s];
  const float hj = h[j];
  vh[s] = make_float4(vel ? vel[3 * j] : 0.f, vel ? vel[3 * j + 1] : 0.f,
                      vel ? vel[3 * j + 2] : 0.f, hj);
  if (aux) {
    const float uj = u[j], rj = rho[j];
    // A = P / (Omega rho^2) with P = (gamma - 1) rho u
    const float A = (gamma - 1.0f) * uj / (omega[j] * rj);
    aux[s] = make_float4(A, sqrtf(gamma * (gamma - 1.0f) * uj), rj, 1.0f / hj);
  }
}

struct HydroTile {
  float4 xm[kWpb][kTile];
  float4 vh[kWpb][kTile];
  float4 aux[kWpb][kTile];
};

__global__ __launch_bounds__(kBlock) void k_hydro(
    const Node *__restrict__ nodes, int nnodes, const float4 *__restrict__ xm,
    const float4 *__restrict__ vh, const float4 *__restrict__ aux,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ targets,
    const uint32_t *__restrict__ dcount, int64_t ntmax, float alpha, int walk_leaf,
    float *__restrict__ acc, float *__restrict__ dudt, float *__restrict__ vsig,
    int32_t *__restrict__ npairs) {
  __shared__ HydroTile T;
  const int w = (int)(threadIdx.x >> 6), lane = lane_id();
  const int64_t ntarg = targets ? (int64_t)(*dcount) : ntmax;
  const int64_t g0 = (xcd_block() * kWpb + w) * kWave;
  if (g0 >= ntarg) return;
  const int64_t t = g0 + lane;
  const bool valid = t < ntarg;
  const int s = valid ? (targets ? targets[t] : (int)t) : 0;
  const float4 me = xm[s], mv = vh[s], ma = aux[s];
  const float3 xi = make_float3(me.x, me.y, me.z);
  const float hi = valid ? mv.w : -1.0f;  // invalid lanes never want anything
  const float Ai = ma.x, ci = ma.y, rhoi = ma.z, hinvi = ma.w;
  const float ki = kF * (hinvi * hinvi) * (hinvi * hinvi) * hinvi;
  // totals with Neumaier compensation terms; per-tile partials are plain
  float ax = 0.f, ay = 0.f, az = 0.f, du = 0.f, vs = 0.f;
  float cax = 0.f, cay = 0.f, caz = 0.f, cdu = 0.f;
  int np = 0, tc = 0, cand = 0;

  auto flush = [&](int nc) {
    if (lane < nc) {
      T.xm[w][lane] = xm[cand];
      T.vh[w][lane] = vh[cand];
      T.aux[w][lane] = aux[cand];
    } else {  // unused slots sit at infinity and fail every neighbour test
      T.xm[w][lane] = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
      T.vh[w][lane] = make_float4(0.f, 0.f, 0.f, 0.f);
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
          const float gi = ki * wc6_f(r * hinvi);
          const float gj = kF * hj5 * wc6_f(r * qa.w);
          // x_ij = x_i - x_j = -(dx, dy, dz); v_ij = v_i - v_j
          const float vdx = (mv.x - qv.x) * dx + (mv.y - qv.y) * dy + (mv.z - qv.z) * dz;
          const float vx = -vdx;  // v_ij . x_ij
          const float wv = vx * rinv;
          const float wneg = fminf(wv, 0.0f);
          const float vsig_ij = ci + qa.y - 3.0f * wneg;
          vs = fmaxf(vs, vsig_ij);
          const float Pi = alpha * vsig_ij * (-wneg) / (rhoi + qa.z);
          const float gbar = 0.5f * (gi + gj);
          const float mj = q.w;
          const float coef = mj * (Ai * gi + qa.x * gj + Pi * gbar);  // a_i -= coef x_ij
          px += coef * dx;
          py += coef * dy;
          pz += coef * dz;
          pu += mj * (Ai * gi + 0.5f * Pi * gbar) * vx;
        }
      }
    };
    // every lane tests every entry (read by broadcast)
    for (int k = 0; k < nc; ++k) {
      const float4 q = T.xm[w][k];
      const float4 qv = T.vh[w][k];
      const float dx = sub_exact(q.x, xi.x), dy = sub_exact(q.y, xi.y),
                  dz = sub_exact(q.z, xi.z);
      const float r2 = dist2_exact(dx, dy, dz);
      if (r2 < sq_exact(fmaxf(hi, qv.w))) {
        ++np;
        pair(k, q, qv, dx, dy, dz, r2);
      }
    }
    neumaier_add(ax, cax, px);
    neumaier_add(ay, cay, py);
    neumaier_add(az, caz, pz);
    neumaier_add(du, cdu, pu);
    wave_sync();
  };

  int cur = 0;
  while (cur < nnodes) {
    const Node nd = nodes[cur];
    const float hm = fmaxf(hi, nd.lo_h.w);
    const bool want = hi > 0.0f && box_dist2(xi, nd.lo_h, nd.hi_l) < sq_exact(hm);
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
}

inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_density(const Octree &gas, const int32_t *targets, const uint32_t *dcount,
                          int64_t max_targets, const SphParams &sp, int solve_h, float *h,
                          float *rho, float *drho_dh, float *omega, int32_t *nngb,
                          unsigned long long *counters, hipStream_t s, float hcap) {
  if (max_targets <= 0 || gas.nnodes == 0) return hipSuccess;
  k_density<<<nblk(max_targets, kBlock), kBlock, 0, s>>>(
      gas.nodes, (int)gas.nnodes, gas.xm, gas.perm, targets, dcount, max_targets, sp.n_ngb,
      sp.h_tol, hcap, solve_h, sp.max_iter, sp.walk_leaf, h, rho, drho_dh, omega, nngb,
      counters);
  return hipGetLastError();
}

hipError_t launch_hydro_prep(Octree &gas, const float *vel, const float *u, const float *h,
                             const float *rho, const float *omega, float gamma,
                             hipStream_t s) {
  if (gas.n == 0) return hipSuccess;
  k_hydro_prep<<<nblk(gas.n, 256), 256, 0, s>>>(gas.perm, gas.n, vel, u, h, rho, omega,
                                                 gamma, gas.vh, rho ? gas.aux : nullptr);
  return hipGetLastError();
}

hipError_t launch_hydro(const Octree &gas, const int32_t *targets, const uint32_t *dcount,
                        int64_t max_targets, const SphParams &sp, float *acc, float *dudt,
                        float *vsig, int32_t *npairs, hipStream_t s) {
  if (max_targets <= 0 || gas.nnodes == 0) return hipSuccess;
  k_hydro<<<nblk(max_targets, kBlock), kBlock, 0, s>>>(
      gas.nodes, (int)gas.nnodes, gas.xm, gas.vh, gas.aux, gas.perm, targets, dcount,
      max_targets, sp.alpha, sp.walk_leaf, acc, dudt, vsig, npairs);
  return hipGetLastError();
}

}  // namespace g3
