// Thermal conduction: the paper's third ported SPH module (section 1, the
// list of modules moved to the GPU). The paper prints no formula; Gadget's
// conduction (Jubelgas, Springel & Dolag 2004) uses the SPH form of
// rho du/dt = div(kappa grad u) of Brookshaw (1985):
//   du_i/dt = sum_j m_j (kappa_i + kappa_j) (u_i - u_j) Fbar_ij / (rho_i rho_j),
//   Fbar_ij = (F(r, h_i) + F(r, h_j)) / 2,  F = (1/r) dW/dr,
// over gas j with r < max(h_i, h_j): the hydro force's symmetric pairs, so
// the kernel is the hydro force's walk and tiles with a lighter pair.
//
// One wavefront serves a group of up to 64 Morton-consecutive targets; the
// walk opens a node when some lane's radius max(h_i, hmax(node)) reaches
// its box; accepted leaves and small subtrees are staged as 64-entry tiles
// in LDS after the group-box cull and scanned by every lane with the exact
// symmetric test.
#include <cmath>

#include "g3_device.h"
#include "g3_internal.h"

namespace g3 {
namespace {

constexpr int kBlock = 256;
constexpr int kWpb = kBlock / kWave;
constexpr int kTile = kWave;

// Sorted-order inputs of the pair: ch[s] = (h, u, kappa, 1/rho) with
// kappa = kappa0 u^kappa_exp.
template <typename HT>
__global__ void k_cond_prep(const int32_t *__restrict__ perm, int64_t m,
                            const float *__restrict__ u, const HT *__restrict__ h,
                            const float *__restrict__ rho, float kappa0, float kappa_exp,
                            float4 *__restrict__ ch) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= m) return;
  const int j = perm[s];
  const float uj = fmaxf(u[j], 0.0f);
  const float kj = kappa_exp == 0.0f ? kappa0 : kappa0 * powf(uj, kappa_exp);
  ch[s] = make_float4((float)h[j], u[j], kj, 1.0f / rho[j]);
}

struct CondTile {
  float4 xm[kWpb][kTile];
  float4 ch[kWpb][kTile];
};

__global__ __launch_bounds__(kBlock) void k_conduction(
    const Node *__restrict__ nodes, const float4 *__restrict__ xm,
    const float4 *__restrict__ ch, const int32_t *__restrict__ perm, const Groups gs,
    int walk_leaf, float *__restrict__ dudt, int32_t *__restrict__ npairs) {
  __shared__ CondTile T;
  const int w = (int)(threadIdx.x >> 6), lane = lane_id();
  int range = 0;
  for (int g; (g = next_group(gs, range)) >= 0;) {
    const Group grp = group_at(gs, g);
    const int64_t t = grp.t0 + lane;
    const bool valid = lane < grp.count;
    const int s = valid ? (gs.targets ? gs.targets[t] : (int)t) : 0;
    const float4 me = xm[s], mc = ch[s];
    const float3 xi = make_float3(me.x, me.y, me.z);
    const float hi = valid ? mc.x : -1.0f;  // invalid lanes never want anything
    const float hi2 = valid ? sq_exact(hi) : -1.0f;
    const float ui = mc.y, kappai = mc.z, rinvi = mc.w;
    const float hinvi = 1.0f / mc.x;
    const float fi5 = kWendlandF * (hinvi * hinvi) * (hinvi * hinvi) * hinvi;
    float du = 0.f, cdu = 0.f;
    int np = 0, tc = 0, cand = 0;
    // the group's target box and largest squared radius (group-box cull)
    float4 tlo = make_float4(valid ? xi.x : INFINITY, valid ? xi.y : INFINITY,
                             valid ? xi.z : INFINITY, 0.f);
    float4 thi = make_float4(valid ? xi.x : -INFINITY, valid ? xi.y : -INFINITY,
                             valid ? xi.z : -INFINITY, 0.f);
    float hmax2 = hi2;
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
    auto su = [](float v) {
      return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
    };
    tlo = make_float4(su(tlo.x), su(tlo.y), su(tlo.z), 0.f);
    thi = make_float4(su(thi.x), su(thi.y), su(thi.z), 0.f);
    hmax2 = su(hmax2);

    auto flush = [&](int nc) {
      {
        float4 vx = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
        float4 vc = make_float4(0.f, 0.f, 0.f, 0.f);
        if (lane < nc) {
          vx = xm[cand];
          vc = ch[cand];
        }
        // a candidate beyond both the group's largest radius and its own h
        // fails every lane's symmetric test
        const float d2 = box_dist2(make_float3(vx.x, vx.y, vx.z), tlo, thi);
        const bool keep = lane < nc && (d2 < hmax2 || d2 < sq_exact(vc.x));
        const uint64_t km = __ballot(keep);
        const int slot = (int)__builtin_amdgcn_mbcnt_hi(
            (uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
        if (keep) {
          T.xm[w][slot] = vx;
          T.ch[w][slot] = vc;
        }
        nc = __popcll(km);
      }
      wave_sync();
      float pu = 0.f;
      for (int k = 0; k < nc; ++k) {
        const float4 q = T.xm[w][k];
        const float4 qc = T.ch[w][k];
        const float dx = sub_exact(q.x, xi.x), dy = sub_exact(q.y, xi.y),
                    dz = sub_exact(q.z, xi.z);
        const float r2 = dist2_exact(dx, dy, dz);
        // r2 < fl(max(h_i, h_j)^2) as two compares (rounding is monotone)
        if (r2 < hi2 || r2 < sq_exact(qc.x)) {
          ++np;
          if (r2 > 0.0f) {
            const float r = r2 * __builtin_amdgcn_rsqf(r2);
            const float hinvj = __builtin_amdgcn_rcpf(qc.x);
            const float hj5 = (hinvj * hinvj) * (hinvj * hinvj) * hinvj;
            const float fi = fi5 * wendland_f(r * hinvi);
            const float fj = kWendlandF * hj5 * wendland_f(r * hinvj);
            pu += q.w * (kappai + qc.z) * (ui - qc.y) * (0.5f * (fi + fj)) * (rinvi * qc.w);
          }
        }
      }
      neumaier_add(du, cdu, pu);
      wave_sync();
    };

    int cur = grp.root;
    while (cur < grp.end) {
      const Node nd = nodes[cur];
      const float hm = fmaxf(hi, nd.lo_h.w);
      const bool want = hi > 0.0f && box_dist2(xi, nd.lo_h, nd.hi_l) < sq_exact(hm);
      if (__ballot(want) == 0ull) {
        cur = nd.meta.x;
        continue;
      }
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
    du += cdu;
    if (valid) {
      const int cid = perm[s];
      if (dudt) dudt[cid] = du;
      if (npairs) npairs[cid] = np - 1;  // the self pair passes the test
    }
  }  // groups
}

inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_conduction_prep(Octree &gas, const float *u, const void *h, int f64,
                                  const float *rho, float kappa0, float kappa_exp,
                                  float4 *ch, hipStream_t s) {
  if (gas.n == 0) return hipSuccess;
  if (f64)
    k_cond_prep<double><<<nblk(gas.n, 256), 256, 0, s>>>(
        gas.perm, gas.n, u, (const double *)h, rho, kappa0, kappa_exp, ch);
  else
    k_cond_prep<float><<<nblk(gas.n, 256), 256, 0, s>>>(
        gas.perm, gas.n, u, (const float *)h, rho, kappa0, kappa_exp, ch);
  return hipGetLastError();
}

hipError_t launch_conduction(const Octree &gas, const Groups &gs, int64_t max_groups,
                             int walk_leaf, const float4 *ch, float *dudt, int32_t *npairs,
                             hipStream_t s) {
  if (max_groups <= 0 || gas.nnodes == 0) return hipSuccess;
  k_conduction<<<persistent_grid((const void *)k_conduction, kBlock, max_groups), kBlock, 0,
                 s>>>(gas.nodes, gas.xm, ch, gas.perm, gs, walk_leaf, dudt, npairs);
  return hipGetLastError();
}

}  // namespace g3
