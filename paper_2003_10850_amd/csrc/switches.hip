// The improved-SPH switches of the hydro force Gadget3 ran (Beck et al.
// 2016; the paper names that SPH variant in section 1): the velocity
// divergence and curl estimates, the Balsara (1995) factor and the
// time-dependent viscosity strength (Morris & Monaghan 1997, with the source
// factor of Rosswog et al. 2000). The per-pair use of the strengths and the
// artificial conduction sit in the hydro kernel (sph.hip, kExt).
#include <cmath>

#include "g3_device.h"
#include "g3_internal.h"

namespace g3 {
namespace {

constexpr int kBlock = 256;
constexpr int kWpb = kBlock / kWave;
constexpr int kTile = kWave;

struct VelTile {
  float4 xm[kWpb][kTile];
  float4 vh[kWpb][kTile];
};

// div v_i  =  (1/(Omega_i rho_i)) sum_j m_j (v_j - v_i) . grad_i W(r, h_i)
// curl v_i = -(1/(Omega_i rho_i)) sum_j m_j (v_j - v_i) x grad_i W(r, h_i)
// with grad_i W = F(r, h_i) (x_i - x_j), over gas j with r < h_i (the
// density's gather pairs; the self pair adds nothing). One wave per group
// of up to 64 targets walks the gas octree with each lane's radius h_i,
// stages leaf members as tiles in LDS (after the group-box cull) and every
// lane scans the tile with the exact neighbour test.
__global__ __launch_bounds__(kBlock) void k_velgrad(
    const Node *__restrict__ nodes, const float4 *__restrict__ xm,
    const float4 *__restrict__ vh, const int32_t *__restrict__ perm, const Groups gs,
    int walk_leaf, const float *__restrict__ rho, const float *__restrict__ omega,
    float *__restrict__ div_v, float *__restrict__ curl_v) {
  __shared__ VelTile T;
  const int w = (int)(threadIdx.x >> 6), lane = lane_id();
  int range = 0;
  for (int g; (g = next_group(gs, range)) >= 0;) {
    const Group grp = group_at(gs, g);
    const int64_t t = grp.t0 + lane;
    const bool valid = lane < grp.count;
    const int s = valid ? (gs.targets ? gs.targets[t] : (int)t) : 0;
    const float4 me = xm[s], mv = vh[s];
    const float3 xi = make_float3(me.x, me.y, me.z);
    const float hi = valid ? mv.w : -1.0f;
    const float hi2 = valid ? sq_exact(hi) : -1.0f;
    const float hinv = 1.0f / mv.w;
    const float fi5 = kWendlandF * (hinv * hinv) * (hinv * hinv) * hinv;
    float dv = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
    float cdv = 0.f, ccx = 0.f, ccy = 0.f, ccz = 0.f;
    int tc = 0, cand = 0;
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
        float4 vv = make_float4(0.f, 0.f, 0.f, 0.f);
        if (lane < nc) {
          vx = xm[cand];
          vv = vh[cand];
        }
        // a candidate at or beyond the group's largest radius from its
        // target box fails every lane's gather test
        const bool keep =
            lane < nc && box_dist2(make_float3(vx.x, vx.y, vx.z), tlo, thi) < hmax2;
        const uint64_t km = __ballot(keep);
        const int slot = (int)__builtin_amdgcn_mbcnt_hi(
            (uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
        if (keep) {
          T.xm[w][slot] = vx;
          T.vh[w][slot] = vv;
        }
        nc = __popcll(km);
      }
      wave_sync();
      float pd = 0.f, px = 0.f, py = 0.f, pz = 0.f;
      for (int k = 0; k < nc; ++k) {
        const float4 q = T.xm[w][k];
        const float dx = sub_exact(q.x, xi.x), dy = sub_exact(q.y, xi.y),
                    dz = sub_exact(q.z, xi.z);
        const float r2 = dist2_exact(dx, dy, dz);
        if (r2 < hi2 && r2 > 0.0f) {
          const float4 qv = T.vh[w][k];
          const float r = r2 * __builtin_amdgcn_rsqf(r2);
          // m_j F(r, h_i): grad_i W = F (x_i - x_j) = -F (dx, dy, dz)
          const float mf = q.w * fi5 * wendland_f(r * hinv);
          const float gx = -mf * dx, gy = -mf * dy, gz = -mf * dz;
          const float ux = qv.x - mv.x, uy = qv.y - mv.y, uz = qv.z - mv.z;
          pd += ux * gx + uy * gy + uz * gz;
          px -= uy * gz - uz * gy;
          py -= uz * gx - ux * gz;
          pz -= ux * gy - uy * gx;
        }
      }
      neumaier_add(dv, cdv, pd);
      neumaier_add(cx, ccx, px);
      neumaier_add(cy, ccy, py);
      neumaier_add(cz, ccz, pz);
      wave_sync();
    };

    int cur = grp.root;
    while (cur < grp.end) {
      const Node nd = nodes[cur];
      const bool want = hi > 0.0f && box_dist2(xi, nd.lo_h, nd.hi_l) < hi2;
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
    if (valid) {
      const int cid = perm[s];
      const float norm = 1.0f / (omega[cid] * rho[cid]);
      if (div_v) div_v[cid] = (dv + cdv) * norm;
      if (curl_v) {
        curl_v[3 * cid] = (cx + ccx) * norm;
        curl_v[3 * cid + 1] = (cy + ccy) * norm;
        curl_v[3 * cid + 2] = (cz + ccz) * norm;
      }
    }
  }  // groups
}

// One step dt of the viscosity strength and the Balsara factor of each
// listed particle:
//   f = |div v| / (|div v| + |curl v| + eps c / h),  c = sqrt(gamma (gamma-1) u),
//   d alpha/dt = -(alpha - alpha_min) / tau + s (alpha_max - alpha),
//   tau = h / (decay c),  s = f max(-div v, 0),
// integrated exactly for inputs held over the step (the equation is linear
// in alpha): alpha -> alpha_inf + (alpha - alpha_inf) exp(-(1/tau + s) dt).
template <typename HT>
__global__ void k_alpha_update(int64_t n, int64_t n_act, const int32_t *__restrict__ active,
                               const SwitchStep sw, const float *__restrict__ u,
                               const HT *__restrict__ h, const float *__restrict__ div_v,
                               const float *__restrict__ curl_v, float *__restrict__ alpha,
                               float *__restrict__ balsara) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_act) return;
  const int64_t i = active ? (int64_t)active[a] : a;
  if (i < 0 || i >= n) return;
  const float c = sqrtf(sw.gamma * (sw.gamma - 1.0f) * fmaxf(u[i], 0.0f));
  const float hi = (float)h[i];
  const float d = div_v[i];
  const float cv = sqrtf(curl_v[3 * i] * curl_v[3 * i] + curl_v[3 * i + 1] * curl_v[3 * i + 1] +
                         curl_v[3 * i + 2] * curl_v[3 * i + 2]);
  const float den = fabsf(d) + cv + sw.eps * c / hi;
  const float f = den > 0.0f ? fabsf(d) / den : 0.0f;
  if (balsara) balsara[i] = f;
  if (alpha) {
    const float decay = sw.decay * c / hi;
    const float src = f * fmaxf(-d, 0.0f);
    const float rate = decay + src;
    const float al = alpha[i];
    if (rate > 0.0f) {
      const float ainf = (sw.alpha_min * decay + src * sw.alpha_max) / rate;
      alpha[i] = ainf + (al - ainf) * expf(-rate * sw.dt);
    }
  }
}

inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_velgrad(const Octree &gas, const Groups &gs, int64_t max_groups,
                          int walk_leaf, const float *rho, const float *omega, float *div_v,
                          float *curl_v, hipStream_t s) {
  if (max_groups <= 0 || gas.nnodes == 0) return hipSuccess;
  k_velgrad<<<persistent_grid((const void *)k_velgrad, kBlock, max_groups), kBlock, 0, s>>>(
      gas.nodes, gas.xm, gas.vh, gas.perm, gs, walk_leaf, rho, omega, div_v, curl_v);
  return hipGetLastError();
}

hipError_t launch_alpha_update(int64_t n, int64_t n_act, const int32_t *active,
                               const SwitchStep &sw, int f64, const float *u, const void *h,
                               const float *div_v, const float *curl_v, float *alpha,
                               float *balsara, hipStream_t s) {
  if (n_act <= 0) return hipSuccess;
  if (f64)
    k_alpha_update<double><<<nblk(n_act, 256), 256, 0, s>>>(
        n, n_act, active, sw, u, (const double *)h, div_v, curl_v, alpha, balsara);
  else
    k_alpha_update<float><<<nblk(n_act, 256), 256, 0, s>>>(
        n, n_act, active, sw, u, (const float *)h, div_v, curl_v, alpha, balsara);
  return hipGetLastError();
}

}  // namespace g3
