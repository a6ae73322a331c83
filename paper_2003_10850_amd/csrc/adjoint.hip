// Adjoint (backward) kernels of the density, hydro force and gravity: the
// gradients of a scalar loss with respect to positions, masses, smoothing
// lengths (and the hydro inputs), given its gradients with respect to the
// module outputs at the active particles. Neighbour sets and Barnes-Hut
// decisions are those of the forward call (the forward map is piecewise
// smooth in them) and h is an input; the derivative through the h solve is
// the density adjoint with a seed derived from the solve's constraint.
//
// SPH adjoints are gathered: every gas particle walks its symmetric
// neighbourhood r < max(h_p, h_q) once and adds both what its own sums owe
// to its inputs and what its neighbours' sums owe to them, so each
// gradient is written by one lane in a fixed order (deterministic). The
// gravity adjoint is scattered: a wave sums the source-side terms of a tile
// entry over its lanes with DPP row operations and adds them with one
// atomic per entry, in 64-bit fixed point (integer additions commute, so
// the result does not depend on the order of the waves: deterministic); node
// adjoints are then pushed down to the members.
#include "g3_device.h"
#include "g3_internal.h"

namespace g3 {

namespace {

constexpr int kBlock = 256;
constexpr int kWpb = kBlock / kWave;
constexpr int kTile = kWave;
constexpr float kC = 6.7889530412636603f;  // 1365 / (64 pi)

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Wendland C6 (support h, q = r/h) and the derivatives the adjoints need,
// each zero at and beyond the support:
//   W    = C/h^3 (1-q)^8 (1 + 8q + 25q^2 + 32q^3)
//   W_h  = dW/dh        = C/h^4 (1-q)^7 (-3 - 21q - 29q^2 + 133q^3 + 448q^4)
//   F    = (1/r) dW/dr  = -22 C/h^5 (1-q)^7 (1 + 7q + 16q^2)
//   G    = (1/r) dW_h/dr = dF/dh = 22 C/h^6 (1-q)^6 (5 + 30q + 21q^2 - 224q^3)
//   W_hh = d^2W/dh^2    = 6 C/h^5 (1-q)^6 (2 + 12q - 13q^2 - 218q^3 - 287q^4 + 1120q^5)
struct Wc6 {
  float W, Wh, F, G, Whh;
};

__device__ __forceinline__ Wc6 wc6_all(float r, float hinv) {
  const float q = r * hinv;
  const float t = fmaxf(1.0f - q, 0.0f);
  const float t2 = t * t, t3 = t2 * t, t6 = t3 * t3, t7 = t6 * t;
  const float h2 = hinv * hinv, h3 = h2 * hinv, h4 = h2 * h2, h5 = h4 * hinv, h6 = h3 * h3;
  Wc6 k;
  k.W = kC * h3 * t7 * t * (1.0f + q * (8.0f + q * (25.0f + q * 32.0f)));
  k.Wh = kC * h4 * t7 * (-3.0f + q * (-21.0f + q * (-29.0f + q * (133.0f + q * 448.0f))));
  k.F = -22.0f * kC * h5 * t7 * (1.0f + q * (7.0f + q * 16.0f));
  k.G = 22.0f * kC * h6 * t6 * (5.0f + q * (30.0f + q * (21.0f - q * 224.0f)));
  k.Whh = 6.0f * kC * h5 * t6 *
          (2.0f + q * (12.0f + q * (-13.0f + q * (-218.0f + q * (-287.0f + q * 1120.0f)))));
  return k;
}

// ---------------------------------------------------------------- density

// Upstream gradients of the density outputs folded into the two sums:
// Omega = 1 + h rho' / (3 rho) gives
//   gbar_rho  = g_rho  - g_omega h rho' / (3 rho^2)
//   gbar_rho' = g_rho' + g_omega h / (3 rho)
//   dL/dh    += g_omega rho' / (3 rho)        (the explicit h of Omega)
// written into bw[s] = (h, gbar_rho, gbar_rho', 0) at the active gas rows.
__global__ void k_density_bwd_prep(const int32_t *__restrict__ active, int64_t n_act,
                                   const int32_t *__restrict__ iperm, int64_t n_caller,
                                   const float *__restrict__ h, const float *__restrict__ rho,
                                   const float *__restrict__ drho, const float *__restrict__ g_rho,
                                   const float *__restrict__ g_drho,
                                   const float *__restrict__ g_omega, float4 *__restrict__ bw,
                                   float *__restrict__ g_h) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_act) return;
  const int32_t id = active ? active[a] : (int32_t)a;
  if (id < 0 || (int64_t)id >= n_caller) return;
  const int32_t s = iperm[id];
  if (s < 0) return;
  const float hi = h[id], r = rho[id], rp = drho[id];
  const float go = g_omega ? g_omega[id] : 0.0f;
  const float gr = (g_rho ? g_rho[id] : 0.0f) - go * hi * rp / (3.0f * r * r);
  const float gd = (g_drho ? g_drho[id] : 0.0f) + go * hi / (3.0f * r);
  bw[s] = make_float4(hi, gr, gd, 0.0f);
  if (g_h && go != 0.0f) g_h[id] += go * rp / (3.0f * r);
}

__global__ void k_density_bwd_init(const int32_t *__restrict__ perm, int64_t m,
                                   const float *__restrict__ h, float4 *__restrict__ bw) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < m) bw[s] = make_float4(h[perm[s]], 0.0f, 0.0f, 0.0f);
}

// Adjoint of the smoothing-length solve. Each active gas h_i is the root of
// F_i = N_eff(h_i) - N_ngb with N_eff = (4 pi/3) h^3 rho / m_i. By the
// implicit function theorem an upstream g_h_i reaches the positions and
// masses as the density adjoint seeded with
//   gbar_rho_i = -g_h_i h_i / (3 rho_i + h_i drho_i/dh)
// plus the explicit 1/m_i of N_eff:
//   dL/dm_i += g_h_i h_i rho_i / (m_i (3 rho_i + h_i drho_i/dh)).
// A row whose N_eff misses N_ngb by more than 1e-3 (relative: an h that did
// not converge, or one held at the cap) has no constraint and passes nothing.
__global__ void k_hsolve_bwd_prep(const int32_t *__restrict__ active, int64_t n_act,
                                  const int32_t *__restrict__ iperm, int64_t n_caller,
                                  const float *__restrict__ h, const float *__restrict__ rho,
                                  const float *__restrict__ drho, const float *__restrict__ g_h,
                                  const float4 *__restrict__ xm, float n_ngb,
                                  float4 *__restrict__ bw, float *__restrict__ g_mass) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_act) return;
  const int32_t id = active ? active[a] : (int32_t)a;
  if (id < 0 || (int64_t)id >= n_caller) return;
  const int32_t s = iperm[id];
  if (s < 0) return;
  const float hi = h[id], r = rho[id], rp = drho[id], mi = xm[s].w, gh = g_h[id];
  const float N = 4.18879020f * hi * hi * hi * r / mi;  // (4 pi/3) h^3 rho / m
  const float den = 3.0f * r + hi * rp;                 // 3 rho Omega
  if (!(fabsf(N / n_ngb - 1.0f) <= 1e-3f) || !(den > 0.0f) || gh == 0.0f) return;
  bw[s] = make_float4(hi, -gh * hi / den, 0.0f, 0.0f);
  if (g_mass) g_mass[id] += gh * hi * r / (mi * den);
}

// One lane per gas particle p, over every q with r < max(h_p, h_q):
//   own sums (r < h_p):  a = gbar_rho_p m_q F(r,h_p) + gbar_rho'_p m_q G(r,h_p)
//       dL/dx_p += a (x_p - x_q)
//       dL/dh_p += m_q (gbar_rho_p W_h(r,h_p) + gbar_rho'_p W_hh(r,h_p))
//   q's sums (r < h_q):  b = gbar_rho_q m_p F(r,h_q) + gbar_rho'_q m_p G(r,h_q)
//       dL/dx_p += b (x_p - x_q)
//       dL/dm_p += gbar_rho_q W(r,h_q) + gbar_rho'_q W_h(r,h_q)
// The pair q = p (r = 0) adds the self terms of h and m.
__global__ __launch_bounds__(kBlock) void k_density_bwd(
    const Node *__restrict__ nodes, const float4 *__restrict__ xm,
    const float4 *__restrict__ bw, const int32_t *__restrict__ perm, const Groups gs,
    float *__restrict__ g_pos, float *__restrict__ g_mass, float *__restrict__ g_h) {
  __shared__ float4 tx[kWpb][kTile];
  __shared__ float4 tb[kWpb][kTile];
  const int w = (int)(threadIdx.x >> 6), lane = lane_id();
  int range = 0;
  for (int g; (g = next_group(gs, range)) >= 0;) {
    const Group grp = group_at(gs, g);
    const bool valid = lane < grp.count;
    const int s = valid ? grp.t0 + lane : grp.t0;
    const float4 me = xm[s], mb = bw[s];
    const float hp = valid ? mb.x : -1.0f;
    const float hp2 = sq_exact(hp), hinv = 1.0f / mb.x;
    const bool own_on = valid && (mb.y != 0.0f || mb.z != 0.0f);
    float gx = 0.f, gy = 0.f, gz = 0.f, gm = 0.f, gh = 0.f;
    float cx = 0.f, cy = 0.f, cz = 0.f, cm = 0.f, ch = 0.f;
    int tc = 0, cand = 0;
    // the box of the group's particles and the largest radius of their own
    // sums: a candidate q whose box_dist2 to the box reaches that radius and
    // (when q's sums carry gradients) fl(h_q^2) meets no lane's test, since
    // box_dist2 never exceeds the r2 of a point inside the box
    float4 tlo = make_float4(valid ? me.x : INFINITY, valid ? me.y : INFINITY,
                             valid ? me.z : INFINITY, 0.f);
    float4 thi = make_float4(valid ? me.x : -INFINITY, valid ? me.y : -INFINITY,
                             valid ? me.z : -INFINITY, 0.f);
    float hmax2 = own_on ? hp2 : -1.0f;
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
    {
      auto su = [](float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); };
      tlo = make_float4(su(tlo.x), su(tlo.y), su(tlo.z), 0.f);
      thi = make_float4(su(thi.x), su(thi.y), su(thi.z), 0.f);
      hmax2 = su(hmax2);
    }
    auto flush = [&](int nc) {
      {
        float4 vx = make_float4(INFINITY, INFINITY, INFINITY, 0.f), vb = make_float4(0.f, 0.f, 0.f, 0.f);
        if (lane < nc) {
          vx = xm[cand];
          vb = bw[cand];
        }
        const float d2 = box_dist2(make_float3(vx.x, vx.y, vx.z), tlo, thi);
        const bool keep = lane < nc && (d2 < hmax2 || ((vb.y != 0.0f || vb.z != 0.0f) &&
                                                       d2 < sq_exact(vb.x)));
        const uint64_t km = __ballot(keep);
        const int slot = (int)__builtin_amdgcn_mbcnt_hi(
            (uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
        // kept candidates in their order at the front; the scan stops at nc
        if (keep) {
          tx[w][slot] = vx;
          tb[w][slot] = vb;
        }
        nc = __popcll(km);
      }
      wave_sync();
      float px = 0.f, py = 0.f, pz = 0.f, pm = 0.f, ph = 0.f;
      for (int k = 0; k < nc; ++k) {
        const float4 q = tx[w][k], qb = tb[w][k];
        const float dx = sub_exact(q.x, me.x), dy = sub_exact(q.y, me.y),
                    dz = sub_exact(q.z, me.z);
        const float r2 = dist2_exact(dx, dy, dz);
        const bool own = own_on && r2 < hp2;
        const bool nbr = valid && (qb.y != 0.0f || qb.z != 0.0f) && r2 < sq_exact(qb.x);
        if (own || nbr) {
          const float r = __builtin_amdgcn_sqrtf(r2);
          float a = 0.0f;
          if (own) {
            const Wc6 kp = wc6_all(r, hinv);
            a = q.w * (mb.y * kp.F + mb.z * kp.G);
            ph += q.w * (mb.y * kp.Wh + mb.z * kp.Whh);
          }
          if (nbr) {
            const Wc6 kq = wc6_all(r, 1.0f / qb.x);
            a += me.w * (qb.y * kq.F + qb.z * kq.G);
            pm += qb.y * kq.W + qb.z * kq.Wh;
          }
          // x_p - x_q = -(dx, dy, dz)
          px -= a * dx;
          py -= a * dy;
          pz -= a * dz;
        }
      }
      neumaier_add(gx, cx, px);
      neumaier_add(gy, cy, py);
      neumaier_add(gz, cz, pz);
      neumaier_add(gm, cm, pm);
      neumaier_add(gh, ch, ph);
      wave_sync();
    };
    int cur = grp.root;
    while (cur < grp.end) {
      const Node nd = nodes[cur];
      const float hm = fmaxf(hp, nd.lo_h.w);
      const bool want = valid && box_dist2(make_float3(me.x, me.y, me.z), nd.lo_h, nd.hi_l) <
                                     sq_exact(hm);
      if (__ballot(want) == 0ull) {
        cur = nd.meta.x;
        continue;
      }
      if (!(nd.meta.w & kLeafBit) && nd.meta.z > kTile) {
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
      if (g_pos) {
        g_pos[3 * cid] += gx + cx;
        g_pos[3 * cid + 1] += gy + cy;
        g_pos[3 * cid + 2] += gz + cz;
      }
      if (g_mass) g_mass[cid] += gm + cm;
      if (g_h) g_h[cid] += gh + ch;
    }
  }
}

// ---------------------------------------------------------------- gravity

// v from the lane paired with this one by a DPP permutation (every lane
// active, every lane a source)
template <int kCtrl>
__device__ __forceinline__ float dpp_from(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, 0xf, 0xf,
                                                    false));
}

// Sums over the 64 lanes of v[0..15], spread so that lane l ends with the
// total of value (l >> 2) & 15, by recursive halving: at each of four steps
// the lanes pair off across one lane bit (5, 4, 3, 2), and each keeps the
// half of its values that its bit selects plus its partner's copy of that
// half; two pairwise exchanges (bits 1, 0) then complete the quads' sums.
// Lane pairs: xor 32 and xor 16 by LDS permute, then the DPP row mirror
// (xor 15), half-row mirror (xor 7) and the quad permutations xor 3, xor 1;
// each pairs lanes that differ in the step's bit and agree in the bits
// above it. Every lane must be active.
__device__ __forceinline__ float wave_reduce_scatter16(float (&v)[16], int lane) {
  {
    const bool up = (lane & 32) != 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const float send = up ? v[i] : v[i + 8];
      const float keep = up ? v[i + 8] : v[i];
      v[i] = keep + __shfl_xor(send, 32);
    }
  }
  {
    const bool up = (lane & 16) != 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float send = up ? v[i] : v[i + 4];
      const float keep = up ? v[i + 4] : v[i];
      v[i] = keep + __shfl_xor(send, 16);
    }
  }
  {
    const bool up = (lane & 8) != 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const float send = up ? v[i] : v[i + 2];
      const float keep = up ? v[i + 2] : v[i];
      v[i] = keep + dpp_from<0x140>(send);  // row mirror: lane ^ 15 in its row
    }
  }
  {
    const bool up = (lane & 4) != 0;
    const float send = up ? v[0] : v[1];
    const float keep = up ? v[1] : v[0];
    v[0] = keep + dpp_from<0x141>(send);  // half-row mirror: lane ^ 7
  }
  v[0] += dpp_from<0x1b>(v[0]);  // quad permutation (3, 2, 1, 0): lane ^ 3
  v[0] += dpp_from<0xb1>(v[0]);  // quad permutation (1, 0, 3, 2): lane ^ 1
  return v[0];
}

// Deterministic accumulation of the gravity adjoint's scattered sums. Every
// value v is added as two 64-bit integers, hi = trunc(v 2^F) and
// lo = rint((v 2^F - hi) 2^kFxLoBits), to a pair of counters: integer
// addition is exact and commutes, so the totals do not depend on the order
// in which waves add them. F is one per call, taken from a bound B on every
// counter's partial sums (|sum hi| <= B 2^F <= 2^62): with S = r^2 + eps^2 >=
// eps^2, a term's position part is at most G m (4 |g_a| S^-3/2 + |g_phi|
// S^-1) and its mass part G (|g_a| S^-1 + |g_phi| S^-1/2), |g_a| <= sqrt(3)
// times the largest upstream component, m at most n times the largest mass
// (a node), and a counter takes at most n_act such terms from the source
// side and at most n from its own target side. The overestimate (many
// orders of magnitude) costs nothing: the low counter resolves 2^-(62 + 36)
// of B, about 2^-30 of the largest true total even at 2e7 particles, far
// below the FP32 rounding of the terms; lo stays below 2^63 for up to 2^26
// additions per counter. Needs eps > 0 (else no such bound: FP32 atomics).
constexpr int kFxLoBits = 36;

// The scale 2^F from the device maxima (float bits) of the upstream
// gradient components, the upstream potential gradients and the masses.
__device__ __forceinline__ double fx_scale(const unsigned *__restrict__ mx, float eps2, float G,
                                           int64_t n, int64_t n_act) {
  const double ga = 1.7320508075688772 * (double)__uint_as_float(mx[0]);
  const double gp = (double)__uint_as_float(mx[1]);
  const double mm = (double)__uint_as_float(mx[2]);
  const double e2 = (double)eps2, e1 = sqrt(e2);
  const double T = 4.0 * ga / (e2 * e1) + gp / e2 + ga / e2 + gp / e1;
  const double B = 2.0 * fabs((double)G) * T * ((double)n * mm + 1.0) *
                   ((double)n + (double)n_act + 1.0);
  // (no finite bound, from non-finite inputs: any scale; the sums are then
  // as meaningless as the inputs)
  const int F = (B > 0.0 && B < 1e300) ? 62 - (ilogb(B) + 1) : 0;
  return ldexp(1.0, F);
}

__device__ __forceinline__ void fx_add(unsigned long long *dst, float v, double scale) {
  const double d = (double)v * scale;
  const double hi = trunc(d);  // d - hi is exact
  const long long lo = (long long)rint((d - hi) * (double)(1ll << kFxLoBits));
  atomicAdd(dst, (unsigned long long)(long long)hi);
  atomicAdd(dst + 1, (unsigned long long)lo);
}

// The largest |upstream gradient component|, |upstream potential gradient|
// (over the active rows; ids outside [0, m) are skipped, as by the walk) and
// mass (over every member), as float bits into mx[0..2] (zero on entry).
constexpr int kFxBoundBlocks = 1024;
__global__ __launch_bounds__(kBlock) void k_fx_bound(
    const int32_t *__restrict__ active, int64_t n_act, const float *__restrict__ g_acc,
    const float *__restrict__ g_pot, const float4 *__restrict__ xm, int64_t m,
    unsigned *__restrict__ mx) {
  // a grid-stride pass, then one atomic per block and value (one per wave
  // on three words had serialised)
  __shared__ float part[3][kBlock / kWave];
  float a = 0.0f, p = 0.0f, w = 0.0f;
  const int64_t n = n_act > m ? n_act : m;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t id = i < n_act ? (active ? active[i] : i) : -1;
    if (id >= 0 && id < m) {
      if (g_acc)
        a = fmaxf(a, fmaxf(fabsf(g_acc[3 * id]),
                           fmaxf(fabsf(g_acc[3 * id + 1]), fabsf(g_acc[3 * id + 2]))));
      if (g_pot) p = fmaxf(p, fabsf(g_pot[id]));
    }
    if (i < m) w = fmaxf(w, fabsf(xm[i].w));
  }
#pragma unroll
  for (int k = 1; k < kWave; k <<= 1) {
    a = fmaxf(a, __shfl_xor(a, k));
    p = fmaxf(p, __shfl_xor(p, k));
    w = fmaxf(w, __shfl_xor(w, k));
  }
  const int wv = (int)(threadIdx.x >> 6);
  if ((threadIdx.x & 63u) == 0u) {
    part[0][wv] = a;
    part[1][wv] = p;
    part[2][wv] = w;
  }
  __syncthreads();
  if (threadIdx.x < 3u) {
    float v = part[threadIdx.x][0];
    for (int k = 1; k < kBlock / kWave; ++k) v = fmaxf(v, part[threadIdx.x][k]);
    atomicMax(&mx[threadIdx.x], __float_as_uint(v));
  }
}

// Fixed-point counter pairs (hi, lo) x 4 components back to float4.
__global__ void k_fx_to_f4(const unsigned long long *__restrict__ fx, int64_t m,
                           const unsigned *__restrict__ mx, float eps2, float G, int64_t n,
                           int64_t n_act, float4 *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double inv = 1.0 / fx_scale(mx, eps2, G, n, n_act);
  double v[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const long long hi = (long long)fx[8 * i + 2 * c], lo = (long long)fx[8 * i + 2 * c + 1];
    v[c] = ((double)hi + ldexp((double)lo, -kFxLoBits)) * inv;
  }
  out[i] = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
}

struct __align__(16) GEntry {
  float4 p;   // source position, mass
  int4 meta;  // sorted source index, or -(node + 1); mask low, mask high; unused
};
// a lane's mask word: meta.y (lanes 0..31) or meta.z (lanes 32..63), the
// 32-bit words 5 and 6 of an entry
constexpr int kGMaskWord = 5;

__device__ __forceinline__ bool open_accept(float l, float theta2, float r2) {
#pragma clang fp contract(off)
  const float lhs = l * l;
  const float rhs = theta2 * r2;
  return lhs < rhs;
}

// The Barnes-Hut walk of the forward kernel; each term of target i with
// source s (x = x_i - x_s, S = r^2 + eps^2) and upstream gradients
// (ga, gp) of a_i and phi_i contributes
//   dL/dx  = G m ( -ga / S^(3/2) + 3 (ga . x) x / S^(5/2) + gp x / S^(3/2) )
//   dL/dx_i += dL/dx,  dL/dx_s -= dL/dx,  dL/dm_s = -G ((ga . x) / S^(3/2) + gp / S^(1/2)).
// The source side of a tile entry is summed over the wave's lanes and added
// once: to the particle's sorted slot, or to the node's (dL/dc, dL/dM).
// kFixed: the sums go to fixed-point counter pairs (gsrc_fx [n][4][2],
// gnode_fx [nnodes][4][2], scale from mx), else to FP32 atomics (gsrc,
// gnode).
template <bool kFixed, bool kInside>
__global__ __launch_bounds__(kBlock) void k_gravity_bwd(
    const GNode *__restrict__ nodes, const float4 *__restrict__ xm,
    const uint64_t *__restrict__ keys, const int32_t *__restrict__ perm, const Groups gs,
    float theta2, float eps2, float G, const float *__restrict__ g_acc,
    const float *__restrict__ g_pot, float4 *__restrict__ gsrc, float4 *__restrict__ gnode,
    unsigned long long *__restrict__ gsrc_fx, unsigned long long *__restrict__ gnode_fx,
    const unsigned *__restrict__ mx, int64_t n_all, int64_t n_act) {
  __shared__ GEntry tiles[kWpb][kTile];
  const int w = (int)(threadIdx.x >> 6), lane = lane_id();
  GEntry *tile = tiles[w];
  const double scale = kFixed ? fx_scale(mx, eps2, G, n_all, n_act) : 1.0;
  int range = 0;
  for (int g; (g = next_group(gs, range)) >= 0;) {
    const Group grp = group_at(gs, g);
    const int64_t t = grp.t0 + lane;
    const bool valid = lane < grp.count;
    const int s = valid ? (gs.targets ? gs.targets[t] : (int)t) : 0;
    const float4 me = xm[s];
    const uint64_t ki = keys[s];
    const int cid = perm[s];
    const float gax = valid && g_acc ? g_acc[3 * cid] : 0.f;
    const float gay = valid && g_acc ? g_acc[3 * cid + 1] : 0.f;
    const float gaz = valid && g_acc ? g_acc[3 * cid + 2] : 0.f;
    const float gpp = valid && g_pot ? g_pot[cid] : 0.f;
    float ox = 0.f, oy = 0.f, oz = 0.f, cox = 0.f, coy = 0.f, coz = 0.f;
    int tc = 0;
    const bool hiword = lane >= 32;
    const uint32_t bitpos = (uint32_t)lane & 31u;
    const uint32_t *maskw = (const uint32_t *)tile + kGMaskWord + (hiword ? 1 : 0);
    auto flush = [&](int nc) {
      // padded to a multiple of four with entries no lane uses
      const int n4 = (nc + 3) & ~3;
      if (lane >= nc && lane < n4) {
        tile[lane].p = make_float4(0.f, 0.f, 0.f, 0.f);
        tile[lane].meta = make_int4(0, 0, 0, 0);
      }
      wave_sync();
      float px = 0.f, py = 0.f, pz = 0.f;
      for (int k0 = 0; k0 < n4; k0 += 4) {
        // the source sides of four entries: (-dL/dx_i, dL/dm_s) per entry
        float v[16];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int k = k0 + e;
          const float4 ep = tile[k].p;
          // 0 or all ones: the lane's bit (its own target's bit is clear)
          const int32_t use = __builtin_amdgcn_sbfe(
              (int32_t)maskw[k * (int)(sizeof(GEntry) / 4)], bitpos, 1u);
          const float dx = ep.x - me.x, dy = ep.y - me.y, dz = ep.z - me.z;  // x_s - x_i
          const float S =
              __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
          // masked here, so that an unused entry adds exact zeros even at S = 0
          const float inv = __int_as_float(__float_as_int(__builtin_amdgcn_rsqf(S)) & use);
          const float inv3 = inv * inv * inv;
          const float Gm = G * ep.w;
          const float gx_ = -(gax * dx + gay * dy + gaz * dz);  // ga . x, x = x_i - x_s
          const float c3 = 3.0f * gx_ * inv3 * inv * inv;
          // dL/dx with x = -(dx, dy, dz)
          const float Dx = Gm * (-gax * inv3 - c3 * dx - gpp * dx * inv3);
          const float Dy = Gm * (-gay * inv3 - c3 * dy - gpp * dy * inv3);
          const float Dz = Gm * (-gaz * inv3 - c3 * dz - gpp * dz * inv3);
          const float Dm = -G * (gx_ * inv3 + gpp * inv);
          px += Dx;
          py += Dy;
          pz += Dz;
          v[4 * e] = -Dx;
          v[4 * e + 1] = -Dy;
          v[4 * e + 2] = -Dz;
          v[4 * e + 3] = Dm;
        }
        // lane l holds the wave's total of entry l >> 4, component (l >> 2) & 3
        const float tot = wave_reduce_scatter16(v, lane);
        const int e = lane >> 4, comp = (lane >> 2) & 3;
        if ((lane & 3) == 0 && k0 + e < nc) {
          const int src = tile[k0 + e].meta.x;
          if constexpr (kFixed) {
            unsigned long long *dst = src >= 0 ? gsrc_fx + 8 * (int64_t)src
                                               : gnode_fx + 8 * (int64_t)(-src - 1);
            fx_add(dst + 2 * comp, tot, scale);
          } else {
            float *dst = src >= 0 ? (float *)&gsrc[src] : (float *)&gnode[-src - 1];
            atomicAdd(dst + comp, tot);
          }
        }
      }
      neumaier_add(ox, cox, px);
      neumaier_add(oy, coy, py);
      neumaier_add(oz, coz, pz);
      wave_sync();
    };
    // the walk of the forward kernel over the 32-byte node copies: the same
    // decisions, one compare each without the containment test (an idle
    // lane compares with NaN, for which both are false)
    const int root_exp = ilogbf((float)gs.sbox[grp.snap].w);
    const int groot = __builtin_amdgcn_readfirstlane(grp.root);
    const int gend = __builtin_amdgcn_readfirstlane(grp.end);
    int resume = valid ? groot : INT32_MAX;
    int cur = groot;
    while (cur < gend) {
      const GNode nd = nodes[cur];
      const float l = __int_as_float(nd.meta.w);
      const bool act = cur >= resume;
      const float r2 = dist2_exact(sub_exact(nd.com_m.x, me.x), sub_exact(nd.com_m.y, me.y),
                                   sub_exact(nd.com_m.z, me.z));
      bool accept, open;
      if constexpr (!kInside) {
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
        const int level = root_exp - ilogbf(l);
        const uint64_t nk = keys[nd.meta.y];
        accept = accept && (((ki ^ nk) >> (3 * (kMaxLevel - level))) != 0ull);
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
          GEntry e;
          e.p = nd.com_m;
          e.meta = make_int4(-(cur + 1), (int)(uint32_t)amask, (int)(uint32_t)(amask >> 32), 0);
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
          GEntry e;
          e.p = xm[st + lane];
          e.meta = make_int4(st + lane, (int)(uint32_t)omask, (int)(uint32_t)(omask >> 32), 0);
          tile[tc + lane] = e;
        }
        wave_sync();
        // an opening lane whose own target is among these members clears
        // its bit in that member's entry (one lane per entry)
        const int rel = s - st;
        if (open && rel >= 0 && rel < take) {
          uint32_t *wd = (uint32_t *)&tile[tc + rel] + kGMaskWord + (hiword ? 1 : 0);
          *wd &= ~(1u << bitpos);
        }
        tc += take;
        st += take;
        c -= take;
      }
      cur = nd.meta.x;
    }
    if (tc > 0) flush(tc);
    if (valid) {
      if constexpr (kFixed) {
        fx_add(gsrc_fx + 8 * (int64_t)s, ox + cox, scale);
        fx_add(gsrc_fx + 8 * (int64_t)s + 2, oy + coy, scale);
        fx_add(gsrc_fx + 8 * (int64_t)s + 4, oz + coz, scale);
      } else {
        atomicAdd(&gsrc[s].x, ox + cox);
        atomicAdd(&gsrc[s].y, oy + coy);
        atomicAdd(&gsrc[s].z, oz + coz);
      }
    }
  }
}

__global__ void k_zero_f4(float4 *__restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// Node adjoints (dL/dc, dL/dM) to the members. With c = sum m x / M and
// M = sum m, a member k of node a receives (m_k / M_a) dL/dc_a on x_k and
// dL/dM_a + dL/dc_a . (x_k - c_a) / M_a on m_k. Summed over the ancestors of
// k's leaf l, top-down in FP64:
//   P_n = sum_a dL/dc_a / M_a,  Q_n = sum_a dL/dM_a,
//   R_n = sum_a dL/dc_a . (c_n - c_a) / M_a = R_parent + P_parent . (c_n - c_parent)
// and then x_k gets m_k P_l, m_k gets Q_l + R_l + P_l . (x_k - c_l).
__global__ void k_push_init(const float4 *__restrict__ gnode, const double4 *__restrict__ mom,
                            int64_t nn, double4 *__restrict__ pq, double *__restrict__ rr) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nn) return;
  const float4 g = gnode[k];
  const double M = mom[k].x;
  const double inv = M > 0.0 ? 1.0 / M : 0.0;
  pq[k] = make_double4(g.x * inv, g.y * inv, g.z * inv, (double)g.w);
  rr[k] = 0.0;
}

__global__ void k_push_level(const Node *__restrict__ nodes, const double4 *__restrict__ mom,
                             int64_t nn, int level, double4 *__restrict__ pq,
                             double *__restrict__ rr) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nn) return;
  const int4 meta = nodes[k].meta;
  if ((meta.w & 255) != level || (meta.w & kLeafBit)) return;
  const double4 P = pq[k];
  const double R = rr[k];
  const double4 mk = mom[k];
  const double ik = mk.x > 0.0 ? 1.0 / mk.x : 0.0;
  const double cx = mk.y * ik, cy = mk.z * ik, cz = mk.w * ik;
  int64_t c = k + 1;
  while (c < meta.x) {
    const double4 mc = mom[c];
    const double ic = mc.x > 0.0 ? 1.0 / mc.x : 0.0;
    double4 q = pq[c];
    q.x += P.x;
    q.y += P.y;
    q.z += P.z;
    q.w += P.w;
    pq[c] = q;
    rr[c] = R + P.x * (mc.y * ic - cx) + P.y * (mc.z * ic - cy) + P.z * (mc.w * ic - cz);
    c = nodes[c].meta.x;
  }
}

__global__ void k_push_leaves(const Node *__restrict__ nodes, const double4 *__restrict__ mom,
                              int64_t nn, const float4 *__restrict__ xm,
                              const double4 *__restrict__ pq, const double *__restrict__ rr,
                              float4 *__restrict__ gsrc) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nn) return;
  const int4 meta = nodes[k].meta;
  if (!(meta.w & kLeafBit)) return;
  const double4 P = pq[k];
  const double R = rr[k];
  const double4 mk = mom[k];
  const double ik = mk.x > 0.0 ? 1.0 / mk.x : 0.0;
  const double cx = mk.y * ik, cy = mk.z * ik, cz = mk.w * ik;
  for (int s = meta.y; s < meta.y + meta.z; ++s) {
    const float4 p = xm[s];
    float4 g = gsrc[s];
    g.x += (float)(p.w * P.x);
    g.y += (float)(p.w * P.y);
    g.z += (float)(p.w * P.z);
    g.w += (float)(P.w + R + P.x * (p.x - cx) + P.y * (p.y - cy) + P.z * (p.z - cz));
    gsrc[s] = g;
  }
}

__global__ void k_scatter_grad(const int32_t *__restrict__ perm, int64_t m,
                               const float4 *__restrict__ gsrc, float *__restrict__ g_pos,
                               float *__restrict__ g_mass) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= m) return;
  const int cid = perm[s];
  const float4 g = gsrc[s];
  if (g_pos) {
    g_pos[3 * cid] += g.x;
    g_pos[3 * cid + 1] += g.y;
    g_pos[3 * cid + 2] += g.z;
  }
  if (g_mass) g_mass[cid] += g.w;
}

// ------------------------------------------------------------------ hydro

// F = (1/r) dW/dr and its derivatives dF/dr, dF/dh (= G above):
//   F_r = 528 C/h^6 q (1-q)^6 (1 + 6q)
__device__ __forceinline__ void wc6_f_derivs(float r, float hinv, float &F, float &Fr,
                                             float &Fh) {
  const float q = r * hinv;
  const float t = fmaxf(1.0f - q, 0.0f);
  const float t2 = t * t, t3 = t2 * t, t6 = t3 * t3;
  const float h2 = hinv * hinv, h5 = h2 * h2 * hinv, h6 = h5 * hinv;
  F = -22.0f * kC * h5 * t6 * t * (1.0f + q * (7.0f + q * 16.0f));
  Fr = 528.0f * kC * h6 * t6 * q * (1.0f + 6.0f * q);
  Fh = 22.0f * kC * h6 * t6 * (5.0f + q * (30.0f + q * (21.0f - q * 224.0f)));
}

// One side of a particle's hydro data: position and mass, velocity and h,
// (A, c, rho, 1/h), and the upstream gradients (g_acc, g_dudt) of its sums.
struct HSide {
  float4 xm, vh, aux, up;
};

// Partials of one pair term (target i, neighbour j) of
//   l = g_acc_i . a_ij + g_dudt_i du_ij,
//   a_ij  = -m_j (A_i g_i + A_j g_j + Pi gbar) x,   x = x_i - x_j, v = v_i - v_j
//   du_ij = m_j (A_i g_i + Pi gbar / 2) v.x,        g_k = F(r, h_k), gbar = (g_i + g_j)/2
//   Pi = -alpha (c_i + c_j - 3w) w / (rho_i + rho_j) if w = v.x / r < 0, else 0,
// with respect to the target's inputs (side 0) or the neighbour's (side 1):
// d[0..2] position, d[3..5] velocity, d[6] h, d[7] A, d[8] c, d[9] rho
// through Pi, d[10] m (neighbour only). The chain rules used:
//   dl/dx = coef g_acc + L_vx v + (L_r / r) x,  dl/dv = L_vx x,
//   L_vx = dl/dvx + dl/dPi dPi/dw / r,  L_r = sum_k dl/dg_k F_r(r,h_k) - dl/dPi dPi/dw w / r.
__device__ __forceinline__ void hydro_pair_partials(const HSide &I, const HSide &J, float alpha,
                                                    float dx, float dy, float dz, float r,
                                                    int side, float *d) {
  // x = x_i - x_j (dx, dy, dz given as that difference)
  const float mj = J.xm.w;
  const float vxx = I.vh.x - J.vh.x, vyy = I.vh.y - J.vh.y, vzz = I.vh.z - J.vh.z;
  const float vx = vxx * dx + vyy * dy + vzz * dz;
  const float rinv = 1.0f / r;
  const float w = vx * rinv;
  float gi, gir, gih, gj, gjr, gjh;
  wc6_f_derivs(r, I.aux.w, gi, gir, gih);
  wc6_f_derivs(r, J.aux.w, gj, gjr, gjh);
  const float Ai = I.aux.x, Aj = J.aux.x, ci = I.aux.y, cj = J.aux.y;
  const float rsum = I.aux.z + J.aux.z;
  const bool neg = w < 0.0f;
  const float Pi = neg ? -alpha * (ci + cj - 3.0f * w) * w / rsum : 0.0f;
  const float Pw = neg ? -alpha * (ci + cj - 6.0f * w) / rsum : 0.0f;
  const float Pc = neg ? -alpha * w / rsum : 0.0f;
  const float Prho = neg ? -Pi / rsum : 0.0f;
  const float gbar = 0.5f * (gi + gj);
  const float gax = I.up.x, gay = I.up.y, gaz = I.up.z, gd = I.up.w;
  const float sdot = gax * dx + gay * dy + gaz * dz;
  const float T1 = Ai * gi, T2 = Aj * gj;
  const float dPi = mj * gbar * (0.5f * gd * vx - sdot);
  const float dgb = mj * Pi * (0.5f * gd * vx - sdot);
  const float dgi = mj * Ai * (gd * vx - sdot) + 0.5f * dgb;
  const float dgj = -mj * Aj * sdot + 0.5f * dgb;
  const float coef = -mj * (T1 + T2 + Pi * gbar);
  const float Lvx = gd * mj * (T1 + 0.5f * Pi * gbar) + dPi * Pw * rinv;
  const float Lr = dgi * gir + dgj * gjr - dPi * Pw * w * rinv;
  const float lr = Lr * rinv;
  const float px = coef * gax + Lvx * vxx + lr * dx;
  const float py = coef * gay + Lvx * vyy + lr * dy;
  const float pz = coef * gaz + Lvx * vzz + lr * dz;
  if (side == 0) {
    d[0] = px; d[1] = py; d[2] = pz;
    d[3] = Lvx * dx; d[4] = Lvx * dy; d[5] = Lvx * dz;
    d[6] = dgi * gih;
    d[7] = mj * gi * (gd * vx - sdot);
    d[8] = dPi * Pc;
    d[9] = dPi * Prho;
    d[10] = 0.0f;
  } else {
    d[0] = -px; d[1] = -py; d[2] = -pz;
    d[3] = -Lvx * dx; d[4] = -Lvx * dy; d[5] = -Lvx * dz;
    d[6] = dgj * gjh;
    d[7] = -mj * gj * sdot;
    d[8] = dPi * Pc;
    d[9] = dPi * Prho;
    d[10] = -(T1 + T2 + Pi * gbar) * sdot + gd * (T1 + 0.5f * Pi * gbar) * vx;  // l / m_j
  }
}

__global__ void k_hydro_bwd_up(const int32_t *__restrict__ active, int64_t n_act,
                               const int32_t *__restrict__ iperm, int64_t n_caller,
                               const float *__restrict__ g_acc, const float *__restrict__ g_dudt,
                               float4 *__restrict__ up) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_act) return;
  const int32_t id = active ? active[a] : (int32_t)a;
  if (id < 0 || (int64_t)id >= n_caller) return;
  const int32_t s = iperm[id];
  if (s < 0) return;
  up[s] = make_float4(g_acc ? g_acc[3 * id] : 0.f, g_acc ? g_acc[3 * id + 1] : 0.f,
                      g_acc ? g_acc[3 * id + 2] : 0.f, g_dudt ? g_dudt[id] : 0.f);
}

// One lane per gas particle p over every q != p with r < max(h_p, h_q):
// the pair (target p, neighbour q) if p is active, and (target q,
// neighbour p) if q is active. Then A and c are mapped back to u, rho and
// Omega: A = (gamma-1) u / (Omega rho), c = sqrt(gamma (gamma-1) u).
__global__ __launch_bounds__(kBlock) void k_hydro_bwd(
    const Node *__restrict__ nodes, const float4 *__restrict__ xm,
    const float4 *__restrict__ vh, const float4 *__restrict__ aux,
    const float4 *__restrict__ up, const int32_t *__restrict__ perm, const Groups gs,
    float alpha, float gamma, const float *__restrict__ u, const float *__restrict__ omega,
    float *__restrict__ g_pos, float *__restrict__ g_vel, float *__restrict__ g_mass,
    float *__restrict__ g_h, float *__restrict__ g_u, float *__restrict__ g_rho,
    float *__restrict__ g_omega) {
  __shared__ HSide T[kWpb][kTile];
  const int w = (int)(threadIdx.x >> 6), lane = lane_id();
  int range = 0;
  for (int g; (g = next_group(gs, range)) >= 0;) {
    const Group grp = group_at(gs, g);
    const bool valid = lane < grp.count;
    const int s = valid ? (gs.targets ? gs.targets[grp.t0 + lane] : grp.t0 + lane) : grp.t0;
    HSide P;
    P.xm = xm[s];
    P.vh = vh[s];
    P.aux = aux[s];
    P.up = up[s];
    const float hp = valid ? P.vh.w : -1.0f;
    const bool p_on = valid && (P.up.x != 0.f || P.up.y != 0.f || P.up.z != 0.f || P.up.w != 0.f);
    constexpr int kN = 11;
    float acc[kN], cmp[kN];
#pragma unroll
    for (int k = 0; k < kN; ++k) acc[k] = cmp[k] = 0.0f;
    int tc = 0, cand = 0;
    // the box of the group's particles and their largest fl(h^2): a
    // candidate q whose box_dist2 to the box reaches both that and
    // fl(h_q^2) is in no lane's symmetric neighbourhood, since box_dist2
    // never exceeds the r2 of a point inside the box
    float4 tlo = make_float4(valid ? P.xm.x : INFINITY, valid ? P.xm.y : INFINITY,
                             valid ? P.xm.z : INFINITY, 0.f);
    float4 thi = make_float4(valid ? P.xm.x : -INFINITY, valid ? P.xm.y : -INFINITY,
                             valid ? P.xm.z : -INFINITY, 0.f);
    float hmax2 = valid ? sq_exact(hp) : -1.0f;
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
    {
      auto su = [](float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); };
      tlo = make_float4(su(tlo.x), su(tlo.y), su(tlo.z), 0.f);
      thi = make_float4(su(thi.x), su(thi.y), su(thi.z), 0.f);
      hmax2 = su(hmax2);
    }
    auto flush = [&](int nc) {
      {
        HSide Q;
        Q.xm = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
        Q.vh = make_float4(0.f, 0.f, 0.f, 0.f);
        Q.aux = make_float4(0.f, 0.f, 1.f, 1.f);
        Q.up = make_float4(0.f, 0.f, 0.f, 0.f);
        if (lane < nc) {
          Q.xm = xm[cand];
          Q.vh = vh[cand];
          Q.aux = aux[cand];
          Q.up = up[cand];
        }
        const float d2 = box_dist2(make_float3(Q.xm.x, Q.xm.y, Q.xm.z), tlo, thi);
        const bool keep = lane < nc && (d2 < hmax2 || d2 < sq_exact(Q.vh.w));
        const uint64_t km = __ballot(keep);
        const int slot = (int)__builtin_amdgcn_mbcnt_hi(
            (uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
        // kept candidates in their order at the front; the scan stops at nc
        if (keep) T[w][slot] = Q;
        nc = __popcll(km);
      }
      wave_sync();
      float part[kN];
#pragma unroll
      for (int k = 0; k < kN; ++k) part[k] = 0.0f;
      for (int k = 0; k < nc; ++k) {
        const HSide Q = T[w][k];
        const float dx = sub_exact(Q.xm.x, P.xm.x), dy = sub_exact(Q.xm.y, P.xm.y),
                    dz = sub_exact(Q.xm.z, P.xm.z);  // x_q - x_p
        const float r2 = dist2_exact(dx, dy, dz);
        const bool in = valid && r2 < sq_exact(fmaxf(hp, Q.vh.w)) && r2 > 0.0f;
        const bool q_on = Q.up.x != 0.f || Q.up.y != 0.f || Q.up.z != 0.f || Q.up.w != 0.f;
        if (in && (p_on || q_on)) {
          const float r = __builtin_amdgcn_sqrtf(r2);
          float d[kN];
          if (p_on) {  // target p, neighbour q: x = x_p - x_q
            hydro_pair_partials(P, Q, alpha, -dx, -dy, -dz, r, 0, d);
#pragma unroll
            for (int k = 0; k < kN; ++k) part[k] += d[k];
          }
          if (q_on) {  // target q, neighbour p: x = x_q - x_p
            hydro_pair_partials(Q, P, alpha, dx, dy, dz, r, 1, d);
#pragma unroll
            for (int k = 0; k < kN; ++k) part[k] += d[k];
          }
        }
      }
#pragma unroll
      for (int k = 0; k < kN; ++k) neumaier_add(acc[k], cmp[k], part[k]);
      wave_sync();
    };
    int cur = grp.root;
    while (cur < grp.end) {
      const Node nd = nodes[cur];
      const float hm = fmaxf(hp, nd.lo_h.w);
      const bool want = valid && box_dist2(make_float3(P.xm.x, P.xm.y, P.xm.z), nd.lo_h,
                                           nd.hi_l) < sq_exact(hm);
      if (__ballot(want) == 0ull) {
        cur = nd.meta.x;
        continue;
      }
      if (!(nd.meta.w & kLeafBit) && nd.meta.z > kTile) {
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
      float tot[kN];
#pragma unroll
      for (int k = 0; k < kN; ++k) tot[k] = acc[k] + cmp[k];
      const int cid = perm[s];
      if (g_pos) {
        g_pos[3 * cid] += tot[0];
        g_pos[3 * cid + 1] += tot[1];
        g_pos[3 * cid + 2] += tot[2];
      }
      if (g_vel) {
        g_vel[3 * cid] += tot[3];
        g_vel[3 * cid + 1] += tot[4];
        g_vel[3 * cid + 2] += tot[5];
      }
      if (g_h) g_h[cid] += tot[6];
      if (g_mass) g_mass[cid] += tot[10];
      // A = (gamma-1) u / (Omega rho): dA/du = (gamma-1)/(Omega rho),
      // dA/dOmega = -A/Omega, dA/drho = -A/rho; dc/du = c / (2u)
      const float A = P.aux.x, cc = P.aux.y, rp = P.aux.z, up_ = u[cid], om = omega[cid];
      const float gA = tot[7], gc = tot[8];
      if (g_u) g_u[cid] += gA * (gamma - 1.0f) / (om * rp) + (up_ > 0.0f ? gc * cc / (2.0f * up_) : 0.0f);
      if (g_omega) g_omega[cid] += -gA * A / om;
      if (g_rho) g_rho[cid] += -gA * A / rp + tot[9];
    }
  }
}

}  // namespace

hipError_t launch_hydro_bwd(Octree &gas, const int32_t *iperm, int64_t n_caller,
                            const Groups &all_gas, int64_t max_groups, int64_t n_act,
                            const int32_t *active, float alpha, float gamma, const float *u,
                            const float *omega, const float *g_acc, const float *g_dudt,
                            float4 *up, float *g_pos, float *g_vel, float *g_mass, float *g_h,
                            float *g_u, float *g_rho, float *g_omega, hipStream_t s) {
  const int64_t m = gas.n;
  if (m == 0) return hipSuccess;
  k_zero_f4<<<nblk(m), kBlock, 0, s>>>(up, m);
  const int64_t na = active ? n_act : n_caller;
  if (na > 0)
    k_hydro_bwd_up<<<nblk(na), kBlock, 0, s>>>(active, na, iperm, n_caller, g_acc, g_dudt, up);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_hydro_bwd<<<persistent_grid((const void *)k_hydro_bwd, kBlock, max_groups), kBlock, 0, s>>>(
      gas.nodes, gas.xm, gas.vh, gas.aux, up, gas.perm, all_gas, alpha, gamma, u, omega, g_pos,
      g_vel, g_mass, g_h, g_u, g_rho, g_omega);
  return hipGetLastError();
}

hipError_t launch_gravity_bwd(const Octree &all, const Groups &gs, int64_t max_groups,
                              const GravParams &gp, int64_t n_act, const int32_t *active,
                              const float *g_acc, const float *g_pot, float4 *gsrc,
                              float4 *gnode, unsigned long long *gsrc_fx,
                              unsigned long long *gnode_fx, unsigned *mx, double4 *pq,
                              double *rr, float *g_pos, float *g_mass, hipStream_t s) {
  const int64_t m = all.n, nn = all.nnodes;
  if (m == 0 || nn == 0) return hipSuccess;
  if (!all.gnodes) return hipErrorInvalidValue;
  const int64_t na = active ? n_act : m;
  if (gp.eps2 > 0.0f) {
    // fixed-point counters (two words per component, four components)
    k_zero_f4<<<nblk(4 * m), kBlock, 0, s>>>((float4 *)gsrc_fx, 4 * m);
    k_zero_f4<<<nblk(4 * nn), kBlock, 0, s>>>((float4 *)gnode_fx, 4 * nn);
    k_zero_f4<<<1, kBlock, 0, s>>>((float4 *)mx, 1);
    const int64_t nb = na > m ? na : m;
    const unsigned gb = nblk(nb) < (unsigned)kFxBoundBlocks ? nblk(nb) : (unsigned)kFxBoundBlocks;
    k_fx_bound<<<gb, kBlock, 0, s>>>(active, na, g_acc, g_pot, all.xm, m, mx);
    if (max_groups > 0) {
      auto kern = gp.inside_test ? k_gravity_bwd<true, true> : k_gravity_bwd<true, false>;
      kern<<<persistent_grid((const void *)kern, kBlock, max_groups), kBlock, 0, s>>>(
          all.gnodes, all.xm, all.keys, all.perm, gs, gp.theta2, gp.eps2, gp.G, g_acc, g_pot,
          gsrc, gnode, gsrc_fx, gnode_fx, mx, m, na);
    }
    k_fx_to_f4<<<nblk(m), kBlock, 0, s>>>(gsrc_fx, m, mx, gp.eps2, gp.G, m, na, gsrc);
    k_fx_to_f4<<<nblk(nn), kBlock, 0, s>>>(gnode_fx, nn, mx, gp.eps2, gp.G, m, na, gnode);
  } else {
    k_zero_f4<<<nblk(m), kBlock, 0, s>>>(gsrc, m);
    k_zero_f4<<<nblk(nn), kBlock, 0, s>>>(gnode, nn);
    if (max_groups > 0) {
      auto kern = gp.inside_test ? k_gravity_bwd<false, true> : k_gravity_bwd<false, false>;
      kern<<<persistent_grid((const void *)kern, kBlock, max_groups), kBlock, 0, s>>>(
          all.gnodes, all.xm, all.keys, all.perm, gs, gp.theta2, gp.eps2, gp.G, g_acc, g_pot,
          gsrc, gnode, nullptr, nullptr, nullptr, m, na);
    }
  }
  k_push_init<<<nblk(nn), kBlock, 0, s>>>(gnode, all.mom, nn, pq, rr);
  for (int l = 0; l < all.max_level; ++l)
    k_push_level<<<nblk(nn), kBlock, 0, s>>>(all.nodes, all.mom, nn, l, pq, rr);
  k_push_leaves<<<nblk(nn), kBlock, 0, s>>>(all.nodes, all.mom, nn, all.xm, pq, rr, gsrc);
  k_scatter_grad<<<nblk(m), kBlock, 0, s>>>(all.perm, m, gsrc, g_pos, g_mass);
  return hipGetLastError();
}

hipError_t launch_density_bwd(Octree &gas, const int32_t *iperm, int64_t n_caller,
                              const Groups &all_gas, int64_t max_groups, int64_t n_act,
                              const int32_t *active, const float *h, const float *rho,
                              const float *drho, const float *g_rho, const float *g_drho,
                              const float *g_omega, float *g_pos, float *g_mass, float *g_h,
                              hipStream_t s) {
  const int64_t m = gas.n;
  if (m == 0) return hipSuccess;
  float4 *bw = gas.aux;  // (h, gbar_rho, gbar_rho', 0) per sorted gas member
  k_density_bwd_init<<<nblk(m), kBlock, 0, s>>>(gas.perm, m, h, bw);
  const int64_t na = active ? n_act : n_caller;
  if (na > 0)
    k_density_bwd_prep<<<nblk(na), kBlock, 0, s>>>(active, na, iperm, n_caller, h, rho, drho,
                                                    g_rho, g_drho, g_omega, bw, g_h);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_density_bwd<<<persistent_grid((const void *)k_density_bwd, kBlock, max_groups), kBlock, 0,
                  s>>>(gas.nodes, gas.xm, bw, gas.perm, all_gas, g_pos, g_mass, g_h);
  return hipGetLastError();
}

hipError_t launch_density_solve_bwd(Octree &gas, const int32_t *iperm, int64_t n_caller,
                                    const Groups &all_gas, int64_t max_groups, int64_t n_act,
                                    const int32_t *active, float n_ngb, const float *h,
                                    const float *rho, const float *drho, const float *g_h,
                                    float *g_pos, float *g_mass, hipStream_t s) {
  const int64_t m = gas.n;
  if (m == 0) return hipSuccess;
  float4 *bw = gas.aux;  // (h, gbar_rho, 0, 0) per sorted gas member
  k_density_bwd_init<<<nblk(m), kBlock, 0, s>>>(gas.perm, m, h, bw);
  const int64_t na = active ? n_act : n_caller;
  if (na > 0)
    k_hsolve_bwd_prep<<<nblk(na), kBlock, 0, s>>>(active, na, iperm, n_caller, h, rho, drho, g_h,
                                                   gas.xm, n_ngb, bw, g_mass);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_density_bwd<<<persistent_grid((const void *)k_density_bwd, kBlock, max_groups), kBlock, 0,
                  s>>>(gas.nodes, gas.xm, bw, gas.perm, all_gas, g_pos, g_mass, nullptr);
  return hipGetLastError();
}

}  // namespace g3
