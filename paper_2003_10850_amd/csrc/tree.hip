// Octree build on the GPU: Morton keys, radix sort, permutation into sorted
// float4 arrays, preorder topology computed per particle without recursion,
// and bottom-up FP64 monopoles with tight bounding boxes.
//
// Topology (Barnes & Hut 1986 octree over Morton-sorted members): a node is
// the run of members sharing a 3l-bit key prefix; it is split while it holds
// more than B members and l < 21. Write cpl(a, b) for the number of leading
// 3-bit digits two keys share. Member p starts a node at level l exactly
// when l >= delta_p = cpl(p, p-1) + 1 (delta_0 = 0), and the deepest node
// holding p (its leaf) is at depth d_p = 1 + the B-th largest of
// cpl(p, p +- k), k = 1..B (missing neighbours count -1), capped at 21.
// So p starts the nodes of levels delta_p..d_p, and in preorder (children in
// Morton order) the nodes sorted by (first member, level) are numbered by an
// exclusive scan of the per-member counts. The node after the subtree of a
// node ending before member e is the first node that starts at e.
#include <algorithm>
#include <utility>

#include "g3_device.h"
#include "g3_internal.h"

namespace g3 {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

// key cell in FP64 for FP32 and FP64 positions alike
template <typename T>
__device__ __forceinline__ uint32_t cell_of(T x, double lo, double scale) {
  double f = floor(((double)x - lo) * scale);
  if (!(f >= 0.0)) f = 0.0;
  if (f > (double)((1u << kMaxLevel) - 1u)) f = (double)((1u << kMaxLevel) - 1u);
  return (uint32_t)f;
}

template <typename T>
__device__ __forceinline__ uint64_t morton_key(const T *p, double lx, double ly, double lz,
                                               double scale) {
  return (spread3(cell_of(p[0], lx, scale)) << 2) | (spread3(cell_of(p[1], ly, scale)) << 1) |
         spread3(cell_of(p[2], lz, scale));
}

// keys and identity values for the members selected by sel (nullptr: all),
// each keyed in the box of its snapshot (caller ids [coff[k], coff[k+1]))
template <typename T>
__global__ void k_keys(const T *__restrict__ pos, const int32_t *__restrict__ sel,
                       int64_t m, const int64_t *__restrict__ coff,
                       const double4 *__restrict__ sbox, int n_snap,
                       uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const int64_t i = sel ? sel[k] : k;
  const double4 b = sbox[n_snap > 1 ? segment_of(coff, n_snap, i) : 0];
  const double scale = 2097152.0 / b.w;  // 2^21 / side
  keys[k] = morton_key(pos + 3 * i, b.x, b.y, b.z, scale);
  vals[k] = (uint32_t)i;
}

// Forest: the snapshot of each key-sorted member, for a stable sort by
// snapshot after the sort by key.
__global__ void k_snap_keys(const uint32_t *__restrict__ vals, int64_t m,
                            const int64_t *__restrict__ coff, int n_snap,
                            uint64_t *__restrict__ skey, uint32_t *__restrict__ sidx) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  skey[k] = (uint64_t)segment_of(coff, n_snap, (int64_t)vals[k]);
  sidx[k] = (uint32_t)k;
}

__global__ void k_gather_sorted(const uint32_t *__restrict__ sidx, int64_t m,
                                const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                uint64_t *__restrict__ kout, uint32_t *__restrict__ vout) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const uint32_t j = sidx[k];
  kout[k] = kin[j];
  vout[k] = vin[j];
}

// Sorted start of each snapshot: slot[coff[k]] (members before coff[k]
// selected by the exclusive scan `slot`), or coff[k] when all are members.
__global__ void k_soff(const int64_t *__restrict__ coff, int n_snap,
                       const uint32_t *__restrict__ slot, int32_t *__restrict__ soff) {
  const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (k > n_snap) return;
  soff[k] = slot ? (int32_t)slot[coff[k]] : (int32_t)coff[k];
}

// First node of each snapshot: the first node its first member starts.
__global__ void k_nroot(const uint32_t *__restrict__ off, const int32_t *__restrict__ soff,
                        int n_snap, int32_t *__restrict__ nroot) {
  const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (k > n_snap) return;
  nroot[k] = (int32_t)off[soff[k]];
}

__global__ void k_gas_flags(const uint8_t *__restrict__ type, int64_t n,
                            uint32_t *__restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flags[i] = (type == nullptr || type[i] == 0) ? 1u : 0u;
}

// The gas octree's members in sorted order come from the all-particle
// octree's: filtering its (snapshot, key, caller id) order keeps that order,
// which is exactly the order a sort of the gas members would give.
__global__ void k_gas_of_sorted(const int32_t *__restrict__ perm_all, int64_t n,
                                const uint8_t *__restrict__ type, uint32_t *__restrict__ flags) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) flags[s] = (type == nullptr || type[perm_all[s]] == 0) ? 1u : 0u;
}

__global__ void k_compact_sorted(const uint32_t *__restrict__ flags,
                                 const uint32_t *__restrict__ slot, int64_t n,
                                 const uint64_t *__restrict__ keys_all,
                                 const int32_t *__restrict__ perm_all,
                                 uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n || !flags[s]) return;
  keys[slot[s]] = keys_all[s];
  vals[slot[s]] = (uint32_t)perm_all[s];
}

// Sorted copies: FP32 (x, y, z, m) always; for FP64 positions also the
// exact (x, y, z, m) in FP64.
template <typename T>
__global__ void k_permute(const uint32_t *__restrict__ perm, int64_t m,
                          const T *__restrict__ pos, const float *__restrict__ mass,
                          float4 *__restrict__ xm, double4 *__restrict__ x64,
                          int32_t *__restrict__ iperm) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= m) return;
  const uint32_t j = perm[s];
  xm[s] = make_float4((float)pos[3 * j], (float)pos[3 * j + 1], (float)pos[3 * j + 2], mass[j]);
  if (x64)
    x64[s] = make_double4((double)pos[3 * j], (double)pos[3 * j + 1], (double)pos[3 * j + 2],
                          (double)mass[j]);
  iperm[j] = (int32_t)s;
}

__device__ __forceinline__ int cpl(uint64_t a, uint64_t b) {
  const uint64_t x = a ^ b;
  if (x == 0) return kMaxLevel;
  return (__clzll((long long)x) - 1) / 3;  // bit 63 is never used
}

// nodes started by each member: cnt[p] = max(0, d_p - delta_p + 1)
constexpr int kMaxLeaf = 64;

__global__ __launch_bounds__(kBlock) void k_node_counts(const uint64_t *__restrict__ keys,
                                                        int64_t m,
                                                        const int32_t *__restrict__ soff,
                                                        int n_snap, int B,
                                                        uint32_t *__restrict__ cnt,
                                                        uint8_t *__restrict__ lev,
                                                        int32_t *__restrict__ maxlev) {
  // the block's keys with B neighbours on each side, staged in LDS
  __shared__ uint64_t win[kBlock + 2 * kMaxLeaf];
  __shared__ int32_t block_max;  // deepest leaf level of the block
  if (threadIdx.x == 0) block_max = 0;
  const int64_t b0 = (int64_t)blockIdx.x * kBlock;
  for (int k = threadIdx.x; k < kBlock + 2 * B; k += kBlock) {
    const int64_t q = b0 - B + k;
    win[k] = (q >= 0 && q < m) ? keys[q] : 0ull;
  }
  __syncthreads();
  const int64_t p = b0 + threadIdx.x;
  if (p < m) {
  const uint64_t *kw = win + B + threadIdx.x;  // kw[d] = key of member p + d
  const uint64_t kp = kw[0];
  // members of other snapshots count as missing: each snapshot is a tree
  const int sn = n_snap > 1 ? segment_of(soff, n_snap, p) : 0;
  const int64_t s0 = soff[sn], s1 = soff[sn + 1];
  const int delta = (p == s0) ? 0 : cpl(kp, kw[-1]) + 1;
  // B-th largest of the window prefix lengths: merge two non-increasing runs
  int i = 1, j = 1;
  int val = -1;
  int a = (p - 1 >= s0) ? cpl(kp, kw[-1]) : -1;
  int b = (p + 1 < s1) ? cpl(kp, kw[1]) : -1;
  for (int step = 0; step < B; ++step) {
    if (a >= b) {
      val = a;
      ++i;
      a = (p - i >= s0 && i <= B) ? cpl(kp, kw[-i]) : -1;
    } else {
      val = b;
      ++j;
      b = (p + j < s1 && j <= B) ? cpl(kp, kw[j]) : -1;
    }
  }
  int d = val + 1;
  if (d > kMaxLevel) d = kMaxLevel;
  cnt[p] = (d >= delta) ? (uint32_t)(d - delta + 1) : 0u;
  lev[2 * p] = (uint8_t)delta;
  lev[2 * p + 1] = (uint8_t)d;
  // one device atomic per block: many members start nodes, and atomics on
  // a single address serialise
  if (d >= delta) atomicMax(&block_max, d);
  }
  __syncthreads();
  if (threadIdx.x == 0 && block_max > 0) atomicMax(maxlev, block_max);
}

__global__ void k_nodes(const uint64_t *__restrict__ keys, int64_t m,
                        const int32_t *__restrict__ soff, int n_snap,
                        const double4 *__restrict__ sbox,
                        const uint32_t *__restrict__ off, const uint8_t *__restrict__ lev,
                        int64_t nnodes, Node *__restrict__ nodes) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m) return;
  const int delta = lev[2 * p], d = lev[2 * p + 1];
  if (d < delta) return;
  const uint64_t kp = keys[p];
  const int sn = n_snap > 1 ? segment_of(soff, n_snap, p) : 0;
  const float side = (float)sbox[sn].w;
  int64_t end = soff[sn + 1];  // members of the level-l node: [p, end)
  for (int l = delta; l <= d; ++l) {
    // first q in (p, end] with cpl(p, q) < l (end shrinks as l grows)
    int64_t lo = p + 1, hi = end;  // answer in [lo, hi]
    int64_t step = 1;
    while (lo + step - 1 < hi && cpl(kp, keys[lo + step - 1]) >= l) {
      lo += step;
      step <<= 1;
    }
    if (lo + step - 1 < hi) hi = lo + step - 1;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (cpl(kp, keys[mid]) >= l) lo = mid + 1;
      else hi = mid;
    }
    end = lo;
    const int64_t idx = (int64_t)off[p] + (l - delta);
    const int64_t skip = (end >= m) ? nnodes : (int64_t)off[end];
    Node nd;
    nd.com_m = make_float4(0.f, 0.f, 0.f, 0.f);
    nd.lo_h = make_float4(0.f, 0.f, 0.f, 0.f);
    nd.hi_l = make_float4(0.f, 0.f, 0.f, ldexpf(side, -l));
    nd.meta = make_int4((int)skip, (int)p, (int)(end - p), l | (l == d ? kLeafBit : 0));
    nodes[idx] = nd;
  }
}

// Bottom-up pass for one level: FP64 mass and first moments, tight box.
__global__ void k_moments_level(Node *__restrict__ nodes, double4 *__restrict__ mom,
                                double4 *__restrict__ c64, int64_t nnodes,
                                const float4 *__restrict__ xm,
                                const double4 *__restrict__ x64, int level) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnodes) return;
  const int4 meta = nodes[k].meta;
  if ((meta.w & 255) != level) return;
  double M = 0.0, Sx = 0.0, Sy = 0.0, Sz = 0.0;
  float4 lo = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
  float4 hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.f);
  if (meta.w & kLeafBit) {
    for (int s = meta.y; s < meta.y + meta.z; ++s) {
      const float4 p = xm[s];
      // moments from the exact positions (FP64 ones when the tree has them)
      const double4 q = x64 ? x64[s] : make_double4(p.x, p.y, p.z, p.w);
      M += q.w;
      Sx += q.w * q.x;
      Sy += q.w * q.y;
      Sz += q.w * q.z;
      lo.x = fminf(lo.x, p.x); lo.y = fminf(lo.y, p.y); lo.z = fminf(lo.z, p.z);
      hi.x = fmaxf(hi.x, p.x); hi.y = fmaxf(hi.y, p.y); hi.z = fmaxf(hi.z, p.z);
    }
  } else {
    int64_t c = k + 1;
    while (c < meta.x) {
      const double4 cm = mom[c];
      const float4 clo = nodes[c].lo_h, chi = nodes[c].hi_l;
      M += cm.x;
      Sx += cm.y;
      Sy += cm.z;
      Sz += cm.w;
      lo.x = fminf(lo.x, clo.x); lo.y = fminf(lo.y, clo.y); lo.z = fminf(lo.z, clo.z);
      hi.x = fmaxf(hi.x, chi.x); hi.y = fmaxf(hi.y, chi.y); hi.z = fmaxf(hi.z, chi.z);
      c = nodes[c].meta.x;
    }
  }
  mom[k] = make_double4(M, Sx, Sy, Sz);
  Node &nd = nodes[k];
  if (M > 0.0)
    nd.com_m = make_float4((float)(Sx / M), (float)(Sy / M), (float)(Sz / M), (float)M);
  else  // massless node: its geometric centre
    nd.com_m = make_float4(0.5f * (lo.x + hi.x), 0.5f * (lo.y + hi.y), 0.5f * (lo.z + hi.z), 0.f);
  if (c64)
    c64[k] = M > 0.0 ? make_double4(Sx / M, Sy / M, Sz / M, M)
                     : make_double4(nd.com_m.x, nd.com_m.y, nd.com_m.z, 0.0);
  lo.w = nd.lo_h.w;
  hi.w = nd.hi_l.w;
  nd.lo_h = lo;
  nd.hi_l = hi;
}

// Bottom-up pass for one level: maximum h of the members (vh.w).
__global__ void k_hmax_level(Node *__restrict__ nodes, int64_t nnodes,
                             const float4 *__restrict__ vh, int level) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnodes) return;
  const int4 meta = nodes[k].meta;
  if ((meta.w & 255) != level) return;
  float hm = 0.f;
  if (meta.w & kLeafBit) {
    for (int s = meta.y; s < meta.y + meta.z; ++s) hm = fmaxf(hm, vh[s].w);
  } else {
    int64_t c = k + 1;
    while (c < meta.x) {
      hm = fmaxf(hm, nodes[c].lo_h.w);
      c = nodes[c].meta.x;
    }
  }
  nodes[k].lo_h.w = hm;
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// The largest |coordinate| of the FP64 positions, as float bits (the FP32
// rounding upwards keeps it an upper bound); *out must start at zero. A
// grid-stride loop with one atomic per block: a few thousand atomics on the
// one word instead of one per wave.
constexpr int kAbsmaxBlocks = 2048;
__global__ __launch_bounds__(kBlock) void k_absmax(const double4 *__restrict__ x64, int64_t n,
                                                   unsigned *__restrict__ out) {
  __shared__ float part[kBlock / kWave];
  float m = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double4 v = x64[i];
    const double a = fmax(fabs(v.x), fmax(fabs(v.y), fabs(v.z)));
    float f = (float)a;
    if ((double)f < a) f = nextafterf(f, INFINITY);
    m = fmaxf(m, f);
  }
#pragma unroll
  for (int k = 1; k < kWave; k <<= 1) m = fmaxf(m, __shfl_xor(m, k));
  if ((threadIdx.x & 63u) == 0u) part[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / kWave; ++w) m = fmaxf(m, part[w]);
    if (m > 0.0f) atomicMax(out, __float_as_uint(m));
  }
}

__global__ void k_zero_one(unsigned *p) {
  if (threadIdx.x == 0) *p = 0u;
}

// The gravity walk's 32-byte node copies (after the moments).
__global__ void k_gnodes(const Node *__restrict__ nodes, int64_t nnodes,
                         GNode *__restrict__ gnodes) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnodes) return;
  const Node nd = nodes[k];
  GNode g;
  g.com_m = nd.com_m;
  g.meta = make_int4(nd.meta.x, nd.meta.y, (nd.meta.w & kLeafBit) ? nd.meta.z : -1,
                     __float_as_int(nd.hi_l.w));
  gnodes[k] = g;
}

}  // namespace

// Selects the members (gas only for the gas octree), sorts them and builds
// the topology and moments. SYNCS once to read the node count.
int build_octree(g3_ctx *c, g3_tree *t, Octree &o, const void *pos, int f64,
                 const float *mass, int64_t m, hipStream_t s, const uint8_t *type) {
  o.n = m;
  o.nnodes = 0;
  o.max_level = 0;
  if (m == 0) {  // no members: every snapshot's node range is empty
    const hipError_t e = fill_i32(o.nroot, 0, t->n_snap + 1, s);
    if (e != hipSuccess) { c->err = "fill launch failed"; return G3_EHIP; }
    return G3_OK;
  }
  if (f64 && (!o.x64 || o.cap_x64 < m)) {
    if (o.x64) (void)hipFree(o.x64);
    o.x64 = nullptr;
    o.cap_x64 = 0;
    if (dev_malloc(c, (void **)&o.x64, m * sizeof(double4)) != hipSuccess) {
      c->err = "device allocation of the FP64 positions failed";
      return G3_ENOMEM;
    }
    o.cap_x64 = m;
  }
  double4 *x64 = f64 ? o.x64 : nullptr;
  if (m > o.cap_n) {
    for (void *p : {(void *)o.keys, (void *)o.perm, (void *)o.xm, (void *)o.vh, (void *)o.aux})
      if (p) (void)hipFree(p);
    o.keys = nullptr; o.perm = nullptr; o.xm = nullptr; o.vh = nullptr; o.aux = nullptr;
    o.cap_n = 0;
    if (dev_malloc(c, (void **)&o.keys, m * sizeof(uint64_t)) != hipSuccess ||
        dev_malloc(c, (void **)&o.perm, m * sizeof(int32_t)) != hipSuccess ||
        dev_malloc(c, (void **)&o.xm, m * sizeof(float4)) != hipSuccess ||
        dev_malloc(c, (void **)&o.vh, m * sizeof(float4)) != hipSuccess ||
        dev_malloc(c, (void **)&o.aux, m * sizeof(float4)) != hipSuccess) {
      c->err = "device allocation of the sorted particle arrays failed";
      return G3_ENOMEM;
    }
    o.cap_n = m;
  }
  uint64_t *kalt = (uint64_t *)scratch(c, kSortKeys, m * sizeof(uint64_t));
  uint32_t *valt = (uint32_t *)scratch(c, kSortVals, m * sizeof(uint32_t));
  void *rtmp = scratch(c, kSortTmp, radix_tmp_bytes(m));
  uint32_t *vals = (uint32_t *)scratch(c, kIds, m * sizeof(uint32_t));
  uint32_t *cnt = (uint32_t *)scratch(c, kCounts, (m + 1) * sizeof(uint32_t));
  uint32_t *off = (uint32_t *)scratch(c, kOffsets, (m + 1) * sizeof(uint32_t));
  uint8_t *lev = (uint8_t *)scratch(c, kLevel, 2 * m);
  uint32_t *stmp = (uint32_t *)scratch(c, kScanTmp, scan_tmp_elems(m) * sizeof(uint32_t));
  int32_t *maxlev = (int32_t *)scratch(c, kMisc, 64);
  if (!kalt || !valt || !rtmp || !vals || !cnt || !off || !lev || !stmp || !maxlev) {
    c->err = "device allocation of build scratch failed";
    return G3_ENOMEM;
  }
  const bool gas = (&o == &t->gas);
  hipError_t e;
  if (gas) {
    // filter the all-particle octree's sorted members (built just before)
    const int64_t n = t->n;
    uint32_t *flags = (uint32_t *)scratch(c, kGasFlags, (n + 1) * sizeof(uint32_t));
    uint32_t *slot = (uint32_t *)scratch(c, kGasSlot, (n + 1) * sizeof(uint32_t));
    uint32_t *stmp2 = (uint32_t *)scratch(c, kGasScan, scan_tmp_elems(n) * sizeof(uint32_t));
    if (!flags || !slot || !stmp2) { c->err = "device allocation of build scratch failed"; return G3_ENOMEM; }
    k_gas_of_sorted<<<nblk(n), kBlock, 0, s>>>(t->all.perm, n, type, flags);
    e = scan_u32(flags, slot, n, stmp2, s);
    if (e != hipSuccess) { c->err = "scan launch failed"; return G3_EHIP; }
    k_compact_sorted<<<nblk(n), kBlock, 0, s>>>(flags, slot, n, t->all.keys, t->all.perm, o.keys,
                                                 vals);
  } else {
    if (f64)
      k_keys<double><<<nblk(m), kBlock, 0, s>>>((const double *)pos, nullptr, m, t->coff, t->sbox,
                                                t->n_snap, o.keys, vals);
    else
      k_keys<float><<<nblk(m), kBlock, 0, s>>>((const float *)pos, nullptr, m, t->coff, t->sbox,
                                               t->n_snap, o.keys, vals);
    e = radix_sort_pairs(o.keys, vals, kalt, valt, m, 64, rtmp, s);
    if (e != hipSuccess) { c->err = "radix sort launch failed"; return G3_EHIP; }
    if (t->n_snap > 1) {
      // stable sort of the key-sorted members by snapshot: (snapshot, key) order
      uint64_t *skey = (uint64_t *)scratch(c, kSnapKeys, 2 * m * sizeof(uint64_t));
      uint64_t *skey_alt = (uint64_t *)scratch(c, kSnapKeysAlt, m * sizeof(uint64_t));
      if (!skey || !skey_alt) { c->err = "device allocation of build scratch failed"; return G3_ENOMEM; }
      uint32_t *sidx = (uint32_t *)(skey + m);
      int bits = 8;
      while (bits < 32 && (int64_t(1) << bits) < t->n_snap) bits += 8;
      k_snap_keys<<<nblk(m), kBlock, 0, s>>>(vals, m, t->coff, t->n_snap, skey, sidx);
      e = radix_sort_pairs(skey, sidx, skey_alt, cnt, m, bits, rtmp, s);
      if (e != hipSuccess) { c->err = "radix sort launch failed"; return G3_EHIP; }
      k_gather_sorted<<<nblk(m), kBlock, 0, s>>>(sidx, m, o.keys, vals, kalt, valt);
      e = hipMemcpyAsync(o.keys, kalt, m * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(vals, valt, m * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) { c->err = "snapshot sort copy failed"; return G3_EHIP; }
    }
  }
  int32_t *iperm = gas ? t->iperm_gas : t->iperm_all;
  if (f64)
    k_permute<double><<<nblk(m), kBlock, 0, s>>>(vals, m, (const double *)pos, mass, o.xm, x64,
                                                 iperm);
  else
    k_permute<float><<<nblk(m), kBlock, 0, s>>>(vals, m, (const float *)pos, mass, o.xm, nullptr,
                                                iperm);
  e = hipMemcpyAsync(o.perm, vals, m * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) { c->err = "perm copy failed"; return G3_EHIP; }
  e = fill_i32(maxlev, 0, 1, s);
  if (e != hipSuccess) { c->err = "fill launch failed"; return G3_EHIP; }
  k_node_counts<<<nblk(m), kBlock, 0, s>>>(o.keys, m, o.soff, t->n_snap, t->leaf, cnt, lev,
                                           maxlev);
  e = scan_u32(cnt, off, m, stmp, s);
  if (e != hipSuccess) { c->err = "scan launch failed"; return G3_EHIP; }
  int64_t *pin = c->pinned;
  e = hipMemcpyAsync(&pin[0], off + m, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&pin[1], maxlev, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) { c->err = std::string("node count readback: ") + hipGetErrorString(e); return G3_EHIP; }
  const int64_t nnodes = (int64_t)(uint32_t)(pin[0] & 0xffffffffll);
  const int32_t maxl = (int32_t)(pin[1] & 0xffffffffll);
  if (nnodes <= 0 || nnodes >= (int64_t)INT32_MAX) { c->err = "node count out of range"; return G3_EHIP; }
  const bool grav = (&o == &t->all);
  if (nnodes > o.cap_nodes || (grav && !o.gnodes)) {
    if (o.nodes) (void)hipFree(o.nodes);
    if (o.mom) (void)hipFree(o.mom);
    if (o.gnodes) (void)hipFree(o.gnodes);
    o.nodes = nullptr; o.mom = nullptr; o.gnodes = nullptr; o.cap_nodes = 0;
    const int64_t cap = nnodes + nnodes / 8 + 64;
    if (dev_malloc(c, (void **)&o.nodes, cap * sizeof(Node)) != hipSuccess ||
        dev_malloc(c, (void **)&o.mom, cap * sizeof(double4)) != hipSuccess ||
        (grav && dev_malloc(c, (void **)&o.gnodes, cap * sizeof(GNode)) != hipSuccess)) {
      c->err = "device allocation of the octree nodes failed";
      return G3_ENOMEM;
    }
    o.cap_nodes = cap;
  }
  if (f64 && (!o.c64 || o.cap_c64 < nnodes)) {
    if (o.c64) (void)hipFree(o.c64);
    o.c64 = nullptr;
    o.cap_c64 = 0;
    const int64_t cap = nnodes + nnodes / 8 + 64;
    if (dev_malloc(c, (void **)&o.c64, cap * sizeof(double4)) != hipSuccess) {
      c->err = "device allocation of the FP64 node centres failed";
      return G3_ENOMEM;
    }
    o.cap_c64 = cap;
  }
  o.nnodes = nnodes;
  o.max_level = maxl;
  k_nodes<<<nblk(m), kBlock, 0, s>>>(o.keys, m, o.soff, t->n_snap, t->sbox, off, lev, nnodes,
                                     o.nodes);
  k_nroot<<<nblk(t->n_snap + 1), kBlock, 0, s>>>(off, o.soff, t->n_snap, o.nroot);
  for (int l = maxl; l >= 0; --l)
    k_moments_level<<<nblk(nnodes), kBlock, 0, s>>>(o.nodes, o.mom, f64 ? o.c64 : nullptr,
                                                     nnodes, o.xm, x64, l);
  if (o.gnodes) k_gnodes<<<nblk(nnodes), kBlock, 0, s>>>(o.nodes, nnodes, o.gnodes);
  e = hipGetLastError();
  if (e != hipSuccess) { c->err = std::string("tree build launch: ") + hipGetErrorString(e); return G3_EHIP; }
  return G3_OK;
}

int refit_octree(g3_ctx *c, g3_tree *t, Octree &o, const void *pos, const float *mass,
                 hipStream_t s) {
  if (o.n == 0 || o.nnodes == 0) return G3_OK;
  const bool gas = (&o == &t->gas);
  int32_t *iperm = gas ? t->iperm_gas : t->iperm_all;
  const uint32_t *order = (const uint32_t *)o.perm;
  if (t->f64)
    k_permute<double><<<nblk(o.n), kBlock, 0, s>>>(order, o.n, (const double *)pos, mass, o.xm,
                                                   o.x64, iperm);
  else
    k_permute<float><<<nblk(o.n), kBlock, 0, s>>>(order, o.n, (const float *)pos, mass, o.xm,
                                                  nullptr, iperm);
  for (int l = o.max_level; l >= 0; --l)
    k_moments_level<<<nblk(o.nnodes), kBlock, 0, s>>>(o.nodes, o.mom, t->f64 ? o.c64 : nullptr,
                                                       o.nnodes, o.xm, t->f64 ? o.x64 : nullptr,
                                                       l);
  if (o.gnodes) k_gnodes<<<nblk(o.nnodes), kBlock, 0, s>>>(o.nodes, o.nnodes, o.gnodes);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    c->err = std::string("tree refit launch: ") + hipGetErrorString(e);
    return G3_EHIP;
  }
  return G3_OK;
}

hipError_t update_absmax(g3_tree *t, hipStream_t s) {
  if (!t->f64 || !t->absmax) return hipSuccess;
  k_zero_one<<<1, 64, 0, s>>>(t->absmax);
  if (t->all.n > 0) {
    const unsigned nb = (unsigned)std::min<int64_t>(nblk(t->all.n), kAbsmaxBlocks);
    k_absmax<<<nb, kBlock, 0, s>>>(t->all.x64, t->all.n, t->absmax);
  }
  return hipGetLastError();
}

hipError_t refit_hmax(Octree &o, hipStream_t s) {
  for (int l = o.max_level; l >= 0 && o.nnodes > 0; --l)
    k_hmax_level<<<nblk(o.nnodes), kBlock, 0, s>>>(o.nodes, o.nnodes, o.vh, l);
  return hipGetLastError();
}

// Gas member count and the sorted start of each snapshot in the gas
// octree; returns the count (SYNCS to read it).
// The all-particle octree's snapshot starts are the caller offsets.
int select_members(g3_ctx *c, g3_tree *t, const uint8_t *type, int64_t *m_out, hipStream_t s) {
  const int64_t n = t->n;
  const unsigned sb = nblk(t->n_snap + 1);
  k_soff<<<sb, kBlock, 0, s>>>(t->coff, t->n_snap, nullptr, t->all.soff);
  if (!type) {
    k_soff<<<sb, kBlock, 0, s>>>(t->coff, t->n_snap, nullptr, t->gas.soff);
    *m_out = n;
    return G3_OK;
  }
  uint32_t *flags = (uint32_t *)scratch(c, kCounts, (n + 1) * sizeof(uint32_t));
  uint32_t *slot = (uint32_t *)scratch(c, kOffsets, (n + 1) * sizeof(uint32_t));
  uint32_t *stmp = (uint32_t *)scratch(c, kScanTmp, scan_tmp_elems(n) * sizeof(uint32_t));
  if (!flags || !slot || !stmp) { c->err = "device allocation failed"; return G3_ENOMEM; }
  k_gas_flags<<<nblk(n), kBlock, 0, s>>>(type, n, flags);
  hipError_t e = scan_u32(flags, slot, n, stmp, s);
  if (e != hipSuccess) { c->err = "scan launch failed"; return G3_EHIP; }
  k_soff<<<sb, kBlock, 0, s>>>(t->coff, t->n_snap, slot, t->gas.soff);
  e = hipMemcpyAsync(&c->pinned[2], slot + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) { c->err = std::string("gas count readback: ") + hipGetErrorString(e); return G3_EHIP; }
  *m_out = (int64_t)(uint32_t)(c->pinned[2] & 0xffffffffll);
  return G3_OK;
}

}  // namespace g3
