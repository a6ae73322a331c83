// The C ABI of libg3.so (declared in include/g3.h): argument checks, device
// selection, scratch management and the order of the launches of each call.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "g3_device.h"
#include "g3_internal.h"

namespace g3 {

// A roctx range around each interaction and build call, named after the
// entry point: a timeline under rocprofv3 --marker-trace shows every C-ABI
// call with the kernels it launched (a no-op when no profiler listens).
struct RocTxRange {
  explicit RocTxRange(const char *name) { roctxRangePush(name); }
  ~RocTxRange() { roctxRangePop(); }
  RocTxRange(const RocTxRange &) = delete;
  RocTxRange &operator=(const RocTxRange &) = delete;
};
#define G3_RANGE(name) const ::g3::RocTxRange g3_range_(name)

int select_members(g3_ctx *c, g3_tree *t, const uint8_t *type, int64_t *m_out, hipStream_t s);

hipError_t dev_malloc(g3_ctx *c, void **p, size_t bytes) {
  *p = nullptr;
  if (c->alloc_budget == 0) return hipErrorOutOfMemory;
  if (c->alloc_budget > 0) --c->alloc_budget;
  const hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) *p = nullptr;
  return e;
}

void *scratch(g3_ctx *c, int slot, size_t bytes) {
  g3_ctx::Buf &b = c->scratch[slot + c->bank * g3_ctx::kBankSlots];
  if (b.p && bytes <= b.bytes) return b.p;
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
  const size_t want = bytes + bytes / 4 + 256;
  if (dev_malloc(c, &b.p, want) != hipSuccess) return nullptr;
  b.bytes = want;
  return b.p;
}

void *scratch_in(g3_ctx *c, Arena *a, int slot, size_t bytes) {
  if (!a) return scratch(c, slot, bytes);
  if (a->slot_p[slot]) return bytes <= a->slot_bytes[slot] ? a->slot_p[slot] : nullptr;
  const size_t start = (a->used + 255) & ~(size_t)255;
  if (start > a->cap || bytes > a->cap - start) return nullptr;
  a->used = start + bytes;
  a->slot_p[slot] = a->base + start;
  a->slot_bytes[slot] = bytes;
  return a->slot_p[slot];
}

namespace {

struct DeviceGuard {
  int prev = -1, want;
  explicit DeviceGuard(int d) : want(d) {
    if (hipGetDevice(&prev) == hipSuccess && prev != d) (void)hipSetDevice(d);
  }
  ~DeviceGuard() {
    if (prev >= 0 && prev != want) (void)hipSetDevice(prev);
  }
};

int fail(g3_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(g3_ctx *c, hipError_t e, const char *where) {
  return fail(c, G3_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Clear a pending runtime error from earlier asynchronous work.
int check_pending(g3_ctx *c) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, "earlier device error");
  return G3_OK;
}

// Records the start event of a timed interaction kernel on construction
// and its stop event at stop(); does nothing unless timing is on for the
// kind, the ring has room and the stream is not being captured. A pair
// counts only once stopped (a call whose launch failed leaves its start
// event to be recorded again by the next call).
struct KernelTimer {
  g3_ctx::Timing *tm = nullptr;
  hipStream_t s = nullptr;
  int slot = -1;
  KernelTimer(g3_ctx *c, int kind, hipStream_t stream) : s(stream) {
    g3_ctx::Timing &t = c->timing[kind];
    if (t.capacity == 0 || t.count >= t.capacity) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
      (void)hipGetLastError();
      return;
    }
    if (hipEventRecord(t.ev[2 * t.count], s) != hipSuccess) {
      (void)hipGetLastError();
      return;
    }
    tm = &t;
    slot = t.count;
  }
  void stop() {
    if (!tm) return;
    if (hipEventRecord(tm->ev[2 * slot + 1], s) == hipSuccess) tm->count = slot + 1;
    else (void)hipGetLastError();
    tm = nullptr;
  }
};

bool params_ok(const g3_params *p) {
  return p && p->leaf_size >= 1 && p->leaf_size <= 64 && p->flags == 0 &&
         std::isfinite(p->theta) && p->theta >= 0.0 && std::isfinite(p->eps) &&
         p->eps >= 0.0 && std::isfinite(p->G);
}

__global__ void k_mark(const int32_t *__restrict__ active, int64_t n_act,
                       const int32_t *__restrict__ iperm, int64_t n_caller,
                       uint32_t *__restrict__ mark, int32_t *__restrict__ rowp1) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_act) return;
  const int32_t id = active[a];
  if (id < 0 || (int64_t)id >= n_caller) return;
  const int32_t s = iperm[id];
  if (s < 0) return;
  mark[s] = 1u;
  rowp1[s] = (int32_t)(a + 1);
}

// Targets by the time-bin rule: member s is a target iff the bin of its
// particle is at least kmin (rows are then caller ids).
__global__ void k_mark_bins(const int32_t *__restrict__ perm, int64_t m,
                            const int32_t *__restrict__ bins, int32_t kmin,
                            uint32_t *__restrict__ mark, int32_t *__restrict__ rowp1) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= m) return;
  const int32_t cid = perm[s];
  mark[s] = bins[cid] >= kmin ? 1u : 0u;
  rowp1[s] = cid + 1;
}

__global__ void k_compact(const uint32_t *__restrict__ mark, const uint32_t *__restrict__ slot,
                          const int32_t *__restrict__ rowp1, int64_t m,
                          int32_t *__restrict__ targets, int32_t *__restrict__ rows) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= m || !mark[s]) return;
  targets[slot[s]] = (int32_t)s;
  rows[slot[s]] = rowp1[s] - 1;
}

__global__ void k_zero_u32(uint32_t *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ void k_export_nodes(const Node *__restrict__ nodes, const double4 *__restrict__ mom,
                               int64_t nn, int32_t *start, int32_t *count, int32_t *level,
                               int32_t *skip, double *mass, double *com) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nn) return;
  const int4 m = nodes[k].meta;
  if (start) start[k] = m.y;
  if (count) count[k] = m.z;
  if (level) level[k] = m.w & 255;
  if (skip) skip[k] = m.x;
  const double4 q = mom[k];
  if (mass) mass[k] = q.x;
  if (com) {
    const double M = q.x;
    com[3 * k] = M > 0 ? q.y / M : 0.0;
    com[3 * k + 1] = M > 0 ? q.z / M : 0.0;
    com[3 * k + 2] = M > 0 ? q.w / M : 0.0;
  }
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

namespace {

// Group table of one launch with one segment per snapshot (one
// workgroup): snapshot k's targets start at tstart[k] (its sorted start
// soff[k] counted through the compaction scan `slot`, or soff[k] itself when
// every member is a target) and form ceil(T_k / 64) groups starting at
// gstart[k]. Also clears the work queue.
constexpr int kTableBlock = 1024;
__global__ __launch_bounds__(kTableBlock) void k_group_table(
    const int32_t *__restrict__ soff, int n_snap, const uint32_t *__restrict__ slot,
    int32_t *__restrict__ tstart, int32_t *__restrict__ gstart, int32_t *__restrict__ seg_snap,
    int32_t *__restrict__ nseg, unsigned *__restrict__ queue) {
  __shared__ int32_t part[kTableBlock];
  const int tid = (int)threadIdx.x;
  if (tid < 8) queue[tid] = 0u;
  if (tid == 0) *nseg = n_snap;
  const int per = (n_snap + kTableBlock - 1) / kTableBlock;
  const int k0 = min(tid * per, n_snap), k1 = min(k0 + per, n_snap);
  auto first = [&](int k) { return slot ? (int32_t)slot[soff[k]] : soff[k]; };
  int32_t sum = 0;
  for (int k = k0; k < k1; ++k) sum += (first(k + 1) - first(k) + kWave - 1) / kWave;
  part[tid] = sum;
  __syncthreads();
  for (int d = 1; d < kTableBlock; d <<= 1) {  // inclusive scan of the sums
    const int32_t v = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int32_t base = part[tid] - sum;
  for (int k = k0; k < k1; ++k) {
    const int32_t f = first(k);
    tstart[k] = f;
    gstart[k] = base;
    seg_snap[k] = k;
    base += (first(k + 1) - f + kWave - 1) / kWave;
  }
  if (tid == kTableBlock - 1) {
    tstart[n_snap] = first(n_snap);
    gstart[n_snap] = part[tid];
  }
}

// Split groups: target t starts a segment when it is the first target, or
// its snapshot or its level-`level` key cell differs from target t-1's.
// ntarg: device count of the targets (nullptr: max_t, every member).
__global__ void k_seg_flags(const int32_t *__restrict__ targets,
                            const uint32_t *__restrict__ ntarg, int64_t max_t,
                            const uint64_t *__restrict__ keys, const int32_t *__restrict__ soff,
                            int n_snap, int level, uint32_t *__restrict__ flags) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t > max_t) return;
  const int64_t T = ntarg ? (int64_t)*ntarg : max_t;
  if (t >= T) {
    flags[t] = 0u;
    return;
  }
  if (t == 0) {
    flags[t] = 1u;
    return;
  }
  const int s = targets ? targets[t] : (int)t, p = targets ? targets[t - 1] : (int)(t - 1);
  const int ks = segment_of(soff, n_snap, s);
  if (ks != segment_of(soff, n_snap, p)) {
    flags[t] = 1u;
    return;
  }
  int lv = level;
  if (lv == kSplitAuto) {
    lv = 0;
    for (int64_t m = (int64_t)(soff[ks + 1] - soff[ks]) / 128; m >= 8; m /= 8) ++lv;
    if (lv < 1) {
      flags[t] = 0u;
      return;
    }
  }
  const int sh = 3 * (kMaxLevel - lv);
  flags[t] = (keys[s] >> sh) != (keys[p] >> sh) ? 1u : 0u;
}

__global__ void k_seg_starts(const uint32_t *__restrict__ flags,
                             const uint32_t *__restrict__ segid,
                             const int32_t *__restrict__ targets,
                             const uint32_t *__restrict__ ntarg, int64_t max_t,
                             const int32_t *__restrict__ soff, int n_snap,
                             int32_t *__restrict__ tstart, int32_t *__restrict__ seg_snap,
                             int32_t *__restrict__ nseg, unsigned *__restrict__ queue) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    const int32_t ns = (int32_t)segid[max_t];
    const int64_t T = ntarg ? (int64_t)*ntarg : max_t;
    *nseg = ns;
    tstart[ns] = (int32_t)T;
    for (int r = 0; r < 8; ++r) queue[r] = 0u;
  }
  if (t >= max_t || !flags[t]) return;
  const uint32_t k = segid[t];
  const int s = targets ? targets[t] : (int)t;
  tstart[k] = (int32_t)t;
  seg_snap[k] = segment_of(soff, n_snap, s);
}

__global__ void k_seg_groups(const int32_t *__restrict__ tstart, const int32_t *__restrict__ nseg,
                             int64_t max_seg, uint32_t *__restrict__ gcnt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k > max_seg) return;
  gcnt[k] = k < *nseg ? (uint32_t)((tstart[k + 1] - tstart[k] + kWave - 1) / kWave) : 0u;
}

}  // namespace

// The buffers of one call's group table, taken before its first launch so
// that a failed allocation leaves nothing enqueued. The split tables reuse
// the compaction's mark and row buffers (kFlags, kCounts), which the
// stream has consumed by then; one scan buffer serves every scan.
struct WorkBufs {
  int64_t max_t = 0, max_seg = 0;
  bool split_on = false;
  uint32_t *stmp = nullptr, *mark = nullptr, *slot = nullptr;
  int32_t *rowp1 = nullptr, *tg = nullptr, *rw = nullptr, *tab = nullptr;
  uint32_t *flags = nullptr, *segid = nullptr, *gcnt = nullptr;
};

// listed: targets come from a mark pass (an active list or a bin rule)
// instead of being every member; max_t bounds their number.
int reserve_work(g3_ctx *c, const g3_tree *t, const Octree &o, int64_t max_t_in, bool listed,
                 int split, WorkBufs *b, Arena *arena) {
  // out of memory: G3_ENOMEM from the ctx's scratch, G3_EINVAL (the call is
  // too large) from a caller-given region
  auto no_room = [&](const char *msg) {
    return arena ? fail(c, G3_EINVAL, "the work tables need more than the allocation-free "
                                      "region holds")
                 : fail(c, G3_ENOMEM, msg);
  };
  *b = WorkBufs();
  const int64_t m = o.n;
  if (m == 0) return G3_OK;
  const int n_snap = t->n_snap;
  const int64_t max_t = listed ? std::min<int64_t>(max_t_in, m) : m;
  const bool split_on = split >= 0 || split == kSplitAuto;
  const int64_t max_seg = split_on ? std::max<int64_t>(max_t, 1) : n_snap;
  b->max_t = max_t;
  b->max_seg = max_seg;
  b->split_on = split_on;
  int64_t scan_n = 1;
  if (listed) scan_n = std::max(scan_n, m + 1);
  if (split_on) scan_n = std::max(scan_n, std::max(max_t, max_seg) + 1);
  uint32_t *stmp = nullptr, *mark = nullptr, *slot = nullptr;
  int32_t *rowp1 = nullptr, *tg = nullptr, *rw = nullptr;
  if (listed || split_on) {
    stmp = (uint32_t *)scratch_in(c, arena, kScanTmp, scan_tmp_elems(scan_n) * sizeof(uint32_t));
    if (!stmp) return no_room("device allocation of the scan scratch failed");
  }
  if (listed) {
    mark = (uint32_t *)scratch_in(c, arena, kFlags, (m + 2) * sizeof(uint32_t));
    slot = (uint32_t *)scratch_in(c, arena, kOffsets, (m + 1) * sizeof(uint32_t));
    rowp1 = (int32_t *)scratch_in(c, arena, kCounts, (m + 2) * sizeof(int32_t));
    tg = (int32_t *)scratch_in(c, arena, kTargets, (m + 1) * sizeof(int32_t));
    rw = (int32_t *)scratch_in(c, arena, kRows, (m + 1) * sizeof(int32_t));
    if (!mark || !slot || !rowp1 || !tg || !rw)
      return no_room("device allocation of the active-set scratch failed");
  }
  // tstart, gstart [max_seg + 2] (a scan writes one past its n), seg_snap
  // [max_seg + 1], nseg, queue [8]
  const size_t tab_elems = 3 * ((size_t)max_seg + 2) + 1 + 8;
  int32_t *tab = (int32_t *)scratch_in(c, arena, kGroups, tab_elems * sizeof(int32_t));
  if (!tab) return no_room("device allocation of the group table failed");
  uint32_t *flags = nullptr, *segid = nullptr, *gcnt = nullptr;
  if (split_on) {
    flags = (uint32_t *)scratch_in(c, arena, kCounts, (m + 2) * sizeof(uint32_t));
    segid = (uint32_t *)scratch_in(c, arena, kFlags, (m + 2) * sizeof(uint32_t));
    gcnt = (uint32_t *)scratch_in(c, arena, kIds, (max_seg + 2) * sizeof(uint32_t));
    if (!flags || !segid || !gcnt)
      return no_room("device allocation of the group table failed");
    // the compaction's buffers must not have moved (same slots, same sizes)
    if (listed && (flags != (uint32_t *)rowp1 || segid != mark))
      return fail(c, G3_EHIP, "group table scratch moved");
  }
  b->stmp = stmp; b->mark = mark; b->slot = slot;
  b->rowp1 = rowp1; b->tg = tg; b->rw = rw; b->tab = tab;
  b->flags = flags; b->segid = segid; b->gcnt = gcnt;
  return G3_OK;
}

int prepare_work(g3_ctx *c, const g3_tree *t, const Octree &o, const int32_t *iperm,
                 int64_t n_act, const int32_t *active, Work *w, hipStream_t s, int split,
                 Arena *arena, const int32_t *bins, int32_t kmin) {
  *w = Work();
  const int64_t m = o.n;
  if (m == 0) return G3_OK;
  WorkBufs b;
  const bool listed = active || bins;
  const int st = reserve_work(c, t, o, active ? n_act : m, listed, split, &b, arena);
  if (st) return st;
  const int n_snap = t->n_snap;
  const int64_t max_t = b.max_t, max_seg = b.max_seg;
  const bool split_on = b.split_on;
  uint32_t *stmp = b.stmp, *mark = b.mark, *slot = b.slot;
  int32_t *rowp1 = b.rowp1, *tg = b.tg, *rw = b.rw, *tab = b.tab;
  uint32_t *flags = b.flags, *segid = b.segid, *gcnt = b.gcnt;
  if (listed) {
    if (bins) {
      k_mark_bins<<<nblk(m), 256, 0, s>>>(o.perm, m, bins, kmin, mark, rowp1);
    } else {
      k_zero_u32<<<nblk(m), 256, 0, s>>>(mark, m);
      if (n_act > 0)
        k_mark<<<nblk(n_act), 256, 0, s>>>(active, n_act, iperm, t->n, mark, rowp1);
    }
    hipError_t e = scan_u32(mark, slot, m, stmp, s);
    if (e != hipSuccess) return hip_fail(c, e, "active-set scan");
    k_compact<<<nblk(m), 256, 0, s>>>(mark, slot, rowp1, m, tg, rw);
  }
  const uint32_t *ntarg = listed ? slot + m : nullptr;
  int32_t *tstart = tab, *gstart = tab + max_seg + 2, *seg_snap = gstart + max_seg + 2;
  int32_t *nseg = seg_snap + max_seg + 2;
  unsigned *queue = (unsigned *)(nseg + 1);
  if (!split_on) {
    k_group_table<<<1, kTableBlock, 0, s>>>(o.soff, n_snap, slot, tstart, gstart, seg_snap, nseg,
                                            queue);
  } else {
    const int level = split == kSplitAuto ? split : std::min(split, (int)kMaxLevel);
    k_seg_flags<<<nblk(max_t + 1), 256, 0, s>>>(tg, ntarg, max_t, o.keys, o.soff, n_snap, level,
                                               flags);
    hipError_t e = scan_u32(flags, segid, max_t + 1, stmp, s);
    if (e != hipSuccess) return hip_fail(c, e, "group split scan");
    k_seg_starts<<<nblk(max_t + 1), 256, 0, s>>>(flags, segid, tg, ntarg, max_t, o.soff, n_snap,
                                                 tstart, seg_snap, nseg, queue);
    k_seg_groups<<<nblk(max_seg + 1), 256, 0, s>>>(tstart, nseg, max_seg, gcnt);
    e = scan_u32(gcnt, (uint32_t *)gstart, max_seg + 1, stmp, s);
    if (e != hipSuccess) return hip_fail(c, e, "group split scan");
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, "group table");
  w->gs.targets = tg;
  w->gs.tstart = tstart;
  w->gs.gstart = gstart;
  w->gs.seg_snap = seg_snap;
  w->gs.nseg = nseg;
  w->gs.nroot = o.nroot;
  w->gs.sbox = t->sbox;
  w->gs.queue = queue;
  w->gs.n_snap = n_snap;
  w->rows = rw;
  w->ntarg = ntarg;
  w->max_groups = split_on ? max_t : max_groups_of(max_t, n_snap);
  return G3_OK;
}

unsigned persistent_grid(const void *kern, int block, int64_t max_groups) {
  static std::mutex mu;
  static std::map<std::pair<int, const void *>, int64_t> resident;
  int dev = 0;
  (void)hipGetDevice(&dev);
  int64_t cap;
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = resident.find({dev, kern});
    if (it == resident.end()) {
      int per_cu = 0, ncu = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, 0) != hipSuccess ||
          per_cu < 1)
        per_cu = 1;
      if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
          ncu < 1)
        ncu = 1;
      it = resident.emplace(std::make_pair(dev, kern), (int64_t)per_cu * ncu).first;
    }
    cap = it->second;
  }
  const int64_t waves_per_block = block / kWave;
  const int64_t need = (max_groups + waves_per_block - 1) / waves_per_block;
  return (unsigned)std::max<int64_t>(1, std::min(need, cap));
}

}  // namespace g3

using namespace g3;

extern "C" {

int g3_ctx_create(g3_ctx **out, int device) {
  if (!out) return G3_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return G3_EINVAL;
  DeviceGuard g(device);
  g3_ctx *c = new g3_ctx;
  c->device = device;
  if (dev_malloc(c, (void **)&c->counters, 8 * sizeof(unsigned long long)) != hipSuccess) {
    delete c;
    return G3_ENOMEM;
  }
  if (hipMemset(c->counters, 0, 8 * sizeof(unsigned long long)) != hipSuccess ||
      hipHostMalloc((void **)&c->pinned, 8 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(c->counters);
    delete c;
    return G3_ENOMEM;
  }
  std::memset(c->pinned, 0, 8 * sizeof(int64_t));
  // the allocation-free calls' region on this device (looked up once per
  // device, with the device current)
  if (noalloc_init(device) != (int)hipSuccess) {
    (void)hipFree(c->counters);
    (void)hipHostFree(c->pinned);
    delete c;
    return G3_EHIP;
  }
  *out = c;
  return G3_OK;
}

static void free_octree(Octree &o) {
  for (void *p : {(void *)o.keys, (void *)o.perm, (void *)o.xm, (void *)o.nodes, (void *)o.mom,
                  (void *)o.gnodes, (void *)o.vh, (void *)o.aux, (void *)o.x64, (void *)o.h64,
                  (void *)o.c64, (void *)o.soff, (void *)o.nroot})
    if (p) (void)hipFree(p);
  o = Octree();
}

static void free_tree(g3_tree *t) {
  if (!t) return;
  if (t->iperm_all) (void)hipFree(t->iperm_all);
  if (t->iperm_gas) (void)hipFree(t->iperm_gas);
  if (t->coff) (void)hipFree(t->coff);
  if (t->sbox) (void)hipFree(t->sbox);
  if (t->absmax) (void)hipFree(t->absmax);
  free_octree(t->all);
  free_octree(t->gas);
  delete t;
}

void g3_ctx_destroy(g3_ctx *c) {
  if (!c) return;
  DeviceGuard g(c->device);
  (void)hipDeviceSynchronize();
  for (g3_tree *t : c->trees) free_tree(t);
  for (auto &b : c->scratch)
    if (b.p) (void)hipFree(b.p);
  if (c->counters) (void)hipFree(c->counters);
  if (c->pinned) (void)hipHostFree(c->pinned);
  for (auto &tm : c->timing)
    for (hipEvent_t e : tm.ev) (void)hipEventDestroy(e);
  delete c;
}

const char *g3_last_error(const g3_ctx *c) { return c ? c->err.c_str() : "null context"; }

int g3_ctx_stats(g3_ctx *c, int64_t *stats, int32_t reset) {
  if (!c || !stats) return fail(c, G3_EINVAL, "g3_ctx_stats: null argument");
  DeviceGuard g(c->device);
  hipStream_t s = c->last_stream;
  hipError_t e = hipMemcpyAsync(&c->pinned[4], c->counters, 4 * sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_ctx_stats");
  for (int k = 0; k < 4; ++k) stats[k] = c->pinned[4 + k];
  if (reset) {
    e = hipMemsetAsync(c->counters, 0, 4 * sizeof(unsigned long long), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(c, e, "g3_ctx_stats reset");
  }
  if (stats[0] > 0)
    return fail(c, G3_ENOCONV, std::to_string(stats[0]) +
                                   " particles' h solves did not converge since the last reset");
  return G3_OK;
}

int g3_ctx_kernel_timing(g3_ctx *c, int32_t kind, int32_t capacity) {
  if (!c) return G3_EINVAL;
  if (kind < 0 || kind >= kTuneKinds || capacity < 0 || capacity > G3_TIMING_MAX)
    return fail(c, G3_EINVAL, "g3_ctx_kernel_timing: bad kind or capacity");
  DeviceGuard g(c->device);
  g3_ctx::Timing &t = c->timing[kind];
  t.count = 0;
  t.capacity = 0;
  while ((int)t.ev.size() < 2 * capacity) {
    hipEvent_t e = nullptr;
    const hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return hip_fail(c, r, "g3_ctx_kernel_timing");
    t.ev.push_back(e);
  }
  t.capacity = capacity;
  c->err.clear();
  return G3_OK;
}

int g3_ctx_kernel_times(g3_ctx *c, int32_t kind, float *ms, int32_t *count) {
  if (!c) return G3_EINVAL;
  if (kind < 0 || kind >= kTuneKinds || !count)
    return fail(c, G3_EINVAL, "g3_ctx_kernel_times: bad kind or null count");
  DeviceGuard g(c->device);
  g3_ctx::Timing &t = c->timing[kind];
  const int n = t.count;
  if (n > 0 && !ms) return fail(c, G3_EINVAL, "g3_ctx_kernel_times: null ms");
  for (int k = 0; k < n; ++k) {
    hipError_t r = hipEventSynchronize(t.ev[2 * k + 1]);
    if (r == hipSuccess) r = hipEventElapsedTime(&ms[k], t.ev[2 * k], t.ev[2 * k + 1]);
    if (r != hipSuccess) return hip_fail(c, r, "g3_ctx_kernel_times");
  }
  *count = n;
  t.count = 0;
  c->err.clear();
  return G3_OK;
}

int g3_ctx_inject(g3_ctx *c, int32_t what, int64_t value) {
  if (!c) return G3_EINVAL;
  if (what == G3_INJECT_ALLOC) {
    c->alloc_budget = value < 0 ? -1 : value;
    return G3_OK;
  }
  if (what == G3_INJECT_MAX_ITER) {
    if (value > 64) return fail(c, G3_EINVAL, "g3_ctx_inject: the pass limit is at most 64");
    c->max_iter = value <= 0 ? 64 : (int)value;
    return G3_OK;
  }
  return fail(c, G3_EINVAL, "g3_ctx_inject: unknown injection");
}

static int build_forest_body(g3_ctx *c, g3_tree *t, int32_t n_snap, const int64_t *snap_off,
                             const void *pos, const float *mass, const uint8_t *type,
                             const double *box, const g3_params *p, int32_t pos_t,
                             hipStream_t s);

int g3_build_forest(g3_ctx *c, int32_t n_snap, const int64_t *snap_off, int32_t pos_t,
                    const void *pos, const float *mass, const uint8_t *type, const double *box,
                    const g3_params *p, g3_tree **tree, void *stream) {
  G3_RANGE("g3_build_forest");
  if (!c) return G3_EINVAL;
  if (n_snap < 1 || n_snap > G3_MAX_SNAPSHOTS || !snap_off || !box)
    return fail(c, G3_EINVAL, "g3_build_forest: need 1..G3_MAX_SNAPSHOTS snapshots, offsets and boxes");
  if (snap_off[0] != 0) return fail(c, G3_EINVAL, "g3_build_forest: snap_off[0] must be 0");
  for (int32_t k = 0; k < n_snap; ++k)
    if (snap_off[k + 1] < snap_off[k])
      return fail(c, G3_EINVAL, "g3_build_forest: snap_off must be non-decreasing");
  const int64_t n = snap_off[n_snap];
  if (n < 0 || n >= (int64_t)INT32_MAX) return fail(c, G3_EINVAL, "g3_build_forest: n out of range");
  if (pos_t != G3_F32 && pos_t != G3_F64)
    return fail(c, G3_EINVAL, "g3_build_forest: pos_t must be G3_F32 or G3_F64");
  if (n > 0 && (!pos || !mass)) return fail(c, G3_EINVAL, "g3_build_forest: null pos/mass");
  for (int32_t k = 0; k < n_snap; ++k) {
    const double *b = box + 4 * k;
    if (!(b[3] > 0.0) || !std::isfinite(b[0]) || !std::isfinite(b[1]) || !std::isfinite(b[2]) ||
        !std::isfinite(b[3]))
      return fail(c, G3_EINVAL, "g3_build_forest: every box must be lo xyz and a finite side > 0");
  }
  if (!params_ok(p)) return fail(c, G3_EINVAL, "g3_build_forest: bad params");
  if (!tree) return fail(c, G3_EINVAL, "g3_build_forest: null tree handle");
  g3_tree *t = *tree;
  if (t && t->owner != c) return fail(c, G3_ESTATE, "g3_build_forest: tree of another ctx");
  DeviceGuard g(c->device);
  int st = check_pending(c);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  if (!t) {
    t = new g3_tree;
    t->owner = c;
    t->device = c->device;
    c->trees.push_back(t);
    *tree = t;
  }
  t->built = false;
  st = build_forest_body(c, t, n_snap, snap_off, pos, mass, type, box, p, pos_t, s);
  if (st) {
    // a failed build leaves no work of its own in flight on the stream
    (void)hipStreamSynchronize(s);
    return st;
  }
  t->built = true;
  c->err.clear();
  return G3_OK;
}

// The work of g3_build_forest after its argument checks.
static int build_forest_body(g3_ctx *c, g3_tree *t, int32_t n_snap, const int64_t *snap_off,
                             const void *pos, const float *mass, const uint8_t *type,
                             const double *box, const g3_params *p, int32_t pos_t,
                             hipStream_t s) {
  const int64_t n = snap_off[n_snap];
  int st = G3_OK;
  if (n > t->cap_n || !t->iperm_all) {
    if (t->iperm_all) (void)hipFree(t->iperm_all);
    if (t->iperm_gas) (void)hipFree(t->iperm_gas);
    t->iperm_all = t->iperm_gas = nullptr;
    t->cap_n = 0;
    const int64_t cap = n > 0 ? n : 1;
    if (dev_malloc(c, (void **)&t->iperm_all, cap * sizeof(int32_t)) != hipSuccess ||
        dev_malloc(c, (void **)&t->iperm_gas, cap * sizeof(int32_t)) != hipSuccess)
      return fail(c, G3_ENOMEM, "g3_build_forest: allocation failed");
    t->cap_n = cap;
  }
  if (n_snap > t->cap_snap) {
    for (void *q : {(void *)t->coff, (void *)t->sbox, (void *)t->all.soff, (void *)t->all.nroot,
                    (void *)t->gas.soff, (void *)t->gas.nroot})
      if (q) (void)hipFree(q);
    t->coff = nullptr; t->sbox = nullptr;
    t->all.soff = t->all.nroot = t->gas.soff = t->gas.nroot = nullptr;
    t->cap_snap = 0;
    const size_t k1 = (size_t)n_snap + 1;
    if (dev_malloc(c, (void **)&t->coff, k1 * sizeof(int64_t)) != hipSuccess ||
        dev_malloc(c, (void **)&t->sbox, k1 * sizeof(double4)) != hipSuccess ||
        dev_malloc(c, (void **)&t->all.soff, k1 * sizeof(int32_t)) != hipSuccess ||
        dev_malloc(c, (void **)&t->all.nroot, k1 * sizeof(int32_t)) != hipSuccess ||
        dev_malloc(c, (void **)&t->gas.soff, k1 * sizeof(int32_t)) != hipSuccess ||
        dev_malloc(c, (void **)&t->gas.nroot, k1 * sizeof(int32_t)) != hipSuccess)
      return fail(c, G3_ENOMEM, "g3_build_forest: allocation failed");
    t->cap_snap = n_snap;
  }
  t->n = n;
  t->n_snap = n_snap;
  t->snap_off.assign(snap_off, snap_off + n_snap + 1);
  t->box.assign(box, box + 4 * (size_t)n_snap);
  t->leaf = p->leaf_size;
  t->f64 = pos_t == G3_F64;
  double smax = 0.0;
  for (int32_t k = 0; k < n_snap; ++k) smax = std::max(smax, box[4 * k + 3]);
  t->max_side = smax;
  if (t->f64 && !t->absmax &&
      dev_malloc(c, (void **)&t->absmax, sizeof(unsigned)) != hipSuccess)
    return fail(c, G3_ENOMEM, "g3_build_forest: allocation failed");
  std::vector<double4> hb(n_snap);
  for (int32_t k = 0; k < n_snap; ++k)
    hb[k] = make_double4(box[4 * k], box[4 * k + 1], box[4 * k + 2], box[4 * k + 3]);
  hipError_t e = hipMemcpyAsync(t->coff, t->snap_off.data(), (n_snap + 1) * sizeof(int64_t),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(t->sbox, hb.data(), n_snap * sizeof(double4), hipMemcpyHostToDevice, s);
  // the host staging above is released on return: wait for the copies
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_build_forest: snapshot table upload");
  int64_t mgas = 0;
  st = select_members(c, t, type, &mgas, s);
  if (st) return st;
  st = build_octree(c, t, t->all, pos, t->f64, mass, n, s);
  if (st) return st;
  e = fill_i32(t->iperm_gas, -1, n, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_build_forest");
  st = build_octree(c, t, t->gas, pos, t->f64, mass, mgas, s, type);
  if (st) return st;
  // FP64 positions are walked through their FP32 copies: the walks pad
  // every pruning radius by a bound on their rounding, from the largest
  // coordinate actually held (positions may lie outside the boxes)
  e = update_absmax(t, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_build_forest");
  return G3_OK;
}

int g3_build_tree(g3_ctx *c, int64_t n, int32_t pos_t, const void *pos, const float *mass,
                  const uint8_t *type, const double *box, const g3_params *p, g3_tree **tree,
                  void *stream) {
  if (!c) return G3_EINVAL;
  if (n < 0 || n >= (int64_t)INT32_MAX) return fail(c, G3_EINVAL, "g3_build_tree: n out of range");
  if (!box) return fail(c, G3_EINVAL, "g3_build_tree: null box");
  const int64_t off[2] = {0, n};
  return g3_build_forest(c, 1, off, pos_t, pos, mass, type, box, p, tree, stream);
}

int g3_refit_tree(g3_ctx *c, g3_tree *t, const void *pos, const float *mass, void *stream) {
  G3_RANGE("g3_refit_tree");
  if (!c) return G3_EINVAL;
  if (!t) return fail(c, G3_EINVAL, "g3_refit_tree: null tree");
  if (t->owner != c) return fail(c, G3_ESTATE, "g3_refit_tree: tree of another ctx");
  if (!t->built) return fail(c, G3_ESTATE, "g3_refit_tree: tree not built (its last build failed)");
  if (t->n > 0 && (!pos || !mass)) return fail(c, G3_EINVAL, "g3_refit_tree: null pos/mass");
  DeviceGuard g(c->device);
  int st = check_pending(c);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  st = refit_octree(c, t, t->all, pos, mass, s);
  if (st) return st;
  st = refit_octree(c, t, t->gas, pos, mass, s);
  if (st) return st;
  const hipError_t e = update_absmax(t, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_refit_tree");
  c->err.clear();
  return G3_OK;
}

void g3_tree_destroy(g3_ctx *c, g3_tree *t) {
  if (!c || !t) return;
  DeviceGuard g(c->device);
  (void)hipDeviceSynchronize();
  for (size_t k = 0; k < c->trees.size(); ++k)
    if (c->trees[k] == t) {
      c->trees.erase(c->trees.begin() + (long)k);
      free_tree(t);
      return;
    }
}

int g3_tree_info(const g3_tree *t, int32_t which, int64_t *n_members, int64_t *n_nodes) {
  if (!t || (which != 0 && which != 1)) return G3_EINVAL;
  const Octree &o = which ? t->gas : t->all;
  if (n_members) *n_members = o.n;
  if (n_nodes) *n_nodes = o.nnodes;
  return G3_OK;
}

int g3_tree_export(g3_ctx *c, const g3_tree *t, int32_t which, int32_t *order, uint64_t *keys,
                   int32_t *node_start, int32_t *node_count, int32_t *node_level,
                   int32_t *node_skip, double *node_mass, double *node_com, void *stream) {
  G3_RANGE("g3_tree_export");
  if (!c) return G3_EINVAL;
  if (!t || (which != 0 && which != 1)) return fail(c, G3_EINVAL, "g3_tree_export: bad tree");
  if (t->owner != c) return fail(c, G3_ESTATE, "g3_tree_export: tree of another ctx");
  if (!t->built) return fail(c, G3_ESTATE, "g3_tree_export: tree not built (its last build failed)");
  DeviceGuard g(c->device);
  int st = check_pending(c);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  const Octree &o = which ? t->gas : t->all;
  hipError_t e = hipSuccess;
  if (order && o.n) e = hipMemcpyAsync(order, o.perm, o.n * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && keys && o.n)
    e = hipMemcpyAsync(keys, o.keys, o.n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_tree_export");
  if (o.nnodes)
    k_export_nodes<<<nblk(o.nnodes), 256, 0, s>>>(o.nodes, o.mom, o.nnodes, node_start,
                                                   node_count, node_level, node_skip, node_mass,
                                                   node_com);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, "g3_tree_export");
  return G3_OK;
}

static GravParams grav_params(const g3_params *p, const g3_tree *t) {
  GravParams gp;
  gp.theta2 = (float)(p->theta * p->theta);
  gp.eps2 = (float)(p->eps * p->eps);
  gp.G = (float)p->G;
  // a point inside a node's cube is within sqrt(3) l of its centre of mass,
  // so the containment test can only matter when theta^2 >= 1/3
  gp.inside_test = p->theta * p->theta >= 0.33 ? 1 : 0;
  gp.f64 = t->f64;
  gp.theta = p->theta;
  return gp;
}

static int size_class(int64_t n) {
  int k = 0;
  while (k < 62 && (int64_t(1) << (k + 1)) <= n) ++k;
  return k;
}

// Launch choices when none is tuned. The density takes subtrees of up to
// 128 members whole and splits its groups per snapshot at the level whose
// cells hold about 128 members (on clustered all-active sets of 10^6
// targets about 10 % faster than 64 unsplit); hydro and gravity take 64
// members, unsplit.
static Tuning default_tuning(int kind) {
  Tuning tu;
  if (kind == kTuneDensity) {
    tu.walk_leaf = 128;
    tu.split = kSplitAuto;
  }
  return tu;
}

// Launch tuning of a call of `kind` over n targets: the autotuned choice
// of the same size class (floor(log2 n)), else of the nearest tuned class
// of that kind, else the defaults.
static Tuning tuning_for(const g3_ctx *c, int kind, int64_t n) {
  const int cls = size_class(n);
  const Tuning *best = nullptr;
  int dist = 1 << 30;
  for (const auto &kv : c->tuning) {
    if (kv.first.first != kind) continue;
    const int d = std::abs(kv.first.second - cls);
    if (d < dist) {
      dist = d;
      best = &kv.second;
    }
  }
  return best ? *best : default_tuning(kind);
}

// FP64 trees: the gas octree's FP64 copy of h in sorted order, grown to
// its member count (before any launch of the call that needs it).
static int ensure_h64(g3_ctx *c, const g3_tree *t, Octree &o) {
  if (!t->f64 || o.n == 0 || (o.h64 && o.cap_h64 >= o.n)) return G3_OK;
  if (o.h64) (void)hipFree(o.h64);
  o.h64 = nullptr;
  o.cap_h64 = 0;
  if (dev_malloc(c, (void **)&o.h64, o.n * sizeof(double)) != hipSuccess)
    return fail(c, G3_ENOMEM, "device allocation of the FP64 smoothing lengths failed");
  o.cap_h64 = o.n;
  return G3_OK;
}

static SphParams sph_params(const g3_ctx *c, const g3_params *p, const g3_tree *t,
                            const Tuning &tu) {
  SphParams sp;
  sp.n_ngb = (float)p->n_ngb;
  sp.h_tol = (float)p->h_tol;
  sp.gamma = (float)p->gamma;
  sp.alpha = (float)p->alpha;
  sp.max_iter = c->max_iter;
  sp.walk_leaf = tu.walk_leaf;
  // candidate streams exist for the FP32 density only
  sp.streams = (!t->f64 && tu.streams == 4) ? 4 : 1;
  sp.f64 = t->f64;
  sp.absmax = t->absmax;
  return sp;
}

static int active_args_ok(g3_ctx *c, const g3_tree *t, int64_t n_act, const int32_t *active,
                          const char *who) {
  if (!t) return fail(c, G3_EINVAL, std::string(who) + ": null tree");
  if (t->owner != c) return fail(c, G3_ESTATE, std::string(who) + ": tree of another ctx");
  if (!t->built)
    return fail(c, G3_ESTATE, std::string(who) + ": tree not built (its last build failed)");
  if (n_act < 0) return fail(c, G3_EINVAL, std::string(who) + ": n_act < 0");
  if (!active && n_act != t->n)
    return fail(c, G3_EINVAL, std::string(who) + ": active == NULL needs n_act == n");
  return G3_OK;
}

int g3_walk(g3_ctx *c, const g3_tree *tc, int32_t kind, int64_t n_act, const int32_t *active,
            const void *h, const g3_params *p, int64_t capacity, int64_t *offsets,
            int32_t *list, int64_t *total, void *stream) {
  G3_RANGE("g3_walk");
  if (!c) return G3_EINVAL;
  int st = active_args_ok(c, tc, n_act, active, "g3_walk");
  if (st) return st;
  if (kind != G3_GATHER && kind != G3_SYMMETRIC && kind != G3_GRAVITY)
    return fail(c, G3_EINVAL, "g3_walk: unknown kind");
  if (!params_ok(p) || !offsets || !total || capacity < 0 || (capacity > 0 && !list))
    return fail(c, G3_EINVAL, "g3_walk: bad arguments");
  if (kind != G3_GRAVITY && !h && tc->gas.n > 0)
    return fail(c, G3_EINVAL, "g3_walk: SPH lists need h");
  g3_tree *t = const_cast<g3_tree *>(tc);
  DeviceGuard g(c->device);
  st = check_pending(c);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  Octree &o = (kind == G3_GRAVITY) ? t->all : t->gas;
  const int32_t *iperm = (kind == G3_GRAVITY) ? t->iperm_all : t->iperm_gas;
  int32_t *counts = (int32_t *)scratch(c, kWalkCounts, (n_act + 1) * sizeof(int32_t));
  int64_t *stmp = (int64_t *)scratch(c, kMisc, scan_tmp_elems(n_act) * sizeof(int64_t) + 64);
  if (!counts || !stmp) return fail(c, G3_ENOMEM, "g3_walk: allocation failed");
  if (kind != G3_GRAVITY) {
    st = ensure_h64(c, t, o);
    if (st) return st;
  }
  Work wk;
  st = prepare_work(c, t, o, iperm, n_act, active, &wk, s);
  if (st) return st;
  hipError_t e;
  if (kind != G3_GRAVITY && o.n > 0) {
    e = launch_hydro_prep(o, nullptr, nullptr, h, nullptr, nullptr, 1.0f, t->f64, s);
    if (e == hipSuccess && kind == G3_SYMMETRIC) e = refit_hmax(o, s);
    if (e != hipSuccess) return hip_fail(c, e, "g3_walk prep");
  }
  e = fill_i32(counts, 0, n_act, s);
  GravParams gp = grav_params(p, t);
  if (e == hipSuccess)
    e = launch_walk(o, kind, wk.gs, wk.rows, wk.max_groups, gp, t->absmax, counts, nullptr,
                    nullptr, s);
  if (e == hipSuccess) e = scan_i32_to_i64(counts, offsets, n_act, stmp, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&c->pinned[3], offsets + n_act, sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_walk count pass");
  *total = c->pinned[3];
  if (*total > capacity) return fail(c, G3_EOVERFLOW, "g3_walk: list exceeds capacity");
  if (*total > 0) {
    // the fill pass takes the groups from a fresh queue
    k_zero_u32<<<1, 64, 0, s>>>(wk.gs.queue, 8);
    e = launch_walk(o, kind, wk.gs, wk.rows, wk.max_groups, gp, t->absmax, counts, offsets,
                    list, s);
    if (e != hipSuccess) return hip_fail(c, e, "g3_walk fill pass");
  }
  c->err.clear();
  return G3_OK;
}

int g3_density(g3_ctx *c, const g3_tree *t, int64_t n_act, const int32_t *active,
               const g3_params *p, int32_t solve_h, void *h, float *rho, float *drho_dh,
               float *omega, int32_t *nngb, void *stream) {
  G3_RANGE("g3_density");
  if (!c) return G3_EINVAL;
  int st = active_args_ok(c, t, n_act, active, "g3_density");
  if (st) return st;
  if (!params_ok(p) || !h) return fail(c, G3_EINVAL, "g3_density: bad arguments");
  if (solve_h && !(p->n_ngb > 1365.0 / 48.0 && p->h_tol > 0.0 && p->h_tol < 1.0))
    return fail(c, G3_EINVAL, "g3_density: n_ngb must exceed 1365/48 and 0 < h_tol < 1");
  DeviceGuard g(c->device);
  st = check_pending(c);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  const Octree &o = t->gas;
  const Tuning tu = tuning_for(c, kTuneDensity, active ? std::min<int64_t>(n_act, o.n) : o.n);
  const SphParams sp = sph_params(c, p, t, tu);
  Work wk;
  st = prepare_work(c, t, o, t->iperm_gas, n_act, active, &wk, s, tu.split);
  if (st) return st;
  KernelTimer timer(c, kTuneDensity, s);
  hipError_t e = launch_density(o, wk.gs, wk.max_groups, sp, solve_h ? 1 : 0, h, rho, drho_dh,
                                omega, nngb, c->counters, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_density");
  timer.stop();
  c->err.clear();
  return G3_OK;
}

int g3_hydro_force(g3_ctx *c, g3_tree *t, int64_t n_act, const int32_t *active,
                   const g3_params *p, const float *vel, const float *u, const void *h,
                   const float *rho, const float *omega, float *acc, float *dudt, float *vsig,
                   int32_t *npairs, void *stream) {
  G3_RANGE("g3_hydro_force");
  if (!c) return G3_EINVAL;
  int st = active_args_ok(c, t, n_act, active, "g3_hydro_force");
  if (st) return st;
  if (!params_ok(p)) return fail(c, G3_EINVAL, "g3_hydro_force: bad params");
  if (t->gas.n > 0 && (!vel || !u || !h || !rho || !omega))
    return fail(c, G3_EINVAL, "g3_hydro_force: null input");
  DeviceGuard g(c->device);
  st = check_pending(c);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  Octree &o = t->gas;
  const Tuning tu = tuning_for(c, kTuneHydro, active ? std::min<int64_t>(n_act, o.n) : o.n);
  const SphParams sp = sph_params(c, p, t, tu);
  st = ensure_h64(c, t, o);
  if (st) return st;
  Work wk;
  st = prepare_work(c, t, o, t->iperm_gas, n_act, active, &wk, s, tu.split);
  if (st) return st;
  hipError_t e = launch_hydro_prep(o, vel, u, h, rho, omega, sp.gamma, t->f64, s);
  if (e == hipSuccess) e = refit_hmax(o, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_hydro_force prep");
  KernelTimer timer(c, kTuneHydro, s);
  e = launch_hydro(o, wk.gs, wk.max_groups, sp, acc, dudt, vsig, npairs, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_hydro_force");
  timer.stop();
  c->err.clear();
  return G3_OK;
}

int g3_gravity(g3_ctx *c, const g3_tree *t, int64_t n_act, const int32_t *active,
               const g3_params *p, float *acc, float *pot, int32_t *nterms, void *stream) {
  G3_RANGE("g3_gravity");
  if (!c) return G3_EINVAL;
  int st = active_args_ok(c, t, n_act, active, "g3_gravity");
  if (st) return st;
  if (!params_ok(p)) return fail(c, G3_EINVAL, "g3_gravity: bad params");
  DeviceGuard g(c->device);
  st = check_pending(c);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  // last_stream stays with the SPH calls: only they count into c->counters
  const BankGuard bank(c, 1);
  const Octree &o = t->all;
  const Tuning tu = tuning_for(c, kTuneGravity, active ? std::min<int64_t>(n_act, o.n) : o.n);
  Work wk;
  st = prepare_work(c, t, o, t->iperm_all, n_act, active, &wk, s, tu.split);
  if (st) return st;
  KernelTimer timer(c, kTuneGravity, s);
  hipError_t e = launch_gravity(o, wk.gs, wk.max_groups, grav_params(p, t), acc, pot, nterms, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_gravity");
  timer.stop();
  c->err.clear();
  return G3_OK;
}

int g3_conduction(g3_ctx *c, g3_tree *t, int64_t n_act, const int32_t *active,
                  const g3_params *p, double kappa0, double kappa_exp, const float *u,
                  const void *h, const float *rho, float *dudt, int32_t *npairs,
                  void *stream) {
  G3_RANGE("g3_conduction");
  if (!c) return G3_EINVAL;
  int st = active_args_ok(c, t, n_act, active, "g3_conduction");
  if (st) return st;
  if (!params_ok(p)) return fail(c, G3_EINVAL, "g3_conduction: bad params");
  if (t->f64) return fail(c, G3_EINVAL, "g3_conduction: FP32 trees only");
  if (!std::isfinite(kappa0) || kappa0 < 0.0 || !std::isfinite(kappa_exp))
    return fail(c, G3_EINVAL, "g3_conduction: bad conductivity");
  if (t->gas.n > 0 && (!u || !h || !rho)) return fail(c, G3_EINVAL, "g3_conduction: null input");
  DeviceGuard g(c->device);
  st = check_pending(c);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  Octree &o = t->gas;
  if (o.n == 0) {
    c->err.clear();
    return G3_OK;
  }
  const Tuning tu = tuning_for(c, kTuneHydro, active ? std::min<int64_t>(n_act, o.n) : o.n);
  float4 *ch = (float4 *)scratch(c, kCondCh, (size_t)o.n * sizeof(float4));
  if (!ch) return fail(c, G3_ENOMEM, "g3_conduction: allocation failed");
  Work wk;
  st = prepare_work(c, t, o, t->iperm_gas, n_act, active, &wk, s, tu.split);
  if (st) return st;
  // node hmax from h (the walk's symmetric radius), then the pair inputs
  hipError_t e = launch_hydro_prep(o, nullptr, nullptr, h, nullptr, nullptr, 1.0f, 0, s);
  if (e == hipSuccess) e = refit_hmax(o, s);
  if (e == hipSuccess)
    e = launch_conduction_prep(o, u, h, 0, rho, (float)kappa0, (float)kappa_exp, ch, s);
  if (e == hipSuccess)
    e = launch_conduction(o, wk.gs, wk.max_groups, tu.walk_leaf, ch, dudt, npairs, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_conduction");
  c->err.clear();
  return G3_OK;
}

// ---- improved-SPH switches ----

static bool switch_params_ok(const g3_switch_params *sp) {
  return sp && std::isfinite(sp->alpha_min) && std::isfinite(sp->alpha_max) &&
         sp->alpha_min >= 0.0 && sp->alpha_max >= sp->alpha_min && std::isfinite(sp->decay) &&
         sp->decay >= 0.0 && std::isfinite(sp->balsara_eps) && sp->balsara_eps >= 0.0 &&
         std::isfinite(sp->alpha_u) && sp->alpha_u >= 0.0 && sp->flags == 0;
}

int g3_velocity_gradients(g3_ctx *c, g3_tree *t, int64_t n_act, const int32_t *active,
                          const g3_params *p, const float *vel, const void *h, const float *rho,
                          const float *omega, float *div_v, float *curl_v, void *stream) {
  G3_RANGE("g3_velocity_gradients");
  if (!c) return G3_EINVAL;
  int st = active_args_ok(c, t, n_act, active, "g3_velocity_gradients");
  if (st) return st;
  if (!params_ok(p)) return fail(c, G3_EINVAL, "g3_velocity_gradients: bad params");
  if (t->f64) return fail(c, G3_EINVAL, "g3_velocity_gradients: FP32 trees only");
  if (t->gas.n > 0 && (!vel || !h || !rho || !omega))
    return fail(c, G3_EINVAL, "g3_velocity_gradients: null input");
  DeviceGuard g(c->device);
  st = check_pending(c);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  Octree &o = t->gas;
  if (o.n == 0) {
    c->err.clear();
    return G3_OK;
  }
  const Tuning tu = tuning_for(c, kTuneDensity, active ? std::min<int64_t>(n_act, o.n) : o.n);
  Work wk;
  st = prepare_work(c, t, o, t->iperm_gas, n_act, active, &wk, s, tu.split);
  if (st) return st;
  // (v, h) in sorted order, then the gather walk
  hipError_t e = launch_hydro_prep(o, vel, nullptr, h, nullptr, nullptr, 1.0f, 0, s);
  if (e == hipSuccess)
    e = launch_velgrad(o, wk.gs, wk.max_groups, tu.walk_leaf, rho, omega, div_v, curl_v, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_velocity_gradients");
  c->err.clear();
  return G3_OK;
}

int g3_viscosity_switch(g3_ctx *c, int64_t n, int32_t h_type, int64_t n_act,
                        const int32_t *active, const g3_params *p, const g3_switch_params *sw,
                        double dt, const float *u, const void *h, const float *div_v,
                        const float *curl_v, float *alpha, float *balsara, void *stream) {
  G3_RANGE("g3_viscosity_switch");
  if (!c) return G3_EINVAL;
  if (n < 0 || n_act < 0 || (!active && n_act != n) || (h_type != G3_F32 && h_type != G3_F64))
    return fail(c, G3_EINVAL, "g3_viscosity_switch: bad sizes");
  if (!params_ok(p) || !switch_params_ok(sw) || !std::isfinite(dt) || dt < 0.0)
    return fail(c, G3_EINVAL, "g3_viscosity_switch: bad params");
  if (n_act > 0 && (!u || !h || !div_v || !curl_v || (!alpha && !balsara)))
    return fail(c, G3_EINVAL, "g3_viscosity_switch: null argument");
  DeviceGuard g(c->device);
  int st = check_pending(c);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  SwitchStep step;
  step.gamma = (float)p->gamma;
  step.alpha_min = (float)sw->alpha_min;
  step.alpha_max = (float)sw->alpha_max;
  step.decay = (float)sw->decay;
  step.eps = (float)sw->balsara_eps;
  step.dt = (float)dt;
  hipError_t e = launch_alpha_update(n, n_act, active, step, h_type == G3_F64, u, h, div_v,
                                     curl_v, alpha, balsara, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_viscosity_switch");
  c->err.clear();
  return G3_OK;
}

int g3_hydro_force_switches(g3_ctx *c, g3_tree *t, int64_t n_act, const int32_t *active,
                            const g3_params *p, const g3_switch_params *sw, const float *vel,
                            const float *u, const void *h, const float *rho,
                            const float *omega, const float *alpha, const float *balsara,
                            float *acc, float *dudt, float *vsig, int32_t *npairs,
                            void *stream) {
  G3_RANGE("g3_hydro_force_switches");
  if (!c) return G3_EINVAL;
  int st = active_args_ok(c, t, n_act, active, "g3_hydro_force_switches");
  if (st) return st;
  if (!params_ok(p) || !switch_params_ok(sw))
    return fail(c, G3_EINVAL, "g3_hydro_force_switches: bad params");
  if (t->gas.n > 0 && (!vel || !u || !h || !rho || !omega))
    return fail(c, G3_EINVAL, "g3_hydro_force_switches: null input");
  DeviceGuard g(c->device);
  st = check_pending(c);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  Octree &o = t->gas;
  const Tuning tu = tuning_for(c, kTuneHydro, active ? std::min<int64_t>(n_act, o.n) : o.n);
  const SphParams sp = sph_params(c, p, t, tu);
  st = ensure_h64(c, t, o);
  if (st) return st;
  float4 *ext = (float4 *)scratch(c, kHydroExt, (size_t)std::max<int64_t>(o.n, 1) * sizeof(float4));
  if (!ext) return fail(c, G3_ENOMEM, "g3_hydro_force_switches: allocation failed");
  Work wk;
  st = prepare_work(c, t, o, t->iperm_gas, n_act, active, &wk, s, tu.split);
  if (st) return st;
  hipError_t e = launch_hydro_prep(o, vel, u, h, rho, omega, sp.gamma, t->f64, s);
  if (e == hipSuccess) e = refit_hmax(o, s);
  if (e == hipSuccess)
    e = launch_hydro_ext_prep(o, u, rho, alpha, balsara, sp.alpha, ext, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_hydro_force_switches prep");
  e = launch_hydro(o, wk.gs, wk.max_groups, sp, acc, dudt, vsig, npairs, s, ext,
                   (float)sw->alpha_u);
  if (e != hipSuccess) return hip_fail(c, e, "g3_hydro_force_switches");
  c->err.clear();
  return G3_OK;
}

int g3_gravity_noalloc(g3_ctx *c, const g3_tree *t, int64_t n_act, const int32_t *active,
                       const g3_params *p, float *acc, float *pot, int32_t *nterms,
                       void *stream) {
  if (!c) return G3_EINVAL;
  int st = active_args_ok(c, t, n_act, active, "g3_gravity_noalloc");
  if (st) return st;
  if (!params_ok(p)) return fail(c, G3_EINVAL, "g3_gravity_noalloc: bad params");
  DeviceGuard g(c->device);
  st = check_pending(c);
  if (st) return st;
  Arena arena;
  arena.base = (char *)noalloc_region(c->device);
  arena.cap = kNoAllocBytes;
  if (!arena.base) return fail(c, G3_ESTATE, "g3_gravity_noalloc: no region on this device");
  hipStream_t s = (hipStream_t)stream;
  // last_stream stays with the SPH calls: only they count into c->counters
  const Octree &o = t->all;
  const Tuning tu = tuning_for(c, kTuneGravity, active ? std::min<int64_t>(n_act, o.n) : o.n);
  Work wk;
  st = prepare_work(c, t, o, t->iperm_all, n_act, active, &wk, s, tu.split, &arena);
  if (st) return st;
  hipError_t e = launch_gravity(o, wk.gs, wk.max_groups, grav_params(p, t), acc, pot, nterms, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_gravity_noalloc");
  c->err.clear();
  return G3_OK;
}

// ---- time integration ----

static bool integ_args_ok(g3_ctx *c, int64_t n, int32_t pos_t, const g3_state *st,
                          const double *box, const g3_params *p, const g3_integ_params *ip,
                          const char *who) {
  auto bad = [&](const char *what) {
    fail(c, G3_EINVAL, std::string(who) + ": " + what);
    return false;
  };
  if (n < 0 || n >= (int64_t)INT32_MAX) return bad("n out of range");
  if (pos_t != G3_F32 && pos_t != G3_F64) return bad("unknown pos_t");
  if (!st || !box || !p || !ip) return bad("null argument");
  if (!params_ok(p)) return bad("bad params");
  if (!(p->n_ngb > 1365.0 / 48.0 && p->h_tol > 0.0 && p->h_tol < 1.0))
    return bad("n_ngb must exceed 1365/48 and 0 < h_tol < 1");
  if (!(ip->dt_max > 0.0) || !std::isfinite(ip->dt_max) || ip->bin_depth < 0 ||
      ip->bin_depth > 20 || !(ip->courant > 0.0) || !(ip->eta > 0.0) || ip->flags != 0)
    return bad("bad integration params");
  if (n > 0 && (!st->pos || !st->vel || !st->mass || !st->u || !st->h || !st->rho ||
                !st->omega || !st->acc || !st->dudt || !st->vsig || !st->pot || !st->bin))
    return bad("null state array");
  return true;
}

// Forces of the particles that are active at tick T (every particle at
// T = 0 and with `every`), then their kicks and new bins: the density with
// the smoothing-length solve (active gas), the hydro force from the gas
// velocities and internal energies predicted to T, gravity, and the update.
static int tick_forces(g3_ctx *c, g3_tree *t, int64_t n, const g3_state *st,
                       const g3_params *p, const g3_integ_params *ip, int64_t T, bool every,
                       const IntegUpdate &iu, float *acc_h, float *vp, float *up,
                       int64_t *count_out, hipStream_t s) {
  const int32_t *bins = every ? nullptr : st->bin;
  const int32_t kmin = iu.kmin;
  const double tau = std::ldexp(ip->dt_max, -ip->bin_depth);
  Octree &gas = t->gas;
  int rc = ensure_h64(c, t, gas);
  if (rc) return rc;
  hipError_t e = hipSuccess;
  if (gas.n > 0) {
    const Tuning td = tuning_for(c, kTuneDensity, gas.n);
    const SphParams spd = sph_params(c, p, t, td);
    Work wd;
    rc = prepare_work(c, t, gas, t->iperm_gas, gas.n, nullptr, &wd, s, td.split, nullptr, bins,
                      kmin);
    if (rc) return rc;
    e = launch_density(gas, wd.gs, wd.max_groups, spd, 1, st->h, st->rho, nullptr, st->omega,
                       nullptr, c->counters, s);
    if (e != hipSuccess) return hip_fail(c, e, "density at a tick");
    const float *vh = st->vel, *uh = st->u;
    if (T > 0) {
      e = launch_predict(n, st->type, st->vel, st->u, st->acc, st->dudt, st->bin,
                         ip->bin_depth, T, tau, vp, up, s);
      if (e != hipSuccess) return hip_fail(c, e, "prediction at a tick");
      vh = vp;
      uh = up;
    }
    const Tuning th = tuning_for(c, kTuneHydro, gas.n);
    const SphParams sp = sph_params(c, p, t, th);
    e = launch_hydro_prep(gas, vh, uh, st->h, st->rho, st->omega, sp.gamma, t->f64, s);
    if (e == hipSuccess) e = refit_hmax(gas, s);
    if (e != hipSuccess) return hip_fail(c, e, "hydro prep at a tick");
    Work wh;
    rc = prepare_work(c, t, gas, t->iperm_gas, gas.n, nullptr, &wh, s, th.split, nullptr, bins,
                      kmin);
    if (rc) return rc;
    e = launch_hydro(gas, wh.gs, wh.max_groups, sp, acc_h, st->dudt, st->vsig, nullptr, s);
    if (e != hipSuccess) return hip_fail(c, e, "hydro at a tick");
  }
  const Octree &all = t->all;
  const Tuning tg = tuning_for(c, kTuneGravity, all.n);
  Work wg;
  rc = prepare_work(c, t, all, t->iperm_all, all.n, nullptr, &wg, s, tg.split, nullptr, bins,
                    kmin);
  if (rc) return rc;
  e = launch_gravity(all, wg.gs, wg.max_groups, grav_params(p, t), st->acc, st->pot, nullptr, s);
  if (e == hipSuccess && count_out) e = launch_store_count(wg.ntarg, count_out, s);
  if (e == hipSuccess)
    e = launch_update(n, t->f64, iu, st->type, st->vel, st->u, st->acc, acc_h, st->dudt,
                      st->vsig, st->h, st->bin, s);
  if (e != hipSuccess) return hip_fail(c, e, "gravity and update at a tick");
  return G3_OK;
}

static IntegUpdate integ_update(const g3_params *p, const g3_integ_params *ip) {
  IntegUpdate iu;
  iu.depth = ip->bin_depth;
  iu.dt_max = ip->dt_max;
  iu.eta_eps2 = 2.0 * ip->eta * p->eps;
  iu.courant = ip->courant;
  return iu;
}

// The ctx scratch of the integration calls, taken before their first launch.
static int integ_scratch(g3_ctx *c, int64_t n, float **acc_h, float **vp, float **up) {
  const int64_t m = std::max<int64_t>(n, 1);
  *acc_h = (float *)scratch(c, kIntAccH, (size_t)m * 3 * sizeof(float));
  *vp = (float *)scratch(c, kIntVp, (size_t)m * 3 * sizeof(float));
  *up = (float *)scratch(c, kIntUp, (size_t)m * sizeof(float));
  if (!*acc_h || !*vp || !*up)
    return fail(c, G3_ENOMEM, "device allocation of the integration scratch failed");
  return G3_OK;
}

static int integ_build(g3_ctx *c, g3_tree **tree, int64_t n, int32_t pos_t, const g3_state *st,
                       const double *box, const g3_params *p, void *stream) {
  const int64_t off[2] = {0, n};
  return g3_build_forest(c, 1, off, pos_t, st->pos, st->mass, st->type, box, p, tree, stream);
}

int g3_integrate_start(g3_ctx *c, g3_tree **tree, int64_t n, int32_t pos_t, const g3_state *st,
                       const double *box, const g3_params *p, const g3_integ_params *ip,
                       void *stream) {
  G3_RANGE("g3_integrate_start");
  if (!c) return G3_EINVAL;
  if (!tree) return fail(c, G3_EINVAL, "g3_integrate_start: null tree handle");
  if (!integ_args_ok(c, n, pos_t, st, box, p, ip, "g3_integrate_start")) return G3_EINVAL;
  DeviceGuard g(c->device);
  int rc = check_pending(c);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  float *acc_h, *vp, *up;
  rc = integ_scratch(c, n, &acc_h, &vp, &up);
  if (rc) return rc;
  rc = integ_build(c, tree, n, pos_t, st, box, p, stream);
  if (rc) return rc;
  IntegUpdate iu = integ_update(p, ip);
  iu.every_particle = 1;
  iu.sum = 1;
  iu.rebin = 1;
  iu.kmin = 0;
  rc = tick_forces(c, *tree, n, st, p, ip, 0, true, iu, acc_h, vp, up, nullptr, s);
  if (rc) return rc;
  c->err.clear();
  return G3_OK;
}

int g3_system_step(g3_ctx *c, g3_tree **tree, int64_t n, int32_t pos_t, const g3_state *st,
                   const double *box, const g3_params *p, const g3_integ_params *ip,
                   int64_t *tick_active, void *stream) {
  G3_RANGE("g3_system_step");
  if (!c) return G3_EINVAL;
  if (!tree) return fail(c, G3_EINVAL, "g3_system_step: null tree handle");
  if (!integ_args_ok(c, n, pos_t, st, box, p, ip, "g3_system_step")) return G3_EINVAL;
  DeviceGuard g(c->device);
  int rc = check_pending(c);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  float *acc_h, *vp, *up;
  rc = integ_scratch(c, n, &acc_h, &vp, &up);
  if (rc) return rc;
  // the trees of this system step, from the positions at its start
  rc = integ_build(c, tree, n, pos_t, st, box, p, stream);
  if (rc) return rc;
  g3_tree *t = *tree;
  const int B = ip->bin_depth;
  const int64_t ticks = (int64_t)1 << B;
  const double tau = std::ldexp(ip->dt_max, -B);
  const IntegUpdate base = integ_update(p, ip);
  // opening half kick of every particle with its bin's step
  IntegUpdate open = base;
  open.every_particle = 1;
  open.open = 1;
  hipError_t e = launch_update(n, t->f64, open, st->type, st->vel, st->u, st->acc, acc_h,
                               st->dudt, st->vsig, st->h, st->bin, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_system_step opening kick");
  for (int64_t T = 1; T <= ticks; ++T) {
    e = launch_drift(st->pos, t->f64, st->vel, n, tau, s);
    if (e != hipSuccess) return hip_fail(c, e, "g3_system_step drift");
    rc = refit_octree(c, t, t->all, st->pos, st->mass, s);
    if (rc) return rc;
    rc = refit_octree(c, t, t->gas, st->pos, st->mass, s);
    if (rc) return rc;
    e = update_absmax(t, s);
    if (e != hipSuccess) return hip_fail(c, e, "g3_system_step refit");
    // active at T: bins k with 2^(B-k) | T, i.e. k >= B - min(tz(T), B)
    int tz = 0;
    while (tz < B && ((T >> tz) & 1) == 0) ++tz;
    IntegUpdate iu = base;
    iu.kmin = B - tz;
    iu.sum = 1;
    iu.close = 1;
    iu.rebin = 1;
    iu.open = T < ticks ? 1 : 0;
    rc = tick_forces(c, t, n, st, p, ip, T, false, iu, acc_h, vp, up,
                     tick_active ? tick_active + (T - 1) : nullptr, s);
    if (rc) return rc;
  }
  c->err.clear();
  return G3_OK;
}

static bool tuning_ok(int kind, int walk_leaf, int split, int streams) {
  return kind >= 0 && kind < kTuneKinds && walk_leaf >= 1 && walk_leaf <= 4096 &&
         (split >= -1 || split == kSplitAuto) && split <= kMaxLevel &&
         (streams == 1 || streams == 4);
}

int g3_tuning_get(g3_ctx *c, int32_t kind, int64_t n_targets, int32_t *walk_leaf,
                  int32_t *split, int32_t *streams) {
  if (!c) return G3_EINVAL;
  if (kind < 0 || kind >= kTuneKinds) return fail(c, G3_EINVAL, "g3_tuning_get: bad kind");
  const Tuning tu = tuning_for(c, kind, n_targets);
  if (walk_leaf) *walk_leaf = tu.walk_leaf;
  if (split) *split = tu.split;
  if (streams) *streams = tu.streams;
  return G3_OK;
}

int g3_tuning_set(g3_ctx *c, int32_t kind, int64_t n_targets, int32_t walk_leaf,
                  int32_t split, int32_t streams) {
  if (!c) return G3_EINVAL;
  if (!tuning_ok(kind, walk_leaf, split, streams))
    return fail(c, G3_EINVAL, "g3_tuning_set: bad arguments");
  Tuning tu;
  tu.walk_leaf = walk_leaf;
  tu.split = split;
  tu.streams = kind == kTuneDensity ? streams : 1;
  if (n_targets < 0) {  // every size class of this kind: one entry
    for (auto it = c->tuning.begin(); it != c->tuning.end();)
      it = it->first.first == kind ? c->tuning.erase(it) : std::next(it);
    c->tuning[{kind, 0}] = tu;
  } else {
    c->tuning[{kind, size_class(n_targets)}] = tu;
  }
  return G3_OK;
}

int g3_tuning_save(g3_ctx *c, const char *path) {
  if (!c || !path) return fail(c, G3_EINVAL, "g3_tuning_save: null argument");
  FILE *f = std::fopen(path, "w");
  if (!f) return fail(c, G3_EINVAL, std::string("g3_tuning_save: cannot write ") + path);
  bool ok = std::fprintf(f, "g3-tuning 1\n") > 0;
  for (const auto &kv : c->tuning)
    ok = ok && std::fprintf(f, "%d %d %d %d %d\n", kv.first.first, kv.first.second,
                            kv.second.walk_leaf, kv.second.split, kv.second.streams) > 0;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return fail(c, G3_EINVAL, std::string("g3_tuning_save: write failed: ") + path);
  return G3_OK;
}

int g3_tuning_load(g3_ctx *c, const char *path) {
  if (!c || !path) return fail(c, G3_EINVAL, "g3_tuning_load: null argument");
  FILE *f = std::fopen(path, "r");
  if (!f) return fail(c, G3_EINVAL, std::string("g3_tuning_load: cannot read ") + path);
  std::map<std::pair<int, int>, Tuning> table;
  int version = 0;
  bool ok = std::fscanf(f, "g3-tuning %d", &version) == 1 && version == 1;
  int kind, cls, leaf, split, streams;
  while (ok) {
    const int got = std::fscanf(f, "%d %d %d %d %d", &kind, &cls, &leaf, &split, &streams);
    if (got == EOF) break;
    if (got != 5 || cls < 0 || cls > 62 || !tuning_ok(kind, leaf, split, streams)) {
      ok = false;
      break;
    }
    Tuning tu;
    tu.walk_leaf = leaf;
    tu.split = split;
    tu.streams = kind == kTuneDensity ? streams : 1;
    table[{kind, cls}] = tu;
  }
  std::fclose(f);
  if (!ok) return fail(c, G3_EINVAL, std::string("g3_tuning_load: malformed file ") + path);
  c->tuning = table;
  return G3_OK;
}

// Time one candidate: `run` enqueues the kernel(s); the second of two runs
// is timed with events on the stream.
static int time_candidate(g3_ctx *c, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                          const std::function<hipError_t()> &run, float *ms) {
  hipError_t e = run();
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  if (e == hipSuccess) e = run();
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  if (e != hipSuccess) return hip_fail(c, e, "g3_autotune");
  return G3_OK;
}

int g3_autotune(g3_ctx *c, g3_tree *t, int64_t n_act, const int32_t *active, const g3_params *p,
                const void *h, const float *vel, const float *u, const float *rho,
                const float *omega, void *stream) {
  G3_RANGE("g3_autotune");
  if (!c) return G3_EINVAL;
  int st = active_args_ok(c, t, n_act, active, "g3_autotune");
  if (st) return st;
  if (!params_ok(p)) return fail(c, G3_EINVAL, "g3_autotune: bad params");
  DeviceGuard g(c->device);
  st = check_pending(c);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  static const int kLeaves[] = {16, 32, 64, 128};
  static const int kSplits[] = {-1, kSplitAuto, 2, 3, 4, 5};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(c, G3_EHIP, "g3_autotune: event");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(c, G3_EHIP, "g3_autotune: event");
  }
  // the tuning runs leave the solve counters as they were
  unsigned long long saved[8];
  hipError_t e = hipMemcpyAsync(saved, c->counters, sizeof(saved), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return hip_fail(c, e, "g3_autotune");
  }
  const size_t hsz = t->f64 ? sizeof(double) : sizeof(float);
  auto finish = [&](int code) {
    (void)hipMemcpyAsync(c->counters, saved, sizeof(saved), hipMemcpyHostToDevice, s);
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return code;
  };
  Octree &gas = t->gas;
  const int64_t ng = active ? std::min<int64_t>(n_act, gas.n) : gas.n;
  // density, with the h solve on a copy of h
  if (gas.n > 0 && h) {
    void *hs = scratch(c, kAdjPQ, (size_t)t->n * hsz);
    if (!hs) return finish(fail(c, G3_ENOMEM, "g3_autotune: allocation failed"));
    Tuning best;
    float best_ms = INFINITY;
    for (int streams : {1, 4})
    for (int leaf : kLeaves)
      for (int split : kSplits) {
        if (streams > 1 && t->f64) continue;
        Tuning tu;
        tu.walk_leaf = leaf;
        tu.split = split;
        tu.streams = streams;
        Work wk;
        float ms = 0.f;
        st = time_candidate(c, s, e0, e1, [&]() -> hipError_t {
          hipError_t r = hipMemcpyAsync(hs, h, (size_t)t->n * hsz, hipMemcpyDeviceToDevice, s);
          if (r != hipSuccess) return r;
          if (prepare_work(c, t, gas, t->iperm_gas, n_act, active, &wk, s, tu.split))
            return hipErrorUnknown;
          return launch_density(gas, wk.gs, wk.max_groups, sph_params(c, p, t, tu), 1, hs,
                                nullptr, nullptr, nullptr, nullptr, c->counters, s);
        }, &ms);
        if (st) return finish(st);
        if (ms < best_ms) {
          best_ms = ms;
          best = tu;
        }
      }
    c->tuning[{kTuneDensity, size_class(ng)}] = best;
  }
  // hydro, when its inputs are given
  if (gas.n > 0 && h && vel && u && rho && omega) {
    const SphParams base = sph_params(c, p, t, Tuning());
    st = ensure_h64(c, t, gas);
    if (st) return finish(st);
    e = launch_hydro_prep(gas, vel, u, h, rho, omega, base.gamma, t->f64, s);
    if (e == hipSuccess) e = refit_hmax(gas, s);
    if (e != hipSuccess) return finish(hip_fail(c, e, "g3_autotune"));
    Tuning best;
    float best_ms = INFINITY;
    for (int leaf : kLeaves)
      for (int split : kSplits) {
        Tuning tu;
        tu.walk_leaf = leaf;
        tu.split = split;
        Work wk;
        float ms = 0.f;
        st = time_candidate(c, s, e0, e1, [&]() -> hipError_t {
          if (prepare_work(c, t, gas, t->iperm_gas, n_act, active, &wk, s, tu.split))
            return hipErrorUnknown;
          return launch_hydro(gas, wk.gs, wk.max_groups, sph_params(c, p, t, tu), nullptr, nullptr,
                              nullptr, nullptr, s);
        }, &ms);
        if (st) return finish(st);
        if (ms < best_ms) {
          best_ms = ms;
          best = tu;
        }
      }
    c->tuning[{kTuneHydro, size_class(ng)}] = best;
  }
  // gravity
  const Octree &all = t->all;
  if (all.n > 0) {
    const int64_t na = active ? std::min<int64_t>(n_act, all.n) : all.n;
    Tuning best;
    float best_ms = INFINITY;
    for (int split : kSplits) {
      Tuning tu;
      tu.split = split;
      Work wk;
      float ms = 0.f;
      st = time_candidate(c, s, e0, e1, [&]() -> hipError_t {
        if (prepare_work(c, t, all, t->iperm_all, n_act, active, &wk, s, tu.split))
          return hipErrorUnknown;
        return launch_gravity(all, wk.gs, wk.max_groups, grav_params(p, t), nullptr, nullptr,
                              nullptr, s);
      }, &ms);
      if (st) return finish(st);
      if (ms < best_ms) {
        best_ms = ms;
        best = tu;
      }
    }
    c->tuning[{kTuneGravity, size_class(na)}] = best;
  }
  c->err.clear();
  return finish(G3_OK);
}

int g3_density_backward(g3_ctx *c, g3_tree *t, int64_t n_act, const int32_t *active,
                        const g3_params *p, const float *h, const float *rho,
                        const float *drho_dh, const float *g_rho, const float *g_drho_dh,
                        const float *g_omega, float *g_pos, float *g_mass, float *g_h,
                        void *stream) {
  G3_RANGE("g3_density_backward");
  if (!c) return G3_EINVAL;
  int st = active_args_ok(c, t, n_act, active, "g3_density_backward");
  if (st) return st;
  if (!params_ok(p)) return fail(c, G3_EINVAL, "g3_density_backward: bad params");
  if (t->f64) return fail(c, G3_EINVAL, "g3_density_backward: FP32 trees only");
  if (t->gas.n > 0 && (!h || !rho || !drho_dh))
    return fail(c, G3_EINVAL, "g3_density_backward: h, rho and drho_dh are required");
  DeviceGuard g(c->device);
  st = check_pending(c);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  Octree &o = t->gas;
  if (o.n == 0) return G3_OK;
  Work wk;
  st = prepare_work(c, t, o, t->iperm_gas, o.n, nullptr, &wk, s);
  if (st) return st;
  hipError_t e = launch_hydro_prep(o, nullptr, nullptr, h, nullptr, nullptr, 1.0f, 0, s);
  if (e == hipSuccess) e = refit_hmax(o, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_density_backward prep");
  e = launch_density_bwd(o, t->iperm_gas, t->n, wk.gs, wk.max_groups, n_act, active, h, rho,
                         drho_dh, g_rho, g_drho_dh, g_omega, g_pos, g_mass, g_h, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_density_backward");
  c->err.clear();
  return G3_OK;
}

int g3_density_solve_backward(g3_ctx *c, g3_tree *t, int64_t n_act, const int32_t *active,
                              const g3_params *p, const float *h, const float *rho,
                              const float *drho_dh, const float *g_h, float *g_pos,
                              float *g_mass, void *stream) {
  G3_RANGE("g3_density_solve_backward");
  if (!c) return G3_EINVAL;
  int st = active_args_ok(c, t, n_act, active, "g3_density_solve_backward");
  if (st) return st;
  if (!params_ok(p)) return fail(c, G3_EINVAL, "g3_density_solve_backward: bad params");
  if (t->f64) return fail(c, G3_EINVAL, "g3_density_solve_backward: FP32 trees only");
  if (t->gas.n > 0 && (!h || !rho || !drho_dh || !g_h))
    return fail(c, G3_EINVAL, "g3_density_solve_backward: h, rho, drho_dh and g_h are required");
  DeviceGuard g(c->device);
  st = check_pending(c);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  Octree &o = t->gas;
  if (o.n == 0) return G3_OK;
  Work wk;
  st = prepare_work(c, t, o, t->iperm_gas, o.n, nullptr, &wk, s);
  if (st) return st;
  hipError_t e = launch_hydro_prep(o, nullptr, nullptr, h, nullptr, nullptr, 1.0f, 0, s);
  if (e == hipSuccess) e = refit_hmax(o, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_density_solve_backward prep");
  e = launch_density_solve_bwd(o, t->iperm_gas, t->n, wk.gs, wk.max_groups, n_act, active,
                               (float)p->n_ngb, h, rho, drho_dh, g_h, g_pos, g_mass, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_density_solve_backward");
  c->err.clear();
  return G3_OK;
}

int g3_hydro_force_backward(g3_ctx *c, g3_tree *t, int64_t n_act, const int32_t *active,
                            const g3_params *p, const float *vel, const float *u,
                            const float *h, const float *rho, const float *omega,
                            const float *g_acc, const float *g_dudt, float *g_pos, float *g_vel,
                            float *g_mass, float *g_h, float *g_u, float *g_rho,
                            float *g_omega, void *stream) {
  G3_RANGE("g3_hydro_force_backward");
  if (!c) return G3_EINVAL;
  int st = active_args_ok(c, t, n_act, active, "g3_hydro_force_backward");
  if (st) return st;
  if (!params_ok(p)) return fail(c, G3_EINVAL, "g3_hydro_force_backward: bad params");
  if (t->f64) return fail(c, G3_EINVAL, "g3_hydro_force_backward: FP32 trees only");
  if (t->gas.n > 0 && (!vel || !u || !h || !rho || !omega))
    return fail(c, G3_EINVAL, "g3_hydro_force_backward: null input");
  DeviceGuard g(c->device);
  st = check_pending(c);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  Octree &o = t->gas;
  if (o.n == 0) return G3_OK;
  const SphParams sp = sph_params(c, p, t, Tuning());
  float4 *up = (float4 *)scratch(c, kAdjSrc, o.n * sizeof(float4));
  if (!up) return fail(c, G3_ENOMEM, "g3_hydro_force_backward: scratch allocation failed");
  Work wk;
  st = prepare_work(c, t, o, t->iperm_gas, o.n, nullptr, &wk, s);
  if (st) return st;
  hipError_t e = launch_hydro_prep(o, vel, u, h, rho, omega, sp.gamma, 0, s);
  if (e == hipSuccess) e = refit_hmax(o, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_hydro_force_backward prep");
  e = launch_hydro_bwd(o, t->iperm_gas, t->n, wk.gs, wk.max_groups, n_act, active, sp.alpha,
                       sp.gamma, u, omega, g_acc, g_dudt, up, g_pos, g_vel, g_mass, g_h, g_u,
                       g_rho, g_omega, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_hydro_force_backward");
  c->err.clear();
  return G3_OK;
}

int g3_gravity_backward(g3_ctx *c, const g3_tree *t, int64_t n_act, const int32_t *active,
                        const g3_params *p, const float *g_acc, const float *g_pot,
                        float *g_pos, float *g_mass, void *stream) {
  G3_RANGE("g3_gravity_backward");
  if (!c) return G3_EINVAL;
  int st = active_args_ok(c, t, n_act, active, "g3_gravity_backward");
  if (st) return st;
  if (!params_ok(p)) return fail(c, G3_EINVAL, "g3_gravity_backward: bad params");
  if (t->f64) return fail(c, G3_EINVAL, "g3_gravity_backward: FP32 trees only");
  DeviceGuard g(c->device);
  st = check_pending(c);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  // last_stream stays with the SPH calls: only they count into c->counters
  const BankGuard bank(c, 1);
  const Octree &o = t->all;
  if (o.n == 0) return G3_OK;
  float4 *gsrc = (float4 *)scratch(c, kAdjSrc, o.n * sizeof(float4));
  float4 *gnode = (float4 *)scratch(c, kAdjNode, o.nnodes * sizeof(float4));
  double4 *pq = (double4 *)scratch(c, kAdjPQ, o.nnodes * sizeof(double4));
  double *rr = (double *)scratch(c, kAdjR, o.nnodes * sizeof(double));
  // fixed-point counters (8 words per member / node) and, after the
  // members', the four words of the scale's maxima
  const bool fixed = p->eps > 0.0;
  unsigned long long *gsrc_fx = fixed ? (unsigned long long *)scratch(
                                            c, kAdjSrcFx, (8 * o.n + 2) * sizeof(uint64_t))
                                      : nullptr;
  unsigned long long *gnode_fx =
      fixed ? (unsigned long long *)scratch(c, kAdjNodeFx, 8 * o.nnodes * sizeof(uint64_t))
            : nullptr;
  if (!gsrc || !gnode || !pq || !rr || (fixed && (!gsrc_fx || !gnode_fx)))
    return fail(c, G3_ENOMEM, "g3_gravity_backward: scratch allocation failed");
  Work wk;
  st = prepare_work(c, t, o, t->iperm_all, n_act, active, &wk, s);
  if (st) return st;
  hipError_t e = launch_gravity_bwd(o, wk.gs, wk.max_groups, grav_params(p, t), n_act, active,
                                    g_acc, g_pot, gsrc, gnode, gsrc_fx, gnode_fx,
                                    fixed ? (unsigned *)(gsrc_fx + 8 * o.n) : nullptr, pq, rr,
                                    g_pos, g_mass, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_gravity_backward");
  c->err.clear();
  return G3_OK;
}

}  // extern "C"
