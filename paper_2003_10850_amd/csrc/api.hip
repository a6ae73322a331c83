// The C ABI of libg3.so (declared in include/g3.h): argument checks, device
// selection, scratch management and the order of the launches of each call.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>

#include "g3_device.h"
#include "g3_internal.h"

namespace g3 {

int select_gas(g3_ctx *c, const uint8_t *type, int64_t n, int64_t *m_out, hipStream_t s);

void *scratch(g3_ctx *c, int slot, size_t bytes) {
  g3_ctx::Buf &b = c->scratch[slot];
  if (b.p && bytes <= b.bytes) return b.p;
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
  const size_t want = bytes + bytes / 4 + 256;
  if (hipMalloc(&b.p, want) != hipSuccess) {
    b.p = nullptr;
    return nullptr;
  }
  b.bytes = want;
  return b.p;
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

int compact_targets(g3_ctx *c, const Octree &o, const int32_t *iperm, int64_t n_caller,
                    int64_t n_act, const int32_t *active, int32_t **targets, int32_t **rows,
                    uint32_t **dcount, hipStream_t s) {
  *targets = nullptr;
  *rows = nullptr;
  *dcount = nullptr;
  if (!active || o.n == 0) return G3_OK;
  const int64_t m = o.n;
  uint32_t *mark = (uint32_t *)scratch(c, kFlags, (m + 1) * sizeof(uint32_t));
  uint32_t *slot = (uint32_t *)scratch(c, kOffsets, (m + 1) * sizeof(uint32_t));
  int32_t *rowp1 = (int32_t *)scratch(c, kCounts, (m + 1) * sizeof(int32_t));
  uint32_t *stmp = (uint32_t *)scratch(c, kScanTmp, scan_tmp_elems(m) * sizeof(uint32_t));
  int32_t *tg = (int32_t *)scratch(c, kTargets, (m + 1) * sizeof(int32_t));
  int32_t *rw = (int32_t *)scratch(c, kRows, (m + 1) * sizeof(int32_t));
  if (!mark || !slot || !rowp1 || !stmp || !tg || !rw)
    return fail(c, G3_ENOMEM, "device allocation of the active-set scratch failed");
  k_zero_u32<<<nblk(m), 256, 0, s>>>(mark, m);
  if (n_act > 0)
    k_mark<<<nblk(n_act), 256, 0, s>>>(active, n_act, iperm, n_caller, mark, rowp1);
  hipError_t e = scan_u32(mark, slot, m, stmp, s);
  if (e != hipSuccess) return hip_fail(c, e, "active-set scan");
  k_compact<<<nblk(m), 256, 0, s>>>(mark, slot, rowp1, m, tg, rw);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, "active-set compaction");
  *targets = tg;
  *rows = rw;
  *dcount = slot + m;
  return G3_OK;
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
  if (hipMalloc((void **)&c->counters, 8 * sizeof(unsigned long long)) != hipSuccess) {
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
  *out = c;
  return G3_OK;
}

static void free_octree(Octree &o) {
  for (void *p : {(void *)o.keys, (void *)o.perm, (void *)o.xm, (void *)o.nodes, (void *)o.mom,
                  (void *)o.vh, (void *)o.aux, (void *)o.x64, (void *)o.h64, (void *)o.c64})
    if (p) (void)hipFree(p);
  o = Octree();
}

static void free_tree(g3_tree *t) {
  if (!t) return;
  if (t->iperm_all) (void)hipFree(t->iperm_all);
  if (t->iperm_gas) (void)hipFree(t->iperm_gas);
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
  return G3_OK;
}

int g3_build_tree(g3_ctx *c, int64_t n, int32_t pos_t, const void *pos, const float *mass,
                  const uint8_t *type, const double *box, const g3_params *p, g3_tree **tree,
                  void *stream) {
  if (!c) return G3_EINVAL;
  if (n < 0 || n >= (int64_t)INT32_MAX) return fail(c, G3_EINVAL, "g3_build_tree: n out of range");
  if (pos_t != G3_F32 && pos_t != G3_F64)
    return fail(c, G3_EINVAL, "g3_build_tree: pos_t must be G3_F32 or G3_F64");
  if (n > 0 && (!pos || !mass)) return fail(c, G3_EINVAL, "g3_build_tree: null pos/mass");
  if (!box || !(box[3] > 0.0) || !std::isfinite(box[0]) || !std::isfinite(box[1]) ||
      !std::isfinite(box[2]) || !std::isfinite(box[3]))
    return fail(c, G3_EINVAL, "g3_build_tree: box must be lo xyz and a finite side > 0");
  if (!params_ok(p)) return fail(c, G3_EINVAL, "g3_build_tree: bad params");
  if (!tree) return fail(c, G3_EINVAL, "g3_build_tree: null tree handle");
  g3_tree *t = *tree;
  if (t && t->owner != c) return fail(c, G3_ESTATE, "g3_build_tree: tree of another ctx");
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
  if (n > t->cap_n || !t->iperm_all) {
    if (t->iperm_all) (void)hipFree(t->iperm_all);
    if (t->iperm_gas) (void)hipFree(t->iperm_gas);
    t->iperm_all = t->iperm_gas = nullptr;
    t->cap_n = 0;
    const int64_t cap = n > 0 ? n : 1;
    if (hipMalloc((void **)&t->iperm_all, cap * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void **)&t->iperm_gas, cap * sizeof(int32_t)) != hipSuccess)
      return fail(c, G3_ENOMEM, "g3_build_tree: allocation failed");
    t->cap_n = cap;
  }
  t->n = n;
  std::memcpy(t->box, box, sizeof(t->box));
  t->scale = std::ldexp(1.0, kMaxLevel) / box[3];
  t->leaf = p->leaf_size;
  t->f64 = pos_t == G3_F64;
  // FP64 positions are walked through their FP32 copies: pad every pruning
  // radius by a bound on the rounding of coordinates as large as the box's
  double amax = 0.0;
  for (int a = 0; a < 3; ++a)
    amax = std::max(amax, std::max(std::fabs(box[a]), std::fabs(box[a] + box[3])));
  t->slack = t->f64 ? (float)std::ldexp(amax, -20) : 0.0f;
  st = build_octree(c, t, t->all, pos, t->f64, mass, n, s);
  if (st) return st;
  hipError_t e = fill_i32(t->iperm_gas, -1, n, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_build_tree");
  int64_t mgas = 0;
  st = select_gas(c, type, n, &mgas, s);
  if (st) return st;
  st = build_octree(c, t, t->gas, pos, t->f64, mass, mgas, s);
  if (st) return st;
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
  if (!c) return G3_EINVAL;
  if (!t || (which != 0 && which != 1)) return fail(c, G3_EINVAL, "g3_tree_export: bad tree");
  if (t->owner != c) return fail(c, G3_ESTATE, "g3_tree_export: tree of another ctx");
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
  gp.side = t->box[3];
  return gp;
}

// Tuning knob (never result-defining): SPH walks stop descending at
// subtrees of at most this many members and scan them whole.
static int walk_leaf_from_env() {
  static int v = [] {
    const char *e = std::getenv("G3_WALK_LEAF");
    int x = e ? std::atoi(e) : 64;
    return x < 1 ? 1 : (x > 4096 ? 4096 : x);
  }();
  return v;
}

static SphParams sph_params(const g3_params *p, const g3_tree *t) {
  SphParams sp;
  sp.n_ngb = (float)p->n_ngb;
  sp.h_tol = (float)p->h_tol;
  sp.gamma = (float)p->gamma;
  sp.alpha = (float)p->alpha;
  sp.max_iter = 64;
  sp.walk_leaf = walk_leaf_from_env();
  sp.f64 = t->f64;
  sp.slack = t->slack;
  return sp;
}

static int active_args_ok(g3_ctx *c, const g3_tree *t, int64_t n_act, const int32_t *active,
                          const char *who) {
  if (!t) return fail(c, G3_EINVAL, std::string(who) + ": null tree");
  if (t->owner != c) return fail(c, G3_ESTATE, std::string(who) + ": tree of another ctx");
  if (n_act < 0) return fail(c, G3_EINVAL, std::string(who) + ": n_act < 0");
  if (!active && n_act != t->n)
    return fail(c, G3_EINVAL, std::string(who) + ": active == NULL needs n_act == n");
  return G3_OK;
}

int g3_walk(g3_ctx *c, const g3_tree *tc, int32_t kind, int64_t n_act, const int32_t *active,
            const void *h, const g3_params *p, int64_t capacity, int64_t *offsets,
            int32_t *list, int64_t *total, void *stream) {
  if (!c) return G3_EINVAL;
  int st = active_args_ok(c, tc, n_act, active, "g3_walk");
  if (st) return st;
  if (tc->f64)
    return fail(c, G3_EINVAL, "g3_walk: explicit lists are built for FP32 trees only");
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
  hipError_t e;
  if (kind != G3_GRAVITY && o.n > 0) {
    e = launch_hydro_prep(o, nullptr, nullptr, h, nullptr, nullptr, 1.0f, 0, s);
    if (e == hipSuccess && kind == G3_SYMMETRIC) e = refit_hmax(o, s);
    if (e != hipSuccess) return hip_fail(c, e, "g3_walk prep");
  }
  int32_t *targets, *rows;
  uint32_t *dcount;
  st = compact_targets(c, o, iperm, t->n, n_act, active, &targets, &rows, &dcount, s);
  if (st) return st;
  const int64_t maxt = active ? std::min<int64_t>(n_act, o.n) : o.n;
  int32_t *counts = (int32_t *)scratch(c, kWalkCounts, (n_act + 1) * sizeof(int32_t));
  int64_t *stmp = (int64_t *)scratch(c, kMisc, scan_tmp_elems(n_act) * sizeof(int64_t) + 64);
  if (!counts || !stmp) return fail(c, G3_ENOMEM, "g3_walk: allocation failed");
  e = fill_i32(counts, 0, n_act, s);
  GravParams gp = grav_params(p, t);
  if (e == hipSuccess)
    e = launch_walk(o, kind, targets, rows, dcount, maxt, gp, counts, nullptr, nullptr, s);
  if (e == hipSuccess) e = scan_i32_to_i64(counts, offsets, n_act, stmp, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&c->pinned[3], offsets + n_act, sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_walk count pass");
  *total = c->pinned[3];
  if (*total > capacity) return fail(c, G3_EOVERFLOW, "g3_walk: list exceeds capacity");
  if (*total > 0) {
    e = launch_walk(o, kind, targets, rows, dcount, maxt, gp, counts, offsets, list, s);
    if (e != hipSuccess) return hip_fail(c, e, "g3_walk fill pass");
  }
  c->err.clear();
  return G3_OK;
}

int g3_density(g3_ctx *c, const g3_tree *t, int64_t n_act, const int32_t *active,
               const g3_params *p, int32_t solve_h, void *h, float *rho, float *drho_dh,
               float *omega, int32_t *nngb, void *stream) {
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
  int32_t *targets, *rows;
  uint32_t *dcount;
  st = compact_targets(c, o, t->iperm_gas, t->n, n_act, active, &targets, &rows, &dcount, s);
  if (st) return st;
  const int64_t maxt = active ? std::min<int64_t>(n_act, o.n) : o.n;
  const float hcap = (float)(2.0 * std::sqrt(3.0) * t->box[3]);
  hipError_t e = launch_density(o, targets, dcount, maxt, sph_params(p, t), solve_h ? 1 : 0, h,
                                rho, drho_dh, omega, nngb, c->counters, s, hcap);
  if (e != hipSuccess) return hip_fail(c, e, "g3_density");
  c->err.clear();
  return G3_OK;
}

int g3_hydro_force(g3_ctx *c, g3_tree *t, int64_t n_act, const int32_t *active,
                   const g3_params *p, const float *vel, const float *u, const void *h,
                   const float *rho, const float *omega, float *acc, float *dudt, float *vsig,
                   int32_t *npairs, void *stream) {
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
  const SphParams sp = sph_params(p, t);
  hipError_t e = launch_hydro_prep(o, vel, u, h, rho, omega, sp.gamma, t->f64, s);
  if (e == hipSuccess) e = refit_hmax(o, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_hydro_force prep");
  int32_t *targets, *rows;
  uint32_t *dcount;
  st = compact_targets(c, o, t->iperm_gas, t->n, n_act, active, &targets, &rows, &dcount, s);
  if (st) return st;
  const int64_t maxt = active ? std::min<int64_t>(n_act, o.n) : o.n;
  e = launch_hydro(o, targets, dcount, maxt, sp, acc, dudt, vsig, npairs, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_hydro_force");
  c->err.clear();
  return G3_OK;
}

int g3_gravity(g3_ctx *c, const g3_tree *t, int64_t n_act, const int32_t *active,
               const g3_params *p, float *acc, float *pot, int32_t *nterms, void *stream) {
  if (!c) return G3_EINVAL;
  int st = active_args_ok(c, t, n_act, active, "g3_gravity");
  if (st) return st;
  if (!params_ok(p)) return fail(c, G3_EINVAL, "g3_gravity: bad params");
  DeviceGuard g(c->device);
  st = check_pending(c);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  const Octree &o = t->all;
  int32_t *targets, *rows;
  uint32_t *dcount;
  st = compact_targets(c, o, t->iperm_all, t->n, n_act, active, &targets, &rows, &dcount, s);
  if (st) return st;
  const int64_t maxt = active ? std::min<int64_t>(n_act, o.n) : o.n;
  hipError_t e =
      launch_gravity(o, targets, dcount, maxt, grav_params(p, t), acc, pot, nterms, s);
  if (e != hipSuccess) return hip_fail(c, e, "g3_gravity");
  c->err.clear();
  return G3_OK;
}

}  // extern "C"
