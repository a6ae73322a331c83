// Internal declarations of libg3.so: device data layout, the context and
// tree objects, and the launch wrappers shared by the translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "g3.h"

namespace g3 {

constexpr int kMaxLevel = 21;  // 21 key bits per axis, 63-bit Morton keys
constexpr int kWave = 64;      // CDNA wavefront width

// One octree node, 64 bytes: a walk reads it with one scalar load.
struct __align__(16) Node {
  float4 com_m;  // centre of mass (FP32 copy of the FP64 moment), mass
  float4 lo_h;   // tight bounding box lower corner, max h of gas members
  float4 hi_l;   // tight bounding box upper corner, cube side l
  int4 meta;     // skip, first member, member count, level | leaf << 8
};
static_assert(sizeof(Node) == 64, "node must be 64 bytes");

constexpr int kLeafBit = 256;

// The gravity walk's copy of a node, 32 bytes: two nodes per 64-byte line,
// so a descent to cur + 1 often finds its node in the line just loaded.
//   com_m   centre of mass, mass
//   meta    skip, first member, member count of a leaf (-1: internal), the
//           cube side l as bits; l = side of the root cube * 2^-level
//           exactly, so the level is the difference of the two exponents
struct __align__(16) GNode {
  float4 com_m;
  int4 meta;
};
static_assert(sizeof(GNode) == 32, "gravity node must be 32 bytes");

// One octree over a subset of the particles (all of them, or the gas ones),
// with the members in Morton order.
struct Octree {
  int64_t n = 0;       // members
  int64_t nnodes = 0;
  int32_t max_level = 0;
  int64_t cap_n = 0, cap_nodes = 0;
  uint64_t *keys = nullptr;  // [n] sorted Morton keys
  int32_t *perm = nullptr;   // [n] sorted position -> caller id
  float4 *xm = nullptr;      // [n] sorted (x, y, z, m)
  Node *nodes = nullptr;     // [nnodes] preorder
  GNode *gnodes = nullptr;   // [nnodes] the gravity walk's copy (all-particle octree)
  double4 *mom = nullptr;    // [nnodes] FP64 (M, M x, M y, M z)
  // SPH member data in sorted order (gas octree only, filled by the calls)
  float4 *vh = nullptr;   // (vx, vy, vz, h)
  float4 *aux = nullptr;  // (A, c, rho, 1/h)
  // FP64 positions (x, y, z, m) in sorted order: trees built from FP64 input
  double4 *x64 = nullptr;
  int64_t cap_x64 = 0;
  double *h64 = nullptr;  // FP64 h in sorted order (FP64 trees, SPH calls)
  int64_t cap_h64 = 0;
  double4 *c64 = nullptr;  // [nnodes] FP64 centre of mass and mass (FP64 trees)
  int64_t cap_c64 = 0;
  // forest of snapshots: snapshot k owns the sorted members [soff[k], soff[k+1])
  // and the nodes [nroot[k], nroot[k+1]) (its root first, when it has members)
  int32_t *soff = nullptr;   // [n_snap + 1]
  int32_t *nroot = nullptr;  // [n_snap + 1]
  int64_t cap_snap = 0;
};

// Launch choices that never change a count or a decision (only the order in
// which FP32 partial sums are formed): SPH walks take subtrees of at most
// walk_leaf members whole; split >= 0 cuts groups at level-`split` cells.
// Group split level chosen per snapshot from its member count m:
// floor(log8(m / 128)), the level whose cells hold about 128 members on
// average (no level cut below 1).
constexpr int kSplitAuto = -2;

struct Tuning {
  int walk_leaf = 64;
  int split = -1;  // -1 none, kSplitAuto, or a level
  int streams = 1;  // density: candidate streams per wave (1 or 4)
};
enum TuneKind { kTuneDensity = 0, kTuneHydro = 1, kTuneGravity = 2, kTuneKinds = 3 };

}  // namespace g3

struct g3_tree {
  g3_ctx *owner = nullptr;
  int device = 0;
  int64_t n = 0;  // caller particles
  int64_t cap_n = 0;
  // snapshots: caller ids [snap_off[k], snap_off[k+1]) in box k (lo xyz, side)
  int32_t n_snap = 1;
  std::vector<int64_t> snap_off;  // host [n_snap + 1]
  std::vector<double> box;        // host [n_snap][4]
  int64_t *coff = nullptr;        // device copy of snap_off
  double4 *sbox = nullptr;        // device copy of the boxes
  int64_t cap_snap = 0;
  double max_side = 0;            // largest snapshot side
  int32_t leaf = 8;
  bool built = false;  // false until a build has completed (a failed build leaves it false)
  int32_t f64 = 0;   // positions (and h) are FP64: the mixed-precision path
  // FP64 trees: the largest |coordinate| of any member, as the bits of a
  // non-negative float (device word, set at every build and refit); the
  // walks pad their radii by 2^-20 of it, a bound on the rounding of the
  // FP32 position copies they prune with
  unsigned *absmax = nullptr;
  int32_t *iperm_all = nullptr;  // [n] caller id -> position in `all`
  int32_t *iperm_gas = nullptr;  // [n] caller id -> position in `gas`, or -1
  g3::Octree all, gas;
};

struct g3_ctx {
  int device = 0;
  std::string err;
  std::vector<g3_tree *> trees;
  struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
  };
  // two banks of scratch slots: bank 1 serves the gravity calls, bank 0
  // every other call, so that a gravity call may run on one stream while
  // the SPH calls of the same ctx run on another
  static constexpr int kBankSlots = 32;
  Buf scratch[2 * kBankSlots];
  int bank = 0;  // the bank of the call in progress (host side)
  // autotuned launch choices: (kind, floor(log2(targets))) -> choice
  std::map<std::pair<int, int>, g3::Tuning> tuning;
  unsigned long long *counters = nullptr;  // device [8]: [0] non-converged h
  int64_t *pinned = nullptr;               // host pinned readback slots [8]
  hipStream_t last_stream = nullptr;
  // fault injection (g3_ctx_inject): device allocations left before every
  // later one fails (-1: off), and the h solve's pass limit
  int64_t alloc_budget = -1;
  int max_iter = 64;
  // opt-in kernel timing (g3_ctx_kernel_timing), per kind (density, hydro,
  // gravity): event pairs recorded on the call's stream around its
  // interaction kernel, for the first `capacity` calls after enabling or
  // after the last read
  struct Timing {
    std::vector<hipEvent_t> ev;  // start, stop of pair k at 2k, 2k + 1
    int capacity = 0;
    int count = 0;
  };
  Timing timing[3];  // indexed by g3::TuneKind
};

namespace g3 {

// scratch slots (grow-only buffers owned by the ctx)
enum Slot {
  kSortKeys = 0, kSortVals, kSortTmp, kScanTmp, kCounts, kOffsets,
  kFlags, kTargets, kRows, kIds, kLevel, kWalkCounts, kMisc,
  kSnapKeys, kSnapKeysAlt, kGroups, kAdjSrc, kAdjNode, kAdjPQ, kAdjR,
  kGasFlags, kGasSlot, kGasScan, kIntAccH, kIntVp, kIntUp, kCondCh, kHydroExt,
  kAdjSrcFx, kAdjNodeFx, kNumSlots
};
static_assert(kNumSlots <= g3_ctx::kBankSlots, "more scratch slots than a bank holds");

// Selects the gravity calls' scratch bank for the lifetime of the guard.
struct BankGuard {
  g3_ctx *c;
  int prev;
  BankGuard(g3_ctx *ctx, int bank) : c(ctx), prev(ctx->bank) { c->bank = bank; }
  ~BankGuard() { c->bank = prev; }
  BankGuard(const BankGuard &) = delete;
  BankGuard &operator=(const BankGuard &) = delete;
};

void *scratch(g3_ctx *c, int slot, size_t bytes);  // nullptr on failure

// Device allocation on behalf of a ctx: hipMalloc, unless the ctx's
// allocation-failure injection says this one fails (then *p = nullptr and
// hipErrorOutOfMemory).
hipError_t dev_malloc(g3_ctx *c, void **p, size_t bytes);

// ---- launch wrappers (each returns hipGetLastError() of its launches) ----

// Exclusive scan with the total: out[i] = sum in[0..i), out[n] = sum in[0..n).
// tmp must hold scan_tmp_elems(n) elements of the output type.
int64_t scan_tmp_elems(int64_t n);
hipError_t scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp,
                    hipStream_t s);
hipError_t scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, int64_t *tmp,
                           hipStream_t s);

// Stable LSD radix sort of (key, value) pairs by key bits [0, bits), bits a
// multiple of 8. tmp must hold radix_tmp_bytes(n) bytes. Result ends in
// keys/vals.
size_t radix_tmp_bytes(int64_t n);
hipError_t radix_sort_pairs(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt,
                            uint32_t *vals_alt, int64_t n, int bits, void *tmp, hipStream_t s);

// Tree build of one octree (members already selected in `ids`/`keys`).
// The gas octree (o == t->gas) takes its members from the all-particle
// octree built before it, filtered by `type` (nullptr: all gas).
int build_octree(g3_ctx *c, g3_tree *t, Octree &o, const void *pos, int f64,
                 const float *mass, int64_t m, hipStream_t s, const uint8_t *type = nullptr);
// Keep the octree's order, topology, keys and cube sides; re-read the
// members' positions and masses and recompute every node's moments and box.
int refit_octree(g3_ctx *c, g3_tree *t, Octree &o, const void *pos, const float *mass,
                 hipStream_t s);
hipError_t refit_hmax(Octree &o, hipStream_t s);
// FP64 trees: t->absmax = max |coordinate| over the members of t->all.
hipError_t update_absmax(g3_tree *t, hipStream_t s);

hipError_t fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);

// Work of one interaction launch: groups of up to 64 Morton-consecutive
// targets (one per lane) that never straddle two segments. A segment is a
// run of consecutive targets of one snapshot: the snapshot's whole active
// set, or, when groups are split by a key level L, the run of its targets
// that share one level-L octree cell. Segment k holds targets
// [tstart[k], tstart[k+1]) and groups [gstart[k], gstart[k+1]) and belongs
// to snapshot seg_snap[k], whose octree is the node range
// [nroot[snap], nroot[snap+1]).
struct Groups {
  const int32_t *targets;   // compacted sorted positions; nullptr: every member
  const int32_t *tstart;    // [nseg + 1]
  const int32_t *gstart;    // [nseg + 1]
  const int32_t *seg_snap;  // [nseg]
  const int32_t *nseg;      // device scalar: number of segments
  const int32_t *nroot;     // [n_snap + 1]
  const double4 *sbox;      // [n_snap] snapshot box: lo xyz, side
  unsigned *queue;          // [8] per-XCD counters, zero at launch
  int n_snap;
};

// Upper bound on the groups of max_targets targets in n_snap snapshots.
inline int64_t max_groups_of(int64_t max_targets, int64_t n_snap) {
  return (max_targets + kWave - 1) / kWave + (n_snap < max_targets ? n_snap : max_targets);
}



// Active set -> group table of one octree (scratch owned by the ctx).
// rows[t] is the index in `active` of target t (nullptr with every member
// active: rows are then caller ids). max_groups bounds the group count.
struct Work {
  Groups gs;
  const int32_t *rows;
  int64_t max_groups;
  const uint32_t *ntarg;  // device count of the targets (nullptr: every member)
};
// A caller-given device region that stands in for the ctx's scratch slots:
// each slot is carved from it once per call, 256-byte aligned, in the order
// the slots are first asked for; a slot asked for again gets the same bytes
// (it must not need more than the first time). `base` is a device address.
struct Arena {
  char *base = nullptr;
  size_t cap = 0, used = 0;
  void *slot_p[kNumSlots] = {};
  size_t slot_bytes[kNumSlots] = {};
};
// The slot's buffer from the arena when one is given (nullptr when the
// arena is full), else from the ctx's scratch.
void *scratch_in(g3_ctx *c, Arena *a, int slot, size_t bytes);

int prepare_work(g3_ctx *c, const g3_tree *t, const Octree &o, const int32_t *iperm,
                 int64_t n_act, const int32_t *active, Work *w, hipStream_t s,
                 int split = -1, Arena *arena = nullptr, const int32_t *bins = nullptr,
                 int32_t kmin = 0);
// (bins: the targets are instead the members whose particle's bins[caller
// id] >= kmin, found on the device; active and n_act are then ignored.)

// Bytes of device memory that the allocation-free calls may use per GPU,
// and that region's address on `device` (nullptr until noalloc_init has
// run for it). noalloc_init looks the address up once per device, with
// that device current; later calls return the kept address.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
int noalloc_init(int device);  // hipError_t of the lookup
void *noalloc_region(int device);

// Grid of a persistent launch: the workgroups that can be resident at once
// (occupancy of `kern` x compute units), or fewer if there are few groups.
unsigned persistent_grid(const void *kern, int block, int64_t max_groups);

struct SphParams {
  float n_ngb, h_tol, gamma, alpha;
  int max_iter;
  int walk_leaf;  // SPH walks take subtrees of at most this many members whole
  int streams;    // density candidate streams per wave (1 or 4; FP32 trees)
  int f64;        // FP64 positions and h: mixed-precision kernels
  const unsigned *absmax;  // FP64 trees: device bits of max |x| (walk pad 2^-20 of it)
};

hipError_t launch_density(const Octree &gas, const Groups &gs, int64_t max_groups,
                          const SphParams &sp, int solve_h, void *h, float *rho,
                          float *drho_dh, float *omega, int32_t *nngb,
                          unsigned long long *counters, hipStream_t s);
hipError_t launch_hydro_prep(Octree &gas, const float *vel, const float *u, const void *h,
                             const float *rho, const float *omega, float gamma, int f64,
                             hipStream_t s);
// ext (nullable): the improved-SPH switches' sorted inputs (alpha, Balsara
// factor, u, rho) from launch_hydro_ext_prep, with conduction strength alpha_u.
hipError_t launch_hydro(const Octree &gas, const Groups &gs, int64_t max_groups,
                        const SphParams &sp, float *acc, float *dudt, float *vsig,
                        int32_t *npairs, hipStream_t s, const float4 *ext = nullptr,
                        float alpha_u = 0.0f);
hipError_t launch_hydro_ext_prep(Octree &gas, const float *u, const float *rho,
                                 const float *alpha, const float *balsara, float alpha0,
                                 float4 *ext, hipStream_t s);
// Velocity divergence and curl (switches.hip), after the hydro prep of vh
// (v, h); rho, omega in caller order.
hipError_t launch_velgrad(const Octree &gas, const Groups &gs, int64_t max_groups,
                          int walk_leaf, const float *rho, const float *omega, float *div_v,
                          float *curl_v, hipStream_t s);
// The viscosity strength step and the Balsara factor of the rows `active`
// (nullptr: rows 0..n-1), see switches.hip.
struct SwitchStep {
  float gamma, alpha_min, alpha_max, decay, eps, dt;
};
hipError_t launch_alpha_update(int64_t n, int64_t n_act, const int32_t *active,
                               const SwitchStep &sw, int f64, const float *u, const void *h,
                               const float *div_v, const float *curl_v, float *alpha,
                               float *balsara, hipStream_t s);

struct GravParams {
  float theta2, eps2, G;
  int inside_test;  // evaluate the cube-containment test (theta^2 >= 1/3)
  int f64;          // FP64 positions: mixed-precision kernels, FP64 decisions
  double theta;     // opening angle (FP64 decisions)
};
hipError_t launch_gravity(const Octree &all, const Groups &gs, int64_t max_groups,
                          const GravParams &gp, float *acc, float *pot, int32_t *nterms,
                          hipStream_t s);

// Adjoints. Gradients are ADDED to the caller-order arrays (nullable).
// Density: every gas member walks its symmetric neighbourhood (all_gas:
// the groups of every gas member); the node hmax must be refit from h.
hipError_t launch_density_bwd(Octree &gas, const int32_t *iperm, int64_t n_caller,
                              const Groups &all_gas, int64_t max_groups, int64_t n_act,
                              const int32_t *active, const float *h, const float *rho,
                              const float *drho, const float *g_rho, const float *g_drho,
                              const float *g_omega, float *g_pos, float *g_mass, float *g_h,
                              hipStream_t s);
// Through the smoothing-length solve: the density adjoint seeded from g_h
// by the implicit function theorem on N_eff(h) = N_ngb (rows that did not
// converge pass nothing); hmax refit from h as above.
hipError_t launch_density_solve_bwd(Octree &gas, const int32_t *iperm, int64_t n_caller,
                                    const Groups &all_gas, int64_t max_groups, int64_t n_act,
                                    const int32_t *active, float n_ngb, const float *h,
                                    const float *rho, const float *drho, const float *g_h,
                                    float *g_pos, float *g_mass, hipStream_t s);
// Hydro: like the density (every gas member, symmetric walk) after the
// hydro prep of vh and aux; scratch up [n_gas].
hipError_t launch_hydro_bwd(Octree &gas, const int32_t *iperm, int64_t n_caller,
                            const Groups &all_gas, int64_t max_groups, int64_t n_act,
                            const int32_t *active, float alpha, float gamma, const float *u,
                            const float *omega, const float *g_acc, const float *g_dudt,
                            float4 *up, float *g_pos, float *g_vel, float *g_mass, float *g_h,
                            float *g_u, float *g_rho, float *g_omega, hipStream_t s);
// Gravity over the active targets `gs` (n_act rows of `active`, nullptr:
// every member); scratch gsrc [n], gnode [nnodes], the fixed-point counters
// gsrc_fx [n][8] and gnode_fx [nnodes][8] with mx [4] (used when eps > 0),
// pq [nnodes], rr [nnodes].
hipError_t launch_gravity_bwd(const Octree &all, const Groups &gs, int64_t max_groups,
                              const GravParams &gp, int64_t n_act, const int32_t *active,
                              const float *g_acc, const float *g_pot, float4 *gsrc,
                              float4 *gnode, unsigned long long *gsrc_fx,
                              unsigned long long *gnode_fx, unsigned *mx, double4 *pq,
                              double *rr, float *g_pos, float *g_mass, hipStream_t s);

// Thermal conduction (conduction.hip): ch [n_gas] scratch of the sorted
// pair inputs; the gas octree's node hmax must be refit from h first.
hipError_t launch_conduction_prep(Octree &gas, const float *u, const void *h, int f64,
                                  const float *rho, float kappa0, float kappa_exp,
                                  float4 *ch, hipStream_t s);
hipError_t launch_conduction(const Octree &gas, const Groups &gs, int64_t max_groups,
                             int walk_leaf, const float4 *ch, float *dudt, int32_t *npairs,
                             hipStream_t s);

// Time integration (integrate.hip). One tick's particle update, see
// k_update: a particle takes part iff every_particle or bin >= kmin.
struct IntegUpdate {
  int every_particle = 0, sum = 0, close = 0, rebin = 0, open = 0;
  int32_t kmin = 0, depth = 0;
  double dt_max = 0, eta_eps2 = 0, courant = 0;  // eta_eps2 = 2 eta eps
};
hipError_t launch_drift(void *pos, int f64, const float *vel, int64_t n, double tau,
                        hipStream_t s);
hipError_t launch_predict(int64_t n, const uint8_t *type, const float *vel, const float *u,
                          const float *acc, const float *dudt, const int32_t *bin, int depth,
                          int64_t T, double tau, float *vp, float *up, hipStream_t s);
hipError_t launch_update(int64_t n, int f64, const IntegUpdate &up, const uint8_t *type,
                         float *vel, float *u, float *acc, const float *acc_h, const float *dudt,
                         const float *vsig, const void *h, int32_t *bin, hipStream_t s);
hipError_t launch_store_count(const uint32_t *count, int64_t *out, hipStream_t s);

// Walk lists: counts pass (list == nullptr) or fill pass.
// absmax: the tree's largest coordinate (FP64 trees, SPH kinds).
hipError_t launch_walk(const Octree &o, int kind, const Groups &gs, const int32_t *rows,
                       int64_t max_groups, const GravParams &gp, const unsigned *absmax,
                       int32_t *counts, const int64_t *offsets, int32_t *list, hipStream_t s);

}  // namespace g3
