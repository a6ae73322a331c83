/*
 * g3.h - C ABI of libg3.so, the MI355X (gfx950) interaction phase of the
 * Gadget3 method (Ragagnin et al., "Gadget3 on GPUs with OpenACC",
 * arXiv 2003.10850).
 *
 * Each of the paper's modules evaluates, for the particles active at a step,
 * a sum over the particles that a tree walk, made once per group of active
 * particles, finds (section 1, fifth paragraph): the SPH density found by iterating the
 * smoothing length, the SPH hydrodynamic force, and Barnes-Hut gravity whose
 * node and particle interactions are evaluated inside the walk
 * (section 2.4). Each module receives only the properties it needs, with
 * read-only inputs kept apart from the updated outputs (section 2.1); each
 * entry point below mirrors that: const inputs, separate outputs.
 *
 * Conventions for every call:
 *  - Pointers are DEVICE pointers unless marked (host). Particle arrays are
 *    in the CALLER's order: row i of every [n] array is particle i.
 *  - The caller owns every input and output buffer; the library never frees
 *    or keeps them beyond the call. Outputs must not alias inputs.
 *  - Outputs are written only at the rows of the active particles; other rows
 *    are left untouched. active == NULL means every particle is active
 *    (n_act must then equal n). Active ids must be distinct and in [0, n);
 *    ids out of range are ignored, SPH calls ignore non-gas ids.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream)
 *    and the call returns without waiting, unless its comment says SYNCS.
 *  - Every call returns a g3_status and never aborts; an asynchronous device
 *    error surfaces as G3_EHIP on a later call. g3_last_error() gives text.
 *    A call that fails with G3_EINVAL, G3_ESTATE or G3_ENOMEM leaves no work
 *    of its own on the stream: the interaction calls (g3_walk, g3_density,
 *    g3_hydro_force, g3_gravity and the _backward twins) take every device
 *    buffer before their first launch and enqueue nothing when one cannot
 *    be had; the builds, which SYNC anyway, wait for what they had enqueued
 *    before returning, and a tree whose build failed is unusable (G3_ESTATE)
 *    until a later build of it succeeds. Outputs are then untouched.
 *  - One g3_ctx per host thread. A g3_tree belongs to the ctx that built it.
 *  - Streams: g3_gravity and g3_gravity_backward take their work tables from
 *    scratch of their own (g3_gravity_noalloc from its per-device region),
 *    so one of them may run on one stream while the SPH calls (density,
 *    hydro, conduction, switches and their backward twins) of the same ctx
 *    and tree run on another (gravity reads only the all-particle octree,
 *    the SPH calls only the gas one). Two calls of the same group must not
 *    overlap; a build or refit of the tree must not overlap any call that
 *    reads it.
 *  - Graph capture: g3_density, g3_hydro_force, g3_gravity and the
 *    _backward calls neither wait on the host nor use memset nodes; they
 *    allocate ctx scratch only when a call needs more than an earlier one.
 *    Run each call once outside capture with the same sizes, then capture
 *    it (hipStreamBeginCapture or torch.cuda.graph); replays reproduce the
 *    eager results. Builds, g3_walk, g3_autotune and g3_ctx_stats SYNC and
 *    cannot be captured.
 *
 * Physics (the paper prints no formula; these are the published methods
 * Gadget builds on): Wendland C6 kernel with support radius h (Dehnen & Aly
 * 2012); h from the mass-weighted neighbour number
 * (4 pi/3) h^3 rho / m = n_ngb (Springel & Hernquist 2002); grad-h SPH force
 * with signal-velocity viscosity (Springel 2005; Monaghan 1997);
 * Barnes-Hut octree, geometric opening angle, Plummer softening
 * (Barnes & Hut 1986). Gas particles are SPH sources and targets;
 * collisionless particles take part in gravity only.
 */
#ifndef G3_H
#define G3_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  G3_OK = 0,
  G3_EINVAL = -1,    /* bad argument; nothing enqueued */
  G3_ENOMEM = -2,    /* device allocation failed; nothing enqueued */
  G3_EHIP = -3,      /* HIP runtime or earlier asynchronous device error */
  G3_EOVERFLOW = -4, /* g3_walk: list longer than capacity (total is set) */
  G3_ENOCONV = -5,   /* g3_ctx_stats: some h solve did not converge */
  G3_ESTATE = -6     /* tree/ctx misuse (e.g. tree of another device) */
} g3_status;

typedef enum { G3_F32 = 0, G3_F64 = 1 } g3_dtype;

enum { G3_GATHER = 0, G3_SYMMETRIC = 1, G3_GRAVITY = 2 };

typedef struct g3_ctx g3_ctx;   /* scratch pools, counters, last error */
typedef struct g3_tree g3_tree; /* sorted copies and octrees of a forest of
                                   snapshots (one snapshot: a plain tree) */

enum { G3_MAX_SNAPSHOTS = 1 << 20 };

/* Result-defining parameters (host struct, read during the call only). */
typedef struct {
  double n_ngb;      /* target mass-weighted neighbour number, > 1365/48 */
  double h_tol;      /* relative accuracy of the h root (e.g. 1e-6) */
  double gamma;      /* adiabatic index (5/3) */
  double alpha;      /* artificial-viscosity strength (1) */
  double theta;      /* Barnes-Hut opening angle (0.5) */
  double eps;        /* Plummer softening length */
  double G;          /* gravitational constant */
  int32_t leaf_size; /* octree leaf capacity B, 1..64 (8) */
  int32_t flags;     /* reserved, must be 0 */
} g3_params;

/* Create a context on HIP device `device`. *out receives the handle. */
int g3_ctx_create(g3_ctx **out, int device);
/* Destroy a context and every tree it owns. NULL is ignored. */
void g3_ctx_destroy(g3_ctx *ctx);
/* Text of the last error of this ctx ("" if none). Valid until the next call. */
const char *g3_last_error(const g3_ctx *ctx);
/* Counters of the h solve since the last reset (reset != 0 clears them):
 * stats (host) [4] = particles whose solve hit its pass limit or the
 * bracket cap of twice the box diagonal without converging (their h and
 * density are those of the last pass), walk passes summed over wavefronts,
 * wavefronts, 0. This is where g3_density, which never waits on the host,
 * reports non-convergence: the call returns G3_ENOCONV (stats still filled)
 * when the first counter is above zero, else G3_OK. SYNCS the stream of
 * the ctx's last call other than g3_gravity / g3_gravity_backward (those
 * two count nothing here). */
int g3_ctx_stats(g3_ctx *ctx, int64_t *stats /* host [4] */, int32_t reset);
/* Kernel timing, for benchmarks and profilers. With capacity > 0, the next
 * `capacity` calls of `kind` (G3_TUNE_DENSITY: g3_density, G3_TUNE_HYDRO:
 * g3_hydro_force, G3_TUNE_GRAVITY: g3_gravity) after this call, or after
 * the last g3_ctx_kernel_times of that kind, each record a pair of HIP
 * events on their stream just before and just after their interaction
 * kernel (k_density, k_hydro, k_gravity: not the group-table and prep
 * kernels before it), so that the pair spans that kernel alone also when
 * other streams keep the device busy. Later calls, calls made under
 * stream capture and calls that fail record nothing. capacity 0 turns
 * timing off; at most G3_TIMING_MAX. Creates the events (host call, no
 * device wait). */
enum { G3_TIMING_MAX = 4096 };
int g3_ctx_kernel_timing(g3_ctx *ctx, int32_t kind, int32_t capacity);
/* The durations (ms, host [capacity]) of the kernels recorded since timing
 * of `kind` was enabled or last read, in call order; *count receives their
 * number (0..capacity). Waits for each stop event (SYNCS on them), then
 * starts a new round of up to `capacity` recordings. */
int g3_ctx_kernel_times(g3_ctx *ctx, int32_t kind, float *ms, int32_t *count);
/* Fault injection, for tests of the error paths:
 *   G3_INJECT_ALLOC     value >= 0: the next `value` device allocations the
 *                       ctx makes (trees and scratch) succeed and every
 *                       later one fails, as on a device out of memory, so
 *                       the calls that need one return G3_ENOMEM; value < 0
 *                       turns the injection off.
 *   G3_INJECT_MAX_ITER  value in 1..64: walk passes the h solve may take
 *                       before it stops and counts the particle as not
 *                       converged (g3_ctx_stats); value <= 0 restores 64.
 * Host-side only (no device work, no wait). */
enum { G3_INJECT_ALLOC = 1, G3_INJECT_MAX_ITER = 2 };
int g3_ctx_inject(g3_ctx *ctx, int32_t what, int64_t value);

/*
 * Build (or rebuild in place) the octrees of one particle set (one
 * snapshot, a forest of one tree; see g3_build_forest): one over all
 * particles (gravity) and one over the gas particles (SPH). The octree
 * follows Barnes & Hut (1986): the root is the cube `box`; a node is the set
 * of particles sharing a 3l-bit prefix of their 63-bit Morton key
 * (key = floor((x - lo) * 2^21 / side) per axis, computed in FP64, clamped
 * to [0, 2^21 - 1]); a node is subdivided while it holds more than
 * leaf_size particles and l < 21; single-child chains are kept. Nodes are
 * stored in preorder with children in Morton order. Node monopoles (mass,
 * centre of mass) are summed in FP64.
 *   n      particles (0 allowed)
 *   pos_t  G3_F32 (pos is float[n][3]: the plain path) or G3_F64 (pos is
 *          double[n][3]: the mixed-precision path). With G3_F64 the tree keeps
 *          the FP64 positions; the kernels work on FP32 offsets (the FP64
 *          difference from the target, rounded) with compensated sums, take
 *          every neighbour and opening decision exactly in FP64 (an FP32 test
 *          on the offsets, re-tested in FP64 inside its error band), and
 *          solve h in FP64. The h arrays of that tree's SPH calls are double.
 *   pos    [n][3] positions;  mass [n];  type [n] (0 gas, 1 collisionless;
 *          NULL: all gas)
 *   box    (host) [4] = lower corner xyz, side > 0
 *   tree   (host) in/out: *tree == NULL creates a tree owned by ctx; an
 *          existing tree is rebuilt reusing its buffers.
 * SYNCS (reads back the node counts). The tree keeps sorted copies, so the
 * inputs may change after the call returns. */
int g3_build_tree(g3_ctx *ctx, int64_t n, int32_t pos_t, const void *pos,
                  const float *mass, const uint8_t *type, const double *box,
                  const g3_params *p, g3_tree **tree, void *stream);
/*
 * Build a forest: n_snap independent snapshots in one tree object, so that
 * every later call serves the active particles of all of them in one
 * launch per kernel (the regime of few and uneven active particles, which
 * the paper names as its speedup limit, section 3). Snapshot k is the
 * caller ids [snap_off[k], snap_off[k+1]) with its own root cube
 * box[4k..4k+3]; each snapshot's octrees are exactly those g3_build_tree
 * builds for it alone, and no interaction crosses snapshots. Particle
 * arrays of the other calls span all n = snap_off[n_snap] particles
 * (caller order), active ids are caller ids over the whole forest, and the
 * exported octree is the concatenation of the snapshots' octrees (node
 * skips and first members offset by the earlier snapshots).
 *   n_snap    1..G3_MAX_SNAPSHOTS
 *   snap_off  (host) [n_snap + 1], snap_off[0] = 0, non-decreasing (empty
 *             snapshots allowed)
 *   box       (host) [n_snap][4] = lower corner xyz, side > 0
 * Other arguments as g3_build_tree. SYNCS. */
int g3_build_forest(g3_ctx *ctx, int32_t n_snap, const int64_t *snap_off,
                    int32_t pos_t, const void *pos, const float *mass,
                    const uint8_t *type, const double *box, const g3_params *p,
                    g3_tree **tree, void *stream);
/* Refit a built tree to moved particles without rebuilding it: the drift
 * update a code makes between rebuilds, when particles have moved little
 * since the build (the paper's tree is rebuilt only from time to time, §1).
 * The member order, octree topology, Morton keys and node cube sides of the
 * build stay; the members' positions and masses are re-read and every
 * node's centre of mass, mass and tight bounding box is recomputed, so SPH
 * neighbour sums stay exact at any drift. Barnes-Hut decisions use the
 * build's cube sides (and, for theta^2 >= 1/3, its cells for the
 * containment test), so their accuracy degrades as particles leave their
 * cells: rebuild when they have moved by a fair part of a leaf.
 *   pos   [n][3] in the tree's dtype (as built), caller order
 *   mass  [n] FP32
 * Asynchronous on `stream` (no host wait, no allocation). */
int g3_refit_tree(g3_ctx *ctx, g3_tree *tree, const void *pos, const float *mass,
                  void *stream);
/* Release a tree (also released by g3_ctx_destroy). NULL is ignored. */
void g3_tree_destroy(g3_ctx *ctx, g3_tree *tree);
/* Sizes of one of the tree's octrees: which = 0 all particles, 1 gas.
 * Host outputs, nullable. */
int g3_tree_info(const g3_tree *tree, int32_t which, int64_t *n_members,
                 int64_t *n_nodes);
/* Copy one octree out (device outputs, each nullable): order [n_members]
 * (sorted position -> caller id), keys [n_members], and per node in preorder
 * [n_nodes]: first member, member count, level, skip (index of the next node
 * after the subtree; n_nodes past the end), mass, centre of mass [n_nodes][3]
 * (FP64). */
int g3_tree_export(g3_ctx *ctx, const g3_tree *tree, int32_t which,
                   int32_t *order, uint64_t *keys, int32_t *node_start,
                   int32_t *node_count, int32_t *node_level, int32_t *node_skip,
                   double *node_mass, double *node_com, void *stream);

/*
 * Interaction lists of the active particles (the walk step the SPH modules
 * run before their sums, section 2.4), in CSR form with rows in the order
 * of `active`:
 *   G3_GATHER    gas j with |x_j - x_i| < h_i, self included;
 *   G3_SYMMETRIC gas j != i with |x_j - x_i| < max(h_i, h_j);
 *   G3_GRAVITY   the Barnes-Hut terms of i: particle j as its caller id,
 *                accepted node k (preorder index in the all-particle tree)
 *                as -(k + 1).
 * Neighbour test (exact, FP32): dx = fl(x_j - x_i) per axis,
 * r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx)), neighbour iff r2 < fl(H * H).
 * On trees built from FP64 positions every decision is the FP64 one, the
 * one the mixed-precision g3_density, g3_hydro_force and g3_gravity take:
 * ((dx dx + dy dy) + dz dz) < H H on the FP64 positions and h, and the
 * opening test on the FP64 node centres with the exact cube side.
 *   h        [n] smoothing lengths in the tree's dtype (GATHER, SYMMETRIC;
 *            ignored for GRAVITY)
 *   offsets  [n_act + 1] int64 output
 *   list     [capacity] output; entries of a row in walk order
 *   total    (host) output: offsets[n_act]
 * SYNCS. Returns G3_EOVERFLOW, with *total and offsets valid and list
 * untouched, when *total > capacity. */
int g3_walk(g3_ctx *ctx, const g3_tree *tree, int32_t kind, int64_t n_act,
            const int32_t *active, const void *h, const g3_params *p,
            int64_t capacity, int64_t *offsets, int32_t *list, int64_t *total,
            void *stream);

/*
 * SPH density of the active gas particles (section 1: the density is
 * evaluated repeatedly while each smoothing length is adjusted):
 *   rho_i   = sum_j m_j W(|x_ij|, h_i)     (gas j, self included)
 *   drho_dh = sum_j m_j dW/dh(|x_ij|, h_i)
 *   omega_i = 1 + h_i / (3 rho_i) drho_dh  (grad-h correction)
 *   nngb_i  = number of gas j meeting the neighbour test at h_i
 * solve_h = 1: h_i is first solved from (4 pi/3) h^3 rho(h) / m_i = n_ngb to
 * relative accuracy h_tol (h[i] > 0 on entry is the first guess); h is then
 * an output. solve_h = 0: h is an input. h is float for a tree built from
 * FP32 positions, double for FP64 positions (the h solve then runs in FP64).
 * Output pointers other than h may be NULL. Particles whose solve does not
 * converge (no root below the cap of twice the box diagonal, e.g. a target
 * above what the snapshot's gas can give, or the pass limit reached) keep
 * the h and sums of their last pass and are counted: g3_ctx_stats then
 * returns G3_ENOCONV. */
int g3_density(g3_ctx *ctx, const g3_tree *tree, int64_t n_act,
               const int32_t *active, const g3_params *p, int32_t solve_h,
               void *h, float *rho, float *drho_dh, float *omega,
               int32_t *nngb, void *stream);

/*
 * SPH hydrodynamic force of the active gas particles: grad-h SPH in energy
 * form (Springel 2005) with signal-velocity viscosity (Monaghan 1997), over
 * gas pairs j != i with |x_ij| < max(h_i, h_j):
 *   P = (gamma-1) rho u, c = sqrt(gamma (gamma-1) u), A = P / (omega rho^2)
 *   F(r,h) = dW/dr / r;  g_i = F(r, h_i);  g_j = F(r, h_j)
 *   a_i   -= m_j (A_i g_i + A_j g_j) x_ij
 *   w = v_ij . x_ij / r; if w < 0: Pi = (alpha/2) (c_i + c_j - 3w)(-w) /
 *        ((rho_i + rho_j)/2), else 0;  a_i -= m_j Pi (g_i + g_j)/2 x_ij
 *   du_i/dt += m_j A_i g_i v_ij.x_ij + m_j Pi (g_i + g_j)/4 v_ij.x_ij
 *   vsig_i = max_j (c_i + c_j - 3 min(w, 0))   (0 with no pair)
 * with x_ij = x_i - x_j, v_ij = v_i - v_j; pairs at r = 0 add nothing.
 *   vel [n][3], u [n], h [n], rho [n], omega [n]: inputs for every gas
 *   particle (neighbours need theirs); h is float or double like the
 *   tree's positions; acc [n][3], dudt, vsig, npairs (number of pairs of i)
 *   are outputs, each nullable.
 * Refits the gas octree's per-node maximum h from `h` first. */
int g3_hydro_force(g3_ctx *ctx, g3_tree *tree, int64_t n_act,
                   const int32_t *active, const g3_params *p, const float *vel,
                   const float *u, const void *h, const float *rho,
                   const float *omega, float *acc, float *dudt, float *vsig,
                   int32_t *npairs, void *stream);

/*
 * Thermal conduction, the third SPH module the paper moves to the GPU
 * (paper section 1, the module list; section 3.3). The paper prints no
 * formula; Gadget's conduction module (Jubelgas, Springel & Dolag 2004)
 * discretises rho du/dt = div(kappa grad u) in the form of Brookshaw (1985):
 *   du_i/dt = sum_j m_j (kappa_i + kappa_j) (u_i - u_j) Fbar_ij / (rho_i rho_j),
 *   Fbar_ij = (F(r, h_i) + F(r, h_j)) / 2,  F = (1/r) dW/dr,
 * over gas j != i with r < max(h_i, h_j) (the hydro force's symmetric test);
 * pairs at r = 0 add nothing. The conductivity is in units of the internal
 * energy per mass (the heat capacity absorbed into it) and a power law of
 * it: kappa = kappa0 u^kappa_exp (kappa_exp = 5/2 follows Spitzer's
 * temperature dependence, 0 is a constant conductivity). Every pair's
 * exchange is antisymmetric, so sum_i m_i du_i/dt = 0 over a set that holds
 * every pair of its members.
 *   u [n], h [n] (float, FP32 trees only), rho [n]: inputs of every gas
 *   particle; dudt [n] (the conduction rate alone) and npairs [n]: outputs
 *   at the active gas rows, each nullable.
 * Refits the gas octree's per-node maximum h from `h` first. */
int g3_conduction(g3_ctx *ctx, g3_tree *tree, int64_t n_act,
                  const int32_t *active, const g3_params *p, double kappa0,
                  double kappa_exp, const float *u, const void *h,
                  const float *rho, float *dudt, int32_t *npairs, void *stream);

/*
 * The improved SPH that the paper's code ran (Beck et al. 2016; paper
 * section 1 names it) adds switches to the hydro force; the paper prints
 * none of them, so these are the published methods, in their usual form:
 *   - velocity divergence and curl, the grad-h SPH estimates over the
 *     density's gather pairs (r < h_i):
 *       div v_i  =  (1/(Omega_i rho_i)) sum_j m_j (v_j - v_i) . grad_i W(r, h_i),
 *       curl v_i = -(1/(Omega_i rho_i)) sum_j m_j (v_j - v_i) x grad_i W(r, h_i),
 *     grad_i W = F(r, h_i) (x_i - x_j);
 *   - the Balsara (1995) factor f = |div v| / (|div v| + |curl v| + eps c/h),
 *     c = sqrt(gamma (gamma-1) u), near 1 in compression, near 0 in shear;
 *   - a time-dependent viscosity strength per particle (Morris & Monaghan
 *     1997, with the source factor of Rosswog et al. 2000, the Balsara
 *     factor in the source):
 *       d alpha/dt = -(alpha - alpha_min)/tau + f max(-div v, 0)(alpha_max - alpha),
 *       tau = h / (decay c),
 *     stepped exactly over dt for inputs held fixed (it is linear in alpha);
 *   - in the hydro force the strength alpha of the viscosity term becomes
 *     (alpha_i + alpha_j)/2 * (f_i + f_j)/2, and artificial conduction of the
 *     internal energy (Price 2008, eq. 28) is added:
 *       du_i/dt += m_j alpha_u v_u (u_i - u_j) gbar r / rhobar,
 *       v_u = sqrt(|P_i - P_j| / rhobar), rhobar = (rho_i + rho_j)/2,
 *     gbar = (F(r, h_i) + F(r, h_j))/2, over the hydro force's pairs; every
 *     pair's exchange is antisymmetric, so total energy is conserved.
 */
typedef struct {
  double alpha_min;   /* floor of the viscosity strength (0.025) */
  double alpha_max;   /* ceiling of the viscosity strength (1) */
  double decay;       /* decay parameter l of tau = h / (l c) (0.2) */
  double balsara_eps; /* eps of the Balsara factor's c/h term (1e-4) */
  double alpha_u;     /* artificial conduction strength (1; 0: none) */
  int32_t flags;      /* reserved, must be 0 */
} g3_switch_params;

/* Velocity divergence and curl of the active gas particles (FP32 trees).
 *   vel [n][3], h [n] (float), rho [n], omega [n]: inputs of every gas
 *   particle; div_v [n] and curl_v [n][3]: outputs at the active gas rows,
 *   each nullable. */
int g3_velocity_gradients(g3_ctx *ctx, g3_tree *tree, int64_t n_act,
                          const int32_t *active, const g3_params *p,
                          const float *vel, const void *h, const float *rho,
                          const float *omega, float *div_v, float *curl_v,
                          void *stream);
/* One step dt of the viscosity strength and the Balsara factor of the rows
 * `active` of [n] caller-order arrays (active NULL: every row, n_act == n):
 * u [n], h [n] (float or double after h_type), div_v [n], curl_v [n][3]
 * inputs; alpha [n] in/out (nullable: the factor only), balsara [n] out
 * (nullable). No tree: a per-particle kernel. */
int g3_viscosity_switch(g3_ctx *ctx, int64_t n, int32_t h_type, int64_t n_act,
                        const int32_t *active, const g3_params *p,
                        const g3_switch_params *sw, double dt, const float *u,
                        const void *h, const float *div_v, const float *curl_v,
                        float *alpha, float *balsara, void *stream);
/* g3_hydro_force with the switches: per-particle strengths alpha [n] and
 * Balsara factors balsara [n] of every gas particle (each nullable:
 * p->alpha and 1) and artificial conduction of strength sw->alpha_u (the
 * other fields of sw are not read). Same pairs, outputs and rules as
 * g3_hydro_force, which it equals with one strength, unit factors and
 * alpha_u = 0. */
int g3_hydro_force_switches(g3_ctx *ctx, g3_tree *tree, int64_t n_act,
                            const int32_t *active, const g3_params *p,
                            const g3_switch_params *sw, const float *vel,
                            const float *u, const void *h, const float *rho,
                            const float *omega, const float *alpha,
                            const float *balsara, float *acc, float *dudt,
                            float *vsig, int32_t *npairs, void *stream);

/*
 * Barnes-Hut gravity of the active particles from all particles: walk the
 * all-particle octree in preorder from the root; a node whose cube does not
 * contain x_i and whose side l satisfies l < theta |x_i - c| contributes its
 * monopole (mass M at centre of mass c), an unaccepted leaf contributes each
 * member j != i, other nodes are opened. Every term is Plummer-softened:
 *   a_i -= G m x_ij / (r^2 + eps^2)^(3/2),  pot_i -= G m / (r^2 + eps^2)^(1/2).
 * The opening test is exact in FP32: dx = fl(fl(c) - x_i),
 * r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx)), accept iff
 * fl(fl(l) * fl(l)) < fl(fl(theta^2) * r2).
 *   acc [n][3], pot [n], nterms [n] (terms of i): outputs, each nullable. */
int g3_gravity(g3_ctx *ctx, const g3_tree *tree, int64_t n_act,
               const int32_t *active, const g3_params *p, float *acc,
               float *pot, int32_t *nterms, void *stream);

/*
 * g3_gravity without any device allocation, for callers that cannot
 * allocate (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc): same arguments, kernels and results as g3_gravity.
 * The call's work tables (active-set compaction, group table, per-XCD
 * queues) live in a fixed region of 64 MiB per GPU, a device array that
 * each GPU running the library holds until the process ends; it is looked
 * up at g3_ctx_create. A call whose tables need more returns G3_EINVAL and
 * enqueues nothing: with an active list the tables take about 20 bytes per
 * member of the all-particle octree (36 with groups split at octree cells,
 * see g3_tuning_set), so up to about 3.3e6 members fit; with every particle
 * active (active == NULL) a few bytes per target. The tree must have been
 * built (builds allocate). Every call on one GPU shares that GPU's region
 * and the call clears what it needs at its start, so results never depend
 * on an earlier call; calls whose work overlaps on one GPU (concurrent
 * streams, or several host threads) race on the region and must be
 * serialised by the caller. */
int g3_gravity_noalloc(g3_ctx *ctx, const g3_tree *tree, int64_t n_act,
                       const int32_t *active, const g3_params *p, float *acc,
                       float *pot, int32_t *nterms, void *stream);

/*
 * Time integration around the interaction phase. The paper's code moves
 * only the particles that are active at a step, on adaptive steps, and
 * drifts the tree between rebuilds instead of rebuilding it (paper section 1
 * on adaptive time-stepping, section 2.2). These calls run that loop on the
 * device: the kick-drift-kick leapfrog on power-of-two time bins of
 * Springel (2005, section 5).
 *
 * A system step lasts dt_max and is cut into 2^B ticks of tau = dt_max/2^B.
 * A particle in bin k (0 <= k <= B) takes steps of 2^(B-k) ticks and is
 * active at tick T iff 2^(B-k) divides T. Its step criterion (Springel
 * 2005, eqs. 34 and 16) is dt = sqrt(2 eta eps / |a|), for gas also at most
 * C h / vsig; the bin is the smallest k in [0, B] with dt_max/2^k <= dt (B
 * if none), but at tick T no smaller than B - min(tz(T), B), tz the number
 * of trailing zero bits of T, so that the new step ends on a tick that its
 * bin is active at. The criterion is evaluated in FP64 from the FP32
 * forces.
 *
 * One system step, from a synchronised state whose forces and bins are
 * known (g3_integrate_start, or the end of the previous system step):
 *  1. the trees are built from the positions (the call SYNCS, as builds do);
 *     every particle takes the opening half kick of its bin's step;
 *  2. for T = 1 .. 2^B: every particle drifts x += v tau (in the positions'
 *     precision); both octrees are refit to the new positions
 *     (g3_refit_tree: same order and topology, new moments and boxes); the
 *     active particles get the density with the smoothing-length solve from
 *     their last h (active gas), the hydro force (active gas) from every gas
 *     particle's velocity and internal energy predicted to T from the middle
 *     of its current step, v + a (T - T_mid) tau and
 *     max(u + du/dt (T - T_mid) tau, 0), and the stored h, rho and Omega of
 *     inactive neighbours, and gravity; then acc = gravity + hydro, the
 *     closing half kick with the step they had, the new bin and, unless
 *     T = 2^B, the opening half kick of the new step;
 *  3. at T = 2^B every particle has been active: the state is synchronised.
 * Kicks are v += a dt/2 and, for gas, u = max(u + du/dt dt/2, 0).
 * Active sets are found on the device from the bins (no host wait inside
 * the tick loop).
 */
typedef struct {
  double dt_max;     /* the longest step (bin 0), > 0 */
  double courant;    /* C of the hydrodynamic step criterion (0.15) */
  double eta;        /* accuracy parameter of the gravitational step (0.025) */
  int32_t bin_depth; /* B: bins 0..B, 2^B ticks per system step, 0..20 */
  int32_t flags;     /* reserved, must be 0 */
} g3_integ_params;

/* The particle state (device pointers, caller order, [n] rows). pos and h
 * are float or double after pos_t; the rest FP32. Updated in place. */
typedef struct {
  void *pos;          /* [n][3] in/out */
  float *vel;         /* [n][3] in/out */
  const float *mass;  /* [n] */
  float *u;           /* [n] in/out: internal energy per unit mass (gas rows) */
  const uint8_t *type;/* [n] 0 gas, 1 collisionless; NULL: all gas */
  void *h;            /* [n] in/out: smoothing length (gas rows; <= 0: none yet) */
  float *rho, *omega; /* [n] in/out: density and grad-h factor (gas rows) */
  float *acc;         /* [n][3] in/out: total acceleration, gravity + hydro */
  float *dudt, *vsig; /* [n] in/out: du/dt and max signal velocity (gas rows) */
  float *pot;         /* [n] in/out: gravitational potential */
  int32_t *bin;       /* [n] in/out: time bin */
} g3_state;

/* Forces and bins of a synchronised state at the start of integration:
 * builds the trees into *tree (a new tree when *tree is NULL) and evaluates
 * density with the h solve, hydro and gravity of every particle, then the
 * bins (no kick). SYNCS (a build). */
int g3_integrate_start(g3_ctx *ctx, g3_tree **tree, int64_t n, int32_t pos_t,
                       const g3_state *state, const double *box /* host [4] */,
                       const g3_params *p, const g3_integ_params *ip,
                       void *stream);
/* One system step (see above), rebuilding *tree from the positions at its
 * start. tick_active (device int64 [2^B], nullable) receives the number of
 * active particles at each tick. Non-converged h solves are counted as in
 * g3_density (g3_ctx_stats). SYNCS once, at the build. */
int g3_system_step(g3_ctx *ctx, g3_tree **tree, int64_t n, int32_t pos_t,
                   const g3_state *state, const double *box /* host [4] */,
                   const g3_params *p, const g3_integ_params *ip,
                   int64_t *tick_active, void *stream);

/*
 * Launch tuning (the batching extension's autotuner). Two launch choices
 * change neither a count nor a decision, only the order in which FP32
 * partial sums are formed (so results agree to rounding):
 *   walk_leaf  SPH walks take octree subtrees of at most this many members
 *              whole into a candidate tile instead of descending (1..4096);
 *   split      -1: a group is up to 64 consecutive targets of one snapshot;
 *              L >= 0: groups also break where consecutive targets leave a
 *              level-L octree cell, so a sparse active set gives compact
 *              groups instead of wide ones; G3_SPLIT_AUTO: L is taken per
 *              snapshot from its member count m as floor(log8(m / 128)),
 *              the level whose cells hold about 128 members (no level
 *              break where that is below 1);
 *   streams    density on FP32 trees: 1 or 4 candidate streams per
 *              wavefront; with 4, each quarter of the 64 lanes scans only
 *              the candidates some lane of its quarter can reach (other
 *              kinds and FP64 trees ignore it).
 * Choices are kept per ctx for each kind (G3_TUNE_*) and size class
 * floor(log2(number of targets)); a call uses its class's choice, else the
 * nearest tuned class's, else the defaults: density walk_leaf 128, split
 * G3_SPLIT_AUTO; hydro and gravity walk_leaf 64, split -1; streams 1.
 * Every default depends on per-snapshot quantities only, so a snapshot in a
 * forest forms the same groups as on its own tree. */
enum { G3_TUNE_DENSITY = 0, G3_TUNE_HYDRO = 1, G3_TUNE_GRAVITY = 2 };
enum { G3_SPLIT_AUTO = -2 };
/* Time every candidate (walk_leaf 16, 32, 64, 128 x split -1,
 * G3_SPLIT_AUTO, 2, 3, 4, 5 for the SPH kernels, times streams 1, 4 for the
 * density; split for gravity) on this tree and active set, and keep the
 * fastest per kind for this size class. The density runs its h solve on a
 * copy of h (tree dtype; h[i] > 0 is a first guess); hydro is tuned only
 * when vel, u, rho and omega are given. Writes no output, and leaves the
 * ctx statistics unchanged. SYNCS. */
int g3_autotune(g3_ctx *ctx, g3_tree *tree, int64_t n_act, const int32_t *active,
                const g3_params *p, const void *h, const float *vel,
                const float *u, const float *rho, const float *omega,
                void *stream);
/* The choice a call of `kind` over n_targets targets of one snapshot would
 * use (host outputs, nullable). */
int g3_tuning_get(g3_ctx *ctx, int32_t kind, int64_t n_targets,
                  int32_t *walk_leaf, int32_t *split, int32_t *streams);
/* Set the choice for n_targets' size class; n_targets < 0 replaces every
 * class of `kind` by this one choice. */
int g3_tuning_set(g3_ctx *ctx, int32_t kind, int64_t n_targets,
                  int32_t walk_leaf, int32_t split, int32_t streams);
/* Keep the tuned choices across processes: save writes every tuned class
 * of the ctx to the text file `path` (host string; a header line
 * "g3-tuning 1", then one line "kind class walk_leaf split streams" per
 * class); load replaces the ctx's choices with a file's, after checking
 * every line as g3_tuning_set would (G3_EINVAL, and the ctx unchanged, for
 * an unreadable or malformed file). Choices never change results beyond
 * rounding, so a file from another device is safe, only perhaps slower. */
int g3_tuning_save(g3_ctx *ctx, const char *path);
int g3_tuning_load(g3_ctx *ctx, const char *path);

/*
 * Adjoints (the _backward twins). The paper stops at the forward modules;
 * these give the gradients of a scalar loss L with respect to the modules'
 * inputs, from the gradients of L with respect to their outputs at the
 * active rows (upstream gradients; NULL means zero). Neighbour sets and
 * Barnes-Hut decisions are those the forward call takes at the same inputs
 * (the forward maps are piecewise smooth in them), and h is an input of
 * each; g3_density_solve_backward adds the derivative through the h solve
 * where h came from it. Gradients are ADDED (+=) to the
 * caller's [n] / [n][3] arrays in caller order, each nullable; inactive
 * particles receive what the active particles' sums owe them. FP32 trees
 * only (G3_EINVAL otherwise). Density and hydro adjoints are gathered per
 * particle in a fixed order (run-to-run identical); the gravity adjoint adds
 * the source side of each term across wavefronts, as fixed-point integers
 * when eps > 0 (run-to-run identical) and as float atomics when eps = 0
 * (last bits may vary between runs): see g3_gravity_backward.
 *
 * Density: L's upstream gradients g_rho, g_drho_dh, g_omega; rho and
 * drho_dh are the forward outputs at the active rows (they enter through
 * omega). Outputs dL/dpos, dL/dmass, dL/dh. */
int g3_density_backward(g3_ctx *ctx, g3_tree *tree, int64_t n_act,
                        const int32_t *active, const g3_params *p,
                        const float *h, const float *rho, const float *drho_dh,
                        const float *g_rho, const float *g_drho_dh,
                        const float *g_omega, float *g_pos, float *g_mass,
                        float *g_h, void *stream);
/* Through the smoothing-length solve (the iterations of the paper's SPH
 * density module, section 1): g_h [n] is the upstream gradient of the
 * SOLVED h at the active rows, and h, rho, drho_dh are g3_density's outputs
 * there (solve_h = 1). Each such h_i is the root of
 * N_eff(h_i) = (4 pi/3) h_i^3 rho_i / m_i = N_ngb, so by the implicit
 * function theorem
 *   dL/dtheta = -sum_i lambda_i dN_eff_i/dtheta,
 *   lambda_i  = g_h_i / (dN_eff_i/dh_i) at fixed positions and masses,
 * which is the density adjoint seeded with
 * g_rho_i = -g_h_i h_i / (3 rho_i + h_i drho_i/dh), plus the explicit 1/m_i
 * of N_eff: dL/dm_i += g_h_i h_i rho_i / (m_i (3 rho_i + h_i drho_i/dh)).
 * A row whose N_eff misses p->n_ngb by more than 1e-3 (relative: a solve
 * that did not converge, or an h held at the cap) passes nothing. Outputs
 * dL/dpos [n][3] and dL/dmass [n], added; the gradients of rho, drho_dh and
 * Omega at fixed h are g3_density_backward's (its dL/dh is part of g_h). */
int g3_density_solve_backward(g3_ctx *ctx, g3_tree *tree, int64_t n_act,
                              const int32_t *active, const g3_params *p,
                              const float *h, const float *rho,
                              const float *drho_dh, const float *g_h,
                              float *g_pos, float *g_mass, void *stream);
/* Hydro force: upstream g_acc [n][3], g_dudt [n] (the signal velocity is
 * not differentiated); inputs as g3_hydro_force. Outputs dL/dpos, dL/dvel,
 * dL/dmass, dL/dh, dL/du, dL/drho, dL/domega. */
int g3_hydro_force_backward(g3_ctx *ctx, g3_tree *tree, int64_t n_act,
                            const int32_t *active, const g3_params *p,
                            const float *vel, const float *u, const float *h,
                            const float *rho, const float *omega,
                            const float *g_acc, const float *g_dudt,
                            float *g_pos, float *g_vel, float *g_mass,
                            float *g_h, float *g_u, float *g_rho,
                            float *g_omega, void *stream);
/* Gravity: upstream g_acc [n][3], g_pot [n]. Node monopoles pass their
 * gradients to their members through M = sum m and c = sum m x / M.
 * Outputs dL/dpos, dL/dmass. With eps > 0 the result is deterministic (the
 * same bits on every run): the terms each source collects from many
 * wavefronts are added as 64-bit fixed-point integers, at a scale bounded
 * from the largest upstream gradients, the largest mass and eps, and turned
 * back into floats once. With eps = 0 they are FP32 atomics (order-dependent
 * in the last bits). */
int g3_gravity_backward(g3_ctx *ctx, const g3_tree *tree, int64_t n_act,
                        const int32_t *active, const g3_params *p,
                        const float *g_acc, const float *g_pot, float *g_pos,
                        float *g_mass, void *stream);

#ifdef __cplusplus
}
#endif
#endif
