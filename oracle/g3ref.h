/*
 * g3ref.h - FP64 CPU oracle of the Gadget3 interaction phase.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. It shares no source,
 * header, table or helper with the HIP library and never calls it.
 *
 * Method: the paper (Ragagnin et al., "Gadget3 on GPUs with OpenACC",
 * arXiv 2003.10850) names the physics but prints no formula: Barnes-Hut
 * gravity, the SPH density (evaluated repeatedly while the smoothing length
 * is adjusted) and the SPH hydrodynamic force, each evaluated for the
 * particles active at a step through tree walks made per group of active
 * particles, which collect the neighbours inside a search radius (section 1,
 * fifth paragraph). The formulas below are the published methods Gadget
 * builds on, each cited where it is implemented in g3ref.cpp:
 *   - Wendland C6 kernel, support radius h (Dehnen & Aly 2012, table 1);
 *   - mass-weighted neighbour number (4 pi / 3) h^3 rho / m = N_ngb solved
 *     for h by bisection (Springel & Hernquist 2002, eq. 6);
 *   - grad-h SPH force in energy form with signal-velocity viscosity
 *     (Springel 2005, eqs. 7, 9, 13-14; Monaghan 1997);
 *   - Barnes-Hut octree with the geometric opening test (Barnes & Hut 1986)
 *     and Plummer softening.
 *
 * All sums are FP64. The two decisions that must match the FP32 kernels
 * bit-for-bit (the neighbour predicate and the Barnes-Hut opening test) are
 * evaluated on the FP32 inputs in FP32, with explicit fmaf, unless
 * G3REF_FLAG_FP64_DECISIONS is set.
 */
#ifndef G3REF_H
#define G3REF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Result-defining parameters (same fields and meaning as the product's). */
typedef struct {
  double n_ngb;   /* target mass-weighted neighbour number (> 1365/48) */
  double h_tol;   /* relative bracket width of the h bisection */
  double gamma;   /* adiabatic index */
  double alpha;   /* viscosity strength */
  double theta;   /* Barnes-Hut opening angle */
  double eps;     /* Plummer softening */
  double G;       /* gravitational constant */
  int32_t leaf_size; /* octree leaf capacity B */
  int32_t flags;     /* G3REF_FLAG_* */
} g3ref_params;

#define G3REF_FLAG_FP64_DECISIONS 1 /* predicate and opening test in FP64 */

enum { G3REF_OK = 0, G3REF_EINVAL = -1, G3REF_ENOCONV = -5 };
enum { G3REF_GATHER = 0, G3REF_SYMMETRIC = 1, G3REF_GRAVITY = 2 };

typedef struct g3ref_tree g3ref_tree;

/* Number of OpenMP threads the parallel loops use, and setting it (n > 0). */
int32_t g3ref_threads(void);
void g3ref_set_threads(int32_t n);

/* Wendland C6 and its derivatives at (r, h): W, dW/dr, dW/dh, F = dW/dr / r. */
void g3ref_kernel(double r, double h, double *W, double *dWdr, double *dWdh,
                  double *F);

/* 63-bit Morton key of one position in a box (lo xyz, side L). */
uint64_t g3ref_key(const double *x, const double *box);

/* Octree over all particles (gas_only = 0) or over gas only (gas_only = 1).
 * pos [n][3], mass [n], type [n] (NULL: all gas), box [4] = lo xyz + side. */
g3ref_tree *g3ref_tree_build(int64_t n, const double *pos, const double *mass,
                             const uint8_t *type, const double *box,
                             int32_t leaf_size, int32_t gas_only);
void g3ref_tree_free(g3ref_tree *t);
/* Drift update (the refit of the time integration, paper section 1: tree
 * nodes are drifted rather than rebuilt): take new positions [n][3] and
 * masses [n]; keep the build's member order, keys, cells, topology and node
 * cubes; recompute the node moments and the members' bounding boxes. */
int g3ref_tree_refit(g3ref_tree *t, const double *pos, const double *mass);
int64_t g3ref_tree_nnodes(const g3ref_tree *t);
int64_t g3ref_tree_nmembers(const g3ref_tree *t);
/* Any output pointer may be NULL. order/keys: [nmembers]; node arrays:
 * [nnodes] in preorder (children in Morton order); com: [nnodes][3]. */
void g3ref_tree_export(const g3ref_tree *t, int64_t *order, uint64_t *keys,
                       int64_t *node_start, int64_t *node_count,
                       int32_t *node_level, int64_t *node_skip,
                       double *node_mass, double *node_com);

/* SPH density of the active gas particles. solve_h = 1: bisection for h
 * (h is output); 0: h is input. Outputs at active rows of [n] arrays.
 * *nonconv receives the number of particles whose bracket hit the cap. */
int g3ref_density(const g3ref_tree *gas, int64_t n_act, const int64_t *active,
                  const g3ref_params *p, int32_t solve_h, double *h,
                  double *rho, double *drho_dh, double *omega, int32_t *nngb,
                  int64_t *nonconv);

/* SPH hydro force. S (L1 magnitude of the acceleration terms) and npairs
 * may be NULL. */
int g3ref_hydro(const g3ref_tree *gas, int64_t n_act, const int64_t *active,
                const g3ref_params *p, const double *vel, const double *u,
                const double *h, const double *rho, const double *omega,
                double *acc, double *dudt, double *vsig, double *S,
                int32_t *npairs);

/* The hydro force with the improved-SPH switches (Beck et al. 2016):
 * per-particle viscosity strengths alpha [n] and Balsara factors balsara [n]
 * (each nullable: params->alpha and 1) and artificial conduction of
 * strength alpha_u (0: none). With all three off it is g3ref_hydro. S_du
 * (nullable) receives the L1 sum of the du/dt terms. */
int g3ref_hydro_switches(const g3ref_tree *gas, int64_t n_act, const int64_t *active,
                         const g3ref_params *p, const double *vel, const double *u,
                         const double *h, const double *rho, const double *omega,
                         const double *alpha, const double *balsara, double alpha_u,
                         double *acc, double *dudt, double *vsig, double *S,
                         int32_t *npairs, double *S_du);

/* Velocity divergence [n] and curl [n][3] of the active gas particles (the
 * grad-h SPH estimates over the density's pairs); S_div and S_curl (the L1
 * sums of the terms) nullable. */
int g3ref_velgrad(const g3ref_tree *gas, int64_t n_act, const int64_t *active,
                  const g3ref_params *p, const double *vel, const double *h,
                  const double *rho, const double *omega, double *div_v,
                  double *curl_v, double *S_div, double *S_curl);

/* Thermal conduction rate of the active gas particles. S (L1 magnitude of
 * the terms) and npairs may be NULL. kappa_j = kappa0 u_j^kappa_exp. */
int g3ref_conduction(const g3ref_tree *gas, int64_t n_act, const int64_t *active,
                     const g3ref_params *p, double kappa0, double kappa_exp,
                     const double *u, const double *h, const double *rho,
                     double *dudt, double *S, int32_t *npairs);

/* Barnes-Hut gravity. S and nterms may be NULL. */
int g3ref_gravity(const g3ref_tree *all, int64_t n_act, const int64_t *active,
                  const g3ref_params *p, double *acc, double *pot, double *S,
                  int32_t *nterms);

/* Interaction lists in CSR form. kind: GATHER (gas j with r < h_i, self
 * included), SYMMETRIC (gas j != i with r < max(h_i, h_j)) or GRAVITY
 * (particle j as its caller id, accepted node k as -(k+1)). offsets
 * [n_act+1] always written; list written when non-NULL (size offsets[n_act]). */
int g3ref_lists(const g3ref_tree *t, int32_t kind, int64_t n_act,
                const int64_t *active, const g3ref_params *p, const double *h,
                int64_t *offsets, int64_t *list);

/* Adjoints (gradients) of the three modules for a scalar loss whose
 * derivatives with respect to the outputs are given at the active rows;
 * neighbour sets and Barnes-Hut decisions held fixed, h an input. Results
 * are ADDED to the [n] (or [n][3]) gradient arrays; every pointer argument
 * named g_* is nullable. Partials come from forward-mode dual numbers over
 * each pair's or term's inputs. S (nullable) receives, per gradient entry,
 * the sum of the magnitudes of the contributions added to it, laid out as
 * the gradient arguments concatenated in order ([n][3] before [n]). */
int g3ref_density_backward(const g3ref_tree *gas, int64_t n_act, const int64_t *active,
                           const g3ref_params *p, const double *h, const double *g_rho,
                           const double *g_drho, const double *g_omega, double *g_pos,
                           double *g_mass, double *g_h, double *S);
int g3ref_hydro_backward(const g3ref_tree *gas, int64_t n_act, const int64_t *active,
                         const g3ref_params *p, const double *vel, const double *u,
                         const double *h, const double *rho, const double *omega,
                         const double *g_acc, const double *g_dudt, double *g_pos,
                         double *g_vel, double *g_mass, double *g_h, double *g_u,
                         double *g_rho, double *g_omega, double *S);
int g3ref_gravity_backward(const g3ref_tree *all, int64_t n_act, const int64_t *active,
                           const g3ref_params *p, const double *g_acc, const double *g_pot,
                           double *g_pos, double *g_mass, double *S);

#ifdef __cplusplus
}
#endif
#endif
