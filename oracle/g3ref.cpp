/*
 * g3ref.cpp - FP64 CPU oracle of the Gadget3 interaction phase.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path. It shares no code
 * with the HIP library. Written for clarity, not speed: every function is the
 * plain definition (for sums over neighbours) or the algorithm's steps in the
 * order the method states them (Barnes-Hut walk, bisection for h).
 *
 * The paper (arXiv 2003.10850) names the modules but prints no formula; the
 * published methods used are cited at each function.
 */
#include "g3ref.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

const double kPi = 3.14159265358979323846;
/* Wendland C6 normalisation in 3D: 1365 / (64 pi) (Dehnen & Aly 2012, tab. 1) */
const double kWc6 = 1365.0 / (64.0 * kPi);
const int kMaxLevel = 21; /* 21 bits per axis, 63-bit Morton keys */

/* ------------------------------------------------------------------ kernel */

/* Wendland C6 with compact support radius h (Gadget convention):
 *   W(r,h)   = C/h^3 (1-q)^8 (1 + 8q + 25q^2 + 32q^3),  q = r/h < 1
 *   dW/dr    = -22 C/h^4 q (1-q)^7 (1 + 7q + 16q^2)
 *   F        = (1/r) dW/dr = -22 C/h^5 (1-q)^7 (1 + 7q + 16q^2)
 *   dW/dh    = C/h^4 (1-q)^7 (448q^4 + 133q^3 - 29q^2 - 21q - 3)
 * (the last equals -(3W + r dW/dr)/h; both are pinned by tests). */
void wc6(double r, double h, double *W, double *dWdr, double *dWdh, double *F) {
  const double q = r / h;
  if (!(q < 1.0)) {
    *W = *dWdr = *dWdh = *F = 0.0;
    return;
  }
  const double t = 1.0 - q;
  const double t2 = t * t, t4 = t2 * t2, t7 = t4 * t2 * t, t8 = t7 * t;
  const double h3 = h * h * h, h4 = h3 * h, h5 = h4 * h;
  const double p8 = 1.0 + q * (8.0 + q * (25.0 + q * 32.0));
  const double p7 = 1.0 + q * (7.0 + q * 16.0);
  const double ph = -3.0 + q * (-21.0 + q * (-29.0 + q * (133.0 + q * 448.0)));
  *W = kWc6 / h3 * t8 * p8;
  *dWdr = -22.0 * kWc6 / h4 * q * t7 * p7;
  *F = -22.0 * kWc6 / h5 * t7 * p7;
  *dWdh = kWc6 / h4 * t7 * ph;
}

double wc6_W(double r, double h) {
  double W, a, b, c;
  wc6(r, h, &W, &a, &b, &c);
  return W;
}

/* ------------------------------------------------------------------- keys */

uint32_t cell_of(double x, double lo, double scale) {
  double f = std::floor((x - lo) * scale);
  const double top = (double)((1u << kMaxLevel) - 1u);
  if (!(f >= 0.0)) f = 0.0;
  if (f > top) f = top;
  return (uint32_t)f;
}

/* Interleave three 21-bit integers, x highest within each 3-bit digit, most
 * significant digit first: digit l (1-based level) selects the child octant
 * at tree level l. */
uint64_t interleave(uint32_t ix, uint32_t iy, uint32_t iz) {
  uint64_t k = 0;
  for (int b = kMaxLevel - 1; b >= 0; --b)
    k = (k << 3) | ((uint64_t)((ix >> b) & 1u) << 2) |
        ((uint64_t)((iy >> b) & 1u) << 1) | (uint64_t)((iz >> b) & 1u);
  return k;
}

double key_scale(double L) { return std::ldexp(1.0, kMaxLevel) / L; }

} // namespace

/* ------------------------------------------------------------------- tree */

struct RefNode {
  int64_t start = 0, count = 0, skip = 0;
  int32_t level = 0;
  uint32_t cx = 0, cy = 0, cz = 0; /* integer cube coordinates at level */
  double l = 0.0;                  /* cube side */
  double clo[3] = {0, 0, 0};       /* cube lower corner */
  double M = 0.0, com[3] = {0, 0, 0};
  double blo[3] = {0, 0, 0}, bhi[3] = {0, 0, 0}; /* members' bounding box */
  std::vector<int64_t> child;      /* preorder indices, Morton order */
};

struct g3ref_tree {
  int64_t n = 0;              /* length of the caller arrays */
  std::vector<double> pos;    /* [n][3] */
  std::vector<double> mass;   /* [n] */
  std::vector<uint8_t> type;  /* [n] */
  std::vector<uint32_t> cell; /* [n][3] integer key coordinates */
  double box[4] = {0, 0, 0, 1};
  int32_t leaf = 8;
  std::vector<int64_t> order; /* sorted member -> caller id */
  std::vector<uint64_t> keys; /* sorted member keys */
  std::vector<RefNode> nodes; /* preorder */
};

namespace {

/* A node is the set of members sharing a 3*level-bit key prefix; it is
 * subdivided while it holds more than leaf members and level < 21; empty
 * octants make no node and single-child chains are kept (Barnes & Hut 1986
 * octree, here over Morton-sorted members). */
int64_t subdivide(g3ref_tree &t, int64_t s, int64_t e, int32_t level) {
  const int64_t idx = (int64_t)t.nodes.size();
  t.nodes.emplace_back();
  std::vector<int64_t> kids;
  if (e - s > t.leaf && level < kMaxLevel) {
    const int shift = 3 * (kMaxLevel - level - 1);
    int64_t a = s;
    while (a < e) {
      const uint64_t d = (t.keys[a] >> shift) & 7u;
      int64_t b = a;
      while (b < e && ((t.keys[b] >> shift) & 7u) == d) ++b;
      kids.push_back(subdivide(t, a, b, level + 1));
      a = b;
    }
  }
  RefNode &nd = t.nodes[idx];
  nd.start = s;
  nd.count = e - s;
  nd.level = level;
  nd.child = kids;
  nd.skip = (int64_t)t.nodes.size();
  const int64_t first = t.order[s];
  const int sh = kMaxLevel - level;
  nd.cx = t.cell[3 * first + 0] >> sh;
  nd.cy = t.cell[3 * first + 1] >> sh;
  nd.cz = t.cell[3 * first + 2] >> sh;
  nd.l = std::ldexp(t.box[3], -level);
  nd.clo[0] = t.box[0] + nd.cx * nd.l;
  nd.clo[1] = t.box[1] + nd.cy * nd.l;
  nd.clo[2] = t.box[2] + nd.cz * nd.l;
  return idx;
}

/* Monopole moments in FP64 (M = sum m, com = sum m x / M) and the members'
 * bounding box of every node. */
void node_moments(g3ref_tree &t) {
  for (RefNode &nd : t.nodes) {
    double M = 0.0, S[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
      nd.blo[a] = INFINITY;
      nd.bhi[a] = -INFINITY;
    }
    for (int64_t k = nd.start; k < nd.start + nd.count; ++k) {
      const int64_t j = t.order[k];
      M += t.mass[j];
      for (int a = 0; a < 3; ++a) {
        const double x = t.pos[3 * j + a];
        S[a] += t.mass[j] * x;
        nd.blo[a] = std::min(nd.blo[a], x);
        nd.bhi[a] = std::max(nd.bhi[a], x);
      }
    }
    nd.M = M;
    for (int a = 0; a < 3; ++a) nd.com[a] = M > 0.0 ? S[a] / M : nd.clo[a] + 0.5 * nd.l;
  }
}

bool inside_cube(const g3ref_tree &t, int64_t i, const RefNode &nd) {
  const int sh = kMaxLevel - nd.level;
  return (t.cell[3 * i + 0] >> sh) == nd.cx && (t.cell[3 * i + 1] >> sh) == nd.cy &&
         (t.cell[3 * i + 2] >> sh) == nd.cz;
}

/* squared distance from x to the bounding box of the node's members (0
 * inside); after a refit the members may have left the node's cube, the
 * box always holds them */
double box_dist2(const RefNode &nd, const double *x) {
  double d2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    double d = 0.0;
    if (x[a] < nd.blo[a]) d = nd.blo[a] - x[a];
    else if (x[a] > nd.bhi[a]) d = x[a] - nd.bhi[a];
    d2 += d * d;
  }
  return d2;
}

/* Collect members j of leaves whose bounding box lies within radius
 * R(node) of x (R may depend on the node, e.g. the symmetric search).
 * Pruning only: it never drops a member within R. */
template <class Radius, class Visit>
void walk_leaves(const g3ref_tree &t, int64_t k, const double *x, Radius R, Visit visit) {
  const RefNode &nd = t.nodes[k];
  const double r = R(k);
  if (box_dist2(nd, x) > r * r) return;
  if (nd.child.empty()) {
    for (int64_t s = nd.start; s < nd.start + nd.count; ++s) visit(t.order[s]);
    return;
  }
  for (int64_t c : nd.child) walk_leaves(t, c, x, R, visit);
}

const double kPruneMargin = 1.0 + 1e-5; /* FP32 predicate vs FP64 pruning */

/* Neighbour predicate. FP32 (default): dx = fl32(x_j - x_i) per axis,
 * r2 = fmaf(dz,dz, fmaf(dy,dy, dx*dx)), true iff r2 < fl32(H*H) with H the
 * FP32 radius. FP64 with G3REF_FLAG_FP64_DECISIONS. */
bool within(const g3ref_tree &t, int64_t i, int64_t j, double H, int32_t flags) {
  const double *xi = &t.pos[3 * i], *xj = &t.pos[3 * j];
  if (flags & G3REF_FLAG_FP64_DECISIONS) {
    const double dx = xj[0] - xi[0], dy = xj[1] - xi[1], dz = xj[2] - xi[2];
    return dx * dx + dy * dy + dz * dz < H * H;
  }
  const float dx = (float)xj[0] - (float)xi[0];
  const float dy = (float)xj[1] - (float)xi[1];
  const float dz = (float)xj[2] - (float)xi[2];
  const float r2 = std::fmaf(dz, dz, std::fmaf(dy, dy, dx * dx));
  const float hf = (float)H;
  const float h2 = hf * hf;
  return r2 < h2;
}

double dist(const g3ref_tree &t, int64_t i, int64_t j) {
  const double *xi = &t.pos[3 * i], *xj = &t.pos[3 * j];
  const double dx = xi[0] - xj[0], dy = xi[1] - xj[1], dz = xi[2] - xj[2];
  return std::sqrt(dx * dx + dy * dy + dz * dz);
}

bool is_gas(const g3ref_tree &t, int64_t j) { return t.type[j] == 0; }

/* --------------------------------------------------------------- density */

/* rho(h) = sum_j m_j W(r_ij, h) over gas j with r_ij < h (self included),
 * FP64 membership: the continuous function the root solve works on. */
double rho_at(const g3ref_tree &t, int64_t i, double h) {
  const double *xi = &t.pos[3 * i];
  double rho = 0.0;
  walk_leaves(t, 0, xi, [&](int64_t) { return h * kPruneMargin; }, [&](int64_t j) {
    if (!is_gas(t, j)) return;
    const double r = dist(t, i, j);
    if (r < h) rho += t.mass[j] * wc6_W(r, h);
  });
  return rho;
}

/* Mass-weighted neighbour number N_eff(h) = (4 pi / 3) h^3 rho(h) / m_i
 * (Springel & Hernquist 2002, eq. 6). */
double n_eff(const g3ref_tree &t, int64_t i, double h) {
  return 4.0 * kPi / 3.0 * h * h * h * rho_at(t, i, h) / t.mass[i];
}

/* Root of N_eff(h) = N_ngb by bracketing and bisection:
 *   start at the mean-density estimate h0 = (3 N_ngb m_i / (4 pi rho_bar))^(1/3);
 *   double (or halve) until N_eff(lo) < N_ngb <= N_eff(hi);
 *   bisect while hi - lo > tol * hi; return the midpoint.
 * Returns false if the bracket reaches the cap 2 x box diagonal. */
bool solve_h(const g3ref_tree &t, int64_t i, const g3ref_params &p, double rho_bar,
             double *h_out) {
  const double cap = 2.0 * std::sqrt(3.0) * t.box[3];
  const double target = p.n_ngb;
  double h0 = std::cbrt(3.0 * target * t.mass[i] / (4.0 * kPi * rho_bar));
  if (!(h0 > 0.0) || h0 > cap) h0 = std::min(cap, t.box[3]);
  double lo, hi;
  if (n_eff(t, i, h0) < target) {
    lo = h0;
    hi = 2.0 * h0;
    while (n_eff(t, i, hi) < target) {
      lo = hi;
      hi = 2.0 * hi;
      if (hi > cap) {
        *h_out = cap;
        return false;
      }
    }
  } else {
    hi = h0;
    lo = 0.5 * h0;
    while (n_eff(t, i, lo) >= target) {
      hi = lo;
      lo = 0.5 * lo;
    }
  }
  while (hi - lo > p.h_tol * hi) {
    const double mid = 0.5 * (lo + hi);
    if (n_eff(t, i, mid) < target) lo = mid;
    else hi = mid;
  }
  *h_out = 0.5 * (lo + hi);
  return true;
}

} // namespace

extern "C" {

int32_t g3ref_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

void g3ref_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

void g3ref_kernel(double r, double h, double *W, double *dWdr, double *dWdh, double *F) {
  wc6(r, h, W, dWdr, dWdh, F);
}

uint64_t g3ref_key(const double *x, const double *box) {
  const double s = key_scale(box[3]);
  return interleave(cell_of(x[0], box[0], s), cell_of(x[1], box[1], s),
                    cell_of(x[2], box[2], s));
}

g3ref_tree *g3ref_tree_build(int64_t n, const double *pos, const double *mass,
                             const uint8_t *type, const double *box, int32_t leaf_size,
                             int32_t gas_only) {
  if (n < 0 || (n > 0 && (!pos || !mass)) || !box || !(box[3] > 0.0) || leaf_size < 1)
    return nullptr;
  g3ref_tree *t = new g3ref_tree;
  t->n = n;
  t->pos.assign(pos, pos + 3 * n);
  t->mass.assign(mass, mass + n);
  t->type.assign((size_t)n, 0);
  if (type) t->type.assign(type, type + n);
  std::memcpy(t->box, box, sizeof(t->box));
  t->leaf = leaf_size;
  t->cell.resize(3 * (size_t)n);
  const double s = key_scale(box[3]);
  std::vector<uint64_t> key((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a) t->cell[3 * i + a] = cell_of(pos[3 * i + a], box[a], s);
    key[i] = interleave(t->cell[3 * i], t->cell[3 * i + 1], t->cell[3 * i + 2]);
    if (!gas_only || t->type[i] == 0) t->order.push_back(i);
  }
  /* Morton order; equal keys keep caller order */
  std::sort(t->order.begin(), t->order.end(), [&](int64_t a, int64_t b) {
    return key[a] < key[b] || (key[a] == key[b] && a < b);
  });
  for (int64_t i : t->order) t->keys.push_back(key[i]);
  if (!t->order.empty()) subdivide(*t, 0, (int64_t)t->order.size(), 0);
  node_moments(*t);
  return t;
}

/* A drift update of a built tree: the members' new positions and masses
 * are taken; order, keys, cells, topology and node cubes stay those of the
 * build; moments and bounding boxes are recomputed. */
int g3ref_tree_refit(g3ref_tree *t, const double *pos, const double *mass) {
  if (!t || (t->n > 0 && (!pos || !mass))) return G3REF_EINVAL;
  t->pos.assign(pos, pos + 3 * t->n);
  t->mass.assign(mass, mass + t->n);
  node_moments(*t);
  return G3REF_OK;
}

void g3ref_tree_free(g3ref_tree *t) { delete t; }
int64_t g3ref_tree_nnodes(const g3ref_tree *t) { return t ? (int64_t)t->nodes.size() : 0; }
int64_t g3ref_tree_nmembers(const g3ref_tree *t) { return t ? (int64_t)t->order.size() : 0; }

void g3ref_tree_export(const g3ref_tree *t, int64_t *order, uint64_t *keys,
                       int64_t *node_start, int64_t *node_count, int32_t *node_level,
                       int64_t *node_skip, double *node_mass, double *node_com) {
  for (size_t k = 0; k < t->order.size(); ++k) {
    if (order) order[k] = t->order[k];
    if (keys) keys[k] = t->keys[k];
  }
  for (size_t k = 0; k < t->nodes.size(); ++k) {
    const RefNode &nd = t->nodes[k];
    if (node_start) node_start[k] = nd.start;
    if (node_count) node_count[k] = nd.count;
    if (node_level) node_level[k] = nd.level;
    if (node_skip) node_skip[k] = nd.skip;
    if (node_mass) node_mass[k] = nd.M;
    if (node_com)
      for (int a = 0; a < 3; ++a) node_com[3 * k + a] = nd.com[a];
  }
}

static bool valid_params(const g3ref_params *p) {
  return p && p->leaf_size >= 1;
}

/* Density at the active gas particles (Springel & Hernquist 2002):
 *   rho_i    = sum_j m_j W(r_ij, h_i)            (self included)
 *   drho/dh  = sum_j m_j dW/dh(r_ij, h_i)
 *   Omega_i  = 1 + h_i / (3 rho_i) drho/dh
 *   n_i      = number of gas j meeting the neighbour predicate at h_i.
 * With solve_h, h_i is first found by solve_h() above. */
int g3ref_density(const g3ref_tree *gas, int64_t n_act, const int64_t *active,
                  const g3ref_params *p, int32_t solve, double *h, double *rho,
                  double *drho_dh, double *omega, int32_t *nngb, int64_t *nonconv) {
  if (!gas || !valid_params(p) || n_act < 0 || (n_act > 0 && !active) || !h)
    return G3REF_EINVAL;
  if (solve && !(p->n_ngb > 1365.0 / 48.0)) return G3REF_EINVAL;
  const g3ref_tree &t = *gas;
  double gas_mass = 0.0;
  for (int64_t j : t.order) gas_mass += t.mass[j];
  const double rho_bar = gas_mass / (t.box[3] * t.box[3] * t.box[3]);
  int64_t bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : bad)
  for (int64_t a = 0; a < n_act; ++a) {
    const int64_t i = active[a];
    if (i < 0 || i >= t.n || !is_gas(t, i)) continue;
    if (solve) {
      double hs;
      if (!solve_h(t, i, *p, rho_bar, &hs)) ++bad;
      h[i] = hs;
    }
    const double hi = h[i];
    const double *xi = &t.pos[3 * i];
    double r_ = 0.0, dr = 0.0;
    int32_t cnt = 0;
    walk_leaves(t, 0, xi, [&](int64_t) { return hi * kPruneMargin; }, [&](int64_t j) {
      if (!is_gas(t, j) || !within(t, i, j, hi, p->flags)) return;
      double W, dWdr, dWdh, F;
      wc6(dist(t, i, j), hi, &W, &dWdr, &dWdh, &F);
      r_ += t.mass[j] * W;
      dr += t.mass[j] * dWdh;
      ++cnt;
    });
    if (rho) rho[i] = r_;
    if (drho_dh) drho_dh[i] = dr;
    if (omega) omega[i] = 1.0 + hi / (3.0 * r_) * dr;
    if (nngb) nngb[i] = cnt;
  }
  if (nonconv) *nonconv = bad;
  return bad ? G3REF_ENOCONV : G3REF_OK;
}

/* Hydro acceleration, du/dt and maximum signal velocity of the active gas
 * particles: the grad-h SPH equations in energy form (Springel 2005, eqs.
 * 7 and 13-14) with the signal-velocity viscosity of Monaghan (1997) as used
 * by Gadget-2. Pairs: gas j != i with r < max(h_i, h_j) (neighbour predicate);
 * pairs at zero separation add nothing.
 *   P = (gamma-1) rho u,  c = sqrt(gamma (gamma-1) u),  A = P / (Omega rho^2)
 *   g_i = F(r, h_i), g_j = F(r, h_j), gbar = (g_i + g_j) / 2
 *   a_i   -= m_j (A_i g_i + A_j g_j) x_ij
 *   w = v_ij . x_ij / r;  if w < 0: v_sig = c_i + c_j - 3w,
 *        Pi = -(alpha/2) v_sig w / ((rho_i + rho_j)/2)    else Pi = 0
 *   a_i   -= m_j Pi gbar x_ij
 *   du_i  += m_j A_i g_i v_ij.x_ij + (1/2) m_j Pi gbar v_ij.x_ij
 *   vsig_i = max_j (c_i + c_j - 3 min(w, 0))   (0 with no pair)
 * The switches of the improved SPH that Gadget3 ran (Beck et al. 2016), each
 * a published method, change only the viscosity and add a conduction term:
 *   - per-particle viscosity strengths alpha_i (a time-dependent viscosity,
 *     Morris & Monaghan 1997) and Balsara (1995) factors f_i enter as
 *     alpha -> (alpha_i + alpha_j)/2 * (f_i + f_j)/2 in Pi (alpha_arr and
 *     balsara nullable: p->alpha and 1);
 *   - artificial conduction of the internal energy (Price 2008, eq. 28, with
 *     the pressure-difference signal speed):
 *       du_i += m_j alpha_u v_u (u_i - u_j) gbar r / rhobar,
 *       v_u = sqrt(|P_i - P_j| / rhobar), rhobar = (rho_i + rho_j)/2
 *     (alpha_u = 0: none). */
static int hydro_general(const g3ref_tree *gas, int64_t n_act, const int64_t *active,
                  const g3ref_params *p, const double *vel, const double *u, const double *h,
                  const double *rho, const double *omega, const double *alpha_arr,
                  const double *balsara, double alpha_u, double *acc, double *dudt,
                  double *vsig, double *S, int32_t *npairs, double *S_du) {
  if (!gas || !valid_params(p) || n_act < 0 || (n_act > 0 && !active) || !vel || !u ||
      !h || !rho || !omega || !std::isfinite(alpha_u) || alpha_u < 0.0)
    return G3REF_EINVAL;
  const g3ref_tree &t = *gas;
  const double gm = p->gamma;
  /* node hmax: largest h among the node's gas members (search radius) */
  std::vector<double> hmax(t.nodes.size(), 0.0);
  for (size_t k = 0; k < t.nodes.size(); ++k)
    for (int64_t s = t.nodes[k].start; s < t.nodes[k].start + t.nodes[k].count; ++s)
      hmax[k] = std::max(hmax[k], h[t.order[s]]);
  auto P_of = [&](int64_t j) { return (gm - 1.0) * rho[j] * u[j]; };
  auto A_of = [&](int64_t j) { return P_of(j) / (omega[j] * rho[j] * rho[j]); };
  auto c_of = [&](int64_t j) { return std::sqrt(gm * (gm - 1.0) * u[j]); };
  auto alpha_of = [&](int64_t j) { return alpha_arr ? alpha_arr[j] : p->alpha; };
  auto f_of = [&](int64_t j) { return balsara ? balsara[j] : 1.0; };
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t a = 0; a < n_act; ++a) {
    const int64_t i = active[a];
    if (i < 0 || i >= t.n || !is_gas(t, i)) continue;
    const double *xi = &t.pos[3 * i];
    const double Ai = A_of(i), ci = c_of(i), hi = h[i];
    double ax = 0, ay = 0, az = 0, du = 0, vs = 0, s = 0, sdu = 0;
    int32_t cnt = 0;
    walk_leaves(t, 0, xi, [&](int64_t k) { return std::max(hi, hmax[k]) * kPruneMargin; },
                [&](int64_t j) {
      if (j == i || !is_gas(t, j)) return;
      const double hm = std::max(hi, h[j]);
      if (!within(t, i, j, hm, p->flags)) return;
      ++cnt;
      const double r = dist(t, i, j);
      if (!(r > 0.0)) return;
      const double x[3] = {xi[0] - t.pos[3 * j], xi[1] - t.pos[3 * j + 1],
                           xi[2] - t.pos[3 * j + 2]};
      const double v[3] = {vel[3 * i] - vel[3 * j], vel[3 * i + 1] - vel[3 * j + 1],
                           vel[3 * i + 2] - vel[3 * j + 2]};
      double W, dWdr, dWdh, gi, gj;
      wc6(r, hi, &W, &dWdr, &dWdh, &gi);
      wc6(r, h[j], &W, &dWdr, &dWdh, &gj);
      const double Aj = A_of(j), cj = c_of(j), mj = t.mass[j];
      const double vx = v[0] * x[0] + v[1] * x[1] + v[2] * x[2];
      const double w = vx / r;
      const double rhobar = 0.5 * (rho[i] + rho[j]);
      double du_pair = 0.0;
      double Pi = 0.0;
      if (w < 0.0) {
        const double vsig_ij = ci + cj - 3.0 * w;
        const double alpha_ij = 0.5 * (alpha_of(i) + alpha_of(j)) * 0.5 * (f_of(i) + f_of(j));
        Pi = -0.5 * alpha_ij * vsig_ij * w / rhobar;
      }
      vs = std::max(vs, ci + cj - 3.0 * std::min(w, 0.0));
      const double gbar = 0.5 * (gi + gj);
      const double tp = -mj * (Ai * gi + Aj * gj);
      const double tv = -mj * Pi * gbar;
      ax += (tp + tv) * x[0];
      ay += (tp + tv) * x[1];
      az += (tp + tv) * x[2];
      du_pair = mj * Ai * gi * vx + 0.5 * mj * Pi * gbar * vx;
      sdu += std::fabs(mj * Ai * gi * vx) + std::fabs(0.5 * mj * Pi * gbar * vx);
      if (alpha_u > 0.0) {
        const double vu = std::sqrt(std::fabs(P_of(i) - P_of(j)) / rhobar);
        const double cond = mj * alpha_u * vu * (u[i] - u[j]) * gbar * r / rhobar;
        du_pair += cond;
        sdu += std::fabs(cond);
      }
      du += du_pair;
      s += (std::fabs(tp) + std::fabs(tv)) * r;
    });
    if (acc) {
      acc[3 * i] = ax;
      acc[3 * i + 1] = ay;
      acc[3 * i + 2] = az;
    }
    if (dudt) dudt[i] = du;
    if (vsig) vsig[i] = vs;
    if (S) S[i] = s;
    if (npairs) npairs[i] = cnt;
    if (S_du) S_du[i] = sdu;
  }
  return G3REF_OK;
}

int g3ref_hydro(const g3ref_tree *gas, int64_t n_act, const int64_t *active,
                const g3ref_params *p, const double *vel, const double *u, const double *h,
                const double *rho, const double *omega, double *acc, double *dudt,
                double *vsig, double *S, int32_t *npairs) {
  return hydro_general(gas, n_act, active, p, vel, u, h, rho, omega, nullptr, nullptr, 0.0, acc,
                       dudt, vsig, S, npairs, nullptr);
}

int g3ref_hydro_switches(const g3ref_tree *gas, int64_t n_act, const int64_t *active,
                         const g3ref_params *p, const double *vel, const double *u,
                         const double *h, const double *rho, const double *omega,
                         const double *alpha, const double *balsara, double alpha_u,
                         double *acc, double *dudt, double *vsig, double *S, int32_t *npairs,
                         double *S_du) {
  return hydro_general(gas, n_act, active, p, vel, u, h, rho, omega, alpha, balsara, alpha_u,
                       acc, dudt, vsig, S, npairs, S_du);
}

/* Velocity divergence and curl of the active gas particles: the grad-h SPH
 * estimates (as the Balsara 1995 and Cullen & Dehnen 2010 switches take
 * them; Price 2012, eqs. 103-104):
 *   div v_i  =  (1/(Omega_i rho_i)) sum_j m_j (v_j - v_i) . grad_i W(r_ij, h_i)
 *   curl v_i = -(1/(Omega_i rho_i)) sum_j m_j (v_j - v_i) x grad_i W(r_ij, h_i)
 * with grad_i W = F(r, h_i) (x_i - x_j), over gas j with r < h_i (the
 * density's pairs; the self pair adds nothing). Outputs div_v [n] and
 * curl_v [n][3] at the active rows; S_div (nullable) the sum of the
 * magnitudes of the divergence's terms, S_curl (nullable) of the curl's. */
int g3ref_velgrad(const g3ref_tree *gas, int64_t n_act, const int64_t *active,
                  const g3ref_params *p, const double *vel, const double *h, const double *rho,
                  const double *omega, double *div_v, double *curl_v, double *S_div,
                  double *S_curl) {
  if (!gas || !valid_params(p) || n_act < 0 || (n_act > 0 && !active) || !vel || !h || !rho ||
      !omega)
    return G3REF_EINVAL;
  const g3ref_tree &t = *gas;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t a = 0; a < n_act; ++a) {
    const int64_t i = active[a];
    if (i < 0 || i >= t.n || !is_gas(t, i)) continue;
    const double *xi = &t.pos[3 * i];
    const double hi = h[i];
    double dv = 0, cx = 0, cy = 0, cz = 0, sd = 0, sc = 0;
    walk_leaves(t, 0, xi, [&](int64_t) { return hi * kPruneMargin; }, [&](int64_t j) {
      if (j == i || !is_gas(t, j)) return;
      if (!within(t, i, j, hi, p->flags)) return;
      const double r = dist(t, i, j);
      if (!(r > 0.0)) return;
      double W, dWdr, dWdh, F;
      wc6(r, hi, &W, &dWdr, &dWdh, &F);
      const double mj = t.mass[j];
      const double g[3] = {F * (xi[0] - t.pos[3 * j]), F * (xi[1] - t.pos[3 * j + 1]),
                           F * (xi[2] - t.pos[3 * j + 2])};
      const double d[3] = {vel[3 * j] - vel[3 * i], vel[3 * j + 1] - vel[3 * i + 1],
                           vel[3 * j + 2] - vel[3 * i + 2]};
      const double td = mj * (d[0] * g[0] + d[1] * g[1] + d[2] * g[2]);
      const double c[3] = {-mj * (d[1] * g[2] - d[2] * g[1]), -mj * (d[2] * g[0] - d[0] * g[2]),
                           -mj * (d[0] * g[1] - d[1] * g[0])};
      dv += td;
      cx += c[0];
      cy += c[1];
      cz += c[2];
      sd += std::fabs(td);
      sc += std::fabs(c[0]) + std::fabs(c[1]) + std::fabs(c[2]);
    });
    const double norm = 1.0 / (omega[i] * rho[i]);
    if (div_v) div_v[i] = dv * norm;
    if (curl_v) {
      curl_v[3 * i] = cx * norm;
      curl_v[3 * i + 1] = cy * norm;
      curl_v[3 * i + 2] = cz * norm;
    }
    if (S_div) S_div[i] = sd * norm;
    if (S_curl) S_curl[i] = sc * norm;
  }
  return G3REF_OK;
}

/* Thermal conduction of the active gas particles: the SPH form of
 * rho du/dt = div(kappa grad u) of Brookshaw (1985), as Gadget's conduction
 * module uses it (Jubelgas, Springel & Dolag 2004), with the conductivity in
 * units of the internal energy per mass (the heat capacity absorbed) and a
 * power law of it, kappa = kappa0 u^kappa_exp (kappa_exp = 5/2: Spitzer's
 * temperature dependence, 0: constant):
 *   du_i/dt = sum_j m_j (kappa_i + kappa_j) (u_i - u_j) Fbar_ij / (rho_i rho_j),
 *   Fbar_ij = (F(r, h_i) + F(r, h_j)) / 2,  F = (1/r) dW/dr <= 0,
 * over gas j != i with r < max(h_i, h_j) (the hydro force's pairs); pairs at
 * zero separation add nothing. Each pair's exchange is antisymmetric, so
 * sum_i m_i du_i/dt = 0 over a set that holds every pair of its members. */
int g3ref_conduction(const g3ref_tree *gas, int64_t n_act, const int64_t *active,
                     const g3ref_params *p, double kappa0, double kappa_exp,
                     const double *u, const double *h, const double *rho, double *dudt,
                     double *S, int32_t *npairs) {
  if (!gas || !valid_params(p) || n_act < 0 || (n_act > 0 && !active) || !u || !h || !rho ||
      !std::isfinite(kappa0) || kappa0 < 0.0 || !std::isfinite(kappa_exp))
    return G3REF_EINVAL;
  const g3ref_tree &t = *gas;
  std::vector<double> hmax(t.nodes.size(), 0.0);
  for (size_t k = 0; k < t.nodes.size(); ++k)
    for (int64_t s = t.nodes[k].start; s < t.nodes[k].start + t.nodes[k].count; ++s)
      hmax[k] = std::max(hmax[k], h[t.order[s]]);
  auto kappa = [&](int64_t j) { return kappa0 * std::pow(std::max(u[j], 0.0), kappa_exp); };
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t a = 0; a < n_act; ++a) {
    const int64_t i = active[a];
    if (i < 0 || i >= t.n || !is_gas(t, i)) continue;
    const double *xi = &t.pos[3 * i];
    const double hi = h[i], ki = kappa(i);
    double du = 0.0, s = 0.0;
    int32_t cnt = 0;
    walk_leaves(t, 0, xi, [&](int64_t k) { return std::max(hi, hmax[k]) * kPruneMargin; },
                [&](int64_t j) {
      if (j == i || !is_gas(t, j)) return;
      if (!within(t, i, j, std::max(hi, h[j]), p->flags)) return;
      ++cnt;
      const double r = dist(t, i, j);
      if (!(r > 0.0)) return;
      double W, dWdr, dWdh, Fi, Fj;
      wc6(r, hi, &W, &dWdr, &dWdh, &Fi);
      wc6(r, h[j], &W, &dWdr, &dWdh, &Fj);
      const double term = t.mass[j] * (ki + kappa(j)) * (u[i] - u[j]) * 0.5 * (Fi + Fj) /
                          (rho[i] * rho[j]);
      du += term;
      s += std::fabs(term);
    });
    if (dudt) dudt[i] = du;
    if (S) S[i] = s;
    if (npairs) npairs[i] = cnt;
  }
  return G3REF_OK;
}

} // extern "C"

namespace {

/* Barnes-Hut opening test for target i and node nd (Barnes & Hut 1986):
 * accept the monopole iff x_i is outside the node's half-open cube and
 * l < theta |x_i - c|. FP32 (default): dx = fl32(fl32(c) - x_i),
 * r2 = fmaf(dz,dz, fmaf(dy,dy, dx*dx)), accept iff fl32(l)^2 < fl32(theta^2) r2
 * with every product rounded to FP32. */
bool bh_accept(const g3ref_tree &t, int64_t i, const RefNode &nd, double theta, int32_t flags) {
  if (inside_cube(t, i, nd)) return false;
  const double *xi = &t.pos[3 * i];
  if (flags & G3REF_FLAG_FP64_DECISIONS) {
    const double dx = nd.com[0] - xi[0], dy = nd.com[1] - xi[1], dz = nd.com[2] - xi[2];
    return nd.l * nd.l < theta * theta * (dx * dx + dy * dy + dz * dz);
  }
  const float dx = (float)nd.com[0] - (float)xi[0];
  const float dy = (float)nd.com[1] - (float)xi[1];
  const float dz = (float)nd.com[2] - (float)xi[2];
  const float r2 = std::fmaf(dz, dz, std::fmaf(dy, dy, dx * dx));
  const float lf = (float)nd.l;
  const float lhs = lf * lf;
  const float th2 = (float)(theta * theta);
  const float rhs = th2 * r2;
  return lhs < rhs;
}

/* Per-particle Barnes-Hut walk: preorder from the root, children in Morton
 * order; an accepted node contributes its monopole, a leaf that is not
 * accepted contributes each member j != i, other nodes are opened. */
template <class Term>
void bh_walk(const g3ref_tree &t, int64_t k, int64_t i, double theta, int32_t flags, Term term) {
  const RefNode &nd = t.nodes[k];
  if (bh_accept(t, i, nd, theta, flags)) {
    term(nd.M, nd.com, -(k + 1));
    return;
  }
  if (nd.child.empty()) {
    for (int64_t s = nd.start; s < nd.start + nd.count; ++s) {
      const int64_t j = t.order[s];
      if (j != i) term(t.mass[j], &t.pos[3 * j], j);
    }
    return;
  }
  for (int64_t c : nd.child) bh_walk(t, c, i, theta, flags, term);
}

} // namespace

extern "C" {

/* Softened gravity of the active particles from every particle:
 *   a_i   += -G m x_ij / (r^2 + eps^2)^(3/2)
 *   phi_i += -G m / (r^2 + eps^2)^(1/2)
 * for each particle term (j != i) and each accepted node (mass M, at its
 * centre of mass), with x_ij = x_i - x_source. */
int g3ref_gravity(const g3ref_tree *all, int64_t n_act, const int64_t *active,
                  const g3ref_params *p, double *acc, double *pot, double *S,
                  int32_t *nterms) {
  if (!all || !valid_params(p) || n_act < 0 || (n_act > 0 && !active)) return G3REF_EINVAL;
  const g3ref_tree &t = *all;
  const double e2 = p->eps * p->eps, G = p->G;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t a = 0; a < n_act; ++a) {
    const int64_t i = active[a];
    if (i < 0 || i >= t.n) continue;
    const double *xi = &t.pos[3 * i];
    double ax = 0, ay = 0, az = 0, ph = 0, s = 0;
    int32_t cnt = 0;
    if (!t.nodes.empty())
      bh_walk(t, 0, i, p->theta, p->flags, [&](double m, const double *c, int64_t) {
        const double x[3] = {xi[0] - c[0], xi[1] - c[1], xi[2] - c[2]};
        const double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
        const double inv = 1.0 / std::sqrt(r2 + e2);
        const double inv3 = inv * inv * inv;
        ax -= G * m * x[0] * inv3;
        ay -= G * m * x[1] * inv3;
        az -= G * m * x[2] * inv3;
        ph -= G * m * inv;
        s += G * m * std::sqrt(r2) * inv3;
        ++cnt;
      });
    if (acc) {
      acc[3 * i] = ax;
      acc[3 * i + 1] = ay;
      acc[3 * i + 2] = az;
    }
    if (pot) pot[i] = ph;
    if (S) S[i] = s;
    if (nterms) nterms[i] = cnt;
  }
  return G3REF_OK;
}

int g3ref_lists(const g3ref_tree *tp, int32_t kind, int64_t n_act, const int64_t *active,
                const g3ref_params *p, const double *h, int64_t *offsets, int64_t *list) {
  if (!tp || !valid_params(p) || n_act < 0 || (n_act > 0 && !active) || !offsets)
    return G3REF_EINVAL;
  if ((kind == G3REF_GATHER || kind == G3REF_SYMMETRIC) && !h) return G3REF_EINVAL;
  if (kind < G3REF_GATHER || kind > G3REF_GRAVITY) return G3REF_EINVAL;
  const g3ref_tree &t = *tp;
  std::vector<double> hmax;
  if (kind == G3REF_SYMMETRIC) {
    hmax.assign(t.nodes.size(), 0.0);
    for (size_t k = 0; k < t.nodes.size(); ++k)
      for (int64_t s = t.nodes[k].start; s < t.nodes[k].start + t.nodes[k].count; ++s)
        hmax[k] = std::max(hmax[k], h[t.order[s]]);
  }
  std::vector<std::vector<int64_t>> out((size_t)n_act);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t a = 0; a < n_act; ++a) {
    const int64_t i = active[a];
    std::vector<int64_t> &L = out[a];
    if (i < 0 || i >= t.n || t.nodes.empty()) continue;
    const double *xi = &t.pos[3 * i];
    if (kind == G3REF_GRAVITY) {
      bh_walk(t, 0, i, p->theta, p->flags,
              [&](double, const double *, int64_t id) { L.push_back(id); });
    } else {
      if (!is_gas(t, i)) continue;
      const double hi = h[i];
      if (kind == G3REF_GATHER) {
        walk_leaves(t, 0, xi, [&](int64_t) { return hi * kPruneMargin; }, [&](int64_t j) {
          if (is_gas(t, j) && within(t, i, j, hi, p->flags)) L.push_back(j);
        });
      } else {
        walk_leaves(t, 0, xi, [&](int64_t k) { return std::max(hi, hmax[k]) * kPruneMargin; },
                    [&](int64_t j) {
          if (j != i && is_gas(t, j) && within(t, i, j, std::max(hi, h[j]), p->flags))
            L.push_back(j);
        });
      }
    }
    std::sort(L.begin(), L.end());
  }
  offsets[0] = 0;
  for (int64_t a = 0; a < n_act; ++a) offsets[a + 1] = offsets[a] + (int64_t)out[a].size();
  if (list)
    for (int64_t a = 0; a < n_act; ++a)
      std::copy(out[a].begin(), out[a].end(), list + offsets[a]);
  return G3REF_OK;
}

} // extern "C"

/* ================================================================ adjoints
 *
 * Gradients of the three modules with respect to their inputs, for a
 * scalar loss whose derivatives with respect to the module outputs (the
 * upstream gradients) are given at the active rows. Neighbour sets and
 * Barnes-Hut decisions are held fixed (the forward is piecewise smooth in
 * them), h is an input (no derivative through its solve), and the results
 * are ADDED to the caller's gradient arrays.
 *
 * Every derivative below is taken mechanically: each pair's (or term's)
 * contribution is evaluated once more in forward-mode dual numbers seeded
 * on that pair's input variables, so the partials are those of the forward
 * formula as written, with no hand-derived expression. Only the two plain
 * chain rules that tie pairs to particle data are written out: a node
 * monopole's dependence on its members (M = sum m, c = sum m x / M) and the
 * sum over pairs.
 */

namespace {

/* value and K partial derivatives */
template <int K>
struct Dual {
  double v;
  double d[K];
  Dual() : v(0.0) { std::fill(d, d + K, 0.0); }
  Dual(double x) : v(x) { std::fill(d, d + K, 0.0); }  // NOLINT: constants
  static Dual var(double x, int k) {
    Dual r(x);
    r.d[k] = 1.0;
    return r;
  }
};

template <int K> Dual<K> operator+(const Dual<K> &a, const Dual<K> &b) {
  Dual<K> r(a.v + b.v);
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <int K> Dual<K> operator-(const Dual<K> &a, const Dual<K> &b) {
  Dual<K> r(a.v - b.v);
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <int K> Dual<K> operator-(const Dual<K> &a) {
  Dual<K> r(-a.v);
  for (int k = 0; k < K; ++k) r.d[k] = -a.d[k];
  return r;
}
template <int K> Dual<K> operator*(const Dual<K> &a, const Dual<K> &b) {
  Dual<K> r(a.v * b.v);
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <int K> Dual<K> operator/(const Dual<K> &a, const Dual<K> &b) {
  Dual<K> r(a.v / b.v);
  for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
  return r;
}
template <int K> Dual<K> operator+(const Dual<K> &a, double b) { return a + Dual<K>(b); }
template <int K> Dual<K> operator+(double a, const Dual<K> &b) { return Dual<K>(a) + b; }
template <int K> Dual<K> operator-(const Dual<K> &a, double b) { return a - Dual<K>(b); }
template <int K> Dual<K> operator-(double a, const Dual<K> &b) { return Dual<K>(a) - b; }
template <int K> Dual<K> operator*(const Dual<K> &a, double b) { return a * Dual<K>(b); }
template <int K> Dual<K> operator*(double a, const Dual<K> &b) { return Dual<K>(a) * b; }
template <int K> Dual<K> operator/(const Dual<K> &a, double b) { return a / Dual<K>(b); }
template <int K> Dual<K> operator/(double a, const Dual<K> &b) { return Dual<K>(a) / b; }
template <int K> Dual<K> sqrt(const Dual<K> &a) {
  const double s = std::sqrt(a.v);
  Dual<K> r(s);
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] / (2.0 * s);
  return r;
}

/* Wendland C6 value, dW/dh and F = (1/r) dW/dr at q = r/h < 1 (the forward
 * formulas of wc6), on any scalar type; zero at and beyond the support. */
template <class T>
void wc6_t(const T &r, const T &h, T *W, T *Wh, T *F) {
  const T q = r / h;
  if (!(q.v < 1.0)) {
    *W = T(0.0);
    *Wh = T(0.0);
    *F = T(0.0);
    return;
  }
  const T t = 1.0 - q;
  const T t2 = t * t, t4 = t2 * t2, t7 = t4 * t2 * t, t8 = t7 * t;
  const T h3 = h * h * h, h4 = h3 * h, h5 = h4 * h;
  const T p8 = 1.0 + q * (8.0 + q * (25.0 + q * 32.0));
  const T p7 = 1.0 + q * (7.0 + q * 16.0);
  const T ph = -3.0 + q * (-21.0 + q * (-29.0 + q * (133.0 + q * 448.0)));
  *W = kWc6 / h3 * t8 * p8;
  *Wh = kWc6 / h4 * t7 * ph;
  *F = -22.0 * kWc6 / h5 * t7 * p7;
}

/* |x_i - x_j| in duals; a pair at zero separation has r = 0 with no
 * position derivative (the kernel is even in r, so dW/dx vanishes there) */
template <int K>
Dual<K> separation(const Dual<K> *xi, const Dual<K> *xj) {
  const Dual<K> dx = xi[0] - xj[0], dy = xi[1] - xj[1], dz = xi[2] - xj[2];
  const Dual<K> r2 = dx * dx + dy * dy + dz * dz;
  if (!(r2.v > 0.0)) return Dual<K>(0.0);
  return sqrt(r2);
}

/* Per-thread gradient buffers, summed in thread order at the end. Each
 * entry also sums the magnitudes of the contributions added to it (the
 * scale of its rounding error in any order of summation). */
struct Mine {
  std::vector<double> &v, &a;
  void add(size_t i, double x) {
    v[i] += x;
    a[i] += std::fabs(x);
  }
};

struct GradBuf {
  std::vector<std::vector<double>> b, s;
  GradBuf(int nt, size_t len)
      : b((size_t)nt, std::vector<double>(len, 0.0)), s((size_t)nt, std::vector<double>(len, 0.0)) {}
  Mine mine() {
#ifdef _OPENMP
    const size_t t = (size_t)omp_get_thread_num();
#else
    const size_t t = 0;
#endif
    return Mine{b[t], s[t]};
  }
  void add_to(double *out, double *mag, size_t len) const {
    for (size_t t = 0; t < b.size(); ++t)
      for (size_t i = 0; i < len; ++i) {
        if (out) out[i] += b[t][i];
        if (mag) mag[i] += s[t][i];
      }
  }
};

int nthreads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // namespace

extern "C" {

/* Density adjoint. Loss L = sum_i (g_rho_i rho_i + g_drho_i drho_i/dh +
 * g_omega_i Omega_i) over the active gas i; rho, drho/dh and Omega as in
 * g3ref_density at the given h. Adds dL/dx, dL/dm, dL/dh to g_pos [n][3],
 * g_mass [n], g_h [n] (each nullable). */
int g3ref_density_backward(const g3ref_tree *gas, int64_t n_act, const int64_t *active,
                           const g3ref_params *p, const double *h, const double *g_rho,
                           const double *g_drho, const double *g_omega, double *g_pos,
                           double *g_mass, double *g_h, double *S) {
  if (!gas || !valid_params(p) || n_act < 0 || (n_act > 0 && !active) || !h) return G3REF_EINVAL;
  const g3ref_tree &t = *gas;
  const size_t n = (size_t)t.n;
  const int nt = nthreads();
  GradBuf gx(nt, 3 * n), gm(nt, n), gh(nt, n);
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < n_act; ++a) {
    const int64_t i = active[a];
    if (i < 0 || i >= t.n || !is_gas(t, i)) continue;
    const double hi = h[i];
    std::vector<int64_t> nb;
    walk_leaves(t, 0, &t.pos[3 * i], [&](int64_t) { return hi * kPruneMargin; }, [&](int64_t j) {
      if (is_gas(t, j) && within(t, i, j, hi, p->flags)) nb.push_back(j);
    });
    // the outputs at the given h
    double rho = 0.0, drho = 0.0;
    for (int64_t j : nb) {
      double W, dWdr, Wh, F;
      wc6(dist(t, i, j), hi, &W, &dWdr, &Wh, &F);
      rho += t.mass[j] * W;
      drho += t.mass[j] * Wh;
    }
    // Omega = 1 + h drho / (3 rho): partials by duals in (rho, drho, h)
    using D3 = Dual<3>;
    const D3 R = D3::var(rho, 0), Rp = D3::var(drho, 1), Hh = D3::var(hi, 2);
    const D3 Om = 1.0 + Hh * Rp / (3.0 * R);
    const double go = g_omega ? g_omega[i] : 0.0;
    const double grho = (g_rho ? g_rho[i] : 0.0) + go * Om.d[0];
    const double gdrho = (g_drho ? g_drho[i] : 0.0) + go * Om.d[1];
    Mine GX = gx.mine(), GM = gm.mine(), GH = gh.mine();
    GH.add(i, go * Om.d[2]);
    // each pair: (m_j W(r, h_i), m_j dW/dh(r, h_i)) in duals over
    // x_i (0-2), x_j (3-5), m_j (6), h_i (7)
    using D8 = Dual<8>;
    for (int64_t j : nb) {
      D8 xi[3], xj[3];
      for (int c = 0; c < 3; ++c) {
        xi[c] = D8::var(t.pos[3 * i + c], c);
        xj[c] = D8::var(t.pos[3 * j + c], 3 + c);
      }
      const D8 mj = D8::var(t.mass[j], 6), H = D8::var(hi, 7);
      D8 W, Wh, F;
      wc6_t(separation(xi, xj), H, &W, &Wh, &F);
      const D8 cr = mj * W, cd = mj * Wh;
      for (int c = 0; c < 3; ++c) {
        GX.add(3 * i + c, grho * cr.d[c] + gdrho * cd.d[c]);
        GX.add(3 * j + c, grho * cr.d[3 + c] + gdrho * cd.d[3 + c]);
      }
      GM.add(j, grho * cr.d[6] + gdrho * cd.d[6]);
      GH.add(i, grho * cr.d[7] + gdrho * cd.d[7]);
    }
  }
  gx.add_to(g_pos, S, 3 * n);
  gm.add_to(g_mass, S ? S + 3 * n : nullptr, n);
  gh.add_to(g_h, S ? S + 4 * n : nullptr, n);
  return G3REF_OK;
}

}  // extern "C"

extern "C" {

/* Hydro adjoint. Loss L = sum_i (g_acc_i . a_i + g_dudt_i du_i/dt) over the
 * active gas i, with a and du/dt as in g3ref_hydro (the signal velocity is
 * not differentiated). Adds the derivatives with respect to positions,
 * velocities, masses, h, u, rho and Omega of every gas particle to the
 * caller's arrays (each nullable). */
int g3ref_hydro_backward(const g3ref_tree *gas, int64_t n_act, const int64_t *active,
                         const g3ref_params *p, const double *vel, const double *u,
                         const double *h, const double *rho, const double *omega,
                         const double *g_acc, const double *g_dudt, double *g_pos,
                         double *g_vel, double *g_mass, double *g_h, double *g_u,
                         double *g_rho, double *g_omega, double *S) {
  if (!gas || !valid_params(p) || n_act < 0 || (n_act > 0 && !active) || !vel || !u || !h ||
      !rho || !omega)
    return G3REF_EINVAL;
  const g3ref_tree &t = *gas;
  const size_t n = (size_t)t.n;
  const double gm = p->gamma, alpha = p->alpha;
  std::vector<double> hmax(t.nodes.size(), 0.0);
  for (size_t k = 0; k < t.nodes.size(); ++k)
    for (int64_t s = t.nodes[k].start; s < t.nodes[k].start + t.nodes[k].count; ++s)
      hmax[k] = std::max(hmax[k], h[t.order[s]]);
  const int nt = nthreads();
  GradBuf gx(nt, 3 * n), gv(nt, 3 * n), gms(nt, n), gh(nt, n), gu(nt, n), gr(nt, n), go(nt, n);
  /* duals over the pair's inputs:
   *  0-2 x_i, 3-5 x_j, 6-8 v_i, 9-11 v_j, 12 m_j, 13 h_i, 14 h_j,
   *  15 u_i, 16 u_j, 17 rho_i, 18 rho_j, 19 Omega_i, 20 Omega_j */
  using D = Dual<21>;
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < n_act; ++a) {
    const int64_t i = active[a];
    if (i < 0 || i >= t.n || !is_gas(t, i)) continue;
    const double ga[3] = {g_acc ? g_acc[3 * i] : 0.0, g_acc ? g_acc[3 * i + 1] : 0.0,
                          g_acc ? g_acc[3 * i + 2] : 0.0};
    const double gd = g_dudt ? g_dudt[i] : 0.0;
    if (ga[0] == 0.0 && ga[1] == 0.0 && ga[2] == 0.0 && gd == 0.0) continue;
    const double hi = h[i];
    std::vector<int64_t> nb;
    walk_leaves(t, 0, &t.pos[3 * i], [&](int64_t k) { return std::max(hi, hmax[k]) * kPruneMargin; },
                [&](int64_t j) {
      if (j != i && is_gas(t, j) && within(t, i, j, std::max(hi, h[j]), p->flags)) nb.push_back(j);
    });
    Mine GX = gx.mine(), GV = gv.mine(), GM = gms.mine(), GH = gh.mine(),
                        GU = gu.mine(), GR = gr.mine(), GO = go.mine();
    for (int64_t j : nb) {
      D xi[3], xj[3], vi[3], vj[3];
      for (int c = 0; c < 3; ++c) {
        xi[c] = D::var(t.pos[3 * i + c], c);
        xj[c] = D::var(t.pos[3 * j + c], 3 + c);
        vi[c] = D::var(vel[3 * i + c], 6 + c);
        vj[c] = D::var(vel[3 * j + c], 9 + c);
      }
      const D mj = D::var(t.mass[j], 12), Hi = D::var(hi, 13), Hj = D::var(h[j], 14);
      const D ui = D::var(u[i], 15), uj = D::var(u[j], 16);
      const D ri = D::var(rho[i], 17), rj = D::var(rho[j], 18);
      const D oi = D::var(omega[i], 19), oj = D::var(omega[j], 20);
      const D r = separation(xi, xj);
      if (!(r.v > 0.0)) continue;  // pairs at zero separation add nothing
      const D x[3] = {xi[0] - xj[0], xi[1] - xj[1], xi[2] - xj[2]};
      const D v[3] = {vi[0] - vj[0], vi[1] - vj[1], vi[2] - vj[2]};
      // the forward formulas of g3ref_hydro
      const D Ai = (gm - 1.0) * ri * ui / (oi * ri * ri);
      const D Aj = (gm - 1.0) * rj * uj / (oj * rj * rj);
      const D ci = sqrt(gm * (gm - 1.0) * ui), cj = sqrt(gm * (gm - 1.0) * uj);
      D W, Wh, gi, gj;
      wc6_t(r, Hi, &W, &Wh, &gi);
      wc6_t(r, Hj, &W, &Wh, &gj);
      const D vx = v[0] * x[0] + v[1] * x[1] + v[2] * x[2];
      const D w = vx / r;
      D Pi(0.0);
      if (w.v < 0.0) {
        const D vsig = ci + cj - 3.0 * w;
        Pi = -0.5 * alpha * vsig * w / (0.5 * (ri + rj));
      }
      const D gbar = 0.5 * (gi + gj);
      const D tp = -mj * (Ai * gi + Aj * gj);
      const D tv = -mj * Pi * gbar;
      const D coef = tp + tv;
      const D du = mj * Ai * gi * vx + 0.5 * mj * Pi * gbar * vx;
      // dL/dvar = sum_c ga_c d(coef x_c)/dvar + gd d(du)/dvar
      D L = gd * du;
      for (int c = 0; c < 3; ++c) L = L + ga[c] * (coef * x[c]);
      for (int c = 0; c < 3; ++c) {
        GX.add(3 * i + c, L.d[c]);
        GX.add(3 * j + c, L.d[3 + c]);
        GV.add(3 * i + c, L.d[6 + c]);
        GV.add(3 * j + c, L.d[9 + c]);
      }
      GM.add(j, L.d[12]);
      GH.add(i, L.d[13]);
      GH.add(j, L.d[14]);
      GU.add(i, L.d[15]);
      GU.add(j, L.d[16]);
      GR.add(i, L.d[17]);
      GR.add(j, L.d[18]);
      GO.add(i, L.d[19]);
      GO.add(j, L.d[20]);
    }
  }
  auto at = [&](size_t off) { return S ? S + off : nullptr; };
  gx.add_to(g_pos, at(0), 3 * n);
  gv.add_to(g_vel, at(3 * n), 3 * n);
  gms.add_to(g_mass, at(6 * n), n);
  gh.add_to(g_h, at(7 * n), n);
  gu.add_to(g_u, at(8 * n), n);
  gr.add_to(g_rho, at(9 * n), n);
  go.add_to(g_omega, at(10 * n), n);
  return G3REF_OK;
}

/* Gravity adjoint. Loss L = sum_i (g_acc_i . a_i + g_pot_i phi_i) over the
 * active i, with a and phi as in g3ref_gravity (opening decisions fixed).
 * A particle term depends on x_i, x_j and m_j; an accepted node's monopole
 * term on x_i and the node's M and c, which depend on its members through
 * M = sum_k m_k and c = sum_k m_k x_k / M:
 *   dc/dx_k = (m_k / M) I,  dc/dm_k = (x_k - c) / M,  dM/dm_k = 1.
 * Adds dL/dx and dL/dm to g_pos [n][3] and g_mass [n] (each nullable). */
int g3ref_gravity_backward(const g3ref_tree *all, int64_t n_act, const int64_t *active,
                           const g3ref_params *p, const double *g_acc, const double *g_pot,
                           double *g_pos, double *g_mass, double *S) {
  if (!all || !valid_params(p) || n_act < 0 || (n_act > 0 && !active)) return G3REF_EINVAL;
  const g3ref_tree &t = *all;
  const size_t n = (size_t)t.n, nn = t.nodes.size();
  const double e2 = p->eps * p->eps, G = p->G;
  const int nt = nthreads();
  // per node: dL/dc (3) and dL/dM
  GradBuf gx(nt, 3 * n), gms(nt, n), gc(nt, 3 * nn), gM(nt, nn);
  /* duals: 0-2 x_i, 3-5 source position, 6 source mass */
  using D = Dual<7>;
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < n_act; ++a) {
    const int64_t i = active[a];
    if (i < 0 || i >= t.n || t.nodes.empty()) continue;
    const double ga[3] = {g_acc ? g_acc[3 * i] : 0.0, g_acc ? g_acc[3 * i + 1] : 0.0,
                          g_acc ? g_acc[3 * i + 2] : 0.0};
    const double gp = g_pot ? g_pot[i] : 0.0;
    Mine GX = gx.mine(), GM = gms.mine(), GC = gc.mine(), GMn = gM.mine();
    bh_walk(t, 0, i, p->theta, p->flags, [&](double m, const double *c, int64_t id) {
      D xi[3], xs[3];
      for (int k = 0; k < 3; ++k) {
        xi[k] = D::var(t.pos[3 * i + k], k);
        xs[k] = D::var(c[k], 3 + k);
      }
      const D ms = D::var(m, 6);
      // the forward formulas of g3ref_gravity
      const D x[3] = {xi[0] - xs[0], xi[1] - xs[1], xi[2] - xs[2]};
      const D r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
      const D inv = 1.0 / sqrt(r2 + e2);
      const D inv3 = inv * inv * inv;
      D L = gp * (-G * ms * inv);
      for (int k = 0; k < 3; ++k) L = L + ga[k] * (-G * ms * x[k] * inv3);
      for (int k = 0; k < 3; ++k) GX.add(3 * i + k, L.d[k]);
      if (id >= 0) {
        for (int k = 0; k < 3; ++k) GX.add(3 * id + k, L.d[3 + k]);
        GM.add(id, L.d[6]);
      } else {
        const int64_t nd = -id - 1;
        for (int k = 0; k < 3; ++k) GC.add(3 * nd + k, L.d[3 + k]);
        GMn.add(nd, L.d[6]);
      }
    });
  }
  gx.add_to(g_pos, S, 3 * n);
  gms.add_to(g_mass, S ? S + 3 * n : nullptr, n);
  // node adjoints to their members
  std::vector<double> GCt(3 * nn, 0.0), GMt(nn, 0.0), SCt(3 * nn, 0.0), SMt(nn, 0.0);
  gc.add_to(GCt.data(), SCt.data(), 3 * nn);
  gM.add_to(GMt.data(), SMt.data(), nn);
  for (size_t k = 0; k < nn; ++k) {
    const RefNode &nd = t.nodes[k];
    if (GCt[3 * k] == 0.0 && GCt[3 * k + 1] == 0.0 && GCt[3 * k + 2] == 0.0 && GMt[k] == 0.0)
      continue;
    for (int64_t s = nd.start; s < nd.start + nd.count; ++s) {
      const int64_t j = t.order[s];
      double dot = 0.0, sdot = 0.0;
      for (int c = 0; c < 3; ++c) {
        if (g_pos) g_pos[3 * j + c] += GCt[3 * k + c] * t.mass[j] / nd.M;
        if (S) S[3 * j + c] += SCt[3 * k + c] * t.mass[j] / nd.M;
        dot += GCt[3 * k + c] * (t.pos[3 * j + c] - nd.com[c]);
        sdot += SCt[3 * k + c] * std::fabs(t.pos[3 * j + c] - nd.com[c]);
      }
      if (g_mass) g_mass[j] += GMt[k] + dot / nd.M;
      if (S) S[3 * n + j] += SMt[k] + sdot / nd.M;
    }
  }
  return G3REF_OK;
}

}  // extern "C"
