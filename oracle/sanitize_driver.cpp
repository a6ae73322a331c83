// A driver that runs every entry point of the oracle (g3ref.h) once on a
// small seeded input, for the AddressSanitizer / UndefinedBehaviorSanitizer
// build the CPU tests make of it (tests/test_oracle_sanitizers.py).
//
// TEST INFRASTRUCTURE ONLY, like the oracle itself: no GPU code loads it.
// It checks memory and undefined-behaviour errors only (the sanitizers abort
// the run on the first one) plus that every output is finite; the values
// are pinned by the other oracle tests.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "g3ref.h"

namespace {

// splitmix64: a counter-based generator, for the inputs only
struct Rng {
  uint64_t s;
  double next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53;
  }
};

int bad = 0;

void finite(const char *what, const std::vector<double> &v) {
  for (double x : v)
    if (!std::isfinite(x)) {
      std::printf("non-finite output: %s\n", what);
      ++bad;
      return;
    }
}

}  // namespace

int main() {
  const int64_t n = 600;
  Rng rng{12345};
  std::vector<double> pos(3 * n), mass(n, 1.0 / n), vel(3 * n), u(n), h(n), rho(n), drho(n),
      omega(n);
  std::vector<uint8_t> type(n);
  for (int64_t i = 0; i < n; ++i) {
    // two clumps and a background, half gas
    const double c = i % 3 == 0 ? 0.5 : (i % 3 == 1 ? 0.3 : 0.7);
    const double s = i % 3 == 0 ? 0.45 : 0.05;
    for (int k = 0; k < 3; ++k) {
      pos[3 * i + k] = c + s * (2.0 * rng.next() - 1.0);
      vel[3 * i + k] = 0.1 * (2.0 * rng.next() - 1.0);
    }
    u[i] = 0.5 + rng.next();
    type[i] = (uint8_t)(i & 1);
  }
  const double box[4] = {0.0, 0.0, 0.0, 1.0};
  g3ref_params p{32.0, 1e-6, 5.0 / 3.0, 1.0, 0.5, 1e-3, 1.0, 8, 0};
  g3ref_set_threads(2);

  double W, dWdr, dWdh, F;
  g3ref_kernel(0.3, 1.0, &W, &dWdr, &dWdh, &F);
  (void)g3ref_key(&pos[0], box);

  g3ref_tree *gas = g3ref_tree_build(n, pos.data(), mass.data(), type.data(), box, 8, 1);
  g3ref_tree *all = g3ref_tree_build(n, pos.data(), mass.data(), type.data(), box, 8, 0);
  if (!gas || !all) {
    std::printf("tree build failed\n");
    return 2;
  }
  const int64_t nn = g3ref_tree_nnodes(all), nm = g3ref_tree_nmembers(all);
  std::vector<int64_t> order(nm), nstart(nn), ncount(nn), nskip(nn);
  std::vector<uint64_t> keys(nm);
  std::vector<int32_t> nlevel(nn);
  std::vector<double> nmass(nn), ncom(3 * nn);
  g3ref_tree_export(all, order.data(), keys.data(), nstart.data(), ncount.data(), nlevel.data(),
                    nskip.data(), nmass.data(), ncom.data());
  finite("node moments", ncom);

  std::vector<int64_t> gas_ids, all_ids(n);
  for (int64_t i = 0; i < n; ++i) {
    all_ids[i] = i;
    if (type[i] == 0) gas_ids.push_back(i);
  }
  const int64_t ng = (int64_t)gas_ids.size();
  std::vector<int32_t> nngb(n), npairs(n), nterms(n);
  int64_t nonconv = 0;
  int rc = g3ref_density(gas, ng, gas_ids.data(), &p, 1, h.data(), rho.data(), drho.data(),
                         omega.data(), nngb.data(), &nonconv);
  std::printf("density rc %d nonconv %lld\n", rc, (long long)nonconv);
  std::vector<double> acc(3 * n), dudt(n), vsig(n), S(n), Sdu(n);
  rc |= g3ref_hydro(gas, ng, gas_ids.data(), &p, vel.data(), u.data(), h.data(), rho.data(),
                    omega.data(), acc.data(), dudt.data(), vsig.data(), S.data(), npairs.data());
  finite("hydro", acc);
  std::vector<double> alpha(n, 0.5), balsara(n, 0.8);
  rc |= g3ref_hydro_switches(gas, ng, gas_ids.data(), &p, vel.data(), u.data(), h.data(),
                             rho.data(), omega.data(), alpha.data(), balsara.data(), 1.0,
                             acc.data(), dudt.data(), vsig.data(), S.data(), npairs.data(),
                             Sdu.data());
  finite("hydro with switches", dudt);
  std::vector<double> divv(n), curl(3 * n), Sdiv(n), Scurl(n);
  rc |= g3ref_velgrad(gas, ng, gas_ids.data(), &p, vel.data(), h.data(), rho.data(),
                      omega.data(), divv.data(), curl.data(), Sdiv.data(), Scurl.data());
  finite("velocity gradients", curl);
  rc |= g3ref_conduction(gas, ng, gas_ids.data(), &p, 1e-3, 2.5, u.data(), h.data(), rho.data(),
                         dudt.data(), S.data(), npairs.data());
  finite("conduction", dudt);
  std::vector<double> gacc(3 * n), pot(n), Sg(n);
  for (double theta : {0.5, 0.0, 0.7}) {
    g3ref_params q = p;
    q.theta = theta;
    rc |= g3ref_gravity(all, n, all_ids.data(), &q, gacc.data(), pot.data(), Sg.data(),
                        nterms.data());
    finite("gravity", gacc);
  }
  for (int32_t kind : {G3REF_GATHER, G3REF_SYMMETRIC, G3REF_GRAVITY}) {
    const g3ref_tree *t = kind == G3REF_GRAVITY ? all : gas;
    const int64_t na = kind == G3REF_GRAVITY ? n : ng;
    const int64_t *act = kind == G3REF_GRAVITY ? all_ids.data() : gas_ids.data();
    std::vector<int64_t> off(na + 1);
    rc |= g3ref_lists(t, kind, na, act, &p, h.data(), off.data(), nullptr);
    std::vector<int64_t> list((size_t)off[na] + 1);
    rc |= g3ref_lists(t, kind, na, act, &p, h.data(), off.data(), list.data());
  }
  std::vector<double> g1(n, 1.0), g3v(3 * n, 0.5), gpos(3 * n), gmass(n), gh(n), gvel(3 * n),
      gu(n), grho(n), gom(n), SB(8 * n);
  rc |= g3ref_density_backward(gas, ng, gas_ids.data(), &p, h.data(), g1.data(), g1.data(),
                               g1.data(), gpos.data(), gmass.data(), gh.data(), SB.data());
  rc |= g3ref_hydro_backward(gas, ng, gas_ids.data(), &p, vel.data(), u.data(), h.data(),
                             rho.data(), omega.data(), g3v.data(), g1.data(), gpos.data(),
                             gvel.data(), gmass.data(), gh.data(), gu.data(), grho.data(),
                             gom.data(), nullptr);
  rc |= g3ref_gravity_backward(all, n, all_ids.data(), &p, g3v.data(), g1.data(), gpos.data(),
                               gmass.data(), SB.data());
  finite("gradients", gpos);
  // a drift, then the refit and one more density at the given h
  for (int64_t i = 0; i < 3 * n; ++i) pos[i] += 1e-3 * (2.0 * rng.next() - 1.0);
  rc |= g3ref_tree_refit(gas, pos.data(), mass.data());
  rc |= g3ref_tree_refit(all, pos.data(), mass.data());
  rc |= g3ref_density(gas, ng, gas_ids.data(), &p, 0, h.data(), rho.data(), drho.data(),
                      omega.data(), nngb.data(), &nonconv);
  finite("density after refit", rho);
  g3ref_tree_free(gas);
  g3ref_tree_free(all);
  std::printf("sanitized oracle run: rc %d, %d non-finite outputs\n", rc, bad);
  return (rc == 0 && bad == 0) ? 0 : 1;
}
