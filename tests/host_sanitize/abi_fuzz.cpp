// Host-only exercise of the C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer: lattice validation and scheduling on random
// and broken lattices (out-of-range ids, repeated order entries, bad
// cluster flags, non-finite couplings), gates, workspace sizes and the
// option checks of hmps_create.  Every schedule that is accepted must keep
// each update inside the MPS.  Exit status 0 and a count line on success.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>
#include <algorithm>
#include "hmps.h"

int main() {
  std::mt19937 rng(7);
  long ok = 0, bad = 0;
  for (int trial = 0; trial < 3000; ++trial) {
    int n = 1 + rng() % 12;
    int nb = rng() % 20;
    std::vector<int32_t> bi(nb), bj(nb), order(n);
    std::vector<double> J(nb);
    std::vector<uint8_t> cl(n);
    for (int b = 0; b < nb; ++b) {
      bi[b] = rng() % (n + 1) - (trial % 17 == 0 ? 1 : 0);
      bj[b] = rng() % n;
      J[b] = (trial % 29 == 0) ? NAN : (rng() % 5) * 0.5 - 1.0;
    }
    for (int i = 0; i < n; ++i) order[i] = i;
    std::shuffle(order.begin(), order.end(), rng);
    if (trial % 13 == 0 && n > 1) order[0] = order[1];
    for (int i = 0; i < n; ++i) cl[i] = rng() % 3 == 0;
    if (trial % 31 == 0) cl[0] = 7;
    hmps_lattice lat;
    std::memset(&lat, 0, sizeof lat);
    lat.n_phys = n;
    lat.n_bonds = nb;
    lat.bond_i = nb ? bi.data() : nullptr;
    lat.bond_j = nb ? bj.data() : nullptr;
    lat.bond_J = nb ? J.data() : nullptr;
    lat.mps_order = order.data();
    lat.in_cluster = cl.data();
    int32_t ns = 0, nu = 0;
    hmps_status st = hmps_schedule(&lat, &ns, &nu, nullptr, nullptr, 0);
    if (st == HMPS_OK) {
      ++ok;
      std::vector<int32_t> k(nu + 1), op(nu + 1);
      // cap too small: counts only
      hmps_schedule(&lat, &ns, &nu, k.data(), op.data(), nu - 1);
      st = hmps_schedule(&lat, &ns, &nu, k.data(), op.data(), nu);
      if (st != HMPS_OK) { std::printf("schedule fill failed\n"); return 1; }
      for (int t = 0; t < nu; ++t)
        if (k[t] < 0 || k[t] + 1 >= ns) { std::printf("bad k\n"); return 1; }
    } else {
      ++bad;
    }
  }
  double g[81];
  for (int i = 0; i < 100; ++i)
    hmps_gate((rng() % 7) - 3.0, (rng() % 100) * 0.01, g);
  hmps_gate(NAN, 0.1, g);
  for (int c = 1; c < 100; c += 7)
    for (int chi = 3; chi <= 640; chi += 97)
      (void)hmps_workspace_bytes(c, 40, chi, 60);
  hmps_ctx *ctx = nullptr;
  hmps_options o;
  std::memset(&o, 0, sizeof o);
  hmps_create(&ctx, &o);
  o.max_chains = 70000; o.max_sites = 4; o.chi_cap = 8;
  hmps_create(&ctx, &o);
  std::printf("valid %ld invalid %ld\n", ok, bad);
  return 0;
}
