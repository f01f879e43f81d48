// Host-side runtime code of libqtm under AddressSanitizer and
// UndefinedBehaviorSanitizer (built with g++ by tests/test_sanitizers.py, no
// device code): circuit validation (valid and invalid gate lists), the
// planner and program encoding at every tile size and low-qubit count, the
// plan JSON, the generated source of every specialised sweep kernel in both
// precisions, the parameter lists and the uneven-batch list schedule.
// Exit status 0 when every check holds; a sanitizer report aborts.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "circuit.h"
#include "jit.h"
#include "schedule.h"

using namespace qtm;

namespace {

int g_fail = 0;
void check(bool ok, const std::string &what) {
  if (!ok) {
    std::fprintf(stderr, "FAIL: %s\n", what.c_str());
    ++g_fail;
  }
}

struct Spec {
  int n, n_in, n_w;
  std::vector<Gate> gates;
  std::vector<uint64_t> z, x;
};

// layer: RX(x_q), RY(w), RZ(w) on every qubit, then a CNOT ring or a CZ ladder
Spec layered(int n, int L, bool ring) {
  Spec s{n, n, 2 * n * L, {}, {}, {}};
  for (int l = 0; l < L; ++l) {
    for (int q = 0; q < n; ++q) s.gates.push_back({G_RX, q, 0, S_INPUT, q});
    for (int q = 0; q < n; ++q) s.gates.push_back({G_RY, q, 0, S_WEIGHT, l * 2 * n + q});
    for (int q = 0; q < n; ++q) s.gates.push_back({G_RZ, q, 0, S_WEIGHT, l * 2 * n + n + q});
    if (ring && n > 1)
      for (int q = 0; q < n; ++q) s.gates.push_back({G_CNOT, q, (q + 1) % n, 0, 0});
    if (!ring)
      for (int q = 0; q + 1 < n; ++q) s.gates.push_back({G_CZ, q, q + 1, 0, 0});
  }
  for (int q = 0; q < n; ++q) s.z.push_back((uint64_t)1 << q);
  s.z.push_back(n >= 64 ? ~(uint64_t)0 : ((uint64_t)1 << n) - 1);
  return s;
}

// random gate mix: rotations (input, weight and scaled sources), fixed gates,
// CNOT and CZ; controlled rotations only when crot
Spec random_circuit(std::mt19937 &rng, int n, int g, bool crot, bool pauli) {
  Spec s{n, 4, 5, {}, {}, {}};
  auto qb = [&] { return (int)(rng() % n); };
  for (int k = 0; k < g; ++k) {
    const int r = (int)(rng() % 10);
    if (r < 4) {
      const int src = 1 + (int)(rng() % 3);
      s.gates.push_back({(int)(rng() % 3), qb(), src == S_SCALED ? (int)(rng() % 5) : 0, src,
                         (int)(rng() % (src == S_WEIGHT ? 5 : 4))});
    } else if (r < 6) {
      s.gates.push_back({G_H + (int)(rng() % 9), qb(), 0, 0, 0});
    } else if (n > 1) {
      int a = qb(), b = qb();
      while (b == a) b = qb();
      int t = r < 8 ? G_CNOT : G_CZ;
      if (crot && r == 9) {
        s.gates.push_back({G_CRX + (int)(rng() % 3), a, b, S_WEIGHT, (int)(rng() % 5)});
        continue;
      }
      s.gates.push_back({t, a, b, 0, 0});
    }
  }
  for (int m = 0; m < 3; ++m) {
    const uint64_t all = ((uint64_t)1 << n) - 1;
    s.z.push_back((((uint64_t)rng() << 32) ^ rng()) & all);
    s.x.push_back(pauli ? ((((uint64_t)rng() << 32) ^ rng()) & all) : 0);
  }
  return s;
}

int create(const Spec &s, CircuitDesc &d, std::string &err) {
  return validate_and_build(s.n, s.gates.data(), (int32_t)s.gates.size(), s.n_in, s.n_w, s.z.data(),
                            s.x.empty() ? nullptr : s.x.data(), (int32_t)s.z.size(), d, err);
}

void exercise(const Spec &s, const std::string &name, bool all_tiles) {
  CircuitDesc d;
  std::string err;
  int rc = create(s, d, err);
  check(rc == 0, name + ": validate: " + err);
  if (rc) return;
  ParamCsr pc = param_csr(d);
  check(pc.w_ptr.size() == (size_t)s.n_w + 1 && pc.x_ptr.size() == (size_t)s.n_in + 1, name + ": csr sizes");
  if (d.has_crot() || d.n < kMinTileQubits) return;
  const int kmax = std::min(d.n, kMaxTileQubits);
  for (int kt = all_tiles ? kMinTileQubits : kmax; kt <= kmax; ++kt)
    for (int klo = 0; klo <= std::min(kt, 7); klo += (all_tiles ? 1 : 3))
      for (int zs : {0, 12}) {
      const std::string tag = name + " kt=" + std::to_string(kt) + " klo=" + std::to_string(klo) +
                              " zero_skip=" + std::to_string(zs);
      Plan p = make_plan(d, kt, klo, zs);
      check(check_plan(d, p).empty(), tag + ": check_plan");
      check(!plan_json(d, p).empty(), tag + ": plan_json");
      HostPlan hp;
      const std::string why = build_host_plan(d, kt, klo, hp, zs);
      check(why.empty(), tag + ": build_host_plan: " + why);
      if (!why.empty()) continue;
      for (int dbl = 0; dbl < 2; ++dbl) {
        JitSpec sp;
        sp.n = d.n;
        sp.kt = hp.kt;
        sp.dbl = dbl != 0;
        sp.M = (int)d.masks.size();
        sp.n_blocks = hp.n_blocks;
        sp.masks = d.masks;
        sp.seed_add = d.has_offdiag();
        const int64_t tiles = (int64_t)1 << (d.n - hp.kt);
        sp.nwg_full = (int)std::min<int64_t>(tiles, 512);
        sp.hp = &hp;
        for (int dir = 0; dir < 2; ++dir)
          for (int sw = 0; sw < hp.n_sweeps; ++sw) {
            const std::string src = jit_source(sp, dir, sw);
            check(src.find(jit_kernel_name(sp, dir)) != std::string::npos, tag + ": kernel name in source");
            const SweepLive lv = sweep_live(sp, dir, sw);
            check(lv.tiles >= 1 && lv.nwg >= 1 && lv.nwg <= sp.nwg_full, tag + ": live tiles");
            check(jit_lds_bytes(sp, dir, sw) <= 160 * 1024, tag + ": LDS within a compute unit");
          }
      }
    }
}

void invalid(const Spec &s, const std::string &what) {
  CircuitDesc d;
  std::string err;
  check(create(s, d, err) != 0, "rejected: " + what);
}

}  // namespace

int main() {
  std::mt19937 rng(12345);
  for (int n : {4, 5, 8, 12})
    for (int ring = 0; ring < 2; ++ring) exercise(layered(n, 3, ring), "layered n=" + std::to_string(n), true);
  exercise(layered(20, 8, false), "c3 n=20 ladder", false);
  exercise(layered(16, 4, true), "n=16 ring", false);
  for (int k = 0; k < 12; ++k) {
    const int n = 1 + (int)(rng() % 13);
    exercise(random_circuit(rng, n, 40, k % 3 == 0, k % 4 == 1), "random " + std::to_string(k), k < 4);
  }
  // invalid gate lists
  Spec b = layered(5, 1, true);
  b.gates[0].q0 = 5;
  invalid(b, "qubit out of range");
  b = layered(5, 1, true);
  b.gates.back().q1 = b.gates.back().q0;
  invalid(b, "control == target");
  b = layered(5, 1, true);
  b.gates[1].index = 1 << 20;
  invalid(b, "weight index out of range");
  b = layered(5, 1, true);
  b.gates[0].index = -1;
  invalid(b, "negative input index");
  b = layered(5, 1, true);
  b.gates[2].type = 99;
  invalid(b, "unknown gate type");
  b = layered(5, 1, true);
  b.z[0] = (uint64_t)1 << 5;
  invalid(b, "mask bit beyond the register");
  b = layered(5, 1, true);
  b.n = 31;
  invalid(b, "31 qubits");
  b = layered(5, 1, true);
  b.z.clear();
  invalid(b, "no observable");
  // uneven-batch list schedule: every unit exactly once, dependencies first
  for (int rep = 0; rep < 4; ++rep) {
    std::vector<std::vector<double>> cost;
    std::vector<int> ntiles;
    int total = 0;
    for (int i = 0; i < 30; ++i) {
      const int S = 1 + (int)(rng() % 5), nt = 1 << (rng() % 6);
      std::vector<double> c;
      for (int s = 0; s < S; ++s) c.push_back(1.0 + (double)(rng() % 100));
      cost.push_back(c);
      ntiles.push_back(nt);
      total += S * nt;
    }
    const std::vector<int32_t> q = multi_schedule(cost, ntiles, 1 + (int)(rng() % 64));
    check(q.size() % 4 == 0 && (int)(q.size() / 4) == total, "schedule covers every unit");
    std::vector<std::vector<int>> done(cost.size());
    for (size_t i = 0; i < cost.size(); ++i) done[i].assign(cost[i].size(), 0);
    for (size_t u = 0; u + 3 < q.size(); u += 4) {
      const int it = q[u], sw = q[u + 1], tl = q[u + 2];
      const bool in = it >= 0 && it < (int)cost.size() && sw >= 0 && sw < (int)cost[it].size() &&
                      tl >= 0 && tl < ntiles[it];
      check(in, "schedule unit in range");
      if (!in) break;
      check(sw == 0 || done[it][sw - 1] == ntiles[it], "schedule: previous sweep complete first");
      ++done[it][sw];
    }
  }
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("host driver ok\n");
  return 0;
}
