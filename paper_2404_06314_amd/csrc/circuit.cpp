// Circuit validation, rotation fusion, dependency DAG and sweep/stage planner.
#include "circuit.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <set>
#include <sstream>

#include "qtm.h"

namespace qtm {

int validate_and_build(int32_t n, const Gate *gates, int32_t n_gates, int32_t n_inputs,
                       int32_t n_weights, const uint64_t *masks, const uint64_t *xmasks,
                       int32_t n_obs, CircuitDesc &out, std::string &err) {
  char buf[256];
  if (n > 30) {
    err = "n_qubits > 30 is not supported";
    return QTM_ERR_UNSUPPORTED;
  }
  if (n < 1) {
    err = "n_qubits must be >= 1";
    return QTM_ERR_INVALID_ARG;
  }
  if (n_gates < 0 || n_inputs < 0 || n_weights < 0) {
    err = "negative count";
    return QTM_ERR_INVALID_ARG;
  }
  if (n_gates > 0 && !gates) {
    err = "gates is NULL";
    return QTM_ERR_INVALID_ARG;
  }
  if (n_obs < 1 || !masks) {
    err = "need at least one observable mask";
    return QTM_ERR_INVALID_ARG;
  }
  out = CircuitDesc();
  out.n = n;
  out.n_inputs = n_inputs;
  out.n_weights = n_weights;
  for (int32_t k = 0; k < n_gates; ++k) {
    const Gate &g = gates[k];
    if (g.type < 0 || g.type > G_CRZ) {
      snprintf(buf, sizeof buf, "gate %d: unknown type %d", k, g.type);
      err = buf;
      return QTM_ERR_UNSUPPORTED;
    }
    if (g.q0 < 0 || g.q0 >= n) {
      snprintf(buf, sizeof buf, "gate %d: qubit %d out of range", k, g.q0);
      err = buf;
      return QTM_ERR_INVALID_ARG;
    }
    if (is_param(g.type)) {
      if (is_crot(g.type) && g.src != S_INPUT && g.src != S_WEIGHT) {
        snprintf(buf, sizeof buf, "gate %d: a controlled rotation needs src INPUT or WEIGHT", k);
        err = buf;
        return QTM_ERR_INVALID_ARG;
      }
      if (g.src == S_INPUT) {
        if (g.index < 0 || g.index >= n_inputs) {
          snprintf(buf, sizeof buf, "gate %d: input index %d out of range", k, g.index);
          err = buf;
          return QTM_ERR_INVALID_ARG;
        }
      } else if (g.src == S_WEIGHT) {
        if (g.index < 0 || g.index >= n_weights) {
          snprintf(buf, sizeof buf, "gate %d: weight index %d out of range", k, g.index);
          err = buf;
          return QTM_ERR_INVALID_ARG;
        }
      } else if (g.src == S_SCALED) {
        if (g.index < 0 || g.index >= n_inputs || g.q1 < 0 || g.q1 >= n_weights) {
          snprintf(buf, sizeof buf, "gate %d: scaled input %d / weight %d out of range", k, g.index, g.q1);
          err = buf;
          return QTM_ERR_INVALID_ARG;
        }
      } else {
        snprintf(buf, sizeof buf, "gate %d: rotation needs src INPUT, WEIGHT or SCALED", k);
        err = buf;
        return QTM_ERR_INVALID_ARG;
      }
    }
    if (!is_rotation(g.type) && !is_fixed(g.type)) {  // CNOT, CZ, controlled rotations
      if (g.q1 < 0 || g.q1 >= n) {
        snprintf(buf, sizeof buf, "gate %d: qubit %d out of range", k, g.q1);
        err = buf;
        return QTM_ERR_INVALID_ARG;
      }
      if (g.q1 == g.q0) {
        snprintf(buf, sizeof buf, "gate %d: both qubits are %d", k, g.q0);
        err = buf;
        return QTM_ERR_INVALID_ARG;
      }
    }
    Gate c = g;
    if (!is_param(g.type)) {
      c.src = S_NONE;
      c.index = 0;
    }
    if (is_fixed(g.type) || (is_rotation(g.type) && g.src != S_SCALED)) c.q1 = 0;
    out.gates.push_back(c);
  }
  for (int32_t m = 0; m < n_obs; ++m) {
    const uint64_t xm = xmasks ? xmasks[m] : 0;
    if (n < 64 && ((masks[m] | xm) >> n) != 0) {
      snprintf(buf, sizeof buf, "observable %d: mask has a bit >= n_qubits", m);
      err = buf;
      return QTM_ERR_INVALID_ARG;
    }
    out.masks.push_back(xm ? 0 : masks[m]);
    out.pauli_x.push_back(xm);
    out.pauli_z.push_back(masks[m]);
  }
  out.gate_occ.assign(out.gates.size(), -1);
  for (size_t k = 0; k < out.gates.size(); ++k)
    if (is_param(out.gates[k].type)) {
      out.gate_occ[k] = (int32_t)out.occ_gate.size();
      out.occ_gate.push_back((int32_t)k);
    }
  return QTM_OK;
}

ParamCsr param_csr(const CircuitDesc &c) {
  std::vector<std::vector<std::pair<int32_t, int32_t>>> wl(c.n_weights), xl(c.n_inputs);
  for (size_t k = 0; k < c.occ_gate.size(); ++k) {
    const Gate &g = c.gates[c.occ_gate[k]];
    const int32_t occ = (int32_t)k;
    if (g.src == S_WEIGHT) {
      wl[g.index].push_back({occ, -1});
    } else if (g.src == S_INPUT) {
      xl[g.index].push_back({occ, -1});
    } else {
      wl[g.q1].push_back({occ, g.index});
      xl[g.index].push_back({occ, g.q1});
    }
  }
  ParamCsr r;
  auto put = [](const std::vector<std::vector<std::pair<int32_t, int32_t>>> &lists,
                std::vector<int32_t> &ptr, std::vector<int32_t> &lst, std::vector<int32_t> &fac) {
    ptr.assign(1, 0);
    for (const auto &l : lists) {
      for (const auto &e : l) {
        lst.push_back(e.first);
        fac.push_back(e.second);
      }
      ptr.push_back((int32_t)lst.size());
    }
  };
  put(wl, r.w_ptr, r.w_list, r.w_fac);
  put(xl, r.x_ptr, r.x_list, r.x_fac);
  return r;
}

// --------------------------------------------------------------------------
// fusion and DAG

static std::vector<int> wires(const FOp &o) {
  if (o.kind == FK_BLOCK) return {o.q0};
  return {o.q0, o.q1};
}

static bool commute(const FOp &a, const FOp &b) {
  std::vector<int> wa = wires(a), wb = wires(b);
  bool share = false;
  for (int x : wa)
    for (int y : wb) share |= x == y;
  if (!share) return true;
  if (a.diagonal && b.diagonal) return true;
  auto cnot_diag = [](const FOp &c, const FOp &d) {  // c CNOT, d diagonal
    for (int w : wires(d))
      if (w == c.q1) return false;
    return true;
  };
  if (a.kind == FK_CNOT && b.diagonal) return cnot_diag(a, b);
  if (b.kind == FK_CNOT && a.diagonal) return cnot_diag(b, a);
  if (a.kind == FK_CNOT && b.kind == FK_CNOT) return a.q0 != b.q1 && b.q0 != a.q1;
  return false;
}

static std::vector<FOp> fuse(const CircuitDesc &c) {
  std::vector<FOp> ops;
  std::vector<int> open(c.n, -1);
  for (size_t k = 0; k < c.gates.size(); ++k) {
    const Gate &g = c.gates[k];
    if (is_rotation(g.type) || is_fixed(g.type)) {
      int q = g.q0;
      if (open[q] < 0) {
        FOp o;
        o.kind = FK_BLOCK;
        o.q0 = q;
        o.diagonal = true;
        open[q] = (int)ops.size();
        ops.push_back(o);
      }
      FOp &o = ops[open[q]];
      o.gates.push_back((int32_t)k);
      if (is_rotation(g.type)) o.has_param = true;
      if (!is_diag1(g.type)) o.diagonal = false;
    } else {
      open[g.q0] = -1;
      open[g.q1] = -1;
      FOp o;
      o.kind = g.type == G_CNOT ? FK_CNOT : FK_CZ;
      o.q0 = g.q0;
      o.q1 = g.q1;
      o.gates.push_back((int32_t)k);
      o.diagonal = g.type == G_CZ;
      ops.push_back(o);
    }
  }
  return ops;
}

// predecessors that do not commute (all earlier ones, not only immediate)
static std::vector<std::vector<int>> build_preds(const std::vector<FOp> &ops, int n) {
  std::vector<std::vector<int>> on_wire(n);
  std::vector<std::vector<int>> preds(ops.size());
  for (size_t j = 0; j < ops.size(); ++j) {
    std::set<int> ps;
    for (int w : wires(ops[j]))
      for (int i : on_wire[w])
        if (!commute(ops[i], ops[j])) ps.insert(i);
    preds[j].assign(ps.begin(), ps.end());
    for (int w : wires(ops[j])) on_wire[w].push_back((int)j);
  }
  return preds;
}

namespace {

struct Sched {
  const std::vector<FOp> &ops;
  const std::vector<std::vector<int>> &succ;
  std::vector<int> left;   // unscheduled predecessors
  std::vector<char> done;

  // Execute (or simulate) every op that becomes ready and whose target is in
  // `inset`; `allowed` restricts the op set (sweep scope).  Returns the ops
  // run, in order.
  std::vector<int> run(const std::vector<char> &inset, const std::vector<char> *allowed,
                       bool commit, int max_blocks = 1 << 30) {
    std::vector<int> lft = left;
    std::vector<char> dn = done;
    std::vector<int> order;
    std::vector<int> ready;
    int blocks = 0;
    for (size_t i = 0; i < ops.size(); ++i)
      if (!dn[i] && lft[i] == 0 && (!allowed || (*allowed)[i])) ready.push_back((int)i);
    std::sort(ready.begin(), ready.end());
    bool progress = true;
    while (progress) {
      progress = false;
      std::vector<int> next;
      for (int i : ready) {
        const FOp &o = ops[i];
        int t = o.target();
        if ((t >= 0 && !inset[t]) || (o.kind == FK_BLOCK && blocks >= max_blocks)) {
          next.push_back(i);
          continue;
        }
        if (o.kind == FK_BLOCK) ++blocks;
        dn[i] = 1;
        order.push_back(i);
        progress = true;
        for (int s : succ[i])
          if (--lft[s] == 0 && (!allowed || (*allowed)[s])) next.push_back(s);
      }
      std::sort(next.begin(), next.end());
      next.erase(std::unique(next.begin(), next.end()), next.end());
      ready.swap(next);
    }
    if (commit) {
      left = lft;
      done = dn;
    }
    return order;
  }
};

// Greedy choice of `k` members of a set among `cands`, starting from `base`:
// each step adds the candidate that lets the most ops run (ties: the one whose
// earliest pending op comes first).
std::vector<char> choose_set(Sched &S, const std::vector<char> &base, const std::vector<int> &cands,
                             int k, int nq, const std::vector<char> *allowed) {
  std::vector<char> in = base;
  std::vector<int> first(nq, 1 << 30);
  for (size_t i = 0; i < S.ops.size(); ++i)
    if (!S.done[i] && (!allowed || (*allowed)[i])) {
      int t = S.ops[i].target();
      if (t >= 0) first[t] = std::min(first[t], (int)i);
    }
  int have = 0;
  for (int q : cands) have += in[q] ? 1 : 0;
  while (have < k) {
    int best = -1;
    long best_score = -1;
    for (int q : cands) {
      if (in[q]) continue;
      in[q] = 1;
      long cnt = (long)S.run(in, allowed, false).size();
      in[q] = 0;
      long score = cnt * (1L << 31) - first[q];
      if (score > best_score) {
        best_score = score;
        best = q;
      }
    }
    if (best < 0) break;
    in[best] = 1;
    ++have;
  }
  return in;
}

// Tiles of the greedy planner: each sweep takes the klo low qubits plus the
// kt - klo others that let the most ops run.
std::vector<uint64_t> greedy_tiles(Sched S, int nq, int kt, int klo) {
  std::vector<uint64_t> out;
  std::vector<int> all_q(nq);
  for (int q = 0; q < nq; ++q) all_q[q] = q;
  size_t n_done = 0;
  while (n_done < S.ops.size()) {
    std::vector<char> base(nq, 0);
    for (int q = 0; q < klo; ++q) base[q] = 1;
    std::vector<char> T = choose_set(S, base, all_q, kt, nq, nullptr);
    const size_t ran = S.run(T, nullptr, true, kMaxSweepBlocks).size();
    if (ran == 0) break;
    n_done += ran;
    uint64_t m = 0;
    for (int q = 0; q < nq; ++q)
      if (T[q]) m |= (uint64_t)1 << q;
    out.push_back(m);
  }
  return out;
}

// Estimated cost of one sweep for kernels that skip the tiles whose
// amplitudes are all zero, in units of one fused block applied to the whole
// state by the forward and the backward sweep together.  A full-state sweep
// moves the state through HBM (kSweepIo block units), which the block work
// hides only in part (kOverlap); a sweep over a fraction `live` of the tiles
// costs that fraction, but at least a per-block latency (few tiles run their
// blocks one after another); each sweep adds a launch.  The constants are
// MI355X measurements of the complex64 sweeps at 20 qubits, batch 64: about
// 44 us per block over the whole state (forward + backward), 530 us of
// traffic per full-state sweep pair (io = 12, the default of
// QTM_OPT_PLAN_IO, which the autotuner varies).
double sweep_cost(double live, int blocks, double io) {
  constexpr double kOverlap = 0.3, kLatency = 0.03, kLaunch = 0.25;
  const double b = blocks;
  const double full = std::max(io, b) + kOverlap * std::min(io, b);
  return std::max(live * full, kLatency * b) + kLaunch;
}

// Qubits a run of ops excites: until a qubit is the target of a
// non-diagonal block or of a CNOT, every amplitude with its bit set is 0.
uint64_t excited_by(const std::vector<FOp> &ops, const std::vector<int> &order) {
  uint64_t ex = 0;
  for (int i : order) {
    const FOp &o = ops[i];
    if ((o.kind == FK_BLOCK && !o.diagonal) || o.kind == FK_CNOT) ex |= (uint64_t)1 << o.target();
  }
  return ex;
}

// Fraction of the tiles a sweep with tile mask `tile` runs when the qubits
// in `ex` are excited before it: those whose outer bits are 0 on every
// unexcited outer qubit.
double live_fraction(uint64_t ex, uint64_t tile, int nq, int kt) {
  const uint64_t all = nq >= 64 ? ~(uint64_t)0 : (((uint64_t)1 << nq) - 1);
  const int outer_ex = __builtin_popcountll(ex & ~tile & all);
  return std::ldexp(1.0, outer_ex - (nq - kt));
}

int count_blocks(const std::vector<FOp> &ops, const std::vector<int> &order) {
  int b = 0;
  for (int i : order) b += ops[i].kind == FK_BLOCK ? 1 : 0;
  return b;
}

double tiles_cost(Sched S, const std::vector<uint64_t> &tiles, int nq, int kt, double io) {
  double cost = 0.0;
  uint64_t ex = 0;
  for (uint64_t m : tiles) {
    std::vector<char> T(nq, 0);
    for (int q = 0; q < nq; ++q) T[q] = (m >> q) & 1;
    const std::vector<int> order = S.run(T, nullptr, true, kMaxSweepBlocks);
    cost += sweep_cost(live_fraction(ex, m, nq, kt), count_blocks(S.ops, order), io);
    ex |= excited_by(S.ops, order);
  }
  return cost;
}

// Tile sequence for kernels that skip all-zero tiles: a beam search over
// sweeps.  A sweep that leaves unexcited qubits outside its tile runs only a
// fraction of the tiles, so fewer ops per sweep can cost less than the
// greedy planner's maximal sweeps.  Candidates per step: the greedy tile,
// and the greedy tile with one, or two, unexcited qubits kept out of it.
// Returns the greedy sequence when the search finds nothing cheaper.
std::vector<uint64_t> zero_aware_tiles(const Sched &S0, int nq, int kt, int klo, double io) {
  const std::vector<uint64_t> greedy = greedy_tiles(S0, nq, kt, klo);
  if (nq <= kt) return greedy;
  const double greedy_cost = tiles_cost(S0, greedy, nq, kt, io);
  constexpr int kWidth = 8, kTopSingles = 5, kMaxDepth = 64;
  constexpr double kPerBlockLeft = 1.2;  // ranking: estimated cost of the blocks not yet run
  struct Node {
    std::vector<int> left;
    std::vector<char> done;
    uint64_t ex = 0;
    size_t n_done = 0;
    int blocks_left = 0;
    double cost = 0.0;
    std::vector<uint64_t> tiles;
  };
  int total_blocks = 0;
  for (const FOp &o : S0.ops) total_blocks += o.kind == FK_BLOCK ? 1 : 0;
  std::vector<Node> frontier(1);
  frontier[0].left = S0.left;
  frontier[0].done = S0.done;
  frontier[0].blocks_left = total_blocks;
  std::vector<int> all_q(nq);
  for (int q = 0; q < nq; ++q) all_q[q] = q;
  double best_cost = greedy_cost;
  std::vector<uint64_t> best = greedy;
  for (int depth = 0; depth < kMaxDepth && !frontier.empty(); ++depth) {
    std::map<std::vector<char>, Node> next;
    for (const Node &nd : frontier) {
      Sched S{S0.ops, S0.succ, nd.left, nd.done};
      std::vector<char> base(nq, 0);
      for (int q = 0; q < klo; ++q) base[q] = 1;
      auto tile_without = [&](const std::vector<int> &out) {
        std::vector<int> cands;
        for (int q : all_q)
          if (std::find(out.begin(), out.end(), q) == out.end()) cands.push_back(q);
        return choose_set(S, base, cands, kt, nq, nullptr);
      };
      std::vector<std::vector<char>> tiles;
      tiles.push_back(tile_without({}));
      // unexcited qubits outside the low ones, by the ops the tile without
      // each of them runs
      std::vector<std::pair<long, int>> singles;
      for (int q = klo; q < nq; ++q) {
        if ((nd.ex >> q) & 1) continue;
        std::vector<char> T = tile_without({q});
        singles.push_back({-(long)S.run(T, nullptr, false, kMaxSweepBlocks).size(), q});
        tiles.push_back(T);
      }
      std::sort(singles.begin(), singles.end());
      const int ns = std::min((int)singles.size(), kTopSingles);
      for (int i = 0; i < ns; ++i)
        for (int j = i + 1; j < ns; ++j) tiles.push_back(tile_without({singles[i].second, singles[j].second}));
      std::set<uint64_t> seen;
      for (const std::vector<char> &T : tiles) {
        uint64_t m = 0;
        for (int q = 0; q < nq; ++q)
          if (T[q]) m |= (uint64_t)1 << q;
        if ((int)__builtin_popcountll(m) != kt || !seen.insert(m).second) continue;
        Sched St{S0.ops, S0.succ, nd.left, nd.done};
        const std::vector<int> order = St.run(T, nullptr, true, kMaxSweepBlocks);
        if (order.empty()) continue;
        const int nb = count_blocks(S0.ops, order);
        Node c;
        c.cost = nd.cost + sweep_cost(live_fraction(nd.ex, m, nq, kt), nb, io);
        c.ex = nd.ex | excited_by(S0.ops, order);
        c.n_done = nd.n_done + order.size();
        c.blocks_left = nd.blocks_left - nb;
        c.tiles = nd.tiles;
        c.tiles.push_back(m);
        if (c.n_done == S0.ops.size()) {
          if (c.cost < best_cost - 1e-9) {
            best_cost = c.cost;
            best = c.tiles;
          }
          continue;
        }
        if (c.cost >= best_cost) continue;
        c.left = std::move(St.left);
        c.done = St.done;
        auto it = next.find(St.done);
        if (it == next.end()) next.emplace(std::move(St.done), std::move(c));
        else if (c.cost < it->second.cost) it->second = std::move(c);
      }
    }
    std::vector<Node> nf;
    nf.reserve(next.size());
    for (auto &kv : next) nf.push_back(std::move(kv.second));
    std::sort(nf.begin(), nf.end(), [&](const Node &a, const Node &b) {
      const double ka = a.cost + kPerBlockLeft * a.blocks_left, kb = b.cost + kPerBlockLeft * b.blocks_left;
      if (ka != kb) return ka < kb;
      return a.tiles < b.tiles;
    });
    if ((int)nf.size() > kWidth) nf.resize(kWidth);
    frontier = std::move(nf);
  }
  return best;
}

}  // namespace

Plan make_plan(const CircuitDesc &c, int32_t kt, int32_t klo, int32_t zero_skip) {
  Plan p;
  p.n = c.n;
  p.kt = kt;
  // the tile must have at least one free slot when the state is larger than a tile
  p.klo = std::min(klo, c.n > kt ? kt - 1 : kt);
  p.ops = fuse(c);
  for (size_t i = 0; i < p.ops.size(); ++i)
    if (p.ops[i].kind == FK_BLOCK) {
      p.ops[i].block = p.n_blocks++;
      p.block_op.push_back((int)i);
      if (p.ops[i].has_param) p.ops[i].gslot = p.n_gslots++;
    }
  auto preds = build_preds(p.ops, c.n);
  std::vector<std::vector<int>> succ(p.ops.size());
  std::vector<int> left(p.ops.size());
  for (size_t j = 0; j < p.ops.size(); ++j) {
    left[j] = (int)preds[j].size();
    for (int i : preds[j]) succ[i].push_back((int)j);
  }
  Sched S{p.ops, succ, left, std::vector<char>(p.ops.size(), 0)};
  // tiles: the klo low qubits plus kt - klo others per sweep
  const std::vector<uint64_t> tiles =
      zero_skip > 0 ? zero_aware_tiles(S, c.n, kt, p.klo, zero_skip) : greedy_tiles(S, c.n, kt, p.klo);
  for (uint64_t tm : tiles) {
    std::vector<char> T(c.n, 0);
    for (int q = 0; q < c.n; ++q) T[q] = (tm >> q) & 1;
    std::vector<int> order = S.run(T, nullptr, true, kMaxSweepBlocks);
    if (order.empty()) break;  // cannot happen: every tile of the sequence runs ops
    Sweep sw;
    for (int q = 0; q < c.n; ++q)
      if (T[q]) sw.tile.push_back(q);
    // tile-local position of each global qubit
    std::vector<int> loc(c.n, -1);
    for (size_t k = 0; k < sw.tile.size(); ++k) loc[sw.tile[k]] = (int)k;
    // stages inside the sweep
    std::vector<char> allowed(p.ops.size(), 0);
    for (int i : order) allowed[i] = 1;
    Sched St{p.ops, succ, std::vector<int>(p.ops.size(), 0), std::vector<char>(p.ops.size(), 1)};
    for (int i : order) {
      St.done[i] = 0;
      int cnt = 0;
      for (int pr : preds[i]) cnt += allowed[pr] ? 1 : 0;
      St.left[i] = cnt;
    }
    size_t st_done = 0;
    while (st_done < order.size()) {
      std::vector<char> none(c.n, 0);
      std::vector<char> R = choose_set(St, none, sw.tile, kRegBits, c.n, &allowed);
      // fill to exactly kRegBits register bits
      for (int q : sw.tile) {
        int cnt = 0;
        for (int x : sw.tile) cnt += R[x] ? 1 : 0;
        if (cnt >= kRegBits) break;
        R[q] = 1;
      }
      std::vector<int> sto = St.run(R, &allowed, true);
      if (sto.empty()) break;
      st_done += sto.size();
      Stage st;
      int r = 0;
      for (int q : sw.tile)
        if (R[q]) st.regpos[r++] = loc[q];
      st.ops.assign(sto.begin(), sto.end());
      sw.stages.push_back(st);
    }
    for (int i : order)
      if (p.ops[i].kind == FK_BLOCK && p.ops[i].gslot >= 0) sw.gslots.push_back(p.ops[i].gslot);
    p.sweeps.push_back(sw);
  }
  if (p.sweeps.empty()) {
    // a circuit without gates still needs one sweep: it writes |0...0> and
    // reads the observables
    Sweep sw;
    for (int q = 0; q < kt; ++q) sw.tile.push_back(q);
    p.sweeps.push_back(sw);
  }
  for (Sweep &sw : p.sweeps)
    if (sw.stages.empty()) {
      Stage st;
      for (int r = 0; r < kRegBits; ++r) st.regpos[r] = r;
      sw.stages.push_back(st);
    }
  return p;
}

std::string check_plan(const CircuitDesc &c, const Plan &p) {
  std::vector<int> pos(p.ops.size(), -1);
  int counter = 0;
  for (size_t s = 0; s < p.sweeps.size(); ++s) {
    const Sweep &sw = p.sweeps[s];
    if ((int)sw.tile.size() != p.kt) return "tile size mismatch";
    for (int q = 0; q < p.klo; ++q)
      if (sw.tile[q] != q) return "low qubits not in tile";
    for (const Stage &st : sw.stages) {
      std::set<int> rb(st.regpos, st.regpos + kRegBits);
      if ((int)rb.size() != kRegBits) return "duplicate register bits";
      for (int i : st.ops) {
        if (i < 0 || i >= (int)p.ops.size()) return "bad op index";
        if (pos[i] >= 0) return "op scheduled twice";
        pos[i] = counter++;
        int t = p.ops[i].target();
        if (t >= 0) {
          int l = -1;
          for (int k = 0; k < p.kt; ++k)
            if (sw.tile[k] == t) l = k;
          if (l < 0) return "target outside tile";
          if (!rb.count(l)) return "target outside register bits";
        }
      }
    }
  }
  for (size_t i = 0; i < p.ops.size(); ++i)
    if (pos[i] < 0) return "op never scheduled";
  // every pair of non-commuting ops keeps its order
  auto preds = build_preds(p.ops, c.n);
  for (size_t j = 0; j < p.ops.size(); ++j)
    for (int i : preds[j])
      if (pos[i] > pos[(int)j]) return "dependency order violated";
  size_t ng = 0;
  for (const FOp &o : p.ops) ng += o.gates.size();
  if (ng != c.gates.size()) return "gate count mismatch";
  return "";
}

std::string plan_json(const CircuitDesc &c, const Plan &p) {
  std::ostringstream s;
  s << "{\"n\":" << p.n << ",\"kt\":" << p.kt << ",\"klo\":" << p.klo << ",\"n_blocks\":" << p.n_blocks
    << ",\"n_gslots\":" << p.n_gslots << ",\"sweeps\":[";
  for (size_t i = 0; i < p.sweeps.size(); ++i) {
    const Sweep &sw = p.sweeps[i];
    if (i) s << ",";
    s << "{\"tile\":[";
    for (size_t k = 0; k < sw.tile.size(); ++k) s << (k ? "," : "") << sw.tile[k];
    s << "],\"stages\":[";
    for (size_t t = 0; t < sw.stages.size(); ++t) {
      const Stage &st = sw.stages[t];
      if (t) s << ",";
      s << "{\"regpos\":[" << st.regpos[0] << "," << st.regpos[1] << "," << st.regpos[2] << ","
        << st.regpos[3] << "],\"gates\":[";
      bool first = true;
      for (int o : st.ops)
        for (int g : p.ops[o].gates) {
          s << (first ? "" : ",") << g;
          first = false;
        }
      s << "]}";
    }
    s << "]}";
  }
  s << "]}";
  (void)c;
  return s.str();
}

// --------------------------------------------------------------------------
// program encoding

static uint32_t pdep_bits(uint32_t v, const int *pos, int npos) {
  uint32_t r = 0;
  for (int i = 0; i < npos; ++i)
    if ((v >> i) & 1u) r |= 1u << pos[i];
  return r;
}

static int parity32(uint32_t v) { return __builtin_popcount(v) & 1; }

static void encode_sweep(const CircuitDesc &c, const Plan &p, const Sweep &sw, bool backward,
                         const std::vector<char> &first_on_wire, std::vector<int32_t> &code,
                         std::vector<int32_t> &thr, std::vector<int32_t> &sweep_offs,
                         int32_t &max_gs) {
  const int kt = p.kt, nthr_bits = kt - kRegBits;
  const int off = (int)code.size();
  sweep_offs.push_back(off);
  const int nst = (int)sw.stages.size();
  // sweep-local matrix slots: blocks in order of first use
  std::vector<int> mslots, mslot_of(p.n_blocks, -1);
  for (const Stage &st : sw.stages)
    for (int oi : st.ops)
      if (p.ops[oi].kind == FK_BLOCK && mslot_of[p.ops[oi].block] < 0) {
        mslot_of[p.ops[oi].block] = (int)mslots.size();
        mslots.push_back(p.ops[oi].block);
      }
  int hdr = kSwStages + nst + (int)sw.gslots.size() + (int)mslots.size();
  code.resize(off + hdr, 0);
  int32_t *H = nullptr;
  auto h = [&](int i) -> int32_t & { return code[off + i]; };
  (void)H;
  std::vector<int> outer;
  std::vector<char> intile(c.n, 0);
  for (int q : sw.tile) intile[q] = 1;
  for (int q = 0; q < c.n; ++q)
    if (!intile[q]) outer.push_back(q);
  h(0) = nst;
  h(1) = (int)outer.size();
  h(2) = (int)sw.gslots.size();
  h(3) = (int)mslots.size();
  max_gs = std::max(max_gs, (int)sw.gslots.size());
  for (size_t i = 0; i < outer.size(); ++i) h(kSwOuter + i) = outer[i];
  for (int k = 0; k < kt; ++k) h(kSwTile + k) = sw.tile[k];
  // load layout: local index i = t + 2^(kt-4) * j
  for (int j = 0; j < kRegs; ++j) {
    uint32_t local = (uint32_t)j << nthr_bits;
    h(kSwLoadG + j) = (int32_t)pdep_bits(local, sw.tile.data(), kt);
    h(kSwLoadL + j) = (int32_t)lds_swizzle(local);
  }
  for (int i = 0; i < nthr_bits; ++i) h(kSwLoadTb + i) = sw.tile[i];
  // sweep-local gslot numbering: order of sw.gslots
  std::vector<int> local_gs(p.n_gslots, -1);
  for (size_t i = 0; i < sw.gslots.size(); ++i) {
    local_gs[sw.gslots[i]] = (int)i;
    h(kSwStages + nst + (int)i) = sw.gslots[i];
  }
  for (size_t i = 0; i < mslots.size(); ++i)
    h(kSwStages + nst + (int)sw.gslots.size() + (int)i) = mslots[i];
  for (int si = 0; si < nst; ++si) {
    const Stage &st = sw.stages[backward ? nst - 1 - si : si];
    h(kSwStages + si) = (int32_t)code.size();
    const int so = (int)code.size();
    code.resize(so + kStOps, 0);
    auto sh = [&](int i) -> int32_t & { return code[so + i]; };
    int rp[kRegBits];
    for (int r = 0; r < kRegBits; ++r) rp[r] = st.regpos[r];
    uint32_t W[kRegs];
    for (int j = 0; j < kRegs; ++j) {
      uint32_t local = pdep_bits((uint32_t)j, rp, kRegBits);
      sh(kStLds + j) = (int32_t)lds_swizzle(local);
      W[j] = pdep_bits(local, sw.tile.data(), kt);
      sh(kStGlob + j) = (int32_t)W[j];
    }
    std::vector<char> isreg(kt, 0);
    for (int r = 0; r < kRegBits; ++r) {
      isreg[rp[r]] = 1;
      sh(kStRegPos + r) = rp[r];
    }
    std::vector<int> tpos;  // local positions of the thread bits, ascending
    for (int k = 0; k < kt; ++k)
      if (!isreg[k]) tpos.push_back(k);
    sh(kStThr) = (int32_t)thr.size();
    for (uint32_t t = 0; t < (1u << nthr_bits); ++t) {
      uint32_t lt = pdep_bits(t, tpos.data(), nthr_bits);
      thr.push_back((int32_t)pdep_bits(lt, sw.tile.data(), kt));
    }
    // ops: CZs merged into one diag op at the position of the first CZ of a run
    std::vector<int> ops = st.ops;
    if (backward) std::reverse(ops.begin(), ops.end());
    std::vector<std::vector<int32_t>> enc;
    std::vector<std::vector<int32_t>> diag_recs;
    int32_t stage_flags = 0;
    std::vector<std::pair<int, int>> czrun;
    auto flush_cz = [&]() {
      if (czrun.empty()) return;
      // groups by distance
      std::vector<std::pair<int, uint32_t>> groups;
      for (auto &pr : czrun) {
        int a = std::min(pr.first, pr.second), b = std::max(pr.first, pr.second);
        int d = b - a;
        bool found = false;
        for (auto &g : groups)
          if (g.first == d) {
            g.second ^= 1u << a;  // a pair listed twice cancels (CZ^2 = I)
            found = true;
          }
        if (!found) groups.push_back({d, 1u << a});
      }
      std::vector<int32_t> rec;
      rec.push_back((int32_t)groups.size());
      for (auto &g : groups) {
        rec.push_back(g.first);
        rec.push_back((int32_t)g.second);
      }
      if (!groups.empty()) stage_flags |= 1;
      // linear term of register bit b: C(W_{e_b}) restricted to non-register bits
      uint32_t regmask = W[kRegs - 1];
      for (int b = 0; b < kRegBits; ++b) {
        const uint32_t Wb = W[1 << b];
        uint32_t Cb = 0;
        for (auto &pr : czrun) {
          int a = pr.first, d = pr.second;
          if ((Wb >> d) & 1u) Cb ^= 1u << a;
          if ((Wb >> a) & 1u) Cb ^= 1u << d;
        }
        rec.push_back((int32_t)(Cb & ~regmask));
      }
      uint32_t qmask = 0;
      for (int j = 0; j < kRegs; ++j) {
        int q = 0;
        for (auto &pr : czrun) q ^= (int)(((W[j] >> pr.first) & (W[j] >> pr.second)) & 1u);
        if (q) qmask |= 1u << j;
      }
      rec.push_back((int32_t)qmask);
      enc.push_back({OP_DIAG, (int32_t)diag_recs.size(), 0, 0});
      diag_recs.push_back(rec);
      czrun.clear();
    };
    std::vector<int> regbit_of(kt, -1);
    for (int r = 0; r < kRegBits; ++r) regbit_of[rp[r]] = r;
    std::vector<int> loc(c.n, -1);
    for (int k = 0; k < kt; ++k) loc[sw.tile[k]] = k;
    for (int oi : ops) {
      const FOp &o = p.ops[oi];
      if (o.kind == FK_CZ) {
        czrun.push_back({o.q0, o.q1});
        continue;
      }
      flush_cz();
      if (o.kind == FK_BLOCK) {
        int r = regbit_of[loc[o.q0]];
        const int32_t code_u1 = !first_on_wire[oi] ? OP_U1 : backward ? OP_U1_LAST : OP_U1_FIRST;
        enc.push_back({code_u1, r, mslot_of[o.block], o.gslot >= 0 ? local_gs[o.gslot] : -1});
      } else {
        int r = regbit_of[loc[o.q1]];
        int lc = loc[o.q0];
        if (lc >= 0 && regbit_of[lc] >= 0)
          enc.push_back({OP_CNOT, r, 0, regbit_of[lc]});
        else
          enc.push_back({OP_CNOT, r, 1, o.q0});
      }
    }
    flush_cz();
    sh(0) = (int32_t)enc.size();
    sh(kStFlags) = stage_flags;
    int ops_off = (int)code.size();
    code.resize(ops_off + 4 * enc.size(), 0);
    for (size_t e = 0; e < enc.size(); ++e)
      for (int f = 0; f < 4; ++f) code[ops_off + 4 * e + f] = enc[e][f];
    // diag records after the ops; patch offsets
    for (size_t e = 0; e < enc.size(); ++e)
      if (enc[e][0] == OP_DIAG) {
        int rec_off = (int)code.size();
        const std::vector<int32_t> &rec = diag_recs[enc[e][1]];
        code.insert(code.end(), rec.begin(), rec.end());
        code[ops_off + 4 * e + 1] = rec_off;
      }
  }
}

Program encode_program(const CircuitDesc &c, const Plan &p) {
  Program pr;
  // blocks that are the first op on their qubit in execution order
  std::vector<char> first_on_wire(p.ops.size(), 0), touched(c.n, 0);
  for (const Sweep &sw : p.sweeps)
    for (const Stage &st : sw.stages)
      for (int oi : st.ops) {
        const FOp &o = p.ops[oi];
        if (o.kind == FK_BLOCK) {
          if (!touched[o.q0]) first_on_wire[oi] = 1;
          touched[o.q0] = 1;
        } else {
          touched[o.q0] = touched[o.q1] = 1;
        }
      }
  uint64_t ex = 0;
  for (const Sweep &sw : p.sweeps) {
    for (const Stage &st : sw.stages)
      for (int oi : st.ops) {
        const FOp &o = p.ops[oi];
        if ((o.kind == FK_BLOCK && !o.diagonal) || o.kind == FK_CNOT) ex |= (uint64_t)1 << o.target();
      }
    pr.excited.push_back(ex);
  }
  for (const Sweep &sw : p.sweeps)
    encode_sweep(c, p, sw, false, first_on_wire, pr.code, pr.thr, pr.sweep_off_fwd,
                 pr.max_gslots_per_sweep);
  for (int s = (int)p.sweeps.size() - 1; s >= 0; --s)
    encode_sweep(c, p, p.sweeps[s], true, first_on_wire, pr.code, pr.thr, pr.sweep_off_bwd,
                 pr.max_gslots_per_sweep);
  return pr;
}

std::string build_host_plan(const CircuitDesc &c, int32_t kt, int32_t klo, HostPlan &out, int32_t zero_skip) {
  Plan plan = make_plan(c, kt, klo, zero_skip);
  std::string why = check_plan(c, plan);
  if (!why.empty()) return why;
  HostPlan &h = out;
  h.prog = encode_program(c, plan);
  h.kt = kt;
  h.klo = klo;
  h.zero_skip = zero_skip;
  h.n_blocks = plan.n_blocks;
  h.n_gslots = plan.n_gslots;
  h.max_gslots = h.prog.max_gslots_per_sweep;
  h.n_sweeps = (int32_t)plan.sweeps.size();
  h.blk.clear();
  h.blk_off.clear();
  h.occ_gslot.assign(c.occ_gate.size(), 0);
  for (int b = 0; b < plan.n_blocks; ++b) {
    const FOp &o = plan.ops[plan.block_op[b]];
    h.blk_off.push_back((int32_t)h.blk.size());
    h.blk.push_back(o.q0);
    h.blk.push_back((int32_t)o.gates.size());
    for (int g : o.gates) {
      const Gate &gt = c.gates[g];
      const int occ = c.gate_occ[g];
      h.blk.push_back(gt.type);
      h.blk.push_back(gt.src);
      h.blk.push_back(gt.index);
      h.blk.push_back(gt.src == S_SCALED ? gt.q1 : 0);
      h.blk.push_back(occ);
      if (occ >= 0) h.occ_gslot[occ] = o.gslot;
    }
  }
  // Z-string signs of the register bits of the last forward stage (the
  // thread part is applied by the kernel) and of the first backward load
  const int M = (int)c.masks.size();
  h.obs_sgn.assign((size_t)(M + 1) * kRegs, 1.f);
  h.seed_sgn.assign((size_t)M * kRegs, 1.0);
  if (!plan.sweeps.empty()) {
    const int32_t *H = h.prog.code.data() + h.prog.sweep_off_fwd.back();
    const int32_t *S = h.prog.code.data() + H[kSwStages + H[0] - 1];
    const int32_t *HB = h.prog.code.data() + h.prog.sweep_off_bwd.front();
    for (int m = 0; m < M; ++m)
      for (int j = 0; j < kRegs; ++j) {
        const uint32_t mk = (uint32_t)c.masks[m];
        h.obs_sgn[m * kRegs + j] = (__builtin_popcount((uint32_t)S[kStGlob + j] & mk) & 1) ? -1.f : 1.f;
        h.seed_sgn[m * kRegs + j] = (__builtin_popcount((uint32_t)HB[kSwLoadG + j] & mk) & 1) ? -1.0 : 1.0;
      }
  }
  return "";
}

}  // namespace qtm
