// Queue order of the persistent uneven-batch kernels (host only).
#include "schedule.h"

#include <algorithm>
#include <queue>

namespace qtm {

// List schedule of one pass: P identical workers; a sweep's tiles become
// ready when every tile of the previous sweep of that circuit has finished;
// among ready sweeps the one with the longest remaining chain goes first.
// The order in which tiles are handed out is the queue order.
std::vector<int32_t> multi_schedule(const std::vector<std::vector<double>> &cost,
                                    const std::vector<int> &ntiles, int P) {
  struct Ready {
    double prio;
    int item, sweep;
    bool operator<(const Ready &o) const {
      if (prio != o.prio) return prio < o.prio;
      if (item != o.item) return item > o.item;
      return sweep > o.sweep;
    }
  };
  struct Ev {
    double time;
    int item, sweep;
    bool operator>(const Ev &o) const {
      if (time != o.time) return time > o.time;
      return item > o.item;
    }
  };
  const int N = (int)cost.size();
  std::vector<std::vector<double>> tail(N);
  for (int i = 0; i < N; ++i) {
    const int S = (int)cost[i].size();
    tail[i].assign(S + 1, 0.0);
    for (int s = S - 1; s >= 0; --s) tail[i][s] = tail[i][s + 1] + cost[i][s];
  }
  std::priority_queue<Ready> ready;
  std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> events;
  std::priority_queue<double, std::vector<double>, std::greater<double>> workers;
  for (int p = 0; p < std::max(P, 1); ++p) workers.push(0.0);
  std::vector<int> next_tile(N, 0);
  std::vector<double> sweep_end(N, 0.0);
  size_t total = 0;
  for (int i = 0; i < N; ++i) {
    total += (size_t)cost[i].size() * ntiles[i];
    if (!cost[i].empty()) ready.push({tail[i][0], i, 0});
  }
  std::vector<int32_t> order;
  order.reserve(total * 4);
  while (order.size() < total * 4) {
    double t = workers.top();
    while (!events.empty() && events.top().time <= t) {
      const Ev e = events.top();
      events.pop();
      ready.push({tail[e.item][e.sweep], e.item, e.sweep});
    }
    if (ready.empty()) {
      if (events.empty()) break;  // unreachable: some sweep is always pending
      // idle until the next sweep completes
      workers.pop();
      workers.push(events.top().time);
      continue;
    }
    const Ready r = ready.top();
    const double fin = t + cost[r.item][r.sweep];
    workers.pop();
    workers.push(fin);
    order.push_back(r.item);
    order.push_back(r.sweep);
    order.push_back(next_tile[r.item]);
    order.push_back(0);
    sweep_end[r.item] = std::max(sweep_end[r.item], fin);
    if (++next_tile[r.item] == ntiles[r.item]) {
      ready.pop();
      next_tile[r.item] = 0;
      const double end = sweep_end[r.item];
      sweep_end[r.item] = 0.0;
      if (r.sweep + 1 < (int)cost[r.item].size()) events.push({end, r.item, r.sweep + 1});
    }
  }
  return order;
}

}  // namespace qtm
