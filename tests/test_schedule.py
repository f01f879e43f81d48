"""Queue order of the persistent uneven-batch kernels (host logic, CPU).

The list schedule is compiled from its C++ source with g++ and driven
through a tiny stdin/stdout harness; the checks are properties any valid
queue must have (each tile exactly once, every tile after all tiles of the
previous sweep of its circuit) plus hand-worked small cases.
"""
import os
import random
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2404_06314_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include "schedule.h"
int main() {
  int N, P;
  if (scanf("%d %d", &N, &P) != 2) return 1;
  std::vector<std::vector<double>> cost(N);
  std::vector<int> nt(N);
  for (int i = 0; i < N; ++i) {
    int S;
    if (scanf("%d %d", &S, &nt[i]) != 2) return 1;
    cost[i].resize(S);
    for (int s = 0; s < S; ++s)
      if (scanf("%lf", &cost[i][s]) != 1) return 1;
  }
  std::vector<int32_t> o = qtm::multi_schedule(cost, nt, P);
  for (size_t k = 0; k < o.size(); k += 4) printf("%d %d %d\n", o[k], o[k + 1], o[k + 2]);
  return 0;
}
"""


@pytest.fixture(scope="module")
def sched_bin():
    d = tempfile.mkdtemp(prefix="qtm_sched_")
    src = os.path.join(d, "driver.cpp")
    with open(src, "w") as f:
        f.write(DRIVER)
    exe = os.path.join(d, "driver")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", CSRC, src,
                    os.path.join(CSRC, "schedule.cpp"), "-o", exe], check=True)
    return exe


def run(exe, items, P):
    lines = [f"{len(items)} {P}"]
    for costs, T in items:
        lines.append(f"{len(costs)} {T} " + " ".join(repr(float(c)) for c in costs))
    out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                         check=True).stdout
    return [tuple(map(int, l.split())) for l in out.strip().splitlines()] if out.strip() else []


def check_valid(order, items):
    want = {(i, s, t) for i, (c, T) in enumerate(items) for s in range(len(c)) for t in range(T)}
    assert len(order) == len(want) and set(order) == want
    seen = {}
    for i, s, t in order:
        if s > 0:
            assert seen.get((i, s - 1), 0) == items[i][1], (i, s, t)
        seen[(i, s)] = seen.get((i, s), 0) + 1


def test_hand_worked_single_worker(sched_bin):
    # item 0: chain of three unit sweeps; item 1: one sweep of cost 2.
    # t=0: chains 3 vs 2 -> item 0; t=1: item 0's remaining chain (2) ties
    # item 1 (2), lower index first; t=2: item 1 (2) beats item 0 (1).
    order = run(sched_bin, [([1, 1, 1], 1), ([2], 1)], P=1)
    assert order == [(0, 0, 0), (0, 1, 0), (1, 0, 0), (0, 2, 0)]


def test_hand_worked_tiles_and_idle_workers(sched_bin):
    # two workers; item 0 has two sweeps of 2 tiles (cost 3 each), item 1 a
    # single sweep of cost 1.  Both workers take item 0's first sweep at t=0;
    # at t=3 item 0's second sweep (remaining chain 3) beats item 1 (1).
    items = [([3, 3], 2), ([1], 1)]
    order = run(sched_bin, items, P=2)
    assert order == [(0, 0, 0), (0, 0, 1), (0, 1, 0), (0, 1, 1), (1, 0, 0)]
    # with a third worker item 1 starts at t=0
    order = run(sched_bin, items, P=3)
    assert order == [(0, 0, 0), (0, 0, 1), (1, 0, 0), (0, 1, 0), (0, 1, 1)]


@pytest.mark.parametrize("seed", range(6))
def test_random_queues_are_valid(sched_bin, seed):
    rng = random.Random(seed)
    items = []
    for _ in range(rng.randint(1, 40)):
        S = rng.randint(1, 8)
        T = rng.choice([1, 1, 2, 4, 16])
        items.append(([rng.uniform(0.5, 10.0) for _ in range(S)], T))
    for P in (1, 3, 64):
        check_valid(run(sched_bin, items, P), items)


def test_longest_chain_first(sched_bin):
    # with enough workers for everything ready at t=0, the queue starts with
    # the first sweeps in decreasing order of their whole chain
    items = [([1.0] * k, 1) for k in (2, 5, 3, 1, 4)]
    order = run(sched_bin, items, P=8)
    assert [i for i, s, t in order[:5]] == [1, 4, 2, 0, 3]
    check_valid(order, items)
