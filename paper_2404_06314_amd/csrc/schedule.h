// Queue order of the persistent uneven-batch kernels (host only, no HIP).
#pragma once

#include <cstdint>
#include <vector>

namespace qtm {

// List schedule of sweep chains on P identical workers.  Item i has
// cost[i].size() sweeps of ntiles[i] tiles each; cost[i][s] is the time of
// one tile of sweep s.  The tiles of sweep s + 1 become ready when every tile
// of sweep s has finished; among ready sweeps the one with the longest
// remaining chain (sum of the remaining sweep costs) goes first, ties by item
// index.  Returns [item, sweep, tile, 0] per tile in the order the tiles are
// handed out, which is the queue order: every tile comes after all tiles of
// the previous sweep of its item.
std::vector<int32_t> multi_schedule(const std::vector<std::vector<double>> &cost,
                                    const std::vector<int> &ntiles, int P);

}  // namespace qtm
