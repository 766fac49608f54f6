// Property checks of the host work decomposition, built with g++ (no HIP).
// Prints one JSON object per case; the pytest wrapper checks the properties.
#include "plan_logic.h"

#include <cstdio>
#include <cstdlib>
#include <vector>

int main(int argc, char** argv) {
    // argv: nb followed by per-subgrid counts
    if (argc < 2) return 2;
    const int nb = std::atoi(argv[1]);
    std::vector<int64_t> off(1, 0);
    for (int i = 2; i < argc; ++i) off.push_back(off.back() + std::atoll(argv[i]));
    const int64_t n_sub = (int64_t)off.size() - 1;
    std::vector<dg::Tile> tiles = dg::build_tiles(n_sub, off.data(), nb, 3);
    dg::QueueSpec q = dg::split_queues(tiles);
    std::printf("{\"tiles\": [");
    for (size_t i = 0; i < tiles.size(); ++i)
        std::printf("%s[%lld, %d, %d, %d]", i ? ", " : "", (long long)tiles[i].begin, tiles[i].sub,
                    tiles[i].count, tiles[i].problem);
    std::printf("], \"n_queues\": %d, \"begin\": [", q.n_queues);
    for (int i = 0; i < q.n_queues; ++i) std::printf("%s%d", i ? ", " : "", q.begin[i]);
    std::printf("], \"end\": [");
    for (int i = 0; i < q.n_queues; ++i) std::printf("%s%d", i ? ", " : "", q.end[i]);
    std::printf("]}\n");
    return 0;
}
