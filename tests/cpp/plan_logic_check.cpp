// Property checks of the host work decomposition, built with g++ (no HIP).
// Prints the tiles and queues as JSON; the pytest wrapper checks properties.
//   plan_logic_check <nb> <count>...                    fixed-size tiles
//   plan_logic_check fitted <nb> <cap> <min_fit> <pad_to> <file> tiles cut to fit a box;
//       <file>: line 1 = per-subgrid counts, line 2 = start word per visibility
//   plan_logic_check deal <nb> <blocks> <count>...       static deal of a launch
//   plan_logic_check blocks <n_v> <n_u> <block> <file> output-block lists;
//       <file>: counts, start words, visibility index per work position
#include "plan_logic.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

static void print(const std::vector<dg::Tile>& tiles) {
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
}

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    if (std::strcmp(argv[1], "deal") == 0) {
        // deal <nb> <blocks> <count>...: queues of fixed-size tiles and the
        // static deal of a launch of <blocks> workgroups
        if (argc < 4) return 2;
        const int nb = std::atoi(argv[2]), blocks = std::atoi(argv[3]);
        std::vector<int64_t> off(1, 0);
        for (int i = 4; i < argc; ++i) off.push_back(off.back() + std::atoll(argv[i]));
        const auto tiles = dg::build_tiles((int64_t)off.size() - 1, off.data(), nb, 0);
        const dg::QueueSpec q = dg::split_queues(tiles);
        const dg::StaticDeal d = dg::deal_static(q, blocks, 4);
        std::printf("{\"n_queues\": %d, \"on\": %d, \"all_static\": %d, \"begin\": [", q.n_queues, d.on,
                    d.all_static);
        for (int i = 0; i < q.n_queues; ++i) std::printf("%s%d", i ? ", " : "", q.begin[i]);
        std::printf("], \"end\": [");
        for (int i = 0; i < q.n_queues; ++i) std::printf("%s%d", i ? ", " : "", q.end[i]);
        std::printf("], \"sbase\": [");
        for (int i = 0; i < q.n_queues; ++i) std::printf("%s%d", i ? ", " : "", d.sbase[i]);
        std::printf("], \"stride\": [");
        for (int i = 0; i < q.n_queues; ++i) std::printf("%s%d", i ? ", " : "", d.stride[i]);
        std::printf("]}\n");
        return 0;
    }
    if (std::strcmp(argv[1], "blocks") == 0) {
        if (argc != 6) return 2;
        const int n_v = std::atoi(argv[2]), n_u = std::atoi(argv[3]), block = std::atoi(argv[4]);
        std::ifstream f(argv[5]);
        std::string l1, l2, l3;
        std::getline(f, l1);
        std::getline(f, l2);
        std::getline(f, l3);
        std::vector<int64_t> off(1, 0);
        std::istringstream c(l1), st(l2), vs(l3);
        long long x;
        while (c >> x) off.push_back(off.back() + x);
        std::vector<uint32_t> start, vis;
        unsigned long long w;
        while (st >> w) start.push_back((uint32_t)w);
        while (vs >> w) vis.push_back((uint32_t)w);
        if ((int64_t)start.size() != off.back() || vis.size() != start.size()) return 3;
        dg::BlockLists bl = dg::build_block_lists((int64_t)off.size() - 1, off.data(), vis.data(), start.data(),
                                                  n_v, n_u, block, 8);
        std::printf("{\"offsets\": [");
        for (size_t i = 0; i < bl.offsets.size(); ++i) std::printf("%s%lld", i ? ", " : "", (long long)bl.offsets[i]);
        std::printf("], \"items\": [");
        for (size_t i = 0; i < bl.items.size(); ++i) std::printf("%s%u", i ? ", " : "", bl.items[i]);
        std::printf("]}\n");
        return 0;
    }
    if (std::strcmp(argv[1], "fitted") == 0) {
        if (argc != 7) return 2;
        const int nb = std::atoi(argv[2]);
        const long long cap = std::atoll(argv[3]);
        const int min_fit = std::atoi(argv[4]);
        const int pad_to = std::atoi(argv[5]);
        std::ifstream f(argv[6]);
        std::string l1, l2;
        std::getline(f, l1);
        std::getline(f, l2);
        std::vector<int64_t> off(1, 0);
        std::istringstream c(l1), st(l2);
        long long x;
        while (c >> x) off.push_back(off.back() + x);
        std::vector<uint32_t> start;
        unsigned long long w;
        while (st >> w) start.push_back((uint32_t)w);
        if ((int64_t)start.size() != off.back()) return 3;
        print(dg::build_tiles_fitted((int64_t)off.size() - 1, off.data(), start.data(), nb, 8, cap, min_fit, 3,
                                     pad_to));
        return 0;
    }
    const int nb = std::atoi(argv[1]);
    std::vector<int64_t> off(1, 0);
    for (int i = 2; i < argc; ++i) off.push_back(off.back() + std::atoll(argv[i]));
    print(dg::build_tiles((int64_t)off.size() - 1, off.data(), nb, 3));
    return 0;
}
