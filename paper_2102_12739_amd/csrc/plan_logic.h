// Host-side work decomposition (plain C++, no HIP): the tile list and its
// split into per-XCD queues. Kept free of HIP so that it can be built and
// tested on a machine without a GPU.
//
// Section 2 of the paper gives each thread block N_b visibilities of one
// subgrid and launches max_S(N_vis,S / N_b) x S blocks (Eq. (1)); with uneven
// counts most of those blocks find no work. Here the same N_b-visibility
// tiles form one list that a persistent launch drains.
#pragma once

#include <stdint.h>

#include <vector>

namespace dg {

constexpr int kMaxQueues = 8;   // one tile queue per XCD of an MI355X
constexpr int kMaxNb = 64;      // a tile fits one wavefront's coordinate stage

// One work item: up to n_b consecutive visibilities of one subgrid.
struct Tile {
    int64_t begin;     // first visibility (row of uvw and of the output)
    int32_t sub;       // subgrid index inside its problem
    uint16_t count;    // visibilities in the tile, 1..kMaxNb
    uint16_t problem;  // problem index inside a batch (0 for a single plan)
};
static_assert(sizeof(Tile) == 16, "Tile must stay 16 bytes");

struct QueueSpec {
    int32_t n_queues;
    int32_t begin[kMaxQueues];  // first tile of queue q
    int32_t end[kMaxQueues];    // one past the last tile of queue q
};

// Cut the visibilities of each of n_sub subgrids (CSR offsets off[0..n_sub])
// into tiles of at most nb consecutive visibilities, in subgrid order.
std::vector<Tile> build_tiles(int64_t n_sub, const int64_t* off, int nb, uint16_t problem);

// Marker of a visibility whose neighbourhood leaves its subgrid.
constexpr uint32_t kNoStart = 0xFFFFFFFFu;

// Like build_tiles, but cut where a tile's cells stop fitting a staging box:
// start[p] is the first tap (y0 << 16 | x0) of the visibility at position p
// of the work order, or kNoStart. A tile grows while the bounding box of its
// neighbourhoods ((x1 - x0 + W) x (y1 - y0 + W) cells, W = support) holds at
// most cap_cells cells and it has fewer than nb visibilities. If fewer than
// min_fit visibilities fit, the tile takes nb visibilities anyway (it will
// be gathered without staging) so that sparse regions do not become many
// tiny tiles. Out-of-range visibilities never enlarge a box. pad_to (0 or a
// power of two) pads the box width to the next value congruent to pad_to / 2
// modulo pad_to, as the staging copy in LDS does.
std::vector<Tile> build_tiles_fitted(int64_t n_sub, const int64_t* off, const uint32_t* start, int nb,
                                     int support, int64_t cap_cells, int min_fit, uint16_t problem,
                                     int pad_to = 0);

// Output blocks of the owner-computes adjoint: block b of subgrid s covers
// cells [by * B, by * B + B) x [bx * B, bx * B + B) (b = (s * nby + by) * nbx + bx,
// nby = n_v / B, nbx = n_u / B). items[offsets[b] .. offsets[b+1]) are the
// visibilities whose W x W neighbourhood overlaps the block: first tap
// (x0, y0) with x0 in [bx * B - W + 1, bx * B + B - 1], likewise y0.
// vis_of[p] is the visibility at work position p, start[p] its first tap
// (y0 << 16 | x0) or kNoStart (never listed). Within a block, items keep
// work order.
struct BlockLists {
    std::vector<int64_t> offsets;   // [n_blocks + 1]
    std::vector<uint32_t> items;    // visibility indices
};
BlockLists build_block_lists(int64_t n_sub, const int64_t* off, const uint32_t* vis_of, const uint32_t* start,
                             int n_v, int n_u, int block, int support);

// Split a tile list into up to kMaxQueues contiguous queues holding about
// equal numbers of visibilities (empty queues only when there are fewer
// tiles than queues).
QueueSpec split_queues(const std::vector<Tile>& tiles);

// The same split for work items of the given weights.
QueueSpec split_queues_weighted(const std::vector<int64_t>& weights);

// Static deal of a persistent launch over queues q: workgroup b serves queue
// b mod n_queues, and wavefront r of the workgroups serving a queue takes
// its tiles begin + r, begin + r + stride, ... below sbase without an atomic;
// tiles from sbase on go through the queue's cursor. A queue gets a static
// part (kStaticEighths / 8 of its tiles) only when it holds at least
// kMinTilesPerWave tiles per serving wavefront; otherwise sbase = begin.
// When no queue holds more tiles than wavefronts serve it, every tile is
// dealt statically (sbase = end, all_static = 1): each wavefront takes at
// most one tile, with no cursor atomic and no stealing.
constexpr int kStaticEighths = 6;
constexpr int kMinTilesPerWave = 4;

struct StaticDeal {
    int32_t on;                   // 1 when some queue has a static part
    int32_t all_static;           // 1 when every tile is dealt statically
    int32_t sbase[kMaxQueues];    // first tile of queue q handed out by its cursor
    int32_t stride[kMaxQueues];   // wavefronts serving queue q
};

StaticDeal deal_static(const QueueSpec& q, int blocks, int waves_per_block);

}  // namespace dg
