// Internal types shared by the host runtime and the gfx950 kernels. The tile
// list and queue split they consume are described in plan_logic.h.
#pragma once

#include <stdint.h>
#include <hip/hip_runtime.h>

#include "plan_logic.h"

namespace dg {

constexpr int kSupportUV = 8;   // G_uv support per axis (Section 2)
constexpr int kSupportW = 4;    // G_w support (Section 2)
constexpr int kWave = 64;       // CDNA wavefront
constexpr int kBlockThreads = 256;
constexpr int kWavesPerBlock = kBlockThreads / kWave;
// The table-gradient kernel runs one workgroup of eight wavefronts per CU
// (its registers allow two wavefronts per SIMD), so that eight wavefronts
// share one LDS copy of dL/dG_uv and half as many copies are added to the
// output at the end as with two workgroups of four.
constexpr int kTableGradThreads = 512;

// Invalid-offset sentinel for hardware bounds-checked (buffer) loads: any
// offset at or above a resource's size returns zero. Subgrids and tables are
// limited to less than this many bytes.
constexpr uint32_t kOutOfRange = 0x40000000u;

// Everything a kernel needs to know about one problem.
struct Problem {
    const void* subgrids;   // [S][n_v][n_u][n_w] in the grid dtype
    const void* g_uv;       // [os_uv][os_uv][8][8] in the gcf dtype
    const void* g_w;        // [os_w][4] in the gcf dtype
    const double* uvw;      // [N][3]
    void* vis;              // complex float32 [N]: degrid output / adjoint input
    void* grid_out;         // complex float32 [S][n_v][n_u][n_w]: adjoint output
    const uint32_t* perm;   // work order: tile position -> visibility index; nullptr = identity
    int64_t cells_per_sub;  // n_v * n_u * n_w
    int32_t n_v, n_u, n_w;
    int32_t log2_os_uv, log2_os_w;   // log2 of the oversampling, or -1 if not a power of two
    uint32_t guv_bytes;     // size of G_uv in bytes
    uint32_t sub_bytes;     // size of one subgrid in bytes (grid dtype)
    int32_t os_uv, os_w;    // oversampling factors
    int32_t pad_;
    double hi_u, hi_v, hi_w;  // exclusive upper bounds of in-range coordinates
};

// Device control block of a plan or batch: queue cursors (one 128-byte line
// each, so atomics from different XCDs do not share a line), the count of
// finished workgroups, and the out-of-range counters. The last workgroup of
// every launch resets the cursors and the counters, so a launch needs no
// separate reset and can be replayed from a graph. Atomics on one counter
// take about 20 ns apiece when they queue, so with one counter the end of a
// launch whose workgroups all finish together waits on a chain as long as
// the grid. Such a kernel (the adjoint's fix-up pass), on a grid of more than
// kDoneFlat workgroups, counts their ends in two levels: into one of
// kDoneGroups group counters (workgroup b into b mod kDoneGroups), and the
// last of each group into `done`. Other kernels, and small grids, count into
// `done` directly, which saves the second, dependent atomic.
constexpr int kDoneGroups = 8;
constexpr int kDoneFlat = 64;
struct alignas(128) CtlLine { uint32_t v[32]; };
struct Ctl {
    CtlLine cursor[kMaxQueues];
    CtlLine done;
    CtlLine oob;   // v[0..1]: running count (u64), v[2..3]: count of the last launch
    CtlLine group[kDoneGroups];
};

struct LaunchParams {
    Problem prob;               // used when probs == nullptr
    const Problem* probs;       // per-problem table of a batch
    const Tile* tiles;
    const uint32_t* tile_vis;   // [n_tiles][kMaxNb]: visibility index of each work item
    Ctl* ctl;
    QueueSpec q;
    StaticDeal deal;            // filled by launch_degrid for its grid size
    // Residual mode (one problem only; v_obs == nullptr: plain degrid). The
    // output becomes v_obs - degrid and each tile stores the float64 sum of
    // |residual|^2 of its visibilities in tile_loss[t] (summed afterwards by
    // launch_loss_sum).
    const float2* v_obs;
    double* tile_loss;
};

// One output block of the owner-computes adjoint and its visibility list.
struct OwnerBlock {
    int64_t begin;   // first entry in the item list
    int32_t count;   // entries
    int32_t block;   // block index (s * nby + by) * nbx + bx
};
static_assert(sizeof(OwnerBlock) == 16, "OwnerBlock must stay 16 bytes");

constexpr int kOwnerBlock = 16;   // cells per side of an owner-computes output block

struct OwnerParams {
    Problem prob;                  // g_uv, g_w, uvw, vis (input), grid_out
    const OwnerBlock* blocks;
    const uint32_t* items;         // visibility indices per block
    const uint32_t* plan_start;    // first tap (y0 << 16 | x0) per visibility at plan time
    Ctl* ctl;
    QueueSpec q;
    StaticDeal deal;               // filled by launch_grid_owner for its grid size
    int32_t accumulate;            // 1: add to grid_out, 0: overwrite
    int32_t nby, nbx;              // blocks per subgrid along v and u
};

// Table-gradient pass: dL/dG_uv and dL/dG_w from dL/dV over the tiles of a
// plan (prob.vis holds dL/dV, complex float32 [N]).
struct TableGradParams {
    Problem prob;
    const Tile* tiles;
    const uint32_t* tile_vis;
    int64_t n_tiles;
    float* grad_uv;   // [os_uv][os_uv][8][8], or nullptr
    float* grad_w;    // [os_w][4], or nullptr
};

enum GridKind : int32_t { kGridC64 = 0, kGridCBF16 = 1, kGridCF16 = 2 };
enum GcfKind : int32_t { kGcfF32 = 0, kGcfF16 = 1, kGcfBF16 = 2 };

// Kernel launchers (defined in degrid_kernels.hip, grid_kernels.hip and
// table_grad_kernels.hip).
hipError_t launch_degrid(const LaunchParams& p, int grid_kind, int gcf_kind, int variant,
                         int blocks, hipStream_t stream);
hipError_t launch_grid_adjoint(const LaunchParams& p, int gcf_kind, int variant, int blocks,
                               hipStream_t stream);
hipError_t launch_zero(void* ptr, int64_t bytes, hipStream_t stream);
// Index of the degrid kernel variant for subgrids deeper than the w support
// (no staging; one load per w value).
constexpr int kDeepVariant = 5;
// Index of the variant with the lane mapping of the paper's kernel D1 (two
// visibilities per wavefront, lanes over (t_u, t_w), accumulation along v).
constexpr int kD1Variant = 6;
// *loss = sum of tile_loss[0 .. n_tiles) in a fixed order (same bits every time).
hipError_t launch_loss_sum(const double* tile_loss, int64_t n_tiles, double* loss, hipStream_t stream);
// *p = v (one float64 written by a kernel, so that graphs may capture it).
hipError_t launch_set_f64(double* p, double v, hipStream_t stream);
// Owner-computes adjoint: every output block written once from its list.
hipError_t launch_grid_owner(const OwnerParams& p, int gcf_kind, int blocks, hipStream_t stream);
hipError_t owner_kernel_occupancy(int gcf_kind, int* blocks_per_cu);
// Adds, with atomics, the visibilities whose first tap differs from the
// plan's (those the owner pass skipped), and counts out-of-range ones into
// ctl. n_vis visibilities of one problem; vis_offsets on the device.
// At most max_blocks workgroups (each one's end is an atomic on the control
// block, so the grid is kept near the device's resident capacity).
hipError_t launch_grid_fixup(const Problem& pr, const int64_t* vis_offsets, int64_t n_sub, int64_t n_vis,
                             const uint32_t* plan_start, Ctl* ctl, int gcf_kind, int max_blocks,
                             hipStream_t stream);
// tile_vis[t * kMaxNb + j] = visibility index of item j of tile t: through
// perms[tile.problem] (a work-order permutation, or nullptr for input order)
// at position tile.begin + j; items past the tile's count repeat its first.
hipError_t launch_expand_tiles(const Tile* tiles, int64_t n_tiles, const uint32_t* const* perms,
                               uint32_t* tile_vis, hipStream_t stream);
// start[p] = first tap (y0 << 16 | x0) of the visibility at work position p
// (through pr.perm), or kNoStart when out of range.
hipError_t launch_start_cells(const Problem& pr, int64_t n, uint32_t* start, hipStream_t stream);

// Stable sort of each subgrid's visibilities by the Hilbert-curve position of
// the cell holding (u, v) (defined in plan_sort.hip). Writes perm[n_vis]: the
// visibility index at each position of the new work order. Allocates and
// frees its own temporary buffers; synchronises 'stream'.
hipError_t sort_visibilities(const double* uvw, const int64_t* offsets_host, int64_t n_sub,
                             uint32_t* perm, hipStream_t stream);
hipError_t degrid_kernel_occupancy(int grid_kind, int gcf_kind, int variant, int* blocks_per_cu);
hipError_t adjoint_kernel_occupancy(int gcf_kind, int variant, int* blocks_per_cu);
int degrid_variant_count();
int adjoint_variant_count();
int degrid_variant_box_bytes(int variant);   // LDS staging bytes per wavefront (0: none)
int degrid_variant_max_nb(int variant);      // largest tile the variant accepts
bool degrid_variant_any_depth(int variant);  // reads subgrids with n_w > 4 (one load per w value)
constexpr int kMaxVariants = 8;
// Adds dL/dG_uv and dL/dG_w of every in-range visibility to p.grad_uv and
// p.grad_w (float atomics). deep: subgrids with more w planes than the support.
// max_lds: the device's LDS bytes per workgroup.
hipError_t launch_table_grad(const TableGradParams& p, int grid_kind, int gcf_kind, bool deep, int blocks,
                             size_t max_lds, hipStream_t stream);
// Dynamic LDS bytes of that kernel, and whether it accumulates dL/dG_uv in LDS.
void table_grad_shape(int os_uv, int os_w, bool want_uv, bool want_w, size_t max_lds, bool* lds_uv,
                      size_t* lds_bytes);
// p[0 .. n) = 0.0f (a kernel, so that graphs may capture it).
hipError_t launch_zero_f32(float* p, int64_t n, hipStream_t stream);

// Degridding without a plan (defined in noalloc.hip): its scratch is a
// file-scope device array of kNoAllocBytes per GPU (tile cursor and count,
// the staged offsets and the tile offsets of at most kNoAllocMaxSubgrids
// subgrids). Input-order tiles of nb visibilities; n_tiles = sum over
// subgrids of ceil(N_s / nb). offsets_host [n_sub + 1] is copied into the
// scratch on 'stream'. oob_out (device, may be null) receives the launch's
// out-of-range count. Allocates nothing.
constexpr int64_t kNoAllocMaxSubgrids = 16384;
constexpr size_t kNoAllocBytes = 262656;   // 256 + 2 * 8 * (kNoAllocMaxSubgrids + 1), rounded up to 256
hipError_t launch_degrid_noalloc(const Problem& pr, int grid_kind, int gcf_kind, bool deep,
                                 const int64_t* offsets_host, int64_t n_sub, int nb, int64_t n_tiles,
                                 unsigned long long* oob_out, hipStream_t stream);

}  // namespace dg
