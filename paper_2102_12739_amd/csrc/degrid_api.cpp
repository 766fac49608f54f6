// Host runtime of the degridding library: the C ABI declared in degrid.h.
//
// Plans validate the problem descriptor and the CSR visibility offsets, cut
// every subgrid's visibility list into tiles of n_b (Section 2: a block
// processes N_b visibilities of one subgrid), split the tile list into one
// contiguous queue per XCD balanced by visibility count, and own the device
// scratch (tile list and control block). Execute calls only fill the launch
// parameters and launch, so they allocate nothing.
#include "degrid.h"
#include "dg_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

using namespace dg;

namespace {

thread_local std::string g_last_error;

dg_status fail(dg_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

dg_status hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? DG_ERR_NOMEM : DG_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool fault_injected(const char* what) {
    const char* f = std::getenv("DG_FAULT_INJECT");
    return f && std::strcmp(f, what) == 0;
}

int log2_exact(int32_t x) {
    if (x < 1 || (x & (x - 1)) != 0) return -1;
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

uint32_t grid_elem_bytes(int32_t grid_dtype) { return grid_dtype == DG_GRID_C64 ? 8u : 4u; }
uint32_t gcf_elem_bytes(int32_t gcf_dtype) { return gcf_dtype == DG_GCF_F32 ? 4u : 2u; }

dg_status validate_desc(const dg_desc* d) {
    if (!d) return fail(DG_ERR_INVALID_ARG, "descriptor is NULL");
    if (d->flags != 0) return fail(DG_ERR_INVALID_ARG, "flags must be 0 (got %u)", d->flags);
    if (d->support_uv != kSupportUV || d->support_w != kSupportW)
        return fail(d->support_uv > 0 && d->support_w > 0 ? DG_ERR_UNSUPPORTED : DG_ERR_INVALID_ARG,
                    "supports must be 8 (uv) and 4 (w), got %d and %d", d->support_uv, d->support_w);
    if (d->n_v < kSupportUV || d->n_u < kSupportUV || d->n_w < kSupportW)
        return fail(DG_ERR_INVALID_ARG, "subgrid %dx%dx%d is smaller than the support", d->n_v, d->n_u, d->n_w);
    if (d->os_uv < 1 || d->os_uv > 64 || d->os_w < 1 || d->os_w > 64)
        return fail(DG_ERR_INVALID_ARG, "oversampling must be in [1, 64], got %d and %d", d->os_uv, d->os_w);
    if (d->grid_dtype < DG_GRID_C64 || d->grid_dtype > DG_GRID_CF16)
        return fail(DG_ERR_INVALID_ARG, "unknown grid dtype %d", d->grid_dtype);
    if (d->gcf_dtype < DG_GCF_F32 || d->gcf_dtype > DG_GCF_BF16)
        return fail(DG_ERR_INVALID_ARG, "unknown gcf dtype %d", d->gcf_dtype);
    if (d->n_b < 0 || d->n_b > kMaxNb)
        return fail(DG_ERR_INVALID_ARG, "n_b must be in [0, %d], got %d", kMaxNb, d->n_b);
    const double cells = (double)d->n_v * d->n_u * d->n_w;
    if (cells * 8.0 >= (double)kOutOfRange)
        return fail(DG_ERR_UNSUPPORTED, "one subgrid must be smaller than %u bytes", kOutOfRange);
    // First taps travel packed as (y0 << 16 | x0) in the work-order and
    // owner-computes plans, with 0xFFFFFFFF marking "out of range": x0 must
    // fit 16 bits and y0 must stay below 0xFFFF.
    if (d->n_u - kSupportUV > 0xFFFF || d->n_v - kSupportUV > 0xFFFE)
        return fail(DG_ERR_UNSUPPORTED, "subgrid sides must be at most %d (u) and %d (v), got %d and %d",
                    0xFFFF + kSupportUV, 0xFFFE + kSupportUV, d->n_u, d->n_v);
    return DG_OK;
}

dg_status validate_offsets(int64_t n_sub, const int64_t* off) {
    if (n_sub < 0) return fail(DG_ERR_INVALID_ARG, "n_subgrids is negative");
    if (n_sub > 0x7FFFFFFF) return fail(DG_ERR_UNSUPPORTED, "too many subgrids");
    if (!off) return fail(DG_ERR_INVALID_ARG, "vis_offsets is NULL");
    if (off[0] != 0) return fail(DG_ERR_INVALID_ARG, "vis_offsets[0] must be 0");
    for (int64_t s = 0; s < n_sub; ++s)
        if (off[s + 1] < off[s])
            return fail(DG_ERR_INVALID_ARG, "vis_offsets must be non-decreasing (at %lld)", (long long)s);
    // visibility indices of work items and work orders are 32-bit
    if (off[n_sub] > (int64_t)0xFFFFFFFF)
        return fail(DG_ERR_UNSUPPORTED, "at most 2^32 - 1 visibilities per plan, got %lld", (long long)off[n_sub]);
    return DG_OK;
}

struct DeviceScratch {
    Tile* tiles = nullptr;
    uint32_t* tile_vis = nullptr;           // [n_tiles][kMaxNb]
    const uint32_t** perm_table = nullptr;  // per problem: work-order permutation or nullptr
    double* tile_loss = nullptr;            // [n_tiles]: per-tile sums of the residual mode
    Ctl* ctl = nullptr;
    int64_t n_tiles = 0;
    int32_t n_problems = 0;
};

void free_tiles(DeviceScratch& ds) {
    if (ds.tiles) (void)hipFree(ds.tiles);
    if (ds.tile_vis) (void)hipFree(ds.tile_vis);
    if (ds.perm_table) (void)hipFree(ds.perm_table);
    if (ds.tile_loss) (void)hipFree(ds.tile_loss);
    ds.tile_loss = nullptr;
    ds.tiles = nullptr;
    ds.tile_vis = nullptr;
    ds.perm_table = nullptr;
    ds.n_tiles = 0;
}

// Uploads the tile list and expands it into per-item visibility indices
// (through each problem's permutation). Allocates; synchronises 'stream'.
dg_status alloc_scratch(DeviceScratch& ds, const std::vector<Tile>& tiles,
                        const std::vector<const uint32_t*>& perms, hipStream_t stream) {
    if (fault_injected("alloc")) return fail(DG_ERR_NOMEM, "allocation failure injected (DG_FAULT_INJECT=alloc)");
    hipError_t e;
    if (!ds.ctl) {
        e = hipMalloc(&ds.ctl, sizeof(Ctl));
        if (e != hipSuccess) { ds.ctl = nullptr; return hip_fail(e, "hipMalloc(control block)"); }
        e = hipMemsetAsync(ds.ctl, 0, sizeof(Ctl), stream);
        if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync(control block)");
    }
    (void)hipStreamSynchronize(stream);
    free_tiles(ds);
    ds.n_tiles = (int64_t)tiles.size();
    ds.n_problems = (int32_t)perms.size();
    if (!tiles.empty()) {
        e = hipMalloc(&ds.tiles, tiles.size() * sizeof(Tile));
        if (e != hipSuccess) { ds.tiles = nullptr; return hip_fail(e, "hipMalloc(tile list)"); }
        e = hipMalloc(&ds.tile_vis, tiles.size() * kMaxNb * sizeof(uint32_t));
        if (e != hipSuccess) { ds.tile_vis = nullptr; return hip_fail(e, "hipMalloc(tile items)"); }
        e = hipMalloc(&ds.perm_table, perms.size() * sizeof(const uint32_t*));
        if (e != hipSuccess) { ds.perm_table = nullptr; return hip_fail(e, "hipMalloc(permutation table)"); }
        e = hipMalloc(&ds.tile_loss, tiles.size() * sizeof(double));
        if (e != hipSuccess) { ds.tile_loss = nullptr; return hip_fail(e, "hipMalloc(tile sums)"); }
        e = hipMemcpyAsync(ds.tiles, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ds.perm_table, perms.data(), perms.size() * sizeof(const uint32_t*),
                               hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = launch_expand_tiles(ds.tiles, ds.n_tiles, ds.perm_table, ds.tile_vis, stream);
        if (e != hipSuccess) return hip_fail(e, "uploading the tile list");
    }
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(plan upload)");
    return DG_OK;
}

void free_scratch(DeviceScratch& ds) {
    free_tiles(ds);
    if (ds.ctl) (void)hipFree(ds.ctl);
    ds = DeviceScratch{};
}

}  // namespace

struct dg_plan_ {
    dg_desc desc{};
    int64_t n_sub = 0;
    std::vector<int64_t> offsets;
    int32_t n_b_req = 0;                   // requested tile size
    int32_t n_b = 0;                       // tile size used (at most the variant's limit)
    int32_t variant = 0;
    std::vector<Tile> tiles;               // host copy of the tile list
    int32_t blocks = 0;                    // persistent grid of the degrid kernel
    int32_t blocks_adj = 0;                // persistent grid of the adjoint kernel
    int32_t cap[kMaxVariants] = {};        // resident workgroups per degrid variant
    int32_t cap_adj[kMaxVariants] = {};    // resident workgroups per adjoint variant
    int32_t device = 0;
    int32_t n_cu = 0;
    int32_t grid_div = 1;                  // persistent grid: resident workgroups / grid_div
    std::string device_key;                // architecture and CU count, for the tuning cache
    QueueSpec q{};
    DeviceScratch ds;
    hipStream_t last_stream = nullptr;
    bool launched = false;
    uint32_t* d_perm = nullptr;   // work order from degrid_plan_sort (nullptr: input order)
    std::vector<uint32_t> start;  // first tap per work position (from degrid_plan_sort)
    uint64_t version = 0;         // bumped when tiles or work order change
    // owner-computes adjoint (built by degrid_plan_sort)
    OwnerBlock* d_own_blocks = nullptr;
    uint32_t* d_own_items = nullptr;
    uint32_t* d_plan_start = nullptr;   // first tap per visibility index at sort time
    int64_t* d_offsets = nullptr;
    Ctl* d_own_ctl = nullptr;
    QueueSpec own_q{};
    int32_t own_grid = 0;
    int32_t nby = 0, nbx = 0;
};

namespace {

void free_owner(dg_plan_* p) {
    if (p->d_own_blocks) (void)hipFree(p->d_own_blocks);
    if (p->d_own_items) (void)hipFree(p->d_own_items);
    if (p->d_plan_start) (void)hipFree(p->d_plan_start);
    if (p->d_offsets) (void)hipFree(p->d_offsets);
    if (p->d_own_ctl) (void)hipFree(p->d_own_ctl);
    p->d_own_blocks = nullptr;
    p->d_own_items = nullptr;
    p->d_plan_start = nullptr;
    p->d_offsets = nullptr;
    p->d_own_ctl = nullptr;
    p->own_grid = 0;
}

}  // namespace

struct dg_batch_ {
    std::vector<dg_plan> plans;
    int32_t variant = 0;                 // kernel of the batch launch
    std::vector<uint64_t> plan_versions;
    int32_t grid_dtype = 0, gcf_dtype = 0;
    int32_t device = 0;
    int32_t blocks = 0;
    QueueSpec q{};
    DeviceScratch ds;
    Problem* d_probs = nullptr;
    Problem* h_probs = nullptr;     // pinned staging for argument uploads
    hipEvent_t upload_done = nullptr;
    bool uploaded = false;
    std::vector<const void*> last_args;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t last_stream = nullptr;
    bool launched = false;
};

namespace {

// Alignment of the device pointers: every element naturally aligned, and
// the G_w table on a 4-byte boundary, because its rows are read as whole
// dwords through the scalar cache. Null pointers are not checked here.
dg_status check_alignment(const dg_desc& d, const void* subgrids, const void* g_uv, const void* g_w,
                          const void* uvw, const void* vis, const void* v_obs, const void* grid_out) {
    struct Need {
        const void* ptr;
        uintptr_t align;
        const char* name;
    };
    const Need need[] = {
        {subgrids, grid_elem_bytes(d.grid_dtype), "subgrids"},
        {g_uv, gcf_elem_bytes(d.gcf_dtype), "g_uv"},
        {g_w, 4, "g_w"},
        {uvw, 8, "uvw"},
        {vis, 8, "the visibility array"},
        {v_obs, 8, "v_obs"},
        {grid_out, 8, "subgrids_out"},
    };
    for (const Need& n : need)
        if (n.ptr && reinterpret_cast<uintptr_t>(n.ptr) % n.align != 0)
            return fail(DG_ERR_INVALID_ARG, "%s must be %u-byte aligned", n.name, (unsigned)n.align);
    return DG_OK;
}

Problem problem_of_desc(const dg_desc& d, const uint32_t* perm, const void* subgrids, const void* g_uv,
                        const void* g_w, const double* uvw, void* vis, void* grid_out) {
    Problem pr{};
    pr.subgrids = subgrids;
    pr.g_uv = g_uv;
    pr.g_w = g_w;
    pr.uvw = uvw;
    pr.vis = vis;
    pr.grid_out = grid_out;
    pr.perm = perm;
    pr.cells_per_sub = (int64_t)d.n_v * d.n_u * d.n_w;
    pr.n_v = d.n_v;
    pr.n_u = d.n_u;
    pr.n_w = d.n_w;
    pr.log2_os_uv = log2_exact(d.os_uv);
    pr.log2_os_w = log2_exact(d.os_w);
    pr.os_uv = d.os_uv;
    pr.os_w = d.os_w;
    pr.guv_bytes = (uint32_t)d.os_uv * d.os_uv * kSupportUV * kSupportUV * gcf_elem_bytes(d.gcf_dtype);
    pr.sub_bytes = (uint32_t)(pr.cells_per_sub * grid_elem_bytes(d.grid_dtype));
    // in range: first tap >= 0 and last tap < n along each axis
    pr.hi_u = (double)(d.n_u - kSupportUV / 2);
    pr.hi_v = (double)(d.n_v - kSupportUV / 2);
    pr.hi_w = (double)(d.n_w - kSupportW / 2);
    return pr;
}

Problem problem_of(const dg_plan_* p, const void* subgrids, const void* g_uv, const void* g_w,
                   const double* uvw, void* vis, void* grid_out) {
    return problem_of_desc(p->desc, p->d_perm, subgrids, g_uv, g_w, uvw, vis, grid_out);
}

// Workgroups for a persistent launch over n_tiles tiles: enough to fill the
// device, never more than there are tiles for their wavefronts.
int32_t blocks_for(int32_t cap, int64_t n_tiles) {
    const int64_t useful = (n_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(cap, useful));
}

// Resident workgroups on the whole device for every degrid variant and for
// the adjoint kernel (CU count x occupancy).
dg_status device_capacity(dg_plan_* p) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    int n_cu = 0;
    e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute(CU count)");
    for (int v = 0; v < degrid_variant_count(); ++v) {
        int occ = 0;
        e = degrid_kernel_occupancy(p->desc.grid_dtype, p->desc.gcf_dtype, v, &occ);
        if (e != hipSuccess) return hip_fail(e, "occupancy query (degrid)");
        p->cap[v] = std::max(1, n_cu * std::max(1, occ));
    }
    for (int v = 0; v < adjoint_variant_count(); ++v) {
        int adj = 0;
        e = adjoint_kernel_occupancy(p->desc.gcf_dtype, v, &adj);
        if (e != hipSuccess) return hip_fail(e, "occupancy query (adjoint)");
        p->cap_adj[v] = std::max(1, n_cu * std::max(1, adj));
    }
    p->device = dev;
    p->n_cu = n_cu;
    hipDeviceProp_t prop{};
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    std::string arch(prop.gcnArchName);
    for (char& c : arch)
        if (c == ':' || c == ' ' || c == '\t') c = '-';
    p->device_key = arch + "_" + std::to_string(n_cu) + "cu";
    return DG_OK;
}

std::string tune_key(const dg_plan_* p) {
    std::ostringstream k;
    int64_t n = p->offsets.back();
    int lg = 0;
    while ((int64_t(1) << (lg + 1)) <= std::max<int64_t>(1, n)) ++lg;
    k << p->device_key << "_grid" << p->desc.grid_dtype << "_gcf" << p->desc.gcf_dtype << "_os" << p->desc.os_uv
      << "x" << p->desc.os_w << "_nw" << p->desc.n_w << "_S" << p->n_sub << "_log2N" << lg;
    return k.str();
}

// On-disk tuning cache (DG_TUNE_CACHE): one line per choice, "key n_b
// variant grid_div"; the key names the device (architecture and CU count)
// and the problem's shape class, so a choice is reused only on the device
// type it was timed on. The last line for a key wins.
bool tune_cache_lookup(const std::string& key, int32_t* n_b, int32_t* variant, int32_t* grid_div) {
    const char* path = std::getenv("DG_TUNE_CACHE");
    if (!path) return false;
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        std::istringstream ls(line);
        std::string k;
        int nb = 0, var = 0, div = 1;
        if (ls >> k >> nb >> var && k == key && nb >= 1 && nb <= kMaxNb && var >= 0 &&
            var < degrid_variant_count()) {
            if (!(ls >> div) || div < 1 || div > 2) div = 1;
            *n_b = nb;
            *variant = var;
            *grid_div = div;
            found = true;
        }
    }
    return found;
}

void tune_cache_store(const std::string& key, int32_t n_b, int32_t variant, int32_t grid_div) {
    const char* path = std::getenv("DG_TUNE_CACHE");
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    f << key << " " << n_b << " " << variant << " " << grid_div << "\n";
}

// Default tile size and kernel variant when neither the caller nor the tuning
// cache fixes them: complex float32 stages tiles in 18 KiB LDS boxes; the
// 16-bit storage types gather through the caches (their cells are half as
// wide, and the staging copy costs more than it saves).
constexpr int32_t kDefaultNb = 64;
// Occupancy settings the tuners try: the persistent grid holds every
// resident workgroup (1) or half of them (2).
constexpr int32_t kGridDivs[] = {1, 2};

// Tile size when neither the caller nor the tuning cache chooses: 64, unless
// the plan is so small that tiles of 64 would leave most of the device's
// resident wavefronts without work (fewer than 16 visibilities per resident
// wavefront); then smaller tiles (a multiple of 8, at least 8), about four
// wavefronts' worth of visibilities each, so that more wavefronts share the
// launch and each one's chain of dependent loads is shorter.
int32_t default_nb(int64_t n_vis, int64_t resident_waves) {
    if (resident_waves <= 0 || n_vis >= 16 * resident_waves) return kDefaultNb;
    const int64_t per = (4 * n_vis + resident_waves - 1) / resident_waves;
    return (int32_t)std::min<int64_t>(kDefaultNb, std::max<int64_t>(8, (per + 7) / 8 * 8));
}
int32_t default_variant(const dg_desc& d) { return d.grid_dtype == DG_GRID_C64 ? 4 : 0; }
// Plans with at most two resident wavefronts' worth of visibilities (each
// wavefront then takes at most one tile of at most 8) gather through the
// caches whatever the storage type: the staging copy's wait would sit on the
// critical path of the whole launch (2048 line-shaped visibilities: 5.05
// against 5.81 us per launch replayed from a graph).
bool tiny_plan(int64_t n_vis, int64_t resident_waves) { return n_vis <= 2 * resident_waves; }

// Subgrids with more w planes than the w support have taps that start at any
// w: only the deep variant (no staging, one load per w value) reads them.
bool deep_only(const dg_desc& d) { return d.n_w != kSupportW; }
bool variant_allowed(const dg_desc& d, int v) { return !deep_only(d) || degrid_variant_any_depth(v); }

// Smallest tile worth staging when tiles are cut to fit the box.
constexpr int kMinStagedTile = 16;
// The kernels pad LDS box rows to a width congruent to 8 modulo 16 cells.
constexpr int kBoxRowPad = 16;

dg_status rebuild_tiles(dg_plan_* p, int32_t n_b_req, hipStream_t stream) {
    const int box = degrid_variant_box_bytes(p->variant);
    const int32_t n_b = std::min<int32_t>(n_b_req, degrid_variant_max_nb(p->variant));
    int64_t plain_tiles = 0;   // tiles of n_b visibilities, before building any
    for (int64_t s = 0; s < p->n_sub; ++s) plain_tiles += (p->offsets[s + 1] - p->offsets[s] + n_b - 1) / n_b;
    if (plain_tiles > 0x7FFFFFFF)
        return fail(DG_ERR_UNSUPPORTED, "%lld tiles: at most 2^31 - 1 per plan (use a larger n_b)",
                    (long long)plain_tiles);
    std::vector<Tile> tiles;
    if (box > 0 && !p->start.empty()) {
        const int64_t cap = box / (int64_t)(grid_elem_bytes(p->desc.grid_dtype) * kSupportW);
        tiles = build_tiles_fitted(p->n_sub, p->offsets.data(), p->start.data(), n_b, kSupportUV, cap,
                                   std::min<int>(kMinStagedTile, n_b), 0, kBoxRowPad);
    } else {
        tiles = build_tiles(p->n_sub, p->offsets.data(), n_b, 0);
    }
    if (tiles.size() > (size_t)0x7FFFFFFF)
        return fail(DG_ERR_UNSUPPORTED, "%zu tiles: at most 2^31 - 1 per plan (use a larger n_b)", tiles.size());
    dg_status s = alloc_scratch(p->ds, tiles, {p->d_perm}, stream);
    if (s != DG_OK) return s;
    p->n_b_req = n_b_req;
    p->n_b = n_b;
    p->version++;
    p->q = split_queues(tiles);
    p->tiles.swap(tiles);
    p->blocks = blocks_for(std::max(1, p->cap[p->variant] / p->grid_div), p->ds.n_tiles);
    p->blocks_adj = blocks_for(p->cap_adj[p->variant], p->ds.n_tiles);
    return DG_OK;
}

LaunchParams params_for(const dg_plan_* p, const Problem& pr) {
    LaunchParams lp{};
    lp.prob = pr;
    lp.probs = nullptr;
    lp.tiles = p->ds.tiles;
    lp.tile_vis = p->ds.tile_vis;
    lp.ctl = p->ds.ctl;
    lp.q = p->q;
    return lp;
}

}  // namespace

// Output-block lists for the owner-computes adjoint, from the sorted order
// and first taps. Subgrid sides must be multiples of the block side.
dg_status build_owner(dg_plan_* p, hipStream_t stream) {
    free_owner(p);
    const dg_desc& d = p->desc;
    if (d.n_v % kOwnerBlock != 0 || d.n_u % kOwnerBlock != 0) return DG_OK;
    const int64_t n = p->offsets.back();
    std::vector<uint32_t> perm((size_t)n);
    hipError_t e = hipMemcpy(perm.data(), p->d_perm, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(work order)");
    std::vector<uint32_t> start_of_vis((size_t)n);
    for (int64_t q = 0; q < n; ++q) start_of_vis[perm[(size_t)q]] = p->start[(size_t)q];
    BlockLists bl = build_block_lists(p->n_sub, p->offsets.data(), perm.data(), p->start.data(), d.n_v, d.n_u,
                                      kOwnerBlock, kSupportUV);
    const int64_t n_blocks = (int64_t)bl.offsets.size() - 1;
    std::vector<OwnerBlock> blocks((size_t)n_blocks);
    std::vector<int64_t> weight((size_t)n_blocks);
    for (int64_t b = 0; b < n_blocks; ++b) {
        const int64_t c = bl.offsets[b + 1] - bl.offsets[b];
        if (c > 0x7FFFFFFF) return fail(DG_ERR_UNSUPPORTED, "too many visibilities on one output block");
        blocks[(size_t)b] = OwnerBlock{bl.offsets[b], (int32_t)c, (int32_t)b};
        weight[(size_t)b] = c + 2 * kOwnerBlock;   // visibilities plus the block's load and store
    }
    auto dev = [&](void** ptr, const void* src, size_t bytes, const char* what) -> dg_status {
        hipError_t err = hipMalloc(ptr, std::max<size_t>(bytes, 16));
        if (err != hipSuccess) { *ptr = nullptr; return hip_fail(err, what); }
        if (bytes > 0) err = hipMemcpyAsync(*ptr, src, bytes, hipMemcpyHostToDevice, stream);
        return err == hipSuccess ? DG_OK : hip_fail(err, what);
    };
    dg_status s = dev((void**)&p->d_own_blocks, blocks.data(), blocks.size() * sizeof(OwnerBlock), "owner blocks");
    if (s == DG_OK) s = dev((void**)&p->d_own_items, bl.items.data(), bl.items.size() * sizeof(uint32_t), "owner items");
    if (s == DG_OK) s = dev((void**)&p->d_plan_start, start_of_vis.data(), start_of_vis.size() * sizeof(uint32_t), "plan start");
    if (s == DG_OK) s = dev((void**)&p->d_offsets, p->offsets.data(), p->offsets.size() * sizeof(int64_t), "offsets");
    if (s == DG_OK) {
        e = hipMalloc(&p->d_own_ctl, sizeof(Ctl));
        if (e == hipSuccess) e = hipMemsetAsync(p->d_own_ctl, 0, sizeof(Ctl), stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) s = hip_fail(e, "owner control block");
    }
    if (s != DG_OK) {
        free_owner(p);
        return s;
    }
    int occ = 0;
    e = owner_kernel_occupancy(d.gcf_dtype, &occ);
    if (e != hipSuccess) { free_owner(p); return hip_fail(e, "occupancy query (owner)"); }
    int n_cu = 0;
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, p->device);
    p->own_q = split_queues_weighted(weight);
    p->own_grid = blocks_for(std::max(1, n_cu * std::max(1, occ)), n_blocks);
    p->nby = d.n_v / kOwnerBlock;
    p->nbx = d.n_u / kOwnerBlock;
    return DG_OK;
}

extern "C" {

dg_status degrid_plan(const dg_desc* d, int64_t n_subgrids, const int64_t* vis_offsets,
                      hipStream_t stream, dg_plan* out) {
    if (!out) return fail(DG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    dg_status s = validate_desc(d);
    if (s != DG_OK) return s;
    s = validate_offsets(n_subgrids, vis_offsets);
    if (s != DG_OK) return s;
    dg_plan_* p = new (std::nothrow) dg_plan_();
    if (!p) return fail(DG_ERR_NOMEM, "host allocation of the plan failed");
    p->desc = *d;
    p->n_sub = n_subgrids;
    p->offsets.assign(vis_offsets, vis_offsets + n_subgrids + 1);
    int32_t n_b = d->n_b, variant = default_variant(*d), grid_div = 1;
    s = device_capacity(p);
    if (s == DG_OK && n_b == 0 && !tune_cache_lookup(tune_key(p), &n_b, &variant, &grid_div)) {
        const int64_t resident = (int64_t)p->cap[variant] * kWavesPerBlock;
        n_b = default_nb(p->offsets.back(), resident);
        if (tiny_plan(p->offsets.back(), resident)) variant = 0;
    }
    p->grid_div = grid_div;
    if (!variant_allowed(*d, variant)) variant = kDeepVariant;
    p->variant = variant;
    if (s == DG_OK) s = rebuild_tiles(p, n_b, stream);
    if (s != DG_OK) {
        free_scratch(p->ds);
        delete p;
        return s;
    }
    *out = p;
    g_last_error.clear();
    return DG_OK;
}

dg_status degrid_execute(dg_plan p, const void* subgrids, const void* g_uv, const void* g_w,
                         const double* uvw, void* vis_out, hipStream_t stream) {
    if (!p) return fail(DG_ERR_INVALID_ARG, "plan is NULL");
    if (p->ds.n_tiles == 0) {   // no visibilities: nothing to write, and nothing out of range
        p->launched = false;
        return DG_OK;
    }
    if (!subgrids || !g_uv || !g_w || !uvw || !vis_out)
        return fail(DG_ERR_INVALID_ARG, "a device pointer is NULL");
    if (dg_status s = check_alignment(p->desc, subgrids, g_uv, g_w, uvw, vis_out, nullptr, nullptr); s != DG_OK)
        return s;
    const Problem pr = problem_of(p, subgrids, g_uv, g_w, uvw, vis_out, nullptr);
    hipError_t e = launch_degrid(params_for(p, pr), p->desc.grid_dtype, p->desc.gcf_dtype, p->variant,
                                 p->blocks, stream);
    if (e != hipSuccess) return hip_fail(e, "degrid kernel launch");
    p->last_stream = stream;
    p->launched = true;
    return DG_OK;
}

dg_status degrid_execute_noalloc(const dg_desc* d, int64_t n_subgrids, const int64_t* vis_offsets,
                                 const void* subgrids, const void* g_uv, const void* g_w, const double* uvw,
                                 void* vis_out, int64_t* oob_count, hipStream_t stream) {
    dg_status s = validate_desc(d);
    if (s != DG_OK) return s;
    if (n_subgrids > kNoAllocMaxSubgrids)
        return fail(DG_ERR_UNSUPPORTED, "degrid_execute_noalloc takes at most %lld subgrids (its static scratch "
                    "holds %lld offsets), got %lld", (long long)kNoAllocMaxSubgrids,
                    (long long)kNoAllocMaxSubgrids + 1, (long long)n_subgrids);
    s = validate_offsets(n_subgrids, vis_offsets);
    if (s != DG_OK) return s;
    const int64_t n = vis_offsets[n_subgrids];
    if (n > 0 && (!subgrids || !g_uv || !g_w || !uvw || !vis_out))
        return fail(DG_ERR_INVALID_ARG, "a device pointer is NULL");
    if (s = check_alignment(*d, subgrids, g_uv, g_w, uvw, vis_out, nullptr, nullptr); s != DG_OK) return s;
    if (reinterpret_cast<uintptr_t>(oob_count) % 8 != 0) return fail(DG_ERR_INVALID_ARG, "oob_count must be 8-byte aligned");
    const int nb = d->n_b > 0 ? d->n_b : kMaxNb;
    int64_t n_tiles = 0;
    for (int64_t k = 0; k < n_subgrids; ++k) n_tiles += (vis_offsets[k + 1] - vis_offsets[k] + nb - 1) / nb;
    if (n_tiles > 0x7FFFFFFF)
        return fail(DG_ERR_UNSUPPORTED, "%lld tiles: at most 2^31 - 1 (use a larger n_b)", (long long)n_tiles);
    const Problem pr = problem_of_desc(*d, nullptr, subgrids, g_uv, g_w, uvw, vis_out, nullptr);
    const hipError_t e = launch_degrid_noalloc(pr, d->grid_dtype, d->gcf_dtype, deep_only(*d), vis_offsets, n_subgrids,
                                               nb, n_tiles, reinterpret_cast<unsigned long long*>(oob_count), stream);
    if (e != hipSuccess) return hip_fail(e, "degrid_execute_noalloc launch");
    return DG_OK;
}

dg_status degrid_residual(dg_plan p, const void* subgrids, const void* g_uv, const void* g_w, const double* uvw,
                          const void* v_obs, void* res_out, double* loss_out, hipStream_t stream) {
    if (!p) return fail(DG_ERR_INVALID_ARG, "plan is NULL");
    if (!loss_out) return fail(DG_ERR_INVALID_ARG, "loss_out is NULL");
    if (p->ds.n_tiles == 0) {   // no visibilities: the loss is 0, and nothing is out of range
        hipError_t e = launch_set_f64(loss_out, 0.0, stream);
        if (e != hipSuccess) return hip_fail(e, "loss fill kernel launch");
        p->launched = false;
        return DG_OK;
    }
    if (!subgrids || !g_uv || !g_w || !uvw || !v_obs || !res_out)
        return fail(DG_ERR_INVALID_ARG, "a device pointer is NULL");
    if (dg_status s = check_alignment(p->desc, subgrids, g_uv, g_w, uvw, res_out, v_obs, nullptr); s != DG_OK)
        return s;
    const Problem pr = problem_of(p, subgrids, g_uv, g_w, uvw, res_out, nullptr);
    LaunchParams lp = params_for(p, pr);
    lp.v_obs = static_cast<const float2*>(v_obs);
    lp.tile_loss = p->ds.tile_loss;
    hipError_t e = launch_degrid(lp, p->desc.grid_dtype, p->desc.gcf_dtype, p->variant, p->blocks, stream);
    if (e == hipSuccess) e = launch_loss_sum(p->ds.tile_loss, p->ds.n_tiles, loss_out, stream);
    if (e != hipSuccess) return hip_fail(e, "degrid kernel launch (residual)");
    p->last_stream = stream;
    p->launched = true;
    return DG_OK;
}

dg_status grid_adjoint(dg_plan p, const void* vis, const void* g_uv, const void* g_w,
                       const double* uvw, void* subgrids_out, int32_t accumulate, hipStream_t stream) {
    if (!p) return fail(DG_ERR_INVALID_ARG, "plan is NULL");
    if (accumulate != 0 && accumulate != 1) return fail(DG_ERR_INVALID_ARG, "accumulate must be 0 or 1");
    if (!subgrids_out && p->n_sub > 0) return fail(DG_ERR_INVALID_ARG, "subgrids_out is NULL");
    const int64_t out_bytes = p->n_sub * (int64_t)p->desc.n_v * p->desc.n_u * p->desc.n_w * 8;
    if (p->d_own_blocks && p->offsets.back() > 0) {
        // owner-computes: every output block written once, then the fix-up
        if (!vis || !g_uv || !g_w || !uvw) return fail(DG_ERR_INVALID_ARG, "a device pointer is NULL");
        if (dg_status s = check_alignment(p->desc, nullptr, g_uv, g_w, uvw, vis, nullptr, subgrids_out); s != DG_OK)
            return s;
        OwnerParams op{};
        op.prob = problem_of(p, nullptr, g_uv, g_w, uvw, const_cast<void*>(vis), subgrids_out);
        op.blocks = p->d_own_blocks;
        op.items = p->d_own_items;
        op.plan_start = p->d_plan_start;
        op.ctl = p->d_own_ctl;
        op.q = p->own_q;
        op.accumulate = accumulate;
        op.nby = p->nby;
        op.nbx = p->nbx;
        hipError_t e = launch_grid_owner(op, p->desc.gcf_dtype, p->own_grid, stream);
        if (e == hipSuccess)
            e = launch_grid_fixup(op.prob, p->d_offsets, p->n_sub, p->offsets.back(), p->d_plan_start, p->ds.ctl,
                                  p->desc.gcf_dtype, std::max(1, 2 * p->n_cu), stream);
        if (e != hipSuccess) return hip_fail(e, "adjoint kernel launch");
        p->last_stream = stream;
        p->launched = true;
        return DG_OK;
    }
    if (dg_status s = check_alignment(p->desc, nullptr, g_uv, g_w, uvw, vis, nullptr, subgrids_out); s != DG_OK)
        return s;
    if (!accumulate) {
        hipError_t e = launch_zero(subgrids_out, out_bytes, stream);
        if (e != hipSuccess) return hip_fail(e, "zero-fill kernel launch");
    }
    if (p->ds.n_tiles == 0) {   // nothing to add, and nothing out of range
        p->launched = false;
        return DG_OK;
    }
    if (!vis || !g_uv || !g_w || !uvw) return fail(DG_ERR_INVALID_ARG, "a device pointer is NULL");
    const Problem pr = problem_of(p, nullptr, g_uv, g_w, uvw, const_cast<void*>(vis), subgrids_out);
    hipError_t e = launch_grid_adjoint(params_for(p, pr), p->desc.gcf_dtype, p->variant, p->blocks_adj, stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint kernel launch");
    p->last_stream = stream;
    p->launched = true;
    return DG_OK;
}

dg_status degrid_table_grad(dg_plan p, const void* subgrids, const void* g_uv, const void* g_w, const double* uvw,
                            const void* grad_vis, float* grad_g_uv, float* grad_g_w, int32_t accumulate,
                            hipStream_t stream) {
    if (!p) return fail(DG_ERR_INVALID_ARG, "plan is NULL");
    if (accumulate != 0 && accumulate != 1) return fail(DG_ERR_INVALID_ARG, "accumulate must be 0 or 1");
    if (!grad_g_uv && !grad_g_w) return DG_OK;   // nothing asked for
    for (const void* q : {static_cast<const void*>(grad_g_uv), static_cast<const void*>(grad_g_w)})
        if (q && reinterpret_cast<uintptr_t>(q) % 4 != 0)
            return fail(DG_ERR_INVALID_ARG, "table gradient outputs must be 4-byte aligned");
    const dg_desc& d = p->desc;
    const int64_t n_uv = (int64_t)d.os_uv * d.os_uv * kSupportUV * kSupportUV;
    const int64_t n_w = (int64_t)d.os_w * kSupportW;
    if (p->ds.n_tiles > 0) {
        if (!subgrids || !g_uv || !g_w || !uvw || !grad_vis)
            return fail(DG_ERR_INVALID_ARG, "a device pointer is NULL");
        if (dg_status s = check_alignment(d, subgrids, g_uv, g_w, uvw, nullptr, grad_vis, nullptr); s != DG_OK)
            return s;
    }
    hipError_t e = hipSuccess;
    if (!accumulate) {
        if (grad_g_uv) e = launch_zero_f32(grad_g_uv, n_uv, stream);
        if (e == hipSuccess && grad_g_w) e = launch_zero_f32(grad_g_w, n_w, stream);
        if (e != hipSuccess) return hip_fail(e, "zero-fill kernel launch");
    }
    if (p->ds.n_tiles == 0) return DG_OK;
    TableGradParams tp{};
    tp.prob = problem_of(p, subgrids, g_uv, g_w, uvw, const_cast<void*>(grad_vis), nullptr);
    tp.tiles = p->ds.tiles;
    tp.tile_vis = p->ds.tile_vis;
    tp.n_tiles = p->ds.n_tiles;
    tp.grad_uv = grad_g_uv;
    tp.grad_w = grad_g_w;
    // grid-stride over the tiles with at most as many workgroups as fit at
    // once (each one ends by adding its LDS sums to the outputs)
    int max_lds = 0;
    e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute(LDS per workgroup)");
    // one workgroup of kTableGradThreads per CU (registers allow no second)
    constexpr int64_t waves = kTableGradThreads / kWave;
    const int64_t blocks = std::max<int64_t>(
        1, std::min<int64_t>((p->ds.n_tiles + waves - 1) / waves, (int64_t)std::max(1, p->n_cu)));
    e = launch_table_grad(tp, d.grid_dtype, d.gcf_dtype, deep_only(d), (int)blocks, (size_t)max_lds, stream);
    if (e != hipSuccess) return hip_fail(e, "table gradient kernel launch");
    p->last_stream = stream;
    p->launched = true;
    return DG_OK;
}

dg_status degrid_oob_count(dg_plan p, int64_t* count) {
    if (!p || !count) return fail(DG_ERR_INVALID_ARG, "plan or count is NULL");
    *count = 0;
    if (!p->launched) return DG_OK;
    hipError_t e = hipStreamSynchronize(p->last_stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    unsigned long long v = 0;
    e = hipMemcpy(&v, &p->ds.ctl->oob.v[2], sizeof(v), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(out-of-range count)");
    *count = (int64_t)v;
    return DG_OK;
}

dg_status degrid_plan_get_info(dg_plan p, dg_plan_info* info) {
    if (!p || !info) return fail(DG_ERR_INVALID_ARG, "plan or info is NULL");
    info->n_subgrids = p->n_sub;
    info->n_vis = p->offsets.back();
    info->n_tiles = p->ds.n_tiles;
    info->n_b = p->n_b;
    info->kernel = p->variant;
    info->grid_blocks = p->blocks;
    info->block_threads = kBlockThreads;
    info->n_queues = p->q.n_queues;
    info->device = p->device;
    info->sorted = p->d_perm ? 1 : 0;
    info->n_kernels = degrid_variant_count();
    return DG_OK;
}

dg_status degrid_tune(dg_plan p, const void* subgrids, const void* g_uv, const void* g_w,
                      const double* uvw, void* vis_out, hipStream_t stream) {
    if (!p) return fail(DG_ERR_INVALID_ARG, "plan is NULL");
    if (!subgrids || !g_uv || !g_w || !uvw || !vis_out)
        return fail(DG_ERR_INVALID_ARG, "a device pointer is NULL");
    if (dg_status s = check_alignment(p->desc, subgrids, g_uv, g_w, uvw, vis_out, nullptr, nullptr); s != DG_OK)
        return s;
    if (p->offsets.back() == 0) return DG_OK;
    static const int32_t kCandidates[] = {8, 16, 32, 64};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    if (he != hipSuccess) return hip_fail(he, "hipEventCreate");
    // Axes: the gather kernel variant (tap-per-lane mapping with LDS boxes of
    // several sizes or through the caches, the D1 mapping, the deep-stack
    // reader), the tile size, and the occupancy of the persistent grid (all
    // resident workgroups, or half of them). One visibility per tile is left
    // out: it was 2-12x slower at every count measured.
    float best_ms = 1e30f;
    int32_t best_nb = p->n_b, best_var = p->variant, best_div = p->grid_div;
    dg_status st = DG_OK;
    for (int var = 0; var < degrid_variant_count() && st == DG_OK; ++var) {
        if (!variant_allowed(p->desc, var)) continue;
        for (int32_t nb : kCandidates) {
            p->variant = var;
            st = rebuild_tiles(p, nb, stream);
            if (st != DG_OK) break;
            for (int32_t div : kGridDivs) {
                p->grid_div = div;
                p->blocks = blocks_for(std::max(1, p->cap[p->variant] / div), p->ds.n_tiles);
                const int reps = 5;
                for (int r = 0; r < 2 && st == DG_OK; ++r)
                    st = degrid_execute(p, subgrids, g_uv, g_w, uvw, vis_out, stream);
                (void)hipEventRecord(e0, stream);
                for (int r = 0; r < reps && st == DG_OK; ++r)
                    st = degrid_execute(p, subgrids, g_uv, g_w, uvw, vis_out, stream);
                (void)hipEventRecord(e1, stream);
                he = hipEventSynchronize(e1);
                if (st != DG_OK) break;
                if (he != hipSuccess) { st = hip_fail(he, "hipEventSynchronize"); break; }
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (ms < best_ms) { best_ms = ms; best_nb = nb; best_var = var; best_div = div; }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != DG_OK) return st;
    p->variant = best_var;
    p->grid_div = best_div;
    st = rebuild_tiles(p, best_nb, stream);
    if (st != DG_OK) return st;
    tune_cache_store(tune_key(p), best_nb, best_var, best_div);
    return DG_OK;
}

dg_status degrid_plan_sort(dg_plan p, const double* uvw, hipStream_t stream) {
    if (!p) return fail(DG_ERR_INVALID_ARG, "plan is NULL");
    const int64_t n = p->offsets.back();
    if (!uvw) {
        if (p->d_perm) {
            (void)hipDeviceSynchronize();
            (void)hipFree(p->d_perm);
            p->d_perm = nullptr;
            p->start.clear();
            free_owner(p);
            return rebuild_tiles(p, p->n_b_req, stream);
        }
        return DG_OK;
    }
    if (n >= (int64_t(1) << 32)) return fail(DG_ERR_UNSUPPORTED, "work order needs N < 2^32");
    if (n == 0) return DG_OK;
    if (fault_injected("alloc")) return fail(DG_ERR_NOMEM, "allocation failure injected (DG_FAULT_INJECT=alloc)");
    hipError_t e;
    if (!p->d_perm) {
        e = hipMalloc(&p->d_perm, sizeof(uint32_t) * (size_t)n);
        if (e != hipSuccess) { p->d_perm = nullptr; return hip_fail(e, "hipMalloc(work order)"); }
    }
    e = sort_visibilities(uvw, p->offsets.data(), p->n_sub, p->d_perm, stream);
    if (e != hipSuccess) {
        (void)hipFree(p->d_perm);
        p->d_perm = nullptr;
        return hip_fail(e, "sorting the work order");
    }
    // first taps in the new order, for cutting tiles that fit the LDS box
    uint32_t* d_start = nullptr;
    e = hipMalloc(&d_start, sizeof(uint32_t) * (size_t)n);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(start cells)");
    const Problem pr = problem_of(p, nullptr, nullptr, nullptr, uvw, nullptr, nullptr);
    e = launch_start_cells(pr, n, d_start, stream);
    p->start.resize((size_t)n);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->start.data(), d_start, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    (void)hipFree(d_start);
    if (e != hipSuccess) {
        p->start.clear();
        return hip_fail(e, "computing start cells");
    }
    // owner-computes gridding keeps 4 w values per cell in LDS
    dg_status st = deep_only(p->desc) ? DG_OK : build_owner(p, stream);
    if (st != DG_OK) return st;
    return rebuild_tiles(p, p->n_b_req, stream);
}

dg_status degrid_plan_set_kernel(dg_plan p, int32_t kernel, int32_t n_b, hipStream_t stream) {
    if (!p) return fail(DG_ERR_INVALID_ARG, "plan is NULL");
    if (kernel < -1 || kernel >= degrid_variant_count())
        return fail(DG_ERR_INVALID_ARG, "kernel must be in [-1, %d), got %d", degrid_variant_count(), kernel);
    if (n_b < 0 || n_b > kMaxNb) return fail(DG_ERR_INVALID_ARG, "n_b must be in [0, %d], got %d", kMaxNb, n_b);
    if (kernel >= 0 && !variant_allowed(p->desc, kernel))
        return fail(DG_ERR_UNSUPPORTED, "subgrids with %d w planes need kernel %d or %d (got %d)", p->desc.n_w,
                    kDeepVariant, kD1Variant, kernel);
    if (kernel >= 0) p->variant = kernel;
    return rebuild_tiles(p, n_b > 0 ? n_b : p->n_b_req, stream);
}

dg_status degrid_destroy(dg_plan p) {
    if (!p) return DG_OK;
    (void)hipDeviceSynchronize();
    if (p->d_perm) (void)hipFree(p->d_perm);
    free_owner(p);
    free_scratch(p->ds);
    delete p;
    return DG_OK;
}

dg_status degrid_batch_plan(const dg_plan* plans, int32_t n, dg_batch* out) {
    if (!out) return fail(DG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!plans || n <= 0) return fail(DG_ERR_INVALID_ARG, "need at least one plan");
    if (n > 0xFFFF) return fail(DG_ERR_UNSUPPORTED, "at most 65535 problems per batch");
    for (int32_t i = 0; i < n; ++i) {
        if (!plans[i]) return fail(DG_ERR_INVALID_ARG, "plan %d is NULL", i);
        if (plans[i]->desc.grid_dtype != plans[0]->desc.grid_dtype ||
            plans[i]->desc.gcf_dtype != plans[0]->desc.gcf_dtype)
            return fail(DG_ERR_INVALID_ARG, "plan %d has another grid or gcf dtype than plan 0", i);
        if (plans[i]->device != plans[0]->device)
            return fail(DG_ERR_INVALID_ARG, "plan %d lives on another device", i);
    }
    dg_batch_* b = new (std::nothrow) dg_batch_();
    if (!b) return fail(DG_ERR_NOMEM, "host allocation of the batch failed");
    b->plans.assign(plans, plans + n);
    for (int32_t i = 0; i < n; ++i) b->plan_versions.push_back(plans[i]->version);
    // one kernel for the whole batch: that of the plan with the most
    // visibilities (a tiny plan defaults to the cache gather, which would slow
    // the others down; the tuner gives every plan the same one), or the deep
    // one if any plan has subgrids deeper than the w support
    int32_t lead = 0;
    for (int32_t i = 1; i < n; ++i)
        if (plans[i]->offsets.back() > plans[lead]->offsets.back()) lead = i;
    b->variant = plans[lead]->variant;
    for (int32_t i = 0; i < n; ++i)
        if (!variant_allowed(plans[i]->desc, b->variant)) b->variant = kDeepVariant;
    b->grid_dtype = plans[0]->desc.grid_dtype;
    b->gcf_dtype = plans[0]->desc.gcf_dtype;
    b->device = plans[0]->device;
    const int max_nb = degrid_variant_max_nb(b->variant);
    std::vector<Tile> tiles;
    std::vector<const uint32_t*> perms;
    size_t total_tiles = 0;
    for (int32_t i = 0; i < n; ++i) total_tiles += plans[i]->tiles.size();
    if (total_tiles > (size_t)0x7FFFFFFF) {
        degrid_batch_destroy(b);
        return fail(DG_ERR_UNSUPPORTED, "%zu tiles: at most 2^31 - 1 per batch", total_tiles);
    }
    for (int32_t i = 0; i < n; ++i) {
        for (Tile t : plans[i]->tiles) {
            if (t.count > max_nb) {
                degrid_batch_destroy(b);
                return fail(DG_ERR_INVALID_ARG, "plan %d has tiles of %d visibilities; the batch's kernel takes at most %d",
                            i, (int)t.count, max_nb);
            }
            t.problem = (uint16_t)i;
            tiles.push_back(t);
        }
        perms.push_back(plans[i]->d_perm);
    }
    dg_status s = DG_OK;
    hipError_t e;
    auto bail = [&](dg_status st) {
        degrid_batch_destroy(b);
        return st;
    };
    s = alloc_scratch(b->ds, tiles, perms, nullptr);
    if (s != DG_OK) return bail(s);
    b->q = split_queues(tiles);
    b->blocks = blocks_for(std::max(1, plans[0]->cap[b->variant] / plans[0]->grid_div), b->ds.n_tiles);
    e = hipMalloc(&b->d_probs, sizeof(Problem) * n);
    if (e != hipSuccess) { b->d_probs = nullptr; return bail(hip_fail(e, "hipMalloc(problem table)")); }
    e = hipHostMalloc(&b->h_probs, sizeof(Problem) * n, hipHostMallocDefault);
    if (e != hipSuccess) { b->h_probs = nullptr; return bail(hip_fail(e, "hipHostMalloc(problem table)")); }
    e = hipEventCreateWithFlags(&b->upload_done, hipEventDisableTiming);
    if (e != hipSuccess) { b->upload_done = nullptr; return bail(hip_fail(e, "hipEventCreate")); }
    if (b->ds.n_tiles > 0) {
        // One kernel node whose parameters point at the batch's own device
        // table, queue and control block; arguments change through the table.
        LaunchParams lp{};
        lp.probs = b->d_probs;
        lp.tiles = b->ds.tiles;
        lp.tile_vis = b->ds.tile_vis;
        lp.ctl = b->ds.ctl;
        lp.q = b->q;
        e = hipGraphCreate(&b->graph, 0);
        if (e != hipSuccess) { b->graph = nullptr; return bail(hip_fail(e, "hipGraphCreate")); }
        hipStream_t cap = nullptr;
        e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(hip_fail(e, "hipStreamCreate"));
        e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t le = launch_degrid(lp, b->grid_dtype, b->gcf_dtype, b->variant, b->blocks, cap);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(cap, &g);
            if (le != hipSuccess) e = le;
            if (e == hipSuccess) {
                (void)hipGraphDestroy(b->graph);
                b->graph = g;
            } else if (g) {
                (void)hipGraphDestroy(g);
            }
        }
        (void)hipStreamDestroy(cap);
        if (e != hipSuccess) return bail(hip_fail(e, "capturing the batch launch"));
        e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) { b->exec = nullptr; return bail(hip_fail(e, "hipGraphInstantiate")); }
    }
    *out = b;
    g_last_error.clear();
    return DG_OK;
}

dg_status degrid_batch_execute(dg_batch b, const void* const* args, hipStream_t stream) {
    if (!b || !args) return fail(DG_ERR_INVALID_ARG, "batch or args is NULL");
    const size_t n = b->plans.size();
    for (size_t i = 0; i < n; ++i) {
        if (b->plans[i]->offsets.back() == 0) continue;
        for (int k = 0; k < 5; ++k)
            if (!args[5 * i + k]) return fail(DG_ERR_INVALID_ARG, "args[%zu] is NULL", 5 * i + k);
        const void* const* a = args + 5 * i;
        if (dg_status s = check_alignment(b->plans[i]->desc, a[0], a[1], a[2], a[3], a[4], nullptr, nullptr); s != DG_OK)
            return s;
    }
    for (size_t i = 0; i < n; ++i)
        if (b->plans[i]->version != b->plan_versions[i])
            return fail(DG_ERR_NOT_READY, "plan %zu changed (sorted or tuned) after the batch was planned", i);
    if (b->ds.n_tiles == 0) {   // no visibilities: nothing to write, and nothing out of range
        b->launched = false;
        return DG_OK;
    }
    const bool same = b->uploaded && std::equal(b->last_args.begin(), b->last_args.end(), args);
    hipError_t e;
    if (!same) {
        // the previous upload must have left the pinned staging buffer
        e = hipEventSynchronize(b->upload_done);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize(upload)");
        for (size_t i = 0; i < n; ++i)
            b->h_probs[i] = problem_of(b->plans[i], args[5 * i], args[5 * i + 1], args[5 * i + 2],
                                       static_cast<const double*>(args[5 * i + 3]),
                                       const_cast<void*>(args[5 * i + 4]), nullptr);
        e = hipMemcpyAsync(b->d_probs, b->h_probs, sizeof(Problem) * n, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(problem table)");
        e = hipEventRecord(b->upload_done, stream);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord(upload)");
        b->last_args.assign(args, args + 5 * n);
        b->uploaded = true;
    }
    e = hipGraphLaunch(b->exec, stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    b->last_stream = stream;
    b->launched = true;
    return DG_OK;
}

dg_status degrid_batch_oob_count(dg_batch b, int64_t* count) {
    if (!b || !count) return fail(DG_ERR_INVALID_ARG, "batch or count is NULL");
    *count = 0;
    if (!b->launched) return DG_OK;
    hipError_t e = hipStreamSynchronize(b->last_stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    unsigned long long v = 0;
    e = hipMemcpy(&v, &b->ds.ctl->oob.v[2], sizeof(v), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(out-of-range count)");
    *count = (int64_t)v;
    return DG_OK;
}

dg_status degrid_batch_tune(const dg_plan* plans, int32_t n, const void* const* args, hipStream_t stream,
                            int32_t* best_kernel, int32_t* best_n_b) {
    if (!plans || n <= 0) return fail(DG_ERR_INVALID_ARG, "need at least one plan");
    if (!args) return fail(DG_ERR_INVALID_ARG, "args is NULL");
    for (int32_t i = 0; i < n; ++i)
        if (!plans[i]) return fail(DG_ERR_INVALID_ARG, "plan %d is NULL", i);
    static const int32_t kCandidates[] = {8, 16, 32, 64};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(he, "hipEventCreate");
    }
    float best_ms = 1e30f;
    int32_t best_var = plans[0]->variant, best_nb = plans[0]->n_b, best_div = plans[0]->grid_div;
    dg_status st = DG_OK;
    bool any_deep = false;
    for (int32_t i = 0; i < n; ++i) any_deep = any_deep || deep_only(plans[i]->desc);
    for (int var = 0; var < degrid_variant_count() && st == DG_OK; ++var) {
        if (any_deep && !degrid_variant_any_depth(var)) continue;
        int32_t last_nb = -1;
        for (int32_t nb_req : kCandidates) {
            const int32_t nb = std::min<int32_t>(nb_req, degrid_variant_max_nb(var));
            if (nb == last_nb) continue;   // the variant caps the tile size
            last_nb = nb;
            for (int32_t i = 0; i < n && st == DG_OK; ++i) {
                plans[i]->variant = var;
                st = rebuild_tiles(plans[i], nb, stream);
            }
            if (st != DG_OK) break;
            for (int32_t div : kGridDivs) {
                plans[0]->grid_div = div;   // the batch's grid follows plan 0
                dg_batch b = nullptr;
                st = degrid_batch_plan(plans, n, &b);
                if (st != DG_OK) break;
                const int reps = 5;
                for (int r = 0; r < 2 && st == DG_OK; ++r) st = degrid_batch_execute(b, args, stream);
                (void)hipEventRecord(e0, stream);
                for (int r = 0; r < reps && st == DG_OK; ++r) st = degrid_batch_execute(b, args, stream);
                (void)hipEventRecord(e1, stream);
                he = hipEventSynchronize(e1);
                (void)degrid_batch_destroy(b);
                if (st != DG_OK) break;
                if (he != hipSuccess) { st = hip_fail(he, "hipEventSynchronize"); break; }
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (ms < best_ms) { best_ms = ms; best_var = var; best_nb = nb; best_div = div; }
            }
            if (st != DG_OK) break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (int32_t i = 0; i < n; ++i) {
        plans[i]->variant = best_var;
        plans[i]->grid_div = best_div;
        const dg_status s2 = rebuild_tiles(plans[i], best_nb, stream);
        if (st == DG_OK) st = s2;
    }
    if (st != DG_OK) return st;
    if (best_kernel) *best_kernel = best_var;
    if (best_n_b) *best_n_b = best_nb;
    return DG_OK;
}

dg_status degrid_batch_destroy(dg_batch b) {
    if (!b) return DG_OK;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->upload_done) (void)hipEventDestroy(b->upload_done);
    if (b->d_probs) (void)hipFree(b->d_probs);
    if (b->h_probs) (void)hipHostFree(b->h_probs);
    free_scratch(b->ds);
    delete b;
    return DG_OK;
}

const char* degrid_status_str(dg_status s) {
    switch (s) {
        case DG_OK: return "DG_OK";
        case DG_ERR_INVALID_ARG: return "DG_ERR_INVALID_ARG";
        case DG_ERR_UNSUPPORTED: return "DG_ERR_UNSUPPORTED";
        case DG_ERR_NOMEM: return "DG_ERR_NOMEM";
        case DG_ERR_HIP: return "DG_ERR_HIP";
        case DG_ERR_NOT_READY: return "DG_ERR_NOT_READY";
    }
    return "DG_ERR_UNKNOWN";
}

const char* degrid_last_error(void) { return g_last_error.c_str(); }

int32_t degrid_version(void) { return 100; }

}  // extern "C"
