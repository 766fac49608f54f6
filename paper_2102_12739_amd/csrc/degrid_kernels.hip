// gfx950 kernels for 3D degridding.
//
// Degridding (Section 2 of the paper) forms each visibility as the sum of
// the 8 x 8 x 4 subgrid neighbourhood that starts at g = [x, y, z], weighted
// by G_w[o_w][t_w] * G_uv[o_v][o_u][t_v][t_u]. It is a gather with about
// 0.5 flop per byte, so these kernels are built around memory access, not
// matrix cores:
//
//  * persistent workgroups drain a list of tiles (n_b consecutive
//    visibilities of one subgrid) from per-XCD queues (this replaces the
//    launch grid of Eq. (1)): most of each queue is dealt round-robin to the
//    wavefronts that serve it, without atomics; the rest goes through the
//    queue's atomic cursor, and a wavefront whose queue is empty steals
//    from the others;
//  * each wavefront takes one tile. Its coordinate stage computes, one lane
//    per visibility, the start cell and the oversample indices in float64
//    (k = floor(c * os) of the float64 product: exact for power-of-two
//    oversampling, the stated rounding for other factors); the results stay
//    in the lane's registers and reach the whole wavefront through
//    v_readlane;
//  * when the tile's neighbourhoods fit the wavefront's LDS box, their
//    subgrid cells are first copied there with loads that write LDS
//    directly, and the gather reads LDS; otherwise it reads through the
//    caches;
//  * the gather maps the 64 lanes onto the 8 x 8 (t_v, t_u) taps. Each lane
//    reads the 4 w values of its tap (32 contiguous bytes for complex64; one
//    v-row of the neighbourhood is 256 contiguous bytes) and its G_uv weight
//    (one coalesced 256-byte block per visibility). Loads go through buffer
//    resources, so the hardware bounds check turns any offset outside the
//    subgrid into zeros. 16-bit storage with a G_w table of the same type
//    sums over w with packed dot products;
//  * eight visibilities are reduced across the wavefront together: two
//    permlane swaps (lanes 32 apart, then 16 apart) and one DPP step halve the
//    number of live partial sums at each level, then three DPP steps finish
//    the 8-lane sums (Section 2 uses a warp reduction after a v-axis
//    accumulation; here the reduction is shared between visibilities);
//  * results are staged in LDS per tile, and each lane then writes its
//    visibility's output at the visibility's own index (Section 2 stages
//    outputs in shared memory and writes them in bulk).
#include "dg_device.h"

namespace dg {
namespace {

// ---------------------------------------------------------------------------
// D1 lane mapping (Section 2, kernel D1)
// ---------------------------------------------------------------------------
//
// The wavefront takes two visibilities at once, one per 32-lane half. Lane
// (t_u, t_w) of a half (t_u = lane / 4 mod 8, t_w = lane mod 4) walks the 8
// v-rows of its visibility's neighbourhood: each step reads one value (a
// half reads one v-row, 8 u x 4 w values, contiguous in memory) and its
// G_uv weight, and accumulates along v; the sum is then weighted by
// G_w[o_w][t_w] and reduced over the half. Eight pairs (16 visibilities)
// are reduced together.

// One value per lane for each of the 8 v-rows of one visibility, its 8 G_uv
// weights and its G_w tap.
template <int G>
struct PairFetch {
    uint32_t raw[kSupportUV][GridTraits<G>::kWords / kSupportW];
    float g[kSupportUV];
    float gw;
};

// Lane-dependent selection: visibility j0 + (upper half) of a value that
// lane j holds for visibility j.
__device__ __forceinline__ int half_pick(int x, int j0, bool upper) {
    const int a = __builtin_amdgcn_readlane(x, j0);
    const int b = __builtin_amdgcn_readlane(x, j0 + 1);
    return upper ? b : a;
}

template <int G, int F>
__device__ __forceinline__ void fetch_pair(PairFetch<G>& f, int j0, int count, int a_off, int g_off, int ow,
                                           __amdgpu_buffer_rsrc_t ra, __amdgpu_buffer_rsrc_t rg, const void* g_w,
                                           uint32_t lane_a, uint32_t lane_g, uint32_t row_bytes, int tw) {
    const bool upper = lane_id() >= 32;
    const bool live = j0 + (upper ? 1 : 0) < count;
    const uint32_t aj = live ? (uint32_t)half_pick(a_off, j0, upper) : kOutOfRange;
    const uint32_t gj = (uint32_t)half_pick(g_off, j0, upper);
    const int oj = half_pick(ow, j0, upper);
#pragma unroll
    for (int tv = 0; tv < kSupportUV; ++tv) {
        const uint32_t off = aj == kOutOfRange ? kOutOfRange : aj + (uint32_t)tv * row_bytes + lane_a;
        if constexpr (G == kGridC64) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b64(ra, off, 0, 0);
            f.raw[tv][0] = v[0];
            f.raw[tv][1] = v[1];
        } else {
            f.raw[tv][0] = __builtin_amdgcn_raw_buffer_load_b32(ra, off, 0, 0);
        }
        f.g[tv] = load_gcf_rsrc<F>(rg, gj + lane_g + (uint32_t)(tv * kSupportUV) * GcfTraits<F>::kBytes);
    }
    f.gw = load_gcf<F>(g_w, (int64_t)oj * kSupportW + tw);
}

// v-accumulated, G_w-weighted partial sum of this lane for its visibility.
template <int G>
__device__ __forceinline__ void sum_pair(const PairFetch<G>& f, float& re, float& im) {
    float ar = 0.0f, ai = 0.0f;
#pragma unroll
    for (int tv = 0; tv < kSupportUV; ++tv) {
        float r, i;
        if constexpr (G == kGridC64) {
            r = __uint_as_float(f.raw[tv][0]);
            i = __uint_as_float(f.raw[tv][1]);
        } else if constexpr (G == kGridCBF16) {
            r = __uint_as_float(f.raw[tv][0] << 16);
            i = __uint_as_float(f.raw[tv][0] & 0xFFFF0000u);
        } else {
            const __half2 h = __builtin_bit_cast(__half2, f.raw[tv][0]);
            r = __low2float(h);
            i = __high2float(h);
        }
        ar += f.g[tv] * r;
        ai += f.g[tv] * i;
    }
    re = ar * f.gw;
    im = ai * f.gw;
}

// In: p[k] = this lane's partial sum for pair k (k = 0..7; the lower half
// holds visibility 2k, the upper half 2k + 1). Out: p[0] on lane l = the
// sum over l's half for pair 4 * bit4 + 2 * bit3 + bit2 of l. A permlane16
// swap pairs the two rows of each half (rows 0/2 keep pair k, rows 1/3 take
// pair k + 4), then DPP steps halve the live values by lane bits 3 and 2
// and finish over bits 1 and 0.
__device__ __forceinline__ void reduce_pairs8(float (&p)[8]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) p[k] = swap_add16(p[k], p[k + 4]);
    const int lane = lane_id();
    const bool b3 = (lane & 8) != 0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float keep = b3 ? p[k + 2] : p[k];
        const float give = b3 ? p[k] : p[k + 2];
        p[k] = keep + dpp<kDppRowRor8>(give);
    }
    const bool b2 = (lane & 4) != 0;
    const float keep = b2 ? p[1] : p[0];
    const float give = b2 ? p[0] : p[1];
    float s = keep + dpp<kDppRowHalfMirror>(give);
    s += dpp<kDppQuadXor2>(s);
    s += dpp<kDppQuadXor1>(s);
    p[0] = s;
}

// All visibilities of a tile with the D1 mapping; results land in out[0 ..
// count). a_off: byte offset of each visibility's first tap in its subgrid
// (kOutOfRange when out of range), g_off: byte offset of its G_uv block,
// ow: its G_w row (lane j holds visibility j's).
template <int G, int F, int NB>
__device__ __forceinline__ void gather_tile_d1(float2* out, int count, int a_off, int g_off, int ow,
                                               __amdgpu_buffer_rsrc_t ra, __amdgpu_buffer_rsrc_t rg,
                                               const void* g_w, uint32_t row_bytes, int n_w) {
    static_assert(NB % 16 == 0, "groups of 16 visibilities");
    const int lane = lane_id();
    const int tu = (lane >> 2) & 7, tw = lane & 3;
    const uint32_t lane_a = (uint32_t)(tu * n_w + tw) * GridTraits<G>::kElemBytes;
    const uint32_t lane_g = (uint32_t)tu * GcfTraits<F>::kBytes;
    PairFetch<G> buf[2];
    fetch_pair<G, F>(buf[0], 0, count, a_off, g_off, ow, ra, rg, g_w, lane_a, lane_g, row_bytes, tw);
#pragma unroll
    for (int g0 = 0; g0 < NB; g0 += 16) {
        if (g0 < count) {
            float pre[8], pim[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int j0 = g0 + 2 * k;
                const int nxt = j0 + 2;
                if (nxt < NB && nxt < count)
                    fetch_pair<G, F>(buf[(k + 1) & 1], nxt, count, a_off, g_off, ow, ra, rg, g_w, lane_a, lane_g,
                                     row_bytes, tw);
                sum_pair<G>(buf[k & 1], pre[k], pim[k]);
            }
            reduce_pairs8(pre);
            reduce_pairs8(pim);
            if ((lane & 3) == 0) {
                const int k = ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 + ((lane >> 2) & 1);
                const int j = g0 + 2 * k + (lane >> 5);
                if (j < count) out[j] = make_float2(pre[0], pim[0]);
            }
        }
    }
}

// BOX: bytes of LDS per wavefront for the staged copy of a tile's cells
// (0: always gather through the caches). NB: largest tile; the tile's G_uv
// weights are held in NB registers per lane.
//
// Each wavefront works on one tile while the next one is on its way: the
// next tile's header and visibility indices are requested when the current
// tile starts, its coordinates while the current tile is gathered, and the
// tile after it is popped from the queue one tile ahead.
// Workgroups per CU the register allocation must allow: three for 16-bit
// storage gathered through the caches (no LDS box, and about 170 registers
// before the bound: the third wavefront per SIMD hides more latency than the
// few values moved to scratch cost), two otherwise.
constexpr int degrid_min_blocks(int grid_kind, int box) { return (grid_kind != kGridC64 && box == 0) ? 3 : 2; }

template <int G, int F, int BOX, int NB, bool DEEP, bool D1>
__global__ __launch_bounds__(kBlockThreads, degrid_min_blocks(G, BOX)) void degrid_kernel(LaunchParams P) {
    using GT = GridTraits<G>;
    static_assert(NB % 8 == 0 && NB <= kMaxNb, "tile size");
    static_assert(!D1 || BOX == 0, "the D1 mapping gathers through the caches");
    // the staging copy below fills whole steps of 64 slots, also past the
    // box's last slot (with zeros), so each plane must hold a multiple of 64
    // 16-byte slots: complex64 boxes are multiples of 2 KiB, 16-bit ones of
    // 1 KiB
    static_assert(BOX % (kWave * 16 * (G == kGridC64 ? 2 : 1)) == 0, "box size");
    constexpr int kBoxBytes = BOX > 0 ? BOX : 16;
    constexpr uint32_t kPlane1 = kBoxBytes / 2;   // complex64: w 2-3 of every slot
    __shared__ float2 s_out[kWavesPerBlock][NB];
    __shared__ __attribute__((aligned(16))) char s_box[kWavesPerBlock][kBoxBytes];

    const int lane = lane_id();
    const int wv = (int)(threadIdx.x / kWave);
    TileClaims st = start_claims(P.q, P.deal, wv);
    uint32_t wave_oob = 0;

    // Tiles are taken ahead of need (to hide the queue atomics) only while
    // the queue holds more tiles after them than there are wavefronts per
    // queue; near its end each wavefront takes one tile at a time, so that
    // the last tiles spread over all wavefronts instead of queueing behind
    // the ones that took tiles early.
    const int waves_per_queue = ((int)gridDim.x * kWavesPerBlock + P.q.n_queues - 1) / P.q.n_queues;
    auto ahead_ok = [&](int tile) { return queue_end(P.q, st.q) - tile > waves_per_queue; };

    int t = uniform(claim_tile(P.q, P.deal, P.ctl, st));
    while (t >= 0) {
    // current tile and its coordinates (in flight until the loop needs them)
    Tile tc{};
    int64_t vis_c = 0;
    double u = 0.0, v = 0.0, w = 0.0;
    {
        tc = load_tile(P.tiles, t);
        vis_c = P.tile_vis[(int64_t)t * kMaxNb + lane];
        const double* uvw = problem_uvw(P, tc.problem);
        if (lane < tc.count) {
            u = uvw[3 * vis_c];
            v = uvw[3 * vis_c + 1];
            w = uvw[3 * vis_c + 2];
        }
    }
    int t_nxt = uniform(ahead_ok(t) ? claim_tile(P.q, P.deal, P.ctl, st) : -1);
    // pop of the tile after t_nxt, sent during the previous tile
    bool pend = false;
    uint32_t raw = 0;

    while (t >= 0) {
        const Problem pr = P.probs ? load_problem(P.probs, tc.problem) : P.prob;
        const int count = tc.count;

        // Coordinate stage of the current tile: lane j, visibility j.
        int32_t x0 = 0, y0 = 0, cell = 0, tab = 0, ow = 0;
        bool in_range = false;
        if (lane < count) in_range = coords_from(pr, u, v, w, cell, tab, ow, x0, y0);
        if (!in_range) ow = 0;
        wave_oob += (uint32_t)__popcll(__ballot(lane < count && !in_range));

        // Next tile: header and visibility indices.
        const bool has_next = t_nxt >= 0;
        Tile tn{};
        int64_t vis_n = 0;
        if (has_next) {
            tn = load_tile(P.tiles, t_nxt);
            vis_n = P.tile_vis[(int64_t)t_nxt * kMaxNb + lane];
        }
        // (wave-uniform: both pops return a readfirstlane value; stated so
        // that the tile descriptors derived from it stay in scalar registers)
        const int t_after = uniform(!has_next ? -1
                                              : (pend ? claim_resolve(P.q, P.deal, P.ctl, st, raw)
                                                      : (ahead_ok(t_nxt) ? claim_tile(P.q, P.deal, P.ctl, st) : -1)));
        pend = false;
        // the pop of the tile after next is sent during this tile (below)
        // only when that one is not among the queue's last tiles
        const bool send_ahead = t_after >= 0 && ahead_ok(t_after);

        const char* sub_base = static_cast<const char*>(pr.subgrids) + (int64_t)tc.sub * pr.sub_bytes;
        const __amdgpu_buffer_rsrc_t ra = make_rsrc(sub_base, pr.sub_bytes);
        const __amdgpu_buffer_rsrc_t rg = make_rsrc(pr.g_uv, pr.guv_bytes);
        const uint64_t g_w = uniform_u64((uint64_t)pr.g_w);
        const uint32_t lane_g = (uint32_t)lane * GcfTraits<F>::kBytes;

        // G_uv weights of the whole tile. Visibility k's block offset goes in
        // the load's scalar offset, so no per-visibility address add. An
        // out-of-range visibility reads block 0: its sum is discarded, because
        // the output stage writes 0 for it.
        const int g_off = in_range ? tab * (int)GcfTraits<F>::kBytes : 0;
        float gv[D1 ? 1 : NB];
#pragma unroll
        for (int g0 = 0; g0 < (D1 ? 0 : NB); g0 += 8) {
            if (g0 < count) {
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    gv[g0 + k] = load_gcf_rsrc<F>(rg, lane_g, (uint32_t)__builtin_amdgcn_readlane(g_off, g0 + k));
            }
        }

        bool staged = false;
        int bx0 = 0, by0 = 0, bw = 0, bh = 0, bp = 0;
        if (BOX > 0 && pr.n_w == kSupportW) {
            // bounding box of the tile's neighbourhoods (the box holds w 0..3
            // of each cell, so only subgrids of 4 w planes are staged)
            int bx1 = -1, by1 = -1;
            wave_bbox(in_range, x0, y0, bx0, by0, bx1, by1);
            if (bx1 >= 0) {
                bw = bx1 - bx0 + kSupportUV;
                bh = by1 - by0 + kSupportUV;
                // row pitch of the LDS copy, in 16-byte chunks: congruent to 8
                // mod 16, so two neighbouring rows read in the same LDS cycle
                // fall on opposite halves of the banks
                bp = bw + ((8 - bw) & 15);
                staged = (uint32_t)(bp * bh) * kCellBytes<G> <= (uint32_t)BOX;
            }
        }

        char* box = s_box[wv];
        if (staged) {
            // Copy the box with loads that write LDS directly (lane l of a step
            // fills 16 bytes at 16 * l), all in flight at once. Slot s = row *
            // bp + col holds the cell's first 16 bytes (complex64: w 0-1; else
            // the whole cell) at 16 * s, and complex64's w 2-3 at kPlane1 +
            // 16 * s; columns col >= bw are row padding (filled with zeros).
            const int n_slots = bp * bh;
            const uint32_t row_stride = (uint32_t)pr.n_u * pr.n_w * GT::kElemBytes;
            const uint32_t box_origin = ((uint32_t)by0 * pr.n_u + bx0) * pr.n_w * GT::kElemBytes;
            const int drow = kWave / bp, dcol = kWave - drow * bp;
            int row = lane / bp;
            int col = lane - row * bp;
            for (int s0 = 0; s0 < n_slots; s0 += kWave) {
                const uint32_t off = (s0 + lane < n_slots && col < bw)
                                         ? box_origin + (uint32_t)row * row_stride + (uint32_t)col * kCellBytes<G>
                                         : kOutOfRange;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    ra, (__attribute__((address_space(3))) void*)(box + s0 * 16), 16, off, 0, 0, 0);
                if constexpr (G == kGridC64)
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(
                        ra, (__attribute__((address_space(3))) void*)(box + kPlane1 + s0 * 16), 16, off + 16u, 0, 0,
                        0);
                row += drow;
                col += dcol;
                if (col >= bp) {
                    col -= bp;
                    ++row;
                }
            }
            wait_vmem();
            wave_lds_sync();
            // the pop of the tile after next travels while this tile is gathered
            if (send_ahead) {
                raw = claim_issue(P.ctl, st);
                pend = true;
            }
        }

        // Next tile's coordinates: requested now when the gather below reads
        // only LDS, registers and the scalar cache; after it otherwise.
        double un = 0.0, vn = 0.0, wn = 0.0;
        const double* uvw_n = has_next ? problem_uvw(P, tn.problem) : nullptr;
        if (staged && has_next && lane < tn.count) {
            un = uvw_n[3 * vis_n];
            vn = uvw_n[3 * vis_n + 1];
            wn = uvw_n[3 * vis_n + 2];
        }

        const int a_off = staged ? (in_range ? ((y0 - by0) * bp + (x0 - bx0)) * 16 : 0)
                                 : (in_range ? cell * (int)GT::kElemBytes : (int)kOutOfRange);
        const uint32_t lane_a = staged ? ((uint32_t)(lane >> 3) * bp + (lane & 7)) * 16u
                                       : (uint32_t)(((lane >> 3) * pr.n_u + (lane & 7)) * pr.n_w) * GT::kElemBytes;
        if constexpr (D1) {
            gather_tile_d1<G, F, NB>(s_out[wv], count, a_off, g_off, ow, ra, rg, pr.g_w,
                                     (uint32_t)pr.n_u * pr.n_w * GT::kElemBytes, pr.n_w);
            if (send_ahead) {
                raw = claim_issue(P.ctl, st);
                pend = true;
            }
        } else if (staged) {
            gather_tile<G, F, NB, true, kPlane1, false>(s_out[wv], count, a_off, ow, gv, ra, g_w, lane_a, box);
        } else {
            gather_tile<G, F, NB, false, kPlane1, DEEP>(s_out[wv], count, a_off, ow, gv, ra, g_w, lane_a, box);
            if (send_ahead) {
                raw = claim_issue(P.ctl, st);
                pend = true;
            }
        }
        if (!staged && has_next && lane < tn.count) {
            un = uvw_n[3 * vis_n];
            vn = uvw_n[3 * vis_n + 1];
            wn = uvw_n[3 * vis_n + 2];
        }
        wave_lds_sync();
        double e = 0.0;
        if (lane < count) {
            float2 r = in_range ? s_out[wv][lane] : make_float2(0.f, 0.f);
            if (P.v_obs) {
                // residual of the observed visibility (it may share memory
                // with the output: this lane reads, then writes, element vis_c)
                const float2 o = P.v_obs[vis_c];
                r = make_float2(o.x - r.x, o.y - r.y);
                e = (double)r.x * r.x + (double)r.y * r.y;
            }
            static_cast<float2*>(pr.vis)[vis_c] = r;
        }
        if (P.v_obs) {
            const double tile_sum = wave_sum_f64(e);
            if (lane == 0) P.tile_loss[t] = tile_sum;
        }
        wave_lds_sync();

        t = t_nxt;
        t_nxt = t_after;
        tc = tn;
        vis_c = vis_n;
        u = un;
        v = vn;
        w = wn;
    }
    // the look-ahead stopped (or the queues are empty): take the next tile now
    t = uniform(claim_tile(P.q, P.deal, P.ctl, st));
    }
    finish_launch(P.ctl, wave_oob);
}

// Sum of the per-tile loss sums in a fixed order (one workgroup of
// kLossThreads): thread k adds tiles k, k + kLossThreads, ... in turn
// (loaded eight at a time, so that the loads overlap), then the wavefront
// butterfly, then the wavefronts in order. The same bits on every launch.
constexpr int kLossThreads = 1024;
__global__ __launch_bounds__(kLossThreads) void loss_sum_kernel(const double* tile_loss, int64_t n, double* loss) {
    __shared__ double s_part[kLossThreads / kWave];
    double s = 0.0;
    for (int64_t i0 = threadIdx.x; i0 < n; i0 += 8 * (int64_t)kLossThreads) {
        double x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t i = i0 + (int64_t)k * kLossThreads;
            x[k] = i < n ? tile_loss[i] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) s += x[k];
    }
    s = wave_sum_f64(s);
    if (lane_id() == 0) s_part[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double total = 0.0;
        for (int k = 0; k < kLossThreads / kWave; ++k) total += s_part[k];
        *loss = total;
    }
}

// First tap (y0 << 16 | x0) of the visibility at each position of the work
// order, or kNoStart when it is out of range: plan-time input for cutting
// tiles whose cells fit a staging box.
__global__ void start_cells_kernel(Problem pr, int64_t n, uint32_t* start) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t i = pr.perm ? (int64_t)pr.perm[p] : p;
    int32_t cell = 0, tab = 0, ow = 0, x0 = 0, y0 = 0;
    start[p] = vis_coords(pr, i, cell, tab, ow, x0, y0) ? ((uint32_t)y0 << 16) | (uint32_t)x0 : kNoStart;
}

__global__ void expand_tiles_kernel(const Tile* tiles, int64_t n_tiles, const uint32_t* const* perms,
                                    uint32_t* tile_vis) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_tiles * kMaxNb) return;
    const Tile tl = tiles[k / kMaxNb];
    const int j = (int)(k % kMaxNb);
    const int64_t pos = tl.begin + (j < tl.count ? j : 0);
    const uint32_t* perm = perms ? perms[tl.problem] : nullptr;
    tile_vis[k] = perm ? perm[pos] : (uint32_t)pos;
}

__global__ void set_f64_kernel(double* p, double v) {
    if (threadIdx.x == 0) *p = v;
}

__global__ void zero_kernel(float4* p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

template <int G, int F, int V>
hipError_t launch_degrid_t(const LaunchParams& p, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((degrid_kernel<G, F, kVariants[V].box, kVariants[V].nb, kVariants[V].deep, kVariants[V].d1>),
                       dim3(blocks),
                       dim3(kBlockThreads), 0, s, p);
    return hipGetLastError();
}

template <int G, int F, int V>
hipError_t occ_degrid_t(int* n) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        n, degrid_kernel<G, F, kVariants[V].box, kVariants[V].nb, kVariants[V].deep, kVariants[V].d1>, kBlockThreads,
        0);
}

template <int G, int F>
hipError_t launch_degrid_v(const LaunchParams& p, int variant, int blocks, hipStream_t s) {
    switch (variant) {
        case 0: return launch_degrid_t<G, F, 0>(p, blocks, s);
        case 1: return launch_degrid_t<G, F, 1>(p, blocks, s);
        case 2: return launch_degrid_t<G, F, 2>(p, blocks, s);
        case 3: return launch_degrid_t<G, F, 3>(p, blocks, s);
        case 4: return launch_degrid_t<G, F, 4>(p, blocks, s);
        case 5: return launch_degrid_t<G, F, 5>(p, blocks, s);
        case 6: return launch_degrid_t<G, F, 6>(p, blocks, s);
        default: return hipErrorInvalidValue;
    }
}

template <int G, int F>
hipError_t occ_degrid_v(int variant, int* n) {
    switch (variant) {
        case 0: return occ_degrid_t<G, F, 0>(n);
        case 1: return occ_degrid_t<G, F, 1>(n);
        case 2: return occ_degrid_t<G, F, 2>(n);
        case 3: return occ_degrid_t<G, F, 3>(n);
        case 4: return occ_degrid_t<G, F, 4>(n);
        case 5: return occ_degrid_t<G, F, 5>(n);
        case 6: return occ_degrid_t<G, F, 6>(n);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int degrid_variant_count() { return kNumVariants; }
int degrid_variant_box_bytes(int variant) {
    return (variant >= 0 && variant < kNumVariants) ? kVariants[variant].box : -1;
}
int degrid_variant_max_nb(int variant) {
    return (variant >= 0 && variant < kNumVariants) ? kVariants[variant].nb : -1;
}
bool degrid_variant_any_depth(int variant) {
    return variant >= 0 && variant < kNumVariants && (kVariants[variant].deep || kVariants[variant].d1);
}

hipError_t launch_degrid(const LaunchParams& params, int grid_kind, int gcf_kind, int variant,
                         int blocks, hipStream_t stream) {
    LaunchParams p = params;
    p.deal = deal_static(p.q, blocks, kWavesPerBlock);
    switch (grid_kind * 3 + gcf_kind) {
        case kGridC64 * 3 + kGcfF32: return launch_degrid_v<kGridC64, kGcfF32>(p, variant, blocks, stream);
        case kGridC64 * 3 + kGcfF16: return launch_degrid_v<kGridC64, kGcfF16>(p, variant, blocks, stream);
        case kGridC64 * 3 + kGcfBF16: return launch_degrid_v<kGridC64, kGcfBF16>(p, variant, blocks, stream);
        case kGridCBF16 * 3 + kGcfF32: return launch_degrid_v<kGridCBF16, kGcfF32>(p, variant, blocks, stream);
        case kGridCBF16 * 3 + kGcfF16: return launch_degrid_v<kGridCBF16, kGcfF16>(p, variant, blocks, stream);
        case kGridCBF16 * 3 + kGcfBF16: return launch_degrid_v<kGridCBF16, kGcfBF16>(p, variant, blocks, stream);
        case kGridCF16 * 3 + kGcfF32: return launch_degrid_v<kGridCF16, kGcfF32>(p, variant, blocks, stream);
        case kGridCF16 * 3 + kGcfF16: return launch_degrid_v<kGridCF16, kGcfF16>(p, variant, blocks, stream);
        case kGridCF16 * 3 + kGcfBF16: return launch_degrid_v<kGridCF16, kGcfBF16>(p, variant, blocks, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t degrid_kernel_occupancy(int grid_kind, int gcf_kind, int variant, int* n) {
    switch (grid_kind * 3 + gcf_kind) {
        case kGridC64 * 3 + kGcfF32: return occ_degrid_v<kGridC64, kGcfF32>(variant, n);
        case kGridC64 * 3 + kGcfF16: return occ_degrid_v<kGridC64, kGcfF16>(variant, n);
        case kGridC64 * 3 + kGcfBF16: return occ_degrid_v<kGridC64, kGcfBF16>(variant, n);
        case kGridCBF16 * 3 + kGcfF32: return occ_degrid_v<kGridCBF16, kGcfF32>(variant, n);
        case kGridCBF16 * 3 + kGcfF16: return occ_degrid_v<kGridCBF16, kGcfF16>(variant, n);
        case kGridCBF16 * 3 + kGcfBF16: return occ_degrid_v<kGridCBF16, kGcfBF16>(variant, n);
        case kGridCF16 * 3 + kGcfF32: return occ_degrid_v<kGridCF16, kGcfF32>(variant, n);
        case kGridCF16 * 3 + kGcfF16: return occ_degrid_v<kGridCF16, kGcfF16>(variant, n);
        case kGridCF16 * 3 + kGcfBF16: return occ_degrid_v<kGridCF16, kGcfBF16>(variant, n);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_start_cells(const Problem& pr, int64_t n, uint32_t* start, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(start_cells_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, pr, n, start);
    return hipGetLastError();
}

hipError_t launch_expand_tiles(const Tile* tiles, int64_t n_tiles, const uint32_t* const* perms,
                               uint32_t* tile_vis, hipStream_t stream) {
    if (n_tiles <= 0) return hipSuccess;
    const int64_t n = n_tiles * kMaxNb;
    hipLaunchKernelGGL(expand_tiles_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, tiles, n_tiles,
                       perms, tile_vis);
    return hipGetLastError();
}

hipError_t launch_loss_sum(const double* tile_loss, int64_t n_tiles, double* loss, hipStream_t stream) {
    hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(kLossThreads), 0, stream, tile_loss, n_tiles, loss);
    return hipGetLastError();
}

hipError_t launch_set_f64(double* p, double v, hipStream_t stream) {
    hipLaunchKernelGGL(set_f64_kernel, dim3(1), dim3(64), 0, stream, p, v);
    return hipGetLastError();
}

hipError_t launch_zero(void* ptr, int64_t bytes, hipStream_t stream) {
    if (bytes <= 0) return hipSuccess;
    if (bytes % 16 != 0) return hipErrorInvalidValue;
    const int64_t n = bytes / 16;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, static_cast<float4*>(ptr), n);
    return hipGetLastError();
}

}  // namespace dg
