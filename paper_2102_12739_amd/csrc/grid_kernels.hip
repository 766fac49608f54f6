// gfx950 kernels for gridding, the adjoint of 3D degridding (the transpose
// of the sum in Section 2): the tile kernel with an LDS staging box, the
// owner-computes kernel over plan-time output blocks, and its fix-up pass.
#include "dg_device.h"

namespace dg {
namespace {

// ---------------------------------------------------------------------------
// Adjoint (gridding) kernel
// ---------------------------------------------------------------------------
//
// The transpose of degridding: every in-range visibility V adds
// G_w[o_w][t_w] * G_uv[o_v][o_u][t_v][t_u] * V to the cell (y + t_v, x + t_u,
// z + t_w). Lanes map onto the 8 x 8 (t_v, t_u) taps as in the gather. When
// the tile's cells fit the wavefront's LDS box, contributions are summed
// there first (plain read-modify-write: a visibility's taps are distinct
// cells and LDS operations of one wavefront run in order) and the box is added to the output once
// with global float atomics; otherwise each contribution is a global atomic.

// V times the four G_w taps of one visibility, interleaved (re, im).
struct WeightedVis {
    float c[8];
};

template <int F, int BOX, int NB>
__global__ __launch_bounds__(kBlockThreads) void grid_adjoint_kernel(LaunchParams P) {
    static_assert(NB % 8 == 0 && NB <= kMaxNb, "tile size");
    constexpr int kBoxBytes = BOX > 0 ? BOX : 16;
    constexpr uint32_t kCell = kSupportW * 8;   // complex64 cell of 4 w values
    __shared__ __attribute__((aligned(16))) char s_box[kWavesPerBlock][kBoxBytes];

    const int lane = lane_id();
    const int wv = (int)(threadIdx.x / kWave);
    QueueState st{xcc_id() % P.q.n_queues, 0};
    uint32_t wave_oob = 0;

    int t = pop_tile(P.q, P.ctl, st);
    while (t >= 0) {
        const Tile tc = load_tile(P.tiles, t);
        const int t_next = pop_tile(P.q, P.ctl, st);
        const Problem pr = P.probs ? load_problem(P.probs, tc.problem) : P.prob;
        const int count = tc.count;

        // Coordinate stage; lane j also forms G_w * V of visibility j.
        int32_t x0 = 0, y0 = 0, cell = 0, tab = 0, ow = 0;
        bool in_range = false;
        WeightedVis cw;
#pragma unroll
        for (int q = 0; q < 8; ++q) cw.c[q] = 0.0f;
        if (lane < count) {
            const int64_t i = P.tile_vis[(int64_t)t * kMaxNb + lane];
            in_range = vis_coords(pr, i, cell, tab, ow, x0, y0);
            if (in_range) {
                const float2 vv = static_cast<const float2*>(pr.vis)[i];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float gw = load_gcf<F>(pr.g_w, ow * kSupportW + k);
                    cw.c[2 * k] = gw * vv.x;
                    cw.c[2 * k + 1] = gw * vv.y;
                }
            }
        }
        wave_oob += (uint32_t)__popcll(__ballot(lane < count && !in_range));

        // G_uv weights of the whole tile (zero for out-of-range visibilities).
        const __amdgpu_buffer_rsrc_t rg = make_rsrc(pr.g_uv, pr.guv_bytes);
        const uint32_t lane_g = (uint32_t)lane * GcfTraits<F>::kBytes;
        const int g_off = in_range ? tab * (int)GcfTraits<F>::kBytes : (int)kOutOfRange;
        float gv[NB];
#pragma unroll
        for (int g0 = 0; g0 < NB; g0 += 8) {
            if (g0 < count) {
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    gv[g0 + k] = load_gcf_rsrc<F>(rg, (uint32_t)__builtin_amdgcn_readlane(g_off, g0 + k) + lane_g);
            }
        }

        bool staged = false;
        int bx0 = 0, by0 = 0, bw = 0, bh = 0, bp = 0;
        if (BOX > 0 && pr.n_w == kSupportW) {   // the box holds w 0..3 of each cell
            int bx1 = -1, by1 = -1;
            wave_bbox(in_range, x0, y0, bx0, by0, bx1, by1);
            if (bx1 >= 0) {
                bw = bx1 - bx0 + kSupportUV;
                bh = by1 - by0 + kSupportUV;
                bp = bw + ((8 - bw) & 15);
                staged = (uint32_t)(bp * bh) * kCell <= (uint32_t)BOX;
            }
        }

        float* out = static_cast<float*>(pr.grid_out) + 2 * (int64_t)tc.sub * pr.n_v * pr.n_u * pr.n_w;
        const int tv = lane >> 3, tu = lane & 7;
        if (staged) {
            char* box = s_box[wv];
            const int n_chunks = bp * bh * (int)(kCell / 16);
            for (int c = lane; c < n_chunks; c += kWave)
                *reinterpret_cast<uint4*>(box + (uint32_t)c * 16u) = make_uint4(0u, 0u, 0u, 0u);
            wave_lds_sync();
            const int rel = in_range ? ((y0 - by0) * bp + (x0 - bx0)) : 0;
            const uint32_t lane_box = ((uint32_t)tv * bp + tu) * kCell;
#pragma unroll
            for (int g0 = 0; g0 < NB; g0 += 8) {
                if (g0 < count) {
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const int j = g0 + k;
                        const uint32_t base = lane_box + (uint32_t)__builtin_amdgcn_readlane(rel, j) * kCell;
                        // distinct cells per visibility, in-order LDS: plain
                        // read-modify-write is exact
                        float4* dst = reinterpret_cast<float4*>(box + base);
                        float c[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q)
                            c[q] = gv[j] * __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cw.c[q]), j));
                        float4 a = dst[0], b = dst[1];
                        a.x += c[0]; a.y += c[1]; a.z += c[2]; a.w += c[3];
                        b.x += c[4]; b.y += c[5]; b.z += c[6]; b.w += c[7];
                        dst[0] = a;
                        dst[1] = b;
                    }
                }
            }
            wave_lds_sync();
            // Add the box to the output row by row: a box row is bw * 8
            // consecutive floats both in LDS and in the subgrid, so lane l of
            // a step adds float l and one atomic instruction covers 256
            // contiguous bytes.
            const int row_floats = bw * (int)(kCell / 4);
            const float* lds_rows = reinterpret_cast<const float*>(box);
            for (int row = 0; row < bh; ++row) {
                float* dst = out + 2 * ((int64_t)((by0 + row) * pr.n_u + bx0) * pr.n_w);
                const float* src = lds_rows + (uint32_t)row * bp * (kCell / 4);
                for (int f = lane; f < row_floats; f += kWave) {
                    const float v = src[f];
                    if (v != 0.0f) unsafeAtomicAdd(dst + f, v);
                }
            }
            wave_lds_sync();
        } else {
            const int64_t lane_cell = (int64_t)(tv * pr.n_u + tu) * pr.n_w;
#pragma unroll
            for (int g0 = 0; g0 < NB; g0 += 8) {
                if (g0 < count) {
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const int j = g0 + k;
                        const int cj = __builtin_amdgcn_readlane(in_range ? cell : -1, j);
                        if (cj >= 0) {
                            float* dst = out + 2 * ((int64_t)cj + lane_cell);
#pragma unroll
                            for (int q = 0; q < 8; ++q) {
                                const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cw.c[q]), j));
                                unsafeAtomicAdd(dst + q, gv[j] * c);
                            }
                        }
                    }
                }
            }
        }
        t = t_next;
    }
    finish_launch(P.ctl, wave_oob);
}

// ---------------------------------------------------------------------------
// Owner-computes adjoint
// ---------------------------------------------------------------------------
//
// A wavefront owns one output block of kOwnerBlock x kOwnerBlock cells of
// one subgrid. It walks the block's visibility list (made at plan time from
// the sorted coordinates), adds each visibility's taps that fall inside the
// block to an LDS copy of the block, and writes the block once with plain
// stores: no global atomics, and the sums do not depend on timing. A listed
// visibility whose first tap at run time differs from the plan's is skipped
// here; the fix-up pass adds those with atomics.

typedef const __attribute__((address_space(4))) OwnerBlock* ConstOwnerBlockPtr;

// This lane's G_uv weights of items j0 .. j0+7, whose table offsets lane j
// holds in g_off (kOutOfRange for skipped items: the load returns zero).
template <int F>
__device__ __forceinline__ void load_weights8(float* g, int g_off, int j0, __amdgpu_buffer_rsrc_t rg,
                                              uint32_t lane_g) {
#pragma unroll
    for (int k = 0; k < 8; ++k)
        g[k] = load_gcf_rsrc<F>(rg, (uint32_t)__builtin_amdgcn_readlane(g_off, j0 + k) + lane_g);
}

// Marks eight values as used here, so that their loads stay where they were
// issued (one group ahead) instead of being moved next to each use.
__device__ __forceinline__ void pin8(float* g) {
    asm volatile("" ::"v"(g[0]), "v"(g[1]), "v"(g[2]), "v"(g[3]), "v"(g[4]), "v"(g[5]), "v"(g[6]), "v"(g[7]));
}

// First tap of a skipped item, relative to the block: far enough outside
// that no lane's tap lands in the block.
constexpr int kSkipX = -1024;

template <int F>
__global__ __launch_bounds__(kBlockThreads) void grid_owner_kernel(OwnerParams P) {
    constexpr int B = kOwnerBlock;
    constexpr int kCellFloats = kSupportW * 2;          // complex64 x 4 w
    constexpr int kRowFloats = B * kCellFloats;         // floats of one block row
    constexpr int kRowVec = kRowFloats / 4;             // float4 per block row
    // LDS copy of the block in two planes of 16-byte slots: plane 0 holds w 0-1
    // of every cell, plane 1 (kPlane floats further) w 2-3. Cell (cy, cx) sits
    // in slot cy * B + (cx ^ 8 * (cy & 1)): the eight lanes of a tap row then
    // touch one 128-byte span (at most two runs) of a plane, and the rows of
    // odd and even cy that one LDS cycle serves fall on opposite halves of
    // the banks (no padding needed).
    constexpr int kPlane = B * B * 4;
    __shared__ __attribute__((aligned(16))) float s_box[kWavesPerBlock][2 * kPlane];
    auto slot_of = [](int cy, int cx) { return cy * B + (cx ^ ((cy & 1) << 3)); };

    const int lane = lane_id();
    const int wv = (int)(threadIdx.x / kWave);
    const int tv = lane >> 3, tu = lane & 7;
    TileClaims st = start_claims(P.q, P.deal, wv);
    const Problem& pr = P.prob;
    const __amdgpu_buffer_rsrc_t rg = make_rsrc(pr.g_uv, pr.guv_bytes);
    const uint32_t lane_g = (uint32_t)lane * GcfTraits<F>::kBytes;
    const int64_t row_floats = 2 * (int64_t)pr.n_u * pr.n_w;   // floats per subgrid row
    float* box = s_box[wv];
    // the next block is taken at the start of a block only while its queue
    // holds more blocks than wavefronts per queue (else after the block)
    const int waves_per_queue = ((int)gridDim.x * kWavesPerBlock + P.q.n_queues - 1) / P.q.n_queues;

    int t = uniform(claim_tile(P.q, P.deal, P.ctl, st));
    while (t >= 0) {
        const ConstOwnerBlockPtr pb = (ConstOwnerBlockPtr)uniform_u64((uint64_t)P.blocks) + t;
        const int64_t begin = pb->begin;
        const int count = pb->count;
        const int blk = pb->block;
        const bool ahead = queue_end(P.q, st.q) - t > waves_per_queue;
        const int t_next = uniform(ahead ? claim_tile(P.q, P.deal, P.ctl, st) : -1);
        const int per_sub = P.nby * P.nbx;
        const int s = blk / per_sub;
        const int by = (blk - s * per_sub) / P.nbx;
        const int bx = blk - s * per_sub - by * P.nbx;
        float* out = static_cast<float*>(pr.grid_out) +
                     2 * ((int64_t)s * pr.cells_per_sub + ((int64_t)(by * B) * pr.n_u + bx * B) * pr.n_w);

        // the block's current contents (or zeros), 16 bytes per lane and step:
        // chunk col of a row is half (col & 1) of cell col / 2
#pragma unroll
        for (int f = lane; f < B * kRowVec; f += kWave) {
            const int row = f / kRowVec, col = f - row * kRowVec;
            *reinterpret_cast<float4*>(box + (col & 1) * kPlane + slot_of(row, col >> 1) * 4) =
                P.accumulate ? *reinterpret_cast<const float4*>(out + row * row_floats + col * 4)
                             : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        wave_lds_sync();

        for (int c0 = 0; c0 < count; c0 += kWave) {
            // Lane j prepares item c0 + j: its first tap relative to the block
            // (y in the high, x in the low 16 bits), its G_uv offset and
            // G_w[o_w][t] * V; the whole wavefront reads them with v_readlane.
            int32_t xy = kSkipX & 0xFFFF;
            int32_t g_off = (int)kOutOfRange;
            float c[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) c[q] = 0.0f;
            if (c0 + lane < count) {
                const int64_t i = P.items[begin + c0 + lane];
                const double* uv = pr.uvw + 3 * i;
                int32_t cell = 0, tab = 0, ow = 0, x0 = 0, y0 = 0;
                if (coords_from(pr, uv[0], uv[1], uv[2], cell, tab, ow, x0, y0) &&
                    (((uint32_t)y0 << 16) | (uint32_t)x0) == P.plan_start[i]) {
                    xy = (int32_t)((uint32_t)(y0 - by * B) << 16) | ((x0 - bx * B) & 0xFFFF);
                    g_off = tab * (int)GcfTraits<F>::kBytes;
                    const float2 vv = static_cast<const float2*>(pr.vis)[i];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const float gw = load_gcf<F>(pr.g_w, ow * kSupportW + k);
                        c[2 * k] = gw * vv.x;
                        c[2 * k + 1] = gw * vv.y;
                    }
                }
            }
            const int n = min(kWave, count - c0);
            // G_uv weights one group of eight ahead (items past n are skipped
            // ones, whose loads return zero)
            float g[2][8];
            load_weights8<F>(g[0], g_off, 0, rg, lane_g);
#pragma unroll
            for (int j0 = 0; j0 < kWave; j0 += 8) {
                if (j0 < n) {
                    float* gc = g[(j0 / 8) & 1];
                    if (j0 + 8 < kWave) load_weights8<F>(g[((j0 / 8) + 1) & 1], g_off, j0 + 8, rg, lane_g);
                    pin8(gc);
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const int xyj = __builtin_amdgcn_readlane(xy, j0 + k);
                        const int cy = (xyj >> 16) + tv;
                        const int cx = (int)(int16_t)(xyj & 0xFFFF) + tu;
                        if ((unsigned)cy < (unsigned)B && (unsigned)cx < (unsigned)B) {
                            float cj[8];
#pragma unroll
                            for (int q = 0; q < 8; ++q)
                                cj[q] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(c[q]), j0 + k));
                            // the taps of one visibility are distinct cells and
                            // LDS operations of a wavefront run in order, so a
                            // plain read-modify-write is exact
                            float4* dst0 = reinterpret_cast<float4*>(box + slot_of(cy, cx) * 4);
                            float4* dst1 = reinterpret_cast<float4*>(box + kPlane + slot_of(cy, cx) * 4);
                            float4 a = *dst0, b = *dst1;
                            a.x += gc[k] * cj[0]; a.y += gc[k] * cj[1];
                            a.z += gc[k] * cj[2]; a.w += gc[k] * cj[3];
                            b.x += gc[k] * cj[4]; b.y += gc[k] * cj[5];
                            b.z += gc[k] * cj[6]; b.w += gc[k] * cj[7];
                            *dst0 = a;
                            *dst1 = b;
                        }
                    }
                }
            }
        }
        wave_lds_sync();

        // write the block
#pragma unroll
        for (int f = lane; f < B * kRowVec; f += kWave) {
            const int row = f / kRowVec, col = f - row * kRowVec;
            *reinterpret_cast<float4*>(out + row * row_floats + col * 4) =
                *reinterpret_cast<const float4*>(box + (col & 1) * kPlane + slot_of(row, col >> 1) * 4);
        }
        wave_lds_sync();
        t = ahead ? t_next : uniform(claim_tile(P.q, P.deal, P.ctl, st));
    }
    finish_launch(P.ctl, 0u);
}

// Visibilities the owner pass skipped (first tap differs from the plan's),
// added with atomics by whole wavefronts, and the out-of-range count. Each
// lane loads the coordinates and plan starts of kFixupPerLane visibilities
// (64 apart) before testing any of them, so one pass over the coordinates
// waits out one memory latency per kFixupPerLane visibilities.
constexpr int kFixupPerLane = 4;

template <int F>
__global__ __launch_bounds__(kBlockThreads) void grid_fixup_kernel(Problem pr, const int64_t* offsets,
                                                                   int64_t n_sub, int64_t n_vis,
                                                                   const uint32_t* plan_start, Ctl* ctl) {
    const int lane = lane_id();
    const int tv = lane >> 3, tu = lane & 7;
    const int64_t lane_cell = (int64_t)(tv * pr.n_u + tu) * pr.n_w;
    uint32_t wave_oob = 0;
    const int64_t n_waves = (int64_t)gridDim.x * kWavesPerBlock;
    const int64_t first = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    constexpr int64_t kSpan = (int64_t)kWave * kFixupPerLane;
    for (int64_t w0 = first * kSpan; w0 < n_vis; w0 += n_waves * kSpan) {
        double cu[kFixupPerLane], cv[kFixupPerLane], cw[kFixupPerLane];
        uint32_t ps[kFixupPerLane];
        // branch-free loads (a lane past the end re-reads the last
        // visibility and ignores it), so all of them are in flight at once
#pragma unroll
        for (int k = 0; k < kFixupPerLane; ++k) {
            int64_t i = w0 + k * kWave + lane;
            i = i < n_vis ? i : n_vis - 1;
            const double* uv = pr.uvw + 3 * i;
            cu[k] = uv[0];
            cv[k] = uv[1];
            cw[k] = uv[2];
            ps[k] = plan_start[i];
        }
#pragma unroll
        for (int k = 0; k < kFixupPerLane; ++k) {
            const int64_t i = w0 + k * kWave + lane;
            int32_t cell = 0, tab = 0, ow = 0, x0 = 0, y0 = 0;
            bool in_range = false, redo = false;
            if (i < n_vis) {
                in_range = coords_from(pr, cu[k], cv[k], cw[k], cell, tab, ow, x0, y0);
                redo = in_range && (((uint32_t)y0 << 16) | (uint32_t)x0) != ps[k];
            }
            wave_oob += (uint32_t)__popcll(__ballot(i < n_vis && !in_range));
            uint64_t mask = __ballot(redo);
            if (mask == 0) continue;
            // subgrid of each visibility to redo
            int64_t sub = 0;
            if (redo) {
                int64_t lo = 0, hi = n_sub;
                while (hi - lo > 1) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (offsets[mid] <= i) lo = mid; else hi = mid;
                }
                sub = lo;
            }
            float c[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) c[q] = 0.0f;
            if (redo) {
                const float2 vv = static_cast<const float2*>(pr.vis)[i];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float gw = load_gcf<F>(pr.g_w, ow * kSupportW + t);
                    c[2 * t] = gw * vv.x;
                    c[2 * t + 1] = gw * vv.y;
                }
            }
            while (mask) {
                const int j = __builtin_ctzll(mask);
                mask &= mask - 1;
                const int64_t sj = ((int64_t)__builtin_amdgcn_readlane((int)(sub >> 32), j) << 32) |
                                   (uint32_t)__builtin_amdgcn_readlane((int)sub, j);
                const int cj = __builtin_amdgcn_readlane(cell, j);
                const int tj = __builtin_amdgcn_readlane(tab, j);
                const float g = load_gcf<F>(pr.g_uv, (int64_t)tj + lane);
                float* dst = static_cast<float*>(pr.grid_out) + 2 * (sj * pr.cells_per_sub + cj + lane_cell);
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    unsafeAtomicAdd(dst + q, g * __int_as_float(__builtin_amdgcn_readlane(__float_as_int(c[q]), j)));
            }
        }
    }
    finish_launch<true>(ctl, wave_oob);
}

}  // namespace

int adjoint_variant_count() { return kNumVariants; }

template <int F, int V>
hipError_t launch_adjoint_t(const LaunchParams& p, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((grid_adjoint_kernel<F, kVariants[V].box, kVariants[V].nb>), dim3(blocks), dim3(kBlockThreads),
                       0, s, p);
    return hipGetLastError();
}

template <int F, int V>
hipError_t occ_adjoint_t(int* n) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        n, grid_adjoint_kernel<F, kVariants[V].box, kVariants[V].nb>, kBlockThreads, 0);
}

template <int F>
hipError_t launch_adjoint_v(const LaunchParams& p, int variant, int blocks, hipStream_t s) {
    switch (variant) {
        case 0: return launch_adjoint_t<F, 0>(p, blocks, s);
        case 1: return launch_adjoint_t<F, 1>(p, blocks, s);
        case 2: return launch_adjoint_t<F, 2>(p, blocks, s);
        case 3: return launch_adjoint_t<F, 3>(p, blocks, s);
        case 4: return launch_adjoint_t<F, 4>(p, blocks, s);
        case 5: return launch_adjoint_t<F, 5>(p, blocks, s);
        case 6: return launch_adjoint_t<F, 6>(p, blocks, s);
        default: return hipErrorInvalidValue;
    }
}

template <int F>
hipError_t occ_adjoint_v(int variant, int* n) {
    switch (variant) {
        case 0: return occ_adjoint_t<F, 0>(n);
        case 1: return occ_adjoint_t<F, 1>(n);
        case 2: return occ_adjoint_t<F, 2>(n);
        case 3: return occ_adjoint_t<F, 3>(n);
        case 4: return occ_adjoint_t<F, 4>(n);
        case 5: return occ_adjoint_t<F, 5>(n);
        case 6: return occ_adjoint_t<F, 6>(n);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_grid_adjoint(const LaunchParams& p, int gcf_kind, int variant, int blocks,
                               hipStream_t stream) {
    if (gcf_kind == kGcfF32) return launch_adjoint_v<kGcfF32>(p, variant, blocks, stream);
    if (gcf_kind == kGcfF16) return launch_adjoint_v<kGcfF16>(p, variant, blocks, stream);
    if (gcf_kind == kGcfBF16) return launch_adjoint_v<kGcfBF16>(p, variant, blocks, stream);
    return hipErrorInvalidValue;
}

hipError_t adjoint_kernel_occupancy(int gcf_kind, int variant, int* n) {
    if (gcf_kind == kGcfF32) return occ_adjoint_v<kGcfF32>(variant, n);
    if (gcf_kind == kGcfF16) return occ_adjoint_v<kGcfF16>(variant, n);
    if (gcf_kind == kGcfBF16) return occ_adjoint_v<kGcfBF16>(variant, n);
    return hipErrorInvalidValue;
}

hipError_t launch_grid_owner(const OwnerParams& params, int gcf_kind, int blocks, hipStream_t stream) {
    OwnerParams p = params;
    p.deal = deal_static(p.q, blocks, kWavesPerBlock);
    if (gcf_kind == kGcfF32)
        hipLaunchKernelGGL((grid_owner_kernel<kGcfF32>), dim3(blocks), dim3(kBlockThreads), 0, stream, p);
    else if (gcf_kind == kGcfF16)
        hipLaunchKernelGGL((grid_owner_kernel<kGcfF16>), dim3(blocks), dim3(kBlockThreads), 0, stream, p);
    else if (gcf_kind == kGcfBF16)
        hipLaunchKernelGGL((grid_owner_kernel<kGcfBF16>), dim3(blocks), dim3(kBlockThreads), 0, stream, p);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t owner_kernel_occupancy(int gcf_kind, int* n) {
    if (gcf_kind == kGcfF32)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, grid_owner_kernel<kGcfF32>, kBlockThreads, 0);
    if (gcf_kind == kGcfF16)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, grid_owner_kernel<kGcfF16>, kBlockThreads, 0);
    if (gcf_kind == kGcfBF16)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, grid_owner_kernel<kGcfBF16>, kBlockThreads, 0);
    return hipErrorInvalidValue;
}

hipError_t launch_grid_fixup(const Problem& pr, const int64_t* vis_offsets, int64_t n_sub, int64_t n_vis,
                             const uint32_t* plan_start, Ctl* ctl, int gcf_kind, int max_blocks,
                             hipStream_t stream) {
    const int64_t per_block = (int64_t)kBlockThreads * kFixupPerLane;
    int64_t blocks = (n_vis + per_block - 1) / per_block;
    blocks = blocks < 1 ? 1 : (blocks > max_blocks ? max_blocks : blocks);
    if (gcf_kind == kGcfF32)
        hipLaunchKernelGGL((grid_fixup_kernel<kGcfF32>), dim3((unsigned)blocks), dim3(kBlockThreads), 0, stream, pr,
                           vis_offsets, n_sub, n_vis, plan_start, ctl);
    else if (gcf_kind == kGcfF16)
        hipLaunchKernelGGL((grid_fixup_kernel<kGcfF16>), dim3((unsigned)blocks), dim3(kBlockThreads), 0, stream, pr,
                           vis_offsets, n_sub, n_vis, plan_start, ctl);
    else if (gcf_kind == kGcfBF16)
        hipLaunchKernelGGL((grid_fixup_kernel<kGcfBF16>), dim3((unsigned)blocks), dim3(kBlockThreads), 0, stream, pr,
                           vis_offsets, n_sub, n_vis, plan_start, ctl);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace dg
