// gfx950 kernels for 3D degridding and its adjoint (gridding).
//
// Degridding (Section 2 of the paper) forms each visibility as the sum of
// the 8 x 8 x 4 subgrid neighbourhood that starts at g = [x, y, z], weighted
// by G_w[o_w][t_w] * G_uv[o_v][o_u][t_v][t_u]. It is a gather with about
// 0.5 flop per byte, so these kernels are built around memory access, not
// matrix cores:
//
//  * persistent workgroups drain a list of tiles (n_b consecutive
//    visibilities of one subgrid) from per-XCD queues, stealing from the
//    other queues when their own is empty (this replaces the launch grid of
//    Eq. (1));
//  * each wavefront takes one tile. Its coordinate stage computes, one lane
//    per visibility, the start cell and the oversample indices in float64
//    (exact: the oversampling is a power of two) and stages them in LDS;
//  * the gather maps the 64 lanes onto the 8 x 8 (t_v, t_u) taps. Each lane
//    reads the 4 w values of its tap (32 contiguous bytes for complex64; one
//    v-row of the neighbourhood is 256 contiguous bytes) and its G_uv weight
//    (one coalesced 256-byte block per visibility). Loads go through buffer
//    resources, so the hardware bounds check turns any offset outside the
//    subgrid into zeros;
//  * eight visibilities are reduced across the wavefront together: two
//    permlane swaps (lanes 32 apart, then 16 apart) and one DPP step halve the
//    number of live partial sums at each level, then three DPP steps finish
//    the 8-lane sums (Section 2 uses a warp reduction after a v-axis
//    accumulation; here the reduction is shared between visibilities);
//  * results are staged in LDS and written as one contiguous block per tile
//    (Section 2 stages outputs in shared memory and writes them in bulk).
#include "dg_internal.h"

#include <hip/hip_fp16.h>

namespace dg {
namespace {

constexpr int32_t kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit dwords (gfx9 family)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRsrcWord3);
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// XCD the wavefront runs on (hardware register XCC_ID, bits 3:0).
__device__ __forceinline__ int xcc_id() {
    return (int)(__builtin_amdgcn_s_getreg((3 << 11) | 20) & 7);
}

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Copy of a value that the compiler knows to be the same on every lane (it
// lives in scalar registers). Used for the per-tile descriptors loaded from
// memory, so that addresses and buffer resources built from them stay scalar.
template <class T>
__device__ __forceinline__ T uniform_copy(const T& x) {
    static_assert(sizeof(T) % 4 == 0, "word-sized types only");
    uint32_t w[sizeof(T) / 4];
    __builtin_memcpy(w, &x, sizeof(T));
#pragma unroll
    for (unsigned i = 0; i < sizeof(T) / 4; ++i) w[i] = (uint32_t)__builtin_amdgcn_readfirstlane((int)w[i]);
    T y;
    __builtin_memcpy(&y, w, sizeof(T));
    return y;
}

// Orders this wavefront's LDS accesses around a hand-off between its lanes.
// LDS operations of one wavefront execute in order; this keeps the compiler
// from moving accesses across the hand-off.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// Tile queue
// ---------------------------------------------------------------------------

struct QueueState {
    int q;       // queue currently drained
    int tried;   // queues found empty so far
};

// Next tile for this wavefront, or -1 once every queue is empty.
__device__ __forceinline__ int pop_tile(const QueueSpec& qs, Ctl* ctl, QueueState& st) {
    while (st.tried < qs.n_queues) {
        uint32_t idx = 0;
        if (lane_id() == 0) idx = atomicAdd(&ctl->cursor[st.q].v[0], 1u);
        idx = (uint32_t)uniform((int)idx);
        const int t = qs.begin[st.q] + (int)idx;
        if (t < qs.end[st.q]) return t;
        st.q = (st.q + 1 == qs.n_queues) ? 0 : st.q + 1;
        st.tried++;
    }
    return -1;
}

// Adds this wavefront's out-of-range count; the last workgroup of the launch
// publishes the launch total and resets cursors and counters for the next.
__device__ __forceinline__ void finish_launch(Ctl* ctl, uint32_t wave_oob) {
    auto* oob = reinterpret_cast<unsigned long long*>(&ctl->oob.v[0]);
    if (lane_id() == 0 && wave_oob != 0u) atomicAdd(&oob[0], (unsigned long long)wave_oob);
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t prev = atomicAdd(&ctl->done.v[0], 1u);
        if (prev == gridDim.x - 1) {
            __threadfence();
            const unsigned long long total = atomicExch(&oob[0], 0ull);
            atomicExch(&oob[1], total);
            for (int q = 0; q < kMaxQueues; ++q) atomicExch(&ctl->cursor[q].v[0], 0u);
            atomicExch(&ctl->done.v[0], 0u);
        }
    }
}

// ---------------------------------------------------------------------------
// Storage types
// ---------------------------------------------------------------------------

template <int G> struct GridTraits;
template <> struct GridTraits<kGridC64> {    // complex float32
    static constexpr uint32_t kElemBytes = 8;
    static constexpr int kWords = 8;         // 4 w values x (re, im)
};
template <> struct GridTraits<kGridCBF16> {  // complex bfloat16
    static constexpr uint32_t kElemBytes = 4;
    static constexpr int kWords = 4;
};
template <> struct GridTraits<kGridCF16> {   // complex float16
    static constexpr uint32_t kElemBytes = 4;
    static constexpr int kWords = 4;
};
// bytes of one (v, u) cell: its 4 w values
template <int G> constexpr uint32_t kCellBytes = GridTraits<G>::kElemBytes * kSupportW;

template <int G>
__device__ __forceinline__ void load_w4(__amdgpu_buffer_rsrc_t r, uint32_t off,
                                        uint32_t (&raw)[GridTraits<G>::kWords]) {
    if constexpr (G == kGridC64) {
        auto a = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        auto b = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16u, 0, 0);
        raw[0] = a[0]; raw[1] = a[1]; raw[2] = a[2]; raw[3] = a[3];
        raw[4] = b[0]; raw[5] = b[1]; raw[6] = b[2]; raw[7] = b[3];
    } else {
        auto a = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        raw[0] = a[0]; raw[1] = a[1]; raw[2] = a[2]; raw[3] = a[3];
    }
}

// Widen the 4 w values of one tap to float32 (re[t], im[t]).
template <int G>
__device__ __forceinline__ void widen_w4(const uint32_t (&raw)[GridTraits<G>::kWords],
                                         float (&re)[4], float (&im)[4]) {
    if constexpr (G == kGridC64) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            re[t] = __uint_as_float(raw[2 * t]);
            im[t] = __uint_as_float(raw[2 * t + 1]);
        }
    } else if constexpr (G == kGridCBF16) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            re[t] = __uint_as_float(raw[t] << 16);
            im[t] = __uint_as_float(raw[t] & 0xFFFF0000u);
        }
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const __half2 h = __builtin_bit_cast(__half2, raw[t]);
            re[t] = __low2float(h);
            im[t] = __high2float(h);
        }
    }
}

template <int F> struct GcfTraits;
template <> struct GcfTraits<kGcfF32> { static constexpr uint32_t kBytes = 4; };
template <> struct GcfTraits<kGcfF16> { static constexpr uint32_t kBytes = 2; };

template <int F>
__device__ __forceinline__ float load_gcf_rsrc(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    if constexpr (F == kGcfF32) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    } else {
        const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
        return __half2float(__builtin_bit_cast(__half, h));
    }
}

template <int F>
__device__ __forceinline__ float load_gcf(const void* table, int64_t idx) {
    if constexpr (F == kGcfF32) {
        return static_cast<const float*>(table)[idx];
    } else {
        return __half2float(static_cast<const __half*>(table)[idx]);
    }
}

// ---------------------------------------------------------------------------
// Coordinate stage (Section 2: start point g and oversampled GCF positions)
// ---------------------------------------------------------------------------

// Start cell offset (first tap, inside its subgrid) and table positions of
// visibility i. Per axis k = floor(c * os) in float64, which is exact for a
// power-of-two os; the cell is k / os, the oversample index k mod os, and the
// first tap sits W/2 - 1 cells below the cell. Returns false when the
// neighbourhood leaves the subgrid or the coordinate is not finite.
__device__ __forceinline__ bool coords_from(const Problem& pr, double u, double v, double w, int32_t& cell,
                                            int32_t& tab, int32_t& ow, int32_t& x_start, int32_t& y_start) {
    const bool ok = (u >= 3.0) & (u < pr.hi_u) & (v >= 3.0) & (v < pr.hi_v) &
                    (w >= 1.0) & (w < pr.hi_w);
    if (!ok) return false;
    const int os_uv = 1 << pr.log2_os_uv;
    const int os_w = 1 << pr.log2_os_w;
    const int ku = (int)(u * (double)os_uv);   // non-negative: truncation is floor
    const int kv = (int)(v * (double)os_uv);
    const int kw = (int)(w * (double)os_w);
    const int x0 = (ku >> pr.log2_os_uv) - (kSupportUV / 2 - 1);
    const int y0 = (kv >> pr.log2_os_uv) - (kSupportUV / 2 - 1);
    const int z0 = (kw >> pr.log2_os_w) - (kSupportW / 2 - 1);
    const int ou = ku & (os_uv - 1);
    const int ov = kv & (os_uv - 1);
    ow = kw & (os_w - 1);
    cell = (y0 * pr.n_u + x0) * pr.n_w + z0;
    tab = ((ov << pr.log2_os_uv) + ou) * (kSupportUV * kSupportUV);
    x_start = x0;
    y_start = y0;
    return true;
}

__device__ __forceinline__ bool vis_coords(const Problem& pr, int64_t i, int32_t& cell,
                                           int32_t& tab, int32_t& ow, int32_t& x_start, int32_t& y_start) {
    const double* c = pr.uvw + 3 * i;
    return coords_from(pr, c[0], c[1], c[2], cell, tab, ow, x_start, y_start);
}

// ---------------------------------------------------------------------------
// Cross-lane reduction of eight visibilities
// ---------------------------------------------------------------------------

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
constexpr int kDppQuadXor1 = 0xB1;       // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;       // quad_perm [2,3,0,1]
constexpr int kDppRowRor8 = 0x128;       // rotate by 8 within 16 lanes (= lane xor 8)
constexpr int kDppRowHalfMirror = 0x141; // lane j <-> 7 - j within 8 lanes

// x <- x + (x of the lane 32 away) for the half that keeps x, and the same
// for y on the other half: after the swap, lanes 0-31 hold x's pair sums and
// lanes 32-63 hold y's.
__device__ __forceinline__ float swap_add32(float x, float y) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Same with rows of 16 lanes: rows 0 and 2 keep x's sums, rows 1 and 3 y's.
__device__ __forceinline__ float swap_add16(float x, float y) {
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// In: p[k] = this lane's partial sum for visibility k (k = 0..7).
// Out: p[0] on lane l = full 64-lane sum for visibility l >> 3.
__device__ __forceinline__ void reduce8(float (&p)[8]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) p[k] = swap_add32(p[k], p[k + 4]);   // vis k + 4*bit5
#pragma unroll
    for (int k = 0; k < 2; ++k) p[k] = swap_add16(p[k], p[k + 2]);   // + 2*bit4
    const bool hi = (lane_id() & 8) != 0;
    const float keep = hi ? p[1] : p[0];
    const float give = hi ? p[0] : p[1];
    float s = keep + dpp<kDppRowRor8>(give);                           // + bit3
    s += dpp<kDppRowHalfMirror>(s);
    s += dpp<kDppQuadXor2>(s);
    s += dpp<kDppQuadXor1>(s);
    p[0] = s;
}

// ---------------------------------------------------------------------------
// Degrid kernel
// ---------------------------------------------------------------------------

__device__ __forceinline__ int wave_min(int x) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x = min(x, __shfl_xor(x, m));
    return x;
}
__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x = max(x, __shfl_xor(x, m));
    return x;
}

// Scalar-cache view of read-only data: loads through it with a wave-uniform
// address become scalar loads.
typedef const __attribute__((address_space(4))) float* ConstF32Ptr;
typedef const __attribute__((address_space(4))) uint32_t* ConstU32Ptr;
typedef const __attribute__((address_space(4))) Tile* ConstTilePtr;
typedef const __attribute__((address_space(4))) Problem* ConstProblemPtr;

__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ Tile load_tile(const Tile* tiles, int t) {
    const ConstTilePtr p = (ConstTilePtr)uniform_u64((uint64_t)tiles) + t;
    Tile x;
    x.begin = p->begin;
    x.sub = p->sub;
    x.count = p->count;
    x.problem = p->problem;
    return x;
}

// The fields of a batch problem the degrid kernel uses, read through the
// scalar cache.
__device__ __forceinline__ Problem load_problem(const Problem* probs, int i) {
    const ConstProblemPtr p = (ConstProblemPtr)uniform_u64((uint64_t)probs) + i;
    Problem x{};
    x.subgrids = p->subgrids;
    x.g_uv = p->g_uv;
    x.g_w = p->g_w;
    x.uvw = p->uvw;
    x.vis = p->vis;
    x.n_v = p->n_v;
    x.n_u = p->n_u;
    x.n_w = p->n_w;
    x.log2_os_uv = p->log2_os_uv;
    x.log2_os_w = p->log2_os_w;
    x.guv_bytes = p->guv_bytes;
    x.sub_bytes = p->sub_bytes;
    x.hi_u = p->hi_u;
    x.hi_v = p->hi_v;
    x.hi_w = p->hi_w;
    return x;
}

__device__ __forceinline__ const double* problem_uvw(const LaunchParams& P, int problem) {
    if (!P.probs) return P.prob.uvw;
    const ConstProblemPtr p = (ConstProblemPtr)uniform_u64((uint64_t)P.probs) + problem;
    return p->uvw;
}

// G_w[o_w][0..3] as four floats, read through the scalar cache.
template <int F>
__device__ __forceinline__ float4 load_gw_row(uint64_t g_w, int ow) {
    if constexpr (F == kGcfF32) {
        const ConstF32Ptr p = (ConstF32Ptr)g_w + ow * kSupportW;
        return make_float4(p[0], p[1], p[2], p[3]);
    } else {
        const ConstU32Ptr p = (ConstU32Ptr)g_w + ow * (kSupportW / 2);
        const __half2 a = __builtin_bit_cast(__half2, p[0]);
        const __half2 b = __builtin_bit_cast(__half2, p[1]);
        return make_float4(__low2float(a), __high2float(a), __low2float(b), __high2float(b));
    }
}


// Waits for this wavefront's outstanding vector-memory operations, including
// loads that write LDS directly.
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// LDS box of one wavefront: a copy of the cells of a tile's bounding box,
// row-major. Complex64 cells are split into two planes of 16 bytes (w 0-1
// and w 2-3), plane 1 starting plane1 bytes after plane 0, so that eight
// lanes reading neighbouring cells touch one contiguous 128-byte span.
template <int G>
__device__ __forceinline__ void lds_w4(const char* box, uint32_t off, uint32_t plane1,
                                       uint32_t (&raw)[GridTraits<G>::kWords]) {
    const uint4 a = *reinterpret_cast<const uint4*>(box + off);
    raw[0] = a.x; raw[1] = a.y; raw[2] = a.z; raw[3] = a.w;
    if constexpr (G == kGridC64) {
        const uint4 b = *reinterpret_cast<const uint4*>(box + plane1 + off);
        raw[4] = b.x; raw[5] = b.y; raw[6] = b.z; raw[7] = b.w;
    }
}

// Subgrid values of eight visibilities, fetched ahead of their arithmetic so
// that the loads of one group overlap the sums of the previous one.
template <int G>
struct Fetch8 {
    uint32_t raw[8][GridTraits<G>::kWords];
};

// Lane j holds the coordinate-stage results of visibility j: a_off (byte
// offset of its first tap in the LDS box or in the subgrid) and ow (its G_w
// row); v_readlane hands them to the whole wavefront.
template <int G, bool STAGED>
__device__ __forceinline__ void fetch8(Fetch8<G>& f, int g0, int a_off, __amdgpu_buffer_rsrc_t ra,
                                       uint32_t lane_a, const char* box, uint32_t plane1) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t aj = (uint32_t)__builtin_amdgcn_readlane(a_off, g0 + k);
        if constexpr (STAGED) {
            lds_w4<G>(box, lane_a + aj, plane1, f.raw[k]);
        } else {
            load_w4<G>(ra, lane_a + aj, f.raw[k]);
        }
    }
}

// Weighted sums of visibilities g0 .. g0+7 from their fetched values; gv[k]
// is this lane's G_uv weight of visibility g0 + k, and the G_w rows come
// through the scalar cache. Results land in out[g0 .. g0+7].
template <int G, int F>
__device__ __forceinline__ void sum8(const Fetch8<G>& f, const float* gv, int ow, uint64_t g_w, float2* out,
                                     int g0) {
    const int lane = lane_id();
    float pre[8], pim[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float4 gw = load_gw_row<F>(g_w, __builtin_amdgcn_readlane(ow, g0 + k));
        float re[4], im[4];
        widen_w4<G>(f.raw[k], re, im);
        const float sr = gw.x * re[0] + gw.y * re[1] + gw.z * re[2] + gw.w * re[3];
        const float si = gw.x * im[0] + gw.y * im[1] + gw.z * im[2] + gw.w * im[3];
        pre[k] = gv[k] * sr;
        pim[k] = gv[k] * si;
    }
    reduce8(pre);
    reduce8(pim);
    if ((lane & 7) == 0) out[g0 + (lane >> 3)] = make_float2(pre[0], pim[0]);
}

// All visibilities of a tile, groups of eight in a two-stage pipeline.
template <int G, int F, int NB, bool STAGED>
__device__ __forceinline__ void gather_tile(float2* out, int count, int a_off, int ow, const float* gv,
                                            __amdgpu_buffer_rsrc_t ra, uint64_t g_w, uint32_t lane_a,
                                            const char* box, uint32_t plane1) {
    Fetch8<G> buf[2];
    fetch8<G, STAGED>(buf[0], 0, a_off, ra, lane_a, box, plane1);
#pragma unroll
    for (int g0 = 0; g0 < NB; g0 += 8) {
        if (g0 < count) {
            if (g0 + 8 < NB && g0 + 8 < count)
                fetch8<G, STAGED>(buf[((g0 / 8) + 1) & 1], g0 + 8, a_off, ra, lane_a, box, plane1);
            sum8<G, F>(buf[(g0 / 8) & 1], gv + g0, ow, g_w, out, g0);
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
template <int G, int F, int BOX, int NB>
__global__ __launch_bounds__(kBlockThreads, 2) void degrid_kernel(LaunchParams P) {
    using GT = GridTraits<G>;
    static_assert(NB % 8 == 0 && NB <= kMaxNb, "tile size");
    constexpr int kBoxBytes = BOX > 0 ? BOX : 16;
    __shared__ float2 s_out[kWavesPerBlock][NB];
    __shared__ __attribute__((aligned(16))) char s_box[kWavesPerBlock][kBoxBytes];

    const int lane = lane_id();
    const int wv = (int)(threadIdx.x / kWave);
    QueueState st{xcc_id() % P.q.n_queues, 0};
    uint32_t wave_oob = 0;

    // current tile and its coordinates (in flight until the loop needs them)
    int t = pop_tile(P.q, P.ctl, st);
    Tile tc{};
    int64_t vis_c = 0;
    double u = 0.0, v = 0.0, w = 0.0;
    if (t >= 0) {
        tc = load_tile(P.tiles, t);
        vis_c = P.tile_vis[(int64_t)t * kMaxNb + lane];
        const double* uvw = problem_uvw(P, tc.problem);
        if (lane < tc.count) {
            u = uvw[3 * vis_c];
            v = uvw[3 * vis_c + 1];
            w = uvw[3 * vis_c + 2];
        }
    }
    int t_nxt = t >= 0 ? pop_tile(P.q, P.ctl, st) : -1;

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
        const int t_after = has_next ? pop_tile(P.q, P.ctl, st) : -1;

        const char* sub_base = static_cast<const char*>(pr.subgrids) + (int64_t)tc.sub * pr.sub_bytes;
        const __amdgpu_buffer_rsrc_t ra = make_rsrc(sub_base, pr.sub_bytes);
        const __amdgpu_buffer_rsrc_t rg = make_rsrc(pr.g_uv, pr.guv_bytes);
        const uint64_t g_w = uniform_u64((uint64_t)pr.g_w);
        const uint32_t lane_g = (uint32_t)lane * GcfTraits<F>::kBytes;

        // G_uv weights of the whole tile (zero for out-of-range visibilities).
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
        if constexpr (BOX > 0) {
            // bounding box of the tile's neighbourhoods
            bx0 = uniform(wave_min(in_range ? x0 : 0x7FFFFFFF));
            by0 = uniform(wave_min(in_range ? y0 : 0x7FFFFFFF));
            const int bx1 = uniform(wave_max(in_range ? x0 : -1));
            const int by1 = uniform(wave_max(in_range ? y0 : -1));
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
            // fills 16 bytes at 16 * l), all in flight at once. LDS chunk c is
            // half c / n_slots of slot c mod n_slots (complex64), or slot c;
            // slot (row, col) with col >= bw is row padding (filled with zeros).
            constexpr int kHalves = (int)(kCellBytes<G> / 16);   // 2 for complex64, else 1
            const int n_slots = bp * bh;
            const int total = n_slots * kHalves;
            const float inv_bp = 1.0f / (float)bp;
            const uint32_t row_stride = (uint32_t)pr.n_u * pr.n_w * GT::kElemBytes;
            const uint32_t box_origin = ((uint32_t)by0 * pr.n_u + bx0) * pr.n_w * GT::kElemBytes;
            for (int c0 = 0; c0 < total; c0 += kWave) {
                const int c = c0 + lane;
                const int half = (kHalves == 2 && c >= n_slots) ? 1 : 0;
                const int cc = c - half * n_slots;
                const int row = (int)(((float)cc + 0.5f) * inv_bp);
                const int col = cc - row * bp;
                const uint32_t off = (c < total && col < bw)
                                         ? box_origin + (uint32_t)row * row_stride + (uint32_t)col * kCellBytes<G> +
                                               (uint32_t)half * 16u
                                         : kOutOfRange;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    ra, (__attribute__((address_space(3))) void*)(box + c0 * 16), 16, off, 0, 0, 0);
            }
            wait_vmem();
            wave_lds_sync();
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

        const uint32_t plane1 = (uint32_t)(bp * bh) * 16u;
        const int a_off = staged ? (in_range ? ((y0 - by0) * bp + (x0 - bx0)) * 16 : 0)
                                 : (in_range ? cell * (int)GT::kElemBytes : (int)kOutOfRange);
        const uint32_t lane_a = staged ? ((uint32_t)(lane >> 3) * bp + (lane & 7)) * 16u
                                       : (uint32_t)(((lane >> 3) * pr.n_u + (lane & 7)) * pr.n_w) * GT::kElemBytes;
        if (staged)
            gather_tile<G, F, NB, true>(s_out[wv], count, a_off, ow, gv, ra, g_w, lane_a, box, plane1);
        else
            gather_tile<G, F, NB, false>(s_out[wv], count, a_off, ow, gv, ra, g_w, lane_a, box, plane1);
        if (!staged && has_next && lane < tn.count) {
            un = uvw_n[3 * vis_n];
            vn = uvw_n[3 * vis_n + 1];
            wn = uvw_n[3 * vis_n + 2];
        }
        wave_lds_sync();
        if (lane < count)
            static_cast<float2*>(pr.vis)[vis_c] = in_range ? s_out[wv][lane] : make_float2(0.f, 0.f);
        wave_lds_sync();

        t = t_nxt;
        t_nxt = t_after;
        tc = tn;
        vis_c = vis_n;
        u = un;
        v = vn;
        w = wn;
    }
    finish_launch(P.ctl, wave_oob);
}

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
        if constexpr (BOX > 0) {
            bx0 = uniform(wave_min(in_range ? x0 : 0x7FFFFFFF));
            by0 = uniform(wave_min(in_range ? y0 : 0x7FFFFFFF));
            const int bx1 = uniform(wave_max(in_range ? x0 : -1));
            const int by1 = uniform(wave_max(in_range ? y0 : -1));
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

struct OwnerRec {
    int32_t x0, y0;   // first tap relative to the block origin (x0 far out of range: skipped)
    int32_t g_off;    // byte offset of the G_uv block (kOutOfRange if skipped)
    int32_t pad;
    float c[8];       // G_w[o_w][t] * V, interleaved (re, im) for t = 0..3
};
static_assert(sizeof(OwnerRec) == 48, "OwnerRec layout");

typedef const __attribute__((address_space(4))) OwnerBlock* ConstOwnerBlockPtr;

// This lane's G_uv weights of records j0 .. j0+7 (zero for skipped records).
template <int F>
__device__ __forceinline__ void load_weights8(float* g, const OwnerRec* rec, int j0, __amdgpu_buffer_rsrc_t rg,
                                              uint32_t lane_g) {
#pragma unroll
    for (int k = 0; k < 8; ++k) g[k] = load_gcf_rsrc<F>(rg, (uint32_t)uniform(rec[j0 + k].g_off) + lane_g);
}

// Marks eight values as used here, so that their loads stay where they were
// issued (one group ahead) instead of being moved next to each use.
__device__ __forceinline__ void pin8(float* g) {
    asm volatile("" ::"v"(g[0]), "v"(g[1]), "v"(g[2]), "v"(g[3]), "v"(g[4]), "v"(g[5]), "v"(g[6]), "v"(g[7]));
}

template <int F>
__global__ __launch_bounds__(kBlockThreads) void grid_owner_kernel(OwnerParams P) {
    constexpr int B = kOwnerBlock;
    constexpr int kCellFloats = kSupportW * 2;          // complex64 x 4 w
    constexpr int kRowFloats = B * kCellFloats;         // floats of one block row
    // LDS row pitch: 16 bytes more than a row (cells stay 16-byte aligned and
    // neighbouring rows start on different banks)
    constexpr int kPitch = kRowFloats + 4;
    __shared__ __attribute__((aligned(16))) float s_box[kWavesPerBlock][B * kPitch];
    __shared__ OwnerRec s_rec[kWavesPerBlock][kWave];

    const int lane = lane_id();
    const int wv = (int)(threadIdx.x / kWave);
    const int tv = lane >> 3, tu = lane & 7;
    QueueState st{xcc_id() % P.q.n_queues, 0};
    const Problem& pr = P.prob;
    const __amdgpu_buffer_rsrc_t rg = make_rsrc(pr.g_uv, pr.guv_bytes);
    const uint32_t lane_g = (uint32_t)lane * GcfTraits<F>::kBytes;
    const int64_t row_floats = 2 * (int64_t)pr.n_u * pr.n_w;   // floats per subgrid row
    float* box = s_box[wv];

    int t = pop_tile(P.q, P.ctl, st);
    while (t >= 0) {
        const ConstOwnerBlockPtr pb = (ConstOwnerBlockPtr)uniform_u64((uint64_t)P.blocks) + t;
        const int64_t begin = pb->begin;
        const int count = pb->count;
        const int blk = pb->block;
        const int t_next = pop_tile(P.q, P.ctl, st);
        const int per_sub = P.nby * P.nbx;
        const int s = blk / per_sub;
        const int by = (blk - s * per_sub) / P.nbx;
        const int bx = blk - s * per_sub - by * P.nbx;
        float* out = static_cast<float*>(pr.grid_out) +
                     2 * ((int64_t)s * pr.cells_per_sub + ((int64_t)(by * B) * pr.n_u + bx * B) * pr.n_w);

        // the block's current contents (or zeros): one float per lane and step
#pragma unroll 4
        for (int f = lane; f < B * kRowFloats; f += kWave) {
            const int row = f / kRowFloats, col = f - row * kRowFloats;
            box[row * kPitch + col] = P.accumulate ? out[row * row_floats + col] : 0.0f;
        }

        for (int c0 = 0; c0 < count; c0 += kWave) {
            OwnerRec r;
            r.x0 = -(1 << 20);
            r.y0 = 0;
            r.g_off = (int)kOutOfRange;
            r.pad = 0;
#pragma unroll
            for (int q = 0; q < 8; ++q) r.c[q] = 0.0f;
            if (c0 + lane < count) {
                const int64_t i = P.items[begin + c0 + lane];
                const double* uv = pr.uvw + 3 * i;
                int32_t cell = 0, tab = 0, ow = 0, x0 = 0, y0 = 0;
                if (coords_from(pr, uv[0], uv[1], uv[2], cell, tab, ow, x0, y0) &&
                    (((uint32_t)y0 << 16) | (uint32_t)x0) == P.plan_start[i]) {
                    r.x0 = x0 - bx * B;
                    r.y0 = y0 - by * B;
                    r.g_off = tab * (int)GcfTraits<F>::kBytes;
                    const float2 vv = static_cast<const float2*>(pr.vis)[i];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const float gw = load_gcf<F>(pr.g_w, ow * kSupportW + k);
                        r.c[2 * k] = gw * vv.x;
                        r.c[2 * k + 1] = gw * vv.y;
                    }
                }
            }
            s_rec[wv][lane] = r;
            wave_lds_sync();
            const int n = min(kWave, count - c0);
            // G_uv weights one group of eight ahead (records past n are
            // skipped ones, whose loads return zero)
            float g[2][8];
            load_weights8<F>(g[0], s_rec[wv], 0, rg, lane_g);
#pragma unroll
            for (int j0 = 0; j0 < kWave; j0 += 8) {
                if (j0 < n) {
                    float* gc = g[(j0 / 8) & 1];
                    if (j0 + 8 < kWave) load_weights8<F>(g[((j0 / 8) + 1) & 1], s_rec[wv], j0 + 8, rg, lane_g);
                    pin8(gc);
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const OwnerRec& rj = s_rec[wv][j0 + k];
                        const int cy = rj.y0 + tv, cx = rj.x0 + tu;
                        if ((unsigned)cy < (unsigned)B && (unsigned)cx < (unsigned)B) {
                            // the taps of one visibility are distinct cells and
                            // LDS operations of a wavefront run in order, so a
                            // plain read-modify-write is exact
                            float4* dst = reinterpret_cast<float4*>(box + cy * kPitch + cx * kCellFloats);
                            float4 a = dst[0], b = dst[1];
                            a.x += gc[k] * rj.c[0]; a.y += gc[k] * rj.c[1];
                            a.z += gc[k] * rj.c[2]; a.w += gc[k] * rj.c[3];
                            b.x += gc[k] * rj.c[4]; b.y += gc[k] * rj.c[5];
                            b.z += gc[k] * rj.c[6]; b.w += gc[k] * rj.c[7];
                            dst[0] = a;
                            dst[1] = b;
                        }
                    }
                }
            }
            wave_lds_sync();
        }

        // write the block
#pragma unroll 4
        for (int f = lane; f < B * kRowFloats; f += kWave) {
            const int row = f / kRowFloats, col = f - row * kRowFloats;
            out[row * row_floats + col] = box[row * kPitch + col];
        }
        wave_lds_sync();
        t = t_next;
    }
    finish_launch(P.ctl, 0u);
}

// Visibilities the owner pass skipped (first tap differs from the plan's),
// added with atomics by whole wavefronts, and the out-of-range count.
template <int F>
__global__ __launch_bounds__(kBlockThreads) void grid_fixup_kernel(Problem pr, const int64_t* offsets,
                                                                   int64_t n_sub, int64_t n_vis,
                                                                   const uint32_t* plan_start, Ctl* ctl) {
    const int lane = lane_id();
    const int tv = lane >> 3, tu = lane & 7;
    uint32_t wave_oob = 0;
    const int64_t n_waves = (int64_t)gridDim.x * kWavesPerBlock;
    const int64_t first = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    for (int64_t w0 = first * kWave; w0 < n_vis; w0 += n_waves * kWave) {
        const int64_t i = w0 + lane;
        int32_t cell = 0, tab = 0, ow = 0, x0 = 0, y0 = 0;
        bool in_range = false, redo = false;
        if (i < n_vis) {
            const double* uv = pr.uvw + 3 * i;
            in_range = coords_from(pr, uv[0], uv[1], uv[2], cell, tab, ow, x0, y0);
            redo = in_range && (((uint32_t)y0 << 16) | (uint32_t)x0) != plan_start[i];
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
            for (int k = 0; k < 4; ++k) {
                const float gw = load_gcf<F>(pr.g_w, ow * kSupportW + k);
                c[2 * k] = gw * vv.x;
                c[2 * k + 1] = gw * vv.y;
            }
        }
        const int64_t lane_cell = (int64_t)(tv * pr.n_u + tu) * pr.n_w;
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
    finish_launch(ctl, wave_oob);
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

__global__ void zero_kernel(float4* p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// Kernel variants: (LDS box per wavefront in bytes, largest tile). Box 0
// gathers through the caches only.
struct Variant { int box; int nb; };
constexpr Variant kVariants[] = {{0, 64}, {8192, 32}, {12288, 32}, {16384, 32}, {16384, 64}, {24576, 64}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

template <int G, int F, int V>
hipError_t launch_degrid_t(const LaunchParams& p, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((degrid_kernel<G, F, kVariants[V].box, kVariants[V].nb>), dim3(blocks), dim3(kBlockThreads),
                       0, s, p);
    return hipGetLastError();
}

template <int G, int F, int V>
hipError_t occ_degrid_t(int* n) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, degrid_kernel<G, F, kVariants[V].box, kVariants[V].nb>,
                                                        kBlockThreads, 0);
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
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int degrid_variant_count() { return kNumVariants; }
int adjoint_variant_count() { return kNumVariants; }
int degrid_variant_box_bytes(int variant) {
    return (variant >= 0 && variant < kNumVariants) ? kVariants[variant].box : -1;
}
int degrid_variant_max_nb(int variant) {
    return (variant >= 0 && variant < kNumVariants) ? kVariants[variant].nb : -1;
}

hipError_t launch_degrid(const LaunchParams& p, int grid_kind, int gcf_kind, int variant,
                         int blocks, hipStream_t stream) {
    switch (grid_kind * 2 + gcf_kind) {
        case kGridC64 * 2 + kGcfF32: return launch_degrid_v<kGridC64, kGcfF32>(p, variant, blocks, stream);
        case kGridC64 * 2 + kGcfF16: return launch_degrid_v<kGridC64, kGcfF16>(p, variant, blocks, stream);
        case kGridCBF16 * 2 + kGcfF32: return launch_degrid_v<kGridCBF16, kGcfF32>(p, variant, blocks, stream);
        case kGridCBF16 * 2 + kGcfF16: return launch_degrid_v<kGridCBF16, kGcfF16>(p, variant, blocks, stream);
        case kGridCF16 * 2 + kGcfF32: return launch_degrid_v<kGridCF16, kGcfF32>(p, variant, blocks, stream);
        case kGridCF16 * 2 + kGcfF16: return launch_degrid_v<kGridCF16, kGcfF16>(p, variant, blocks, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t degrid_kernel_occupancy(int grid_kind, int gcf_kind, int variant, int* n) {
    switch (grid_kind * 2 + gcf_kind) {
        case kGridC64 * 2 + kGcfF32: return occ_degrid_v<kGridC64, kGcfF32>(variant, n);
        case kGridC64 * 2 + kGcfF16: return occ_degrid_v<kGridC64, kGcfF16>(variant, n);
        case kGridCBF16 * 2 + kGcfF32: return occ_degrid_v<kGridCBF16, kGcfF32>(variant, n);
        case kGridCBF16 * 2 + kGcfF16: return occ_degrid_v<kGridCBF16, kGcfF16>(variant, n);
        case kGridCF16 * 2 + kGcfF32: return occ_degrid_v<kGridCF16, kGcfF32>(variant, n);
        case kGridCF16 * 2 + kGcfF16: return occ_degrid_v<kGridCF16, kGcfF16>(variant, n);
        default: return hipErrorInvalidValue;
    }
}

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
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_grid_adjoint(const LaunchParams& p, int gcf_kind, int variant, int blocks,
                               hipStream_t stream) {
    if (gcf_kind == kGcfF32) return launch_adjoint_v<kGcfF32>(p, variant, blocks, stream);
    if (gcf_kind == kGcfF16) return launch_adjoint_v<kGcfF16>(p, variant, blocks, stream);
    return hipErrorInvalidValue;
}

hipError_t adjoint_kernel_occupancy(int gcf_kind, int variant, int* n) {
    if (gcf_kind == kGcfF32) return occ_adjoint_v<kGcfF32>(variant, n);
    if (gcf_kind == kGcfF16) return occ_adjoint_v<kGcfF16>(variant, n);
    return hipErrorInvalidValue;
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

hipError_t launch_grid_owner(const OwnerParams& p, int gcf_kind, int blocks, hipStream_t stream) {
    if (gcf_kind == kGcfF32)
        hipLaunchKernelGGL((grid_owner_kernel<kGcfF32>), dim3(blocks), dim3(kBlockThreads), 0, stream, p);
    else if (gcf_kind == kGcfF16)
        hipLaunchKernelGGL((grid_owner_kernel<kGcfF16>), dim3(blocks), dim3(kBlockThreads), 0, stream, p);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t owner_kernel_occupancy(int gcf_kind, int* n) {
    if (gcf_kind == kGcfF32)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, grid_owner_kernel<kGcfF32>, kBlockThreads, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, grid_owner_kernel<kGcfF16>, kBlockThreads, 0);
}

hipError_t launch_grid_fixup(const Problem& pr, const int64_t* vis_offsets, int64_t n_sub, int64_t n_vis,
                             const uint32_t* plan_start, Ctl* ctl, int gcf_kind, hipStream_t stream) {
    int64_t blocks = (n_vis + kBlockThreads - 1) / kBlockThreads;
    blocks = blocks < 1 ? 1 : (blocks > 2048 ? 2048 : blocks);
    if (gcf_kind == kGcfF32)
        hipLaunchKernelGGL((grid_fixup_kernel<kGcfF32>), dim3((unsigned)blocks), dim3(kBlockThreads), 0, stream, pr,
                           vis_offsets, n_sub, n_vis, plan_start, ctl);
    else if (gcf_kind == kGcfF16)
        hipLaunchKernelGGL((grid_fixup_kernel<kGcfF16>), dim3((unsigned)blocks), dim3(kBlockThreads), 0, stream, pr,
                           vis_offsets, n_sub, n_vis, plan_start, ctl);
    else
        return hipErrorInvalidValue;
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
