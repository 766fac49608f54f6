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
__device__ __forceinline__ bool vis_coords(const Problem& pr, int64_t i, int32_t& cell,
                                           int32_t& tab, int32_t& ow) {
    const double* c = pr.uvw + 3 * i;
    const double u = c[0], v = c[1], w = c[2];
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
    return true;
}

// Coordinates of one visibility as staged in LDS for the gather.
struct VisRec {
    int32_t cell;   // first-tap cell offset inside the subgrid; -1 if out of range
    int32_t tab;    // element offset of the 8x8 G_uv block
    int32_t pad0, pad1;
    float gw[4];    // G_w[o_w][0..3]; zeros when out of range
};
static_assert(sizeof(VisRec) == 32, "VisRec layout");

// Coordinates and the G_w-weighted visibility of one visibility (adjoint).
struct AdjRec {
    int32_t cell;
    int32_t tab;
    int32_t pad0, pad1;
    float c[8];     // G_w[o_w][t] * V, interleaved (re, im) for t = 0..3
};
static_assert(sizeof(AdjRec) == 48, "AdjRec layout");

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

template <int G, int F>
__global__ __launch_bounds__(kBlockThreads) void degrid_kernel(LaunchParams P) {
    using GT = GridTraits<G>;
    __shared__ VisRec s_rec[kWavesPerBlock][kMaxNb];
    __shared__ float2 s_out[kWavesPerBlock][kMaxNb];

    const int lane = lane_id();
    const int wv = (int)(threadIdx.x / kWave);
    QueueState st{xcc_id() % P.q.n_queues, 0};
    uint32_t wave_oob = 0;

    int t = pop_tile(P.q, P.ctl, st);
    while (t >= 0) {
        const Tile tile = P.tiles[t];
        const int t_next = pop_tile(P.q, P.ctl, st);
        const Problem pr = P.probs ? P.probs[tile.problem] : P.prob;
        const int count = tile.count;

        // Coordinate stage: lane j handles visibility begin + j.
        {
            VisRec r;
            r.cell = -1;
            r.tab = 0;
            r.pad0 = r.pad1 = 0;
            r.gw[0] = r.gw[1] = r.gw[2] = r.gw[3] = 0.0f;
            bool in_range = false;
            if (lane < count) {
                int32_t ow = 0;
                in_range = vis_coords(pr, tile.begin + lane, r.cell, r.tab, ow);
                if (in_range) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) r.gw[k] = load_gcf<F>(pr.g_w, ow * kSupportW + k);
                } else {
                    r.cell = -1;
                    r.tab = 0;
                }
            }
            wave_oob += (uint32_t)__popcll(__ballot(lane < count && !in_range));
            s_rec[wv][lane] = r;
        }
        wave_lds_sync();

        // Gather: lane = (t_v, t_u); 4 w values per lane.
        const char* sub_base = static_cast<const char*>(pr.subgrids) + (int64_t)tile.sub * pr.sub_bytes;
        const __amdgpu_buffer_rsrc_t ra = make_rsrc(sub_base, pr.sub_bytes);
        const __amdgpu_buffer_rsrc_t rg = make_rsrc(pr.g_uv, pr.guv_bytes);
        const uint32_t lane_a = (uint32_t)(((lane >> 3) * pr.n_u + (lane & 7)) * pr.n_w) * GT::kElemBytes;
        const uint32_t lane_g = (uint32_t)lane * GcfTraits<F>::kBytes;

        for (int g0 = 0; g0 < count; g0 += 8) {
            uint32_t raw[8][GT::kWords];
            float guv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int j = g0 + k;
                const int cell = uniform(s_rec[wv][j].cell);
                const int tab = uniform(s_rec[wv][j].tab);
                const bool live = (j < count) & (cell >= 0);
                const uint32_t oa = live ? (uint32_t)cell * GT::kElemBytes + lane_a : kOutOfRange;
                const uint32_t og = live ? (uint32_t)tab * GcfTraits<F>::kBytes + lane_g : kOutOfRange;
                load_w4<G>(ra, oa, raw[k]);
                guv[k] = load_gcf_rsrc<F>(rg, og);
            }
            float pre[8], pim[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const float4 gw = *reinterpret_cast<const float4*>(s_rec[wv][g0 + k].gw);
                float re[4], im[4];
                widen_w4<G>(raw[k], re, im);
                const float sr = gw.x * re[0] + gw.y * re[1] + gw.z * re[2] + gw.w * re[3];
                const float si = gw.x * im[0] + gw.y * im[1] + gw.z * im[2] + gw.w * im[3];
                pre[k] = guv[k] * sr;
                pim[k] = guv[k] * si;
            }
            reduce8(pre);
            reduce8(pim);
            if ((lane & 7) == 0) s_out[wv][g0 + (lane >> 3)] = make_float2(pre[0], pim[0]);
        }
        wave_lds_sync();
        if (lane < count) static_cast<float2*>(pr.vis)[tile.begin + lane] = s_out[wv][lane];
        wave_lds_sync();
        t = t_next;
    }
    finish_launch(P.ctl, wave_oob);
}

// ---------------------------------------------------------------------------
// Adjoint (gridding) kernel: scatter with float32 atomics
// ---------------------------------------------------------------------------

template <int F>
__global__ __launch_bounds__(kBlockThreads) void grid_adjoint_kernel(LaunchParams P) {
    __shared__ AdjRec s_rec[kWavesPerBlock][kMaxNb];

    const int lane = lane_id();
    const int wv = (int)(threadIdx.x / kWave);
    QueueState st{xcc_id() % P.q.n_queues, 0};
    uint32_t wave_oob = 0;

    int t = pop_tile(P.q, P.ctl, st);
    while (t >= 0) {
        const Tile tile = P.tiles[t];
        const int t_next = pop_tile(P.q, P.ctl, st);
        const Problem pr = P.probs ? P.probs[tile.problem] : P.prob;
        const int count = tile.count;

        {
            AdjRec r;
            r.cell = -1;
            r.tab = 0;
            r.pad0 = r.pad1 = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) r.c[k] = 0.0f;
            bool in_range = false;
            if (lane < count) {
                int32_t ow = 0;
                in_range = vis_coords(pr, tile.begin + lane, r.cell, r.tab, ow);
                if (in_range) {
                    const float2 vv = static_cast<const float2*>(pr.vis)[tile.begin + lane];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const float gw = load_gcf<F>(pr.g_w, ow * kSupportW + k);
                        r.c[2 * k] = gw * vv.x;
                        r.c[2 * k + 1] = gw * vv.y;
                    }
                } else {
                    r.cell = -1;
                    r.tab = 0;
                }
            }
            wave_oob += (uint32_t)__popcll(__ballot(lane < count && !in_range));
            s_rec[wv][lane] = r;
        }
        wave_lds_sync();

        const __amdgpu_buffer_rsrc_t rg = make_rsrc(pr.g_uv, pr.guv_bytes);
        const uint32_t lane_g = (uint32_t)lane * GcfTraits<F>::kBytes;
        float* out = static_cast<float*>(pr.grid_out) + 2 * ((int64_t)tile.sub * pr.cells_per_sub +
                     (int64_t)(((lane >> 3) * pr.n_u + (lane & 7)) * pr.n_w));

        for (int g0 = 0; g0 < count; g0 += 8) {
            float guv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int j = g0 + k;
                const int cell = uniform(s_rec[wv][j].cell);
                const int tab = uniform(s_rec[wv][j].tab);
                const bool live = (j < count) & (cell >= 0);
                guv[k] = load_gcf_rsrc<F>(rg, live ? (uint32_t)tab * GcfTraits<F>::kBytes + lane_g : kOutOfRange);
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int j = g0 + k;
                const int cell = uniform(s_rec[wv][j].cell);
                if (j < count && cell >= 0) {
                    float* dst = out + 2 * (int64_t)cell;
#pragma unroll
                    for (int q = 0; q < 8; ++q) unsafeAtomicAdd(dst + q, guv[k] * s_rec[wv][j].c[q]);
                }
            }
        }
        wave_lds_sync();
        t = t_next;
    }
    finish_launch(P.ctl, wave_oob);
}

__global__ void zero_kernel(float4* p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

template <int G, int F>
hipError_t launch_degrid_t(const LaunchParams& p, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((degrid_kernel<G, F>), dim3(blocks), dim3(kBlockThreads), 0, s, p);
    return hipGetLastError();
}

template <int G, int F>
hipError_t occ_degrid_t(int* n) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, degrid_kernel<G, F>, kBlockThreads, 0);
}

}  // namespace

int degrid_variant_count() { return 1; }
int adjoint_variant_count() { return 1; }

hipError_t launch_degrid(const LaunchParams& p, int grid_kind, int gcf_kind, int variant,
                         int blocks, hipStream_t stream) {
    (void)variant;
    switch (grid_kind * 2 + gcf_kind) {
        case kGridC64 * 2 + kGcfF32: return launch_degrid_t<kGridC64, kGcfF32>(p, blocks, stream);
        case kGridC64 * 2 + kGcfF16: return launch_degrid_t<kGridC64, kGcfF16>(p, blocks, stream);
        case kGridCBF16 * 2 + kGcfF32: return launch_degrid_t<kGridCBF16, kGcfF32>(p, blocks, stream);
        case kGridCBF16 * 2 + kGcfF16: return launch_degrid_t<kGridCBF16, kGcfF16>(p, blocks, stream);
        case kGridCF16 * 2 + kGcfF32: return launch_degrid_t<kGridCF16, kGcfF32>(p, blocks, stream);
        case kGridCF16 * 2 + kGcfF16: return launch_degrid_t<kGridCF16, kGcfF16>(p, blocks, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t degrid_kernel_occupancy(int grid_kind, int gcf_kind, int variant, int* n) {
    (void)variant;
    switch (grid_kind * 2 + gcf_kind) {
        case kGridC64 * 2 + kGcfF32: return occ_degrid_t<kGridC64, kGcfF32>(n);
        case kGridC64 * 2 + kGcfF16: return occ_degrid_t<kGridC64, kGcfF16>(n);
        case kGridCBF16 * 2 + kGcfF32: return occ_degrid_t<kGridCBF16, kGcfF32>(n);
        case kGridCBF16 * 2 + kGcfF16: return occ_degrid_t<kGridCBF16, kGcfF16>(n);
        case kGridCF16 * 2 + kGcfF32: return occ_degrid_t<kGridCF16, kGcfF32>(n);
        case kGridCF16 * 2 + kGcfF16: return occ_degrid_t<kGridCF16, kGcfF16>(n);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_grid_adjoint(const LaunchParams& p, int gcf_kind, int variant, int blocks,
                               hipStream_t stream) {
    (void)variant;
    if (gcf_kind == kGcfF32)
        hipLaunchKernelGGL((grid_adjoint_kernel<kGcfF32>), dim3(blocks), dim3(kBlockThreads), 0, stream, p);
    else if (gcf_kind == kGcfF16)
        hipLaunchKernelGGL((grid_adjoint_kernel<kGcfF16>), dim3(blocks), dim3(kBlockThreads), 0, stream, p);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t adjoint_kernel_occupancy(int gcf_kind, int variant, int* n) {
    (void)variant;
    if (gcf_kind == kGcfF32)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, grid_adjoint_kernel<kGcfF32>, kBlockThreads, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, grid_adjoint_kernel<kGcfF16>, kBlockThreads, 0);
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
