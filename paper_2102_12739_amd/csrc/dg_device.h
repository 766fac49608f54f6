// Device-side pieces shared by the degridding and gridding kernels on
// gfx950: buffer resources, the tile queue, storage types, the coordinate
// stage (Section 2: start point and oversampled table positions), the
// cross-lane reduction and scalar-cache views of read-only data.
#pragma once

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

// Waits until this wavefront's vector-memory operations (loads, stores and
// atomics) have been performed.
__device__ __forceinline__ void wait_vmem_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// ---------------------------------------------------------------------------
// Tile queue
// ---------------------------------------------------------------------------

struct QueueState {
    int q;       // queue currently drained
    int tried;   // queues found empty so far
};

// Next tile for this wavefront, or -1 once every queue is empty. A queue
// found empty is left for the next one (at most n_queues probes at the end).
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

// One past the last tile of queue q (the selection keeps the queue table in
// scalar registers).
__device__ __forceinline__ int queue_end(const QueueSpec& qs, int q) {
    int e = 0;
#pragma unroll
    for (int k = 0; k < kMaxQueues; ++k)
        if (q == k) e = qs.end[k];
    return e;
}

// Tile claims of the degrid and owner-computes adjoint kernels. Every atomic on a queue cursor is served
// one after another where the cursor lives (about 14 ns apiece when they
// queue), so most tiles are dealt without one: the launch's static deal
// (computed on the host for its grid size) gives most of each queue
// round-robin to the wavefronts that serve it, and only the rest goes
// through the cursor, one tile per atomic, with stealing as for pop_tile.
// Round-robin dealing keeps the shares even where tile costs vary along the
// queue.
struct TileClaims {
    int q;        // queue currently drained
    int tried;    // queues found empty so far
    int next;     // static share: tiles next, next + stride, ... below lim
    int lim;
    int stride;
    int dbeg;     // first tile of queue q handed out by its cursor
    int only_static;   // every tile is dealt statically: no cursor, no stealing
};

// Workgroup b serves queue b mod n_queues: workgroups are placed on the XCDs
// round-robin, so that is a queue of its own XCD. Without a static deal the
// first claim goes straight to the cursor.
__device__ __forceinline__ TileClaims start_claims(const QueueSpec& qs, const StaticDeal& d, int wv) {
    TileClaims st;
    st.q = uniform((int)blockIdx.x % qs.n_queues);
    st.tried = 0;
    st.next = 0;
    st.lim = 0;
    st.stride = 0;
    if (d.on) {
        st.next = uniform(qs.begin[st.q] + ((int)blockIdx.x / qs.n_queues) * kWavesPerBlock + wv);
        st.lim = uniform(d.sbase[st.q]);
        st.stride = uniform(d.stride[st.q]);
    }
    st.dbeg = uniform(d.sbase[st.q]);
    st.only_static = uniform(d.all_static);
    return st;
}

// After the cursor of st.q ran dry: the next queue in rotation.
__device__ __forceinline__ void next_queue(const QueueSpec& qs, const StaticDeal& d, TileClaims& st) {
    st.q = (st.q + 1 == qs.n_queues) ? 0 : st.q + 1;
    st.tried++;
    st.dbeg = uniform(d.sbase[st.q]);
}

// Next tile for this wavefront, or -1 once every queue is empty (at most
// n_queues cursor probes at the end).
__device__ __forceinline__ int claim_tile(const QueueSpec& qs, const StaticDeal& d, Ctl* ctl, TileClaims& st) {
    if (st.next < st.lim) {
        const int t = st.next;
        st.next += st.stride;
        return t;
    }
    if (st.only_static) return -1;
    while (st.tried < qs.n_queues) {
        uint32_t idx = 0;
        if (lane_id() == 0) idx = atomicAdd(&ctl->cursor[st.q].v[0], 1u);
        const int t = st.dbeg + uniform((int)idx);
        if (t < qs.end[st.q]) return t;
        next_queue(qs, d, st);
    }
    return -1;
}

// The two halves of a claim whose atomic is left in flight while the
// wavefront works: claim_issue sends the cursor increment (none while the
// static share lasts) and returns without waiting; claim_resolve, called
// before any other claim, turns the result into a tile, or carries on as
// claim_tile when that queue has run dry.
constexpr uint32_t kStaticClaim = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t claim_issue(Ctl* ctl, const TileClaims& st) {
    if (st.next < st.lim || st.only_static) return kStaticClaim;
    uint32_t idx = 0;
    if (lane_id() == 0) idx = atomicAdd(&ctl->cursor[st.q].v[0], 1u);
    return idx;
}

__device__ __forceinline__ int claim_resolve(const QueueSpec& qs, const StaticDeal& d, Ctl* ctl, TileClaims& st,
                                             uint32_t idx) {
    const uint32_t r = (uint32_t)uniform((int)idx);
    if (r == kStaticClaim) return claim_tile(qs, d, ctl, st);
    const int t = st.dbeg + (int)r;
    if (t < qs.end[st.q]) return t;
    next_queue(qs, d, st);
    return claim_tile(qs, d, ctl, st);
}

// Adds this wavefront's out-of-range count; the last workgroup of the launch
// publishes the launch total and resets cursors and counters for the next.
// The workgroups talk through device-scope atomics only, which are performed
// beyond the L2 caches: waiting for this workgroup's count to be performed
// (vmcnt 0) before its increment of the finished-workgroup counter orders
// the two, and the last workgroup's exchange then reads every count. No L2
// write-back is needed (the kernel's own end writes the caches back).
// kGrouped: for kernels whose workgroups all end at about the same time, a
// grid of more than kDoneFlat workgroups counts in two levels (group
// counters, then `done`).
template <bool kGrouped = false>
__device__ __forceinline__ void finish_launch(Ctl* ctl, uint32_t wave_oob) {
    auto* oob = reinterpret_cast<unsigned long long*>(&ctl->oob.v[0]);
    if (lane_id() == 0 && wave_oob != 0u) atomicAdd(&oob[0], (unsigned long long)wave_oob);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    wait_vmem_all();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const uint32_t n = gridDim.x;
    const bool grouped = kGrouped && n > (uint32_t)kDoneFlat;
    bool last;
    if (!grouped) {
        last = atomicAdd(&ctl->done.v[0], 1u) == n - 1;
    } else {
        // the last workgroup of a group has seen every increment of its
        // group, and the last of the groups every group's last
        const uint32_t g = blockIdx.x % kDoneGroups;
        const uint32_t in_group = (n - g + kDoneGroups - 1) / kDoneGroups;
        last = atomicAdd(&ctl->group[g].v[0], 1u) == in_group - 1 &&
               atomicAdd(&ctl->done.v[0], 1u) == (uint32_t)kDoneGroups - 1;
    }
    if (last) {
        const unsigned long long total = atomicExch(&oob[0], 0ull);
        atomicExch(&oob[1], total);
        for (int q = 0; q < kMaxQueues; ++q) atomicExch(&ctl->cursor[q].v[0], 0u);
        if (grouped)
            for (int q = 0; q < kDoneGroups; ++q) atomicExch(&ctl->group[q].v[0], 0u);
        atomicExch(&ctl->done.v[0], 0u);
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

// The same with one load per w value (8 bytes for complex64, 4 otherwise), so
// that the loads are naturally aligned whatever the first w of the tap.
template <int G>
__device__ __forceinline__ void load_w4_narrow(__amdgpu_buffer_rsrc_t r, uint32_t off,
                                               uint32_t (&raw)[GridTraits<G>::kWords]) {
    if constexpr (G == kGridC64) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            auto a = __builtin_amdgcn_raw_buffer_load_b64(r, off + 8u * (uint32_t)t, 0, 0);
            raw[2 * t] = a[0];
            raw[2 * t + 1] = a[1];
        }
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) raw[t] = __builtin_amdgcn_raw_buffer_load_b32(r, off + 4u * (uint32_t)t, 0, 0);
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
template <> struct GcfTraits<kGcfBF16> { static constexpr uint32_t kBytes = 2; };

// One 16-bit table value (the low half of h) widened to float32.
template <int F>
__device__ __forceinline__ float widen_gcf16(uint32_t h) {
    if constexpr (F == kGcfBF16) return __uint_as_float(h << 16);
    else return __half2float(__builtin_bit_cast(__half, (unsigned short)h));
}

// One table value at byte offset off + soff (soff wave-uniform: it travels
// in the load's scalar offset).
template <int F>
__device__ __forceinline__ float load_gcf_rsrc(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff = 0) {
    if constexpr (F == kGcfF32) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
    } else {
        return widen_gcf16<F>(__builtin_amdgcn_raw_buffer_load_b16(r, off, soff, 0));
    }
}

template <int F>
__device__ __forceinline__ float load_gcf(const void* table, int64_t idx) {
    if constexpr (F == kGcfF32) {
        return static_cast<const float*>(table)[idx];
    } else {
        return widen_gcf16<F>(static_cast<const unsigned short*>(table)[idx]);
    }
}

// ---------------------------------------------------------------------------
// Coordinate stage (Section 2: start point g and oversampled GCF positions)
// ---------------------------------------------------------------------------

// Start cell offset (first tap, inside its subgrid) and table positions of
// visibility i. Per axis k = floor(c * os) of the float64 product, which is
// exact for a power-of-two os (for other factors this rounding is the
// contract); the cell is k / os, the oversample index k mod os, and the
// first tap sits W/2 - 1 cells below the cell. Returns false when the
// neighbourhood leaves the subgrid or the coordinate is not finite.
__device__ __forceinline__ bool coords_from(const Problem& pr, double u, double v, double w, int32_t& cell,
                                            int32_t& tab, int32_t& ow, int32_t& x_start, int32_t& y_start) {
    // coarse float64 bounds first (they also reject NaN and values too large
    // for an int), then the exact test on the cells
    const bool near = (u >= 2.0) & (u < pr.hi_u + 1.0) & (v >= 2.0) & (v < pr.hi_v + 1.0) &
                      (w >= 0.0) & (w < pr.hi_w + 1.0);
    if (!near) return false;
    const int os_uv = pr.os_uv;
    const int os_w = pr.os_w;
    // k = floor(c * os) of the float64 product (exact when os is a power of
    // two); non-negative, so truncation is floor
    const int ku = (int)(u * (double)os_uv);
    const int kv = (int)(v * (double)os_uv);
    const int kw = (int)(w * (double)os_w);
    int nu, nv, nw;
    if (pr.log2_os_uv >= 0) {
        nu = ku >> pr.log2_os_uv;
        nv = kv >> pr.log2_os_uv;
    } else {
        nu = ku / os_uv;
        nv = kv / os_uv;
    }
    nw = pr.log2_os_w >= 0 ? kw >> pr.log2_os_w : kw / os_w;
    const int x0 = nu - (kSupportUV / 2 - 1);
    const int y0 = nv - (kSupportUV / 2 - 1);
    const int z0 = nw - (kSupportW / 2 - 1);
    if ((x0 < 0) | (x0 > pr.n_u - kSupportUV) | (y0 < 0) | (y0 > pr.n_v - kSupportUV) | (z0 < 0) |
        (z0 > pr.n_w - kSupportW))
        return false;
    const int ou = ku - nu * os_uv;
    const int ov = kv - nv * os_uv;
    ow = kw - nw * os_w;
    cell = (y0 * pr.n_u + x0) * pr.n_w + z0;
    tab = (ov * os_uv + ou) * (kSupportUV * kSupportUV);
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
    // bound_ctrl: the patterns used never read outside a row, so lanes never
    // take the old value, and none has to be set up
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
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

// Minimum over the 64 lanes of four values at once, on every lane: the lane
// exchanges of reduce8 (permlane swaps 32 and 16 lanes apart, then four DPP
// steps inside rows of 16) with min in place of the sum, the four chains in
// lockstep so that each step's latency hides behind the other three. All
// VALU, no LDS traffic. Call with every lane active.
__device__ __forceinline__ void wave_min4(int (&v)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const auto r = __builtin_amdgcn_permlane32_swap((uint32_t)v[i], (uint32_t)v[i], false, false);
        v[i] = min((int)r[0], (int)r[1]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const auto r = __builtin_amdgcn_permlane16_swap((uint32_t)v[i], (uint32_t)v[i], false, false);
        v[i] = min((int)r[0], (int)r[1]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = min(v[i], __builtin_amdgcn_update_dpp(0, v[i], kDppRowRor8, 0xF, 0xF, false));
#pragma unroll
    for (int i = 0; i < 4; ++i)
        v[i] = min(v[i], __builtin_amdgcn_update_dpp(0, v[i], kDppRowHalfMirror, 0xF, 0xF, false));
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = min(v[i], __builtin_amdgcn_update_dpp(0, v[i], kDppQuadXor2, 0xF, 0xF, false));
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = min(v[i], __builtin_amdgcn_update_dpp(0, v[i], kDppQuadXor1, 0xF, 0xF, false));
}

// Bounding box of the start cells (x, y) of the lanes with valid set, as
// wavefront-uniform values; x1 = -1 when no lane is valid.
__device__ __forceinline__ void wave_bbox(bool valid, int x, int y, int& x0, int& y0, int& x1, int& y1) {
    constexpr int kNone = 0x7FFFFFFF;
    // maxima as minima of the negated values (start cells are >= 0)
    int v[4] = {valid ? x : kNone, valid ? y : kNone, valid ? -x : 1, valid ? -y : 1};
    wave_min4(v);
    x0 = uniform(v[0]);
    y0 = uniform(v[1]);
    x1 = uniform(-v[2]);
    y1 = uniform(-v[3]);
}

// Scalar-cache view of read-only data: loads through it with a wave-uniform
// address become scalar loads.
typedef const __attribute__((address_space(4))) float* ConstF32Ptr;
typedef const __attribute__((address_space(4))) uint32_t* ConstU32Ptr;
typedef uint32_t U32x2 __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(4))) U32x2* ConstU32x2Ptr;
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
    x.os_uv = p->os_uv;
    x.os_w = p->os_w;
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

// Byte offset of G_w row o_w in a table of type F.
template <int F>
__device__ __forceinline__ uint32_t gw_row_offset(int ow) {
    return (uint32_t)ow * (GcfTraits<F>::kBytes * kSupportW);
}

// G_w row of a 16-bit table at byte offset off as two packed pairs (g0, g1),
// (g2, g3), read through the scalar cache.
__device__ __forceinline__ uint2 load_gw_pairs(uint64_t g_w, uint32_t off) {
    const U32x2 v = *(ConstU32x2Ptr)(g_w + off);
    return make_uint2(v.x, v.y);
}

// Storage and table types whose w sums run on the packed 16-bit dot products
// (v_dot2_f32_f16, v_dot2_f32_bf16): storage and G_w of the same 16-bit type.
// Each product of two such values is exact in float32.
template <int G, int F>
constexpr bool kPackedDot = (G == kGridCF16 && F == kGcfF16) || (G == kGridCBF16 && F == kGcfBF16);

typedef _Float16 Half2V __attribute__((ext_vector_type(2)));
typedef __bf16 BF16x2V __attribute__((ext_vector_type(2)));

// a.lo * b.lo + a.hi * b.hi + c, float32 accumulation
template <int G>
__device__ __forceinline__ float dot2(uint32_t a, uint32_t b, float c) {
    static_assert(G == kGridCF16 || G == kGridCBF16, "packed dot products cover 16-bit storage");
    if constexpr (G == kGridCF16)
        return __builtin_amdgcn_fdot2(__builtin_bit_cast(Half2V, a), __builtin_bit_cast(Half2V, b), c, false);
    else
        return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(BF16x2V, a), __builtin_bit_cast(BF16x2V, b), c,
                                               false);
}

// The same with c = 0. The builtin with a zero accumulator becomes a move of
// 0 and the two-operand v_dot2c form; the three-operand form takes 0 as an
// inline constant, which saves the move. b is wavefront-uniform (a G_w pair).
template <int G>
__device__ __forceinline__ float dot2_first(uint32_t a, uint32_t b) {
    static_assert(G == kGridCF16 || G == kGridCBF16, "packed dot products cover 16-bit storage");
    float d;
    if constexpr (G == kGridCF16)
        asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(d) : "s"(b), "v"(a));
    else
        asm("v_dot2_f32_bf16 %0, %1, %2, 0" : "=v"(d) : "s"(b), "v"(a));
    return d;
}

// sum_t G_w[t] * A[t] over the 4 w values of one fetched cell, for 16-bit
// storage with a G_w table of the same type: v_perm pairs the real parts (and
// the imaginary parts) of two adjacent w values so that one dot product
// takes two taps.
template <int G>
__device__ __forceinline__ void wsum_packed(const uint32_t (&raw)[GridTraits<G>::kWords], uint2 gw, float& sr,
                                            float& si) {
    // v_perm_b32 selects bytes of {src0 : src1}; bytes 0-3 are src1's.
    constexpr uint32_t kLowHalves = 0x05040100u;    // (src1.lo, src0.lo)
    constexpr uint32_t kHighHalves = 0x07060302u;   // (src1.hi, src0.hi)
    const uint32_t re01 = __builtin_amdgcn_perm(raw[1], raw[0], kLowHalves);
    const uint32_t im01 = __builtin_amdgcn_perm(raw[1], raw[0], kHighHalves);
    const uint32_t re23 = __builtin_amdgcn_perm(raw[3], raw[2], kLowHalves);
    const uint32_t im23 = __builtin_amdgcn_perm(raw[3], raw[2], kHighHalves);
    sr = dot2<G>(re23, gw.y, dot2_first<G>(re01, gw.x));
    si = dot2<G>(im23, gw.y, dot2_first<G>(im01, gw.x));
}

// G_w row at byte offset off as four floats, read through the scalar cache.
template <int F>
__device__ __forceinline__ float4 load_gw_row(uint64_t g_w, uint32_t off) {
    if constexpr (F == kGcfF32) {
        const ConstF32Ptr p = (ConstF32Ptr)(g_w + off);
        return make_float4(p[0], p[1], p[2], p[3]);
    } else {
        const U32x2 v = *(ConstU32x2Ptr)(g_w + off);
        return make_float4(widen_gcf16<F>(v.x & 0xFFFFu), widen_gcf16<F>(v.x >> 16), widen_gcf16<F>(v.y & 0xFFFFu),
                           widen_gcf16<F>(v.y >> 16));
    }
}


// sum_t g[t] * x[t] for one G_w row, in the order ((g0 x0 + g1 x1) + g2 x2)
// + g3 x3. For a 16-bit table the first product is also a fused
// multiply-add (with 0), so that every product takes the 16-bit weight as
// it is (v_fma_mix_f32) instead of a conversion and a multiply; the sum is
// the same, but for the sign of an exact zero.
template <int F>
__device__ __forceinline__ float wsum4(float4 g, const float (&x)[4]) {
    const float first = F == kGcfF32 ? g.x * x[0] : __builtin_fmaf(g.x, x[0], 0.0f);
    return __builtin_fmaf(g.w, x[3], __builtin_fmaf(g.z, x[2], __builtin_fmaf(g.y, x[1], first)));
}

// Sum over the 64 lanes in float64, in a fixed butterfly order (the same
// bits on every run).
__device__ __forceinline__ double wave_sum_f64(double x) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m);
    return x;
}

// Waits for this wavefront's outstanding vector-memory operations, including
// loads that write LDS directly.
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// LDS box of one wavefront: a copy of the cells of a tile's bounding box,
// row-major. Complex64 cells are split into two planes of 16 bytes (w 0-1
// and w 2-3), plane 1 starting PLANE1 bytes after plane 0 (half the box, a
// constant, so it becomes the LDS instruction's offset field), so that eight
// lanes reading neighbouring cells touch one contiguous 128-byte span.
template <int G, uint32_t PLANE1>
__device__ __forceinline__ void lds_w4(const char* box, uint32_t off, uint32_t (&raw)[GridTraits<G>::kWords]) {
    const uint4 a = *reinterpret_cast<const uint4*>(box + off);
    raw[0] = a.x; raw[1] = a.y; raw[2] = a.z; raw[3] = a.w;
    if constexpr (G == kGridC64) {
        const uint4 b = *reinterpret_cast<const uint4*>(box + off + PLANE1);
        raw[4] = b.x; raw[5] = b.y; raw[6] = b.z; raw[7] = b.w;
    }
}

// ---------------------------------------------------------------------------
// Gather of a tile (degrid kernels)
// ---------------------------------------------------------------------------

// Subgrid values of eight visibilities, fetched ahead of their arithmetic so
// that the loads of one group overlap the sums of the previous one.
template <int G>
struct Fetch8 {
    uint32_t raw[8][GridTraits<G>::kWords];
};

// Lane j holds the coordinate-stage results of visibility j: a_off (byte
// offset of its first tap in the LDS box or in the subgrid) and ow (its G_w
// row); v_readlane hands them to the whole wavefront.
template <int G, bool STAGED, uint32_t PLANE1, bool DEEP>
__device__ __forceinline__ void fetch8(Fetch8<G>& f, int g0, int a_off, __amdgpu_buffer_rsrc_t ra,
                                       uint32_t lane_a, const char* box) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t aj = (uint32_t)__builtin_amdgcn_readlane(a_off, g0 + k);
        if constexpr (STAGED) {
            lds_w4<G, PLANE1>(box, lane_a + aj, f.raw[k]);
        } else if constexpr (DEEP) {
            load_w4_narrow<G>(ra, lane_a + aj, f.raw[k]);
        } else {
            load_w4<G>(ra, lane_a + aj, f.raw[k]);
        }
    }
}

// Weighted sums of visibilities g0 .. g0+7 from their fetched values; gv[k]
// is this lane's G_uv weight of visibility g0 + k, and the G_w rows (lane j
// holds the byte offset gw_off of visibility j's row) come through the
// scalar cache. Results land in out[g0 .. g0+7].
template <int G, int F>
__device__ __forceinline__ void sum8(const Fetch8<G>& f, const float* gv, uint32_t gw_off, uint64_t g_w,
                                     float2* out, int g0) {
    const int lane = lane_id();
    float pre[8], pim[8];
    uint2 gwp[8];
    if constexpr (kPackedDot<G, F>) {
        // the eight rows' scalar loads go out together, ahead of the sums
#pragma unroll
        for (int k = 0; k < 8; ++k)
            gwp[k] = load_gw_pairs(g_w, (uint32_t)__builtin_amdgcn_readlane((int)gw_off, g0 + k));
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        float sr, si;
        if constexpr (kPackedDot<G, F>) {
            wsum_packed<G>(f.raw[k], gwp[k], sr, si);
        } else {
            const float4 gw = load_gw_row<F>(g_w, (uint32_t)__builtin_amdgcn_readlane((int)gw_off, g0 + k));
            float re[4], im[4];
            widen_w4<G>(f.raw[k], re, im);
            sr = wsum4<F>(gw, re);
            si = wsum4<F>(gw, im);
        }
        pre[k] = gv[k] * sr;
        pim[k] = gv[k] * si;
    }
    reduce8(pre);
    reduce8(pim);
    if ((lane & 7) == 0) out[g0 + (lane >> 3)] = make_float2(pre[0], pim[0]);
}

// All visibilities of a tile, groups of eight in a two-stage pipeline.
template <int G, int F, int NB, bool STAGED, uint32_t PLANE1, bool DEEP>
__device__ __forceinline__ void gather_tile(float2* out, int count, int a_off, int ow, const float* gv,
                                            __amdgpu_buffer_rsrc_t ra, uint64_t g_w, uint32_t lane_a,
                                            const char* box) {
    const uint32_t gw_off = gw_row_offset<F>(ow);
    Fetch8<G> buf[2];
    fetch8<G, STAGED, PLANE1, DEEP>(buf[0], 0, a_off, ra, lane_a, box);
#pragma unroll
    for (int g0 = 0; g0 < NB; g0 += 8) {
        if (g0 < count) {
            if (g0 + 8 < NB && g0 + 8 < count)
                fetch8<G, STAGED, PLANE1, DEEP>(buf[((g0 / 8) + 1) & 1], g0 + 8, a_off, ra, lane_a, box);
            sum8<G, F>(buf[(g0 / 8) & 1], gv + g0, gw_off, g_w, out, g0);
        }
    }
}

// Kernel variants: (LDS box per wavefront in bytes, largest tile, deep).
// Box 0 gathers through the caches only. A box is a multiple of 2 KiB (the
// staging copy fills whole steps of 64 slots of 32 bytes). The largest, 18
// KiB, lets two workgroups of four wavefronts (boxes and 512-byte output
// staging) fit the CU's 160 KiB of LDS; it holds dense 64-visibility tiles
// that a 16 KiB box does not (rows of 24 slots: 24 rows instead of 21). A deep variant reads the 4 w values
// of a tap with loads of one value each (naturally aligned at any first w),
// for subgrids with more w planes than the w support; it never stages.
// A D1 variant maps the lanes as the paper's kernel D1 (two visibilities
// per wavefront, lanes over a v-row's (t_u, t_w) values, accumulation along
// v, then a reduction); it reads one value per lane, so it also takes
// subgrids deeper than the w support, and never stages.
struct Variant { int box; int nb; bool deep; bool d1; };
constexpr Variant kVariants[] = {{0, 64, false, false},     {8192, 32, false, false},  {12288, 32, false, false},
                                 {16384, 32, false, false}, {18432, 64, false, false}, {0, 64, true, false},
                                 {0, 64, false, true}};
static_assert(kVariants[kD1Variant].d1 && kVariants[kD1Variant].box == 0, "D1 variant index");
static_assert(kVariants[kDeepVariant].deep && kVariants[kDeepVariant].box == 0, "deep variant index");
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

}  // namespace
}  // namespace dg
