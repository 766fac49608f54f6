// gfx950 kernel for the gradients of a real loss L with respect to the two
// GCF tables, given dL/dV (the chain rule through the weighted sum of
// Section 2; each visibility is linear in each table):
//
//   dL/dG_uv[o_v][o_u][t_v][t_u] += Re(conj(g_i) * sum_tw G_w[o_w][t_w] * A[y+t_v][x+t_u][z+t_w])
//   dL/dG_w[o_w][t_w]            += Re(conj(g_i) * sum_{t_v,t_u} G_uv[o_v][o_u][t_v][t_u] * A[...])
//
// for every in-range visibility i with gradient g_i. The gather is the
// degrid kernel's: each wavefront takes tiles of the plan (grid-stride over
// the tile list), lane j of 64 takes tap (t_v, t_u) = (j / 8, j % 8) and
// reads the 4 w values of its tap through bounds-checked buffer loads.
//
//  * dL/dG_uv: every visibility adds one value per lane to the 64 contiguous
//    entries of its (o_v, o_u) block. When the table fits (os_uv <= 16,
//    64 KiB) the workgroup keeps its own copy in LDS and seven of every
//    sixteen visibilities add there (one LDS float add, no two lanes on one
//    entry; the copy is added to the output once at the end), the others
//    straight to the output with one coalesced float atomic, so that the two
//    atomic units work side by side (7/16 measured faster than 3/8 and 1/2,
//    with caches cold and warm). Float atomics make the order, and so the
//    last bits, depend on timing;
//  * dL/dG_w: per w tap, the shares of a group of eight visibilities are
//    summed over the 64 lanes together (the degrid kernel's eight-way
//    permlane/DPP reduction), and lane 8m adds visibility m's four sums to
//    a private per-wavefront LDS array [o_w][t_w][8] (eight distinct slots
//    per add); at the end each row is summed and added to the output.
#include "dg_device.h"

namespace dg {
namespace {

constexpr int kGroup = 8;   // visibilities whose loads are issued together

template <int G>
struct GradFetch {
    uint32_t raw[kGroup][GridTraits<G>::kWords];
    float gv[kGroup];
};

// The loads of visibilities g0 .. g0+7 (all of them, without branches, so
// that the compiler can count the loads in flight and wait for exactly the
// ones it needs): a visibility out of range or past the tile has the
// out-of-range offset (its subgrid loads return zeros) and table block 0.
template <int G, int F, bool DEEP>
__device__ __forceinline__ void grad_fetch(GradFetch<G>& f, int g0, int a_off, int tab,
                                           __amdgpu_buffer_rsrc_t ra, __amdgpu_buffer_rsrc_t rg, uint32_t lane_a) {
    const int lane = lane_id();
#pragma unroll
    for (int k = 0; k < kGroup; ++k) {
        const uint32_t aj = (uint32_t)__builtin_amdgcn_readlane(a_off, g0 + k);
        if constexpr (DEEP)
            load_w4_narrow<G>(ra, lane_a + aj, f.raw[k]);
        else
            load_w4<G>(ra, lane_a + aj, f.raw[k]);
        f.gv[k] = load_gcf_rsrc<F>(rg, (uint32_t)(__builtin_amdgcn_readlane(tab, g0 + k) + lane) * GcfTraits<F>::kBytes);
    }
}

constexpr int kWGroups = 8;   // per-visibility slots of the dL/dG_w sums in LDS
// bit k: visibility k of a group adds to the LDS copy; even groups take 3
// of their 8 visibilities there, odd groups 4
constexpr uint32_t kLdsShareEven = 0x49u, kLdsShareOdd = 0x55u;

// w value tw of one fetched cell, widened to float32.
template <int G>
__device__ __forceinline__ void widen_one(const uint32_t (&raw)[GridTraits<G>::kWords], int tw, float& re,
                                          float& im) {
    if constexpr (G == kGridC64) {
        re = __uint_as_float(raw[2 * tw]);
        im = __uint_as_float(raw[2 * tw + 1]);
    } else if constexpr (G == kGridCBF16) {
        re = __uint_as_float(raw[tw] << 16);
        im = __uint_as_float(raw[tw] & 0xFFFF0000u);
    } else {
        const __half2 h = __builtin_bit_cast(__half2, raw[tw]);
        re = __low2float(h);
        im = __high2float(h);
    }
}

// LDS_UV: the workgroup accumulates dL/dG_uv in LDS (the table fits).
template <int G, int F, bool DEEP, bool LDS_UV>
__global__ __launch_bounds__(kTableGradThreads) void table_grad_kernel(TableGradParams P) {
    // [n_uv] shared by the workgroup (LDS_UV), then [waves][os_w * 4][8]
    extern __shared__ float s_acc[];
    const int lane = lane_id();
    const int waves = (int)(blockDim.x / kWave);
    // wave-uniform as far as the compiler knows, so that the tile index and
    // the buffer resources built from it stay in scalar registers (a
    // divergent resource would wrap every buffer load in a loop)
    const int wv = uniform((int)(threadIdx.x / kWave));
    const Problem& pr = P.prob;
    const bool want_uv = P.grad_uv != nullptr;
    const bool want_w = P.grad_w != nullptr;
    const int rows_w = pr.os_w * kSupportW;
    const int n_uv = LDS_UV ? pr.os_uv * pr.os_uv * kSupportUV * kSupportUV : 0;
    float* s_uv = s_acc;
    float* acc = s_acc + n_uv + (size_t)wv * rows_w * kWGroups;
    if (LDS_UV)
        for (int i = (int)threadIdx.x; i < n_uv; i += (int)blockDim.x) s_uv[i] = 0.0f;
    if (want_w)
        for (int i = lane; i < rows_w * kWGroups; i += kWave) acc[i] = 0.0f;
    __syncthreads();

    const uint64_t g_w = uniform_u64((uint64_t)pr.g_w);
    const __amdgpu_buffer_rsrc_t rg = make_rsrc(pr.g_uv, pr.guv_bytes);
    const uint32_t lane_a = (uint32_t)(((lane >> 3) * pr.n_u + (lane & 7)) * pr.n_w) * GridTraits<G>::kElemBytes;

    for (int64_t t = (int64_t)blockIdx.x * waves + wv; t < P.n_tiles; t += (int64_t)gridDim.x * waves) {
        const Tile tc = load_tile(P.tiles, (int)t);
        const int count = tc.count;
        const int64_t vis = P.tile_vis[t * kMaxNb + lane];
        int32_t x0 = 0, y0 = 0, cell = 0, tab = 0, ow = 0;
        bool in_range = false;
        float2 g = make_float2(0.f, 0.f);
        if (lane < count) {
            const double* c = pr.uvw + 3 * vis;
            in_range = coords_from(pr, c[0], c[1], c[2], cell, tab, ow, x0, y0);
            if (in_range) g = static_cast<const float2*>(pr.vis)[vis];
        }
        if (!in_range) {
            tab = 0;
            ow = 0;
        }
        const uint64_t live = __ballot(in_range);
        const int a_off = in_range ? cell * (int)GridTraits<G>::kElemBytes : (int)kOutOfRange;
        const uint32_t gw_off = gw_row_offset<F>(ow);
        const char* sub_base = static_cast<const char*>(pr.subgrids) + (int64_t)tc.sub * pr.sub_bytes;
        const __amdgpu_buffer_rsrc_t ra = make_rsrc(sub_base, pr.sub_bytes);

        // groups of eight in a two-stage pipeline, unrolled over the largest
        // tile so that both buffers stay in registers
        GradFetch<G> buf[2];
        grad_fetch<G, F, DEEP>(buf[0], 0, a_off, tab, ra, rg, lane_a);
#pragma unroll
        for (int g0 = 0; g0 < kMaxNb; g0 += kGroup) {
            if (g0 < count) {
                const int cur = (g0 / kGroup) & 1;
                if (g0 + kGroup < kMaxNb && g0 + kGroup < count)
                    grad_fetch<G, F, DEEP>(buf[cur ^ 1], g0 + kGroup, a_off, tab, ra, rg, lane_a);
                // dL/dV of the group's visibilities (zero for the ones out
                // of range or past the tile)
                // (g is 0 on lanes out of range or past the tile, and their
                // subgrid loads returned zeros: their shares below are 0
                // without any branch)
                float gre[kGroup], gim[kGroup];
#pragma unroll
                for (int k = 0; k < kGroup; ++k) {
                    gre[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(g.x), g0 + k));
                    gim[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(g.y), g0 + k));
                }
                if (want_uv) {
                    // the eight G_w rows' scalar loads go out together, then
                    // the eight shares, then the atomics back to back (an
                    // LDS atomic between two scalar loads would make the
                    // second one's wait also wait for the atomic)
                    float4 gwr[kGroup];
#pragma unroll
                    for (int k = 0; k < kGroup; ++k)
                        gwr[k] = load_gw_row<F>(g_w, (uint32_t)__builtin_amdgcn_readlane((int)gw_off, g0 + k));
                    float val[kGroup];
#pragma unroll
                    for (int k = 0; k < kGroup; ++k) {
                        float re[4], im[4];
                        widen_w4<G>(buf[cur].raw[k], re, im);
                        const float4 gw = gwr[k];
                        const float sr = wsum4<F>(gw, re);
                        const float si = wsum4<F>(gw, im);
                        val[k] = gre[k] * sr + gim[k] * si;
                    }
#pragma unroll
                    for (int k = 0; k < kGroup; ++k) {
                        const int j = g0 + k;
                        if (!((live >> j) & 1ull)) continue;   // wave-uniform: no atomic for nothing
                        const int e = __builtin_amdgcn_readlane(tab, j) + lane;
                        // LDS float atomics and global float atomics run in
                        // different units: 7 of every 16 visibilities go to
                        // LDS, the others to global memory, so that the two
                        // overlap
                        const uint32_t lds_share = ((g0 / kGroup) & 1) ? kLdsShareOdd : kLdsShareEven;
                        if (LDS_UV && ((lds_share >> k) & 1u))
                            atomicAdd(s_uv + e, val[k]);
                        else
                            atomicAdd(P.grad_uv + e, val[k]);
                    }
                }
                if (want_w) {
                    // per w tap: the eight visibilities' shares summed over
                    // the 64 lanes together (reduce8: lane l ends with
                    // visibility l / 8's sum), then one add per visibility
                    // by lane 8m into this wavefront's own slots (LDS
                    // operations of a wavefront run in order)
                    float r[kSupportW];
#pragma unroll
                    for (int tw = 0; tw < kSupportW; ++tw) {
                        float x[kGroup];
#pragma unroll
                        for (int k = 0; k < kGroup; ++k) {
                            float re1, im1;
                            widen_one<G>(buf[cur].raw[k], tw, re1, im1);
                            x[k] = buf[cur].gv[k] * (gre[k] * re1 + gim[k] * im1);
                        }
                        reduce8(x);
                        r[tw] = x[0];
                    }
                    int row = 0;   // G_w row of visibility g0 + lane / 8
#pragma unroll
                    for (int k = 0; k < kGroup; ++k) {
                        const int o = __builtin_amdgcn_readlane(ow, g0 + k);
                        row = (lane >> 3) == k ? o : row;
                    }
                    if ((lane & (kWGroups - 1)) == 0) {
#pragma unroll
                        for (int tw = 0; tw < kSupportW; ++tw)
                            acc[(row * kSupportW + tw) * kWGroups + (lane >> 3)] += r[tw];
                    }
                }
            }
        }
    }
    __syncthreads();
    // Every workgroup ends at about the same time; each starts its flush at
    // its own place in the table, so that the adds to one entry spread out
    // instead of queueing behind each other.
    if (LDS_UV) {
        const int rot = (int)(((int64_t)blockIdx.x * n_uv) / (int64_t)gridDim.x);
        for (int k = (int)threadIdx.x; k < n_uv; k += (int)blockDim.x) {
            const int i = k + rot < n_uv ? k + rot : k + rot - n_uv;
            const float v = s_uv[i];
            if (v != 0.0f) atomicAdd(P.grad_uv + i, v);   // entries no visibility reached stay as they are
        }
    }
    if (want_w) {
        // the workgroup's rows summed over its wavefronts and lane groups,
        // then one add per row
        const float* acc0 = s_acc + n_uv;
        for (int r = (int)threadIdx.x; r < rows_w; r += (int)blockDim.x) {
            float s = 0.0f;
            for (int w = 0; w < waves; ++w)
#pragma unroll
                for (int m = 0; m < kWGroups; ++m) s += acc0[((size_t)w * rows_w + r) * kWGroups + m];
            if (s != 0.0f) atomicAdd(P.grad_w + r, s);
        }
    }
}

__global__ void zero_f32_kernel(float* p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0f;
}

template <int G, int F, bool DEEP, bool LDS_UV>
hipError_t launch_tg(const TableGradParams& p, int blocks, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((table_grad_kernel<G, F, DEEP, LDS_UV>), dim3(blocks), dim3(kTableGradThreads), lds, s, p);
    return hipGetLastError();
}

template <int G, int F>
hipError_t launch_tg_d(const TableGradParams& p, bool deep, bool lds_uv, int blocks, size_t lds, hipStream_t s) {
    if (deep)
        return lds_uv ? launch_tg<G, F, true, true>(p, blocks, lds, s) : launch_tg<G, F, true, false>(p, blocks, lds, s);
    return lds_uv ? launch_tg<G, F, false, true>(p, blocks, lds, s) : launch_tg<G, F, false, false>(p, blocks, lds, s);
}

}  // namespace

// LDS of the table-gradient kernel: the workgroup's copy of dL/dG_uv when it
// is wanted, takes at most 64 KiB (os_uv <= 16) and the total fits max_lds
// (the device's LDS per workgroup), and os_w * 4 * 8 floats per wavefront
// for dL/dG_w.
void table_grad_shape(int os_uv, int os_w, bool want_uv, bool want_w, size_t max_lds, bool* lds_uv,
                      size_t* lds_bytes) {
    const size_t uv = (size_t)os_uv * os_uv * kSupportUV * kSupportUV * sizeof(float);
    const size_t w = want_w ? (size_t)(kTableGradThreads / kWave) * os_w * kSupportW * kWGroups * sizeof(float) : 0;
    *lds_uv = want_uv && uv <= 65536 && uv + w <= max_lds;
    *lds_bytes = (*lds_uv ? uv : 0) + w;
}

hipError_t launch_table_grad(const TableGradParams& p, int grid_kind, int gcf_kind, bool deep, int blocks,
                             size_t max_lds, hipStream_t stream) {
    bool lds_uv = false;
    size_t lds = 0;
    table_grad_shape(p.prob.os_uv, p.prob.os_w, p.grad_uv != nullptr, p.grad_w != nullptr, max_lds, &lds_uv, &lds);
    switch (grid_kind * 3 + gcf_kind) {
        case kGridC64 * 3 + kGcfF32: return launch_tg_d<kGridC64, kGcfF32>(p, deep, lds_uv, blocks, lds, stream);
        case kGridC64 * 3 + kGcfF16: return launch_tg_d<kGridC64, kGcfF16>(p, deep, lds_uv, blocks, lds, stream);
        case kGridC64 * 3 + kGcfBF16: return launch_tg_d<kGridC64, kGcfBF16>(p, deep, lds_uv, blocks, lds, stream);
        case kGridCBF16 * 3 + kGcfF32: return launch_tg_d<kGridCBF16, kGcfF32>(p, deep, lds_uv, blocks, lds, stream);
        case kGridCBF16 * 3 + kGcfF16: return launch_tg_d<kGridCBF16, kGcfF16>(p, deep, lds_uv, blocks, lds, stream);
        case kGridCBF16 * 3 + kGcfBF16: return launch_tg_d<kGridCBF16, kGcfBF16>(p, deep, lds_uv, blocks, lds, stream);
        case kGridCF16 * 3 + kGcfF32: return launch_tg_d<kGridCF16, kGcfF32>(p, deep, lds_uv, blocks, lds, stream);
        case kGridCF16 * 3 + kGcfF16: return launch_tg_d<kGridCF16, kGcfF16>(p, deep, lds_uv, blocks, lds, stream);
        case kGridCF16 * 3 + kGcfBF16: return launch_tg_d<kGridCF16, kGcfBF16>(p, deep, lds_uv, blocks, lds, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_zero_f32(float* p, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(zero_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

}  // namespace dg
