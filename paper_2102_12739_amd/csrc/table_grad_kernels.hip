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
//    entries of its (o_v, o_u) block: one coalesced float atomic per
//    visibility (the table is small and shared by all visibilities, so the
//    adds have to meet in memory; float atomics make the order, and so the
//    last bits, depend on timing);
//  * dL/dG_w: each wavefront keeps a private LDS array [o_w][t_w][lane] and
//    adds its lane's share of every visibility there (no two lanes share a
//    slot, so there are no bank conflicts and no atomics); at the end it sums
//    each row over the lanes and adds it to the output with one float atomic
//    per row.
#include "dg_device.h"

namespace dg {
namespace {

constexpr int kGroup = 8;   // visibilities whose loads are issued together

template <int G>
struct GradFetch {
    uint32_t raw[kGroup][GridTraits<G>::kWords];
    float gv[kGroup];
};

template <int G, int F, bool DEEP>
__device__ __forceinline__ void grad_fetch(GradFetch<G>& f, int g0, int count, int a_off, int tab,
                                           __amdgpu_buffer_rsrc_t ra, __amdgpu_buffer_rsrc_t rg, uint32_t lane_a,
                                           bool want_w) {
    const int lane = lane_id();
#pragma unroll
    for (int k = 0; k < kGroup; ++k) {
        if (g0 + k < count) {
            const uint32_t aj = (uint32_t)__builtin_amdgcn_readlane(a_off, g0 + k);
            if constexpr (DEEP)
                load_w4_narrow<G>(ra, lane_a + aj, f.raw[k]);
            else
                load_w4<G>(ra, lane_a + aj, f.raw[k]);
            f.gv[k] = want_w ? load_gcf_rsrc<F>(rg, (uint32_t)(__builtin_amdgcn_readlane(tab, g0 + k) + lane) *
                                                        GcfTraits<F>::kBytes)
                             : 0.0f;
        }
    }
}

template <int G, int F, bool DEEP>
__global__ __launch_bounds__(kBlockThreads) void table_grad_kernel(TableGradParams P) {
    extern __shared__ float s_acc[];   // [waves][os_w * 4][64] when grad_w is wanted
    const int lane = lane_id();
    const int waves = (int)(blockDim.x / kWave);
    const int wv = (int)(threadIdx.x / kWave);
    const Problem& pr = P.prob;
    const bool want_uv = P.grad_uv != nullptr;
    const bool want_w = P.grad_w != nullptr;
    const int rows_w = pr.os_w * kSupportW;
    float* acc = s_acc + (size_t)wv * rows_w * kWave;
    if (want_w)
        for (int r = 0; r < rows_w; ++r) acc[r * kWave + lane] = 0.0f;

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
        grad_fetch<G, F, DEEP>(buf[0], 0, count, a_off, tab, ra, rg, lane_a, want_w);
#pragma unroll
        for (int g0 = 0; g0 < kMaxNb; g0 += kGroup) {
            if (g0 < count) {
                const int cur = (g0 / kGroup) & 1;
                if (g0 + kGroup < kMaxNb && g0 + kGroup < count)
                    grad_fetch<G, F, DEEP>(buf[cur ^ 1], g0 + kGroup, count, a_off, tab, ra, rg, lane_a, want_w);
#pragma unroll
                for (int k = 0; k < kGroup; ++k) {
                    const int j = g0 + k;
                    if (j >= count || !((live >> j) & 1ull)) continue;   // wave-uniform
                    float re[4], im[4];
                    widen_w4<G>(buf[cur].raw[k], re, im);
                    const float gre = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(g.x), j));
                    const float gim = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(g.y), j));
                    if (want_uv) {
                        const float4 gw = load_gw_row<F>(g_w, (uint32_t)__builtin_amdgcn_readlane((int)gw_off, j));
                        const float sr = gw.x * re[0] + gw.y * re[1] + gw.z * re[2] + gw.w * re[3];
                        const float si = gw.x * im[0] + gw.y * im[1] + gw.z * im[2] + gw.w * im[3];
                        atomicAdd(P.grad_uv + __builtin_amdgcn_readlane(tab, j) + lane, gre * sr + gim * si);
                    }
                    if (want_w) {
                        const int row = __builtin_amdgcn_readlane(ow, j) * kSupportW;
                        const float gv = buf[cur].gv[k];
#pragma unroll
                        for (int tw = 0; tw < kSupportW; ++tw) {
                            float* slot = acc + (row + tw) * kWave + lane;
                            *slot += gv * (gre * re[tw] + gim * im[tw]);
                        }
                    }
                }
            }
        }
    }
    if (want_w) {
        wave_lds_sync();
        // lane r sums row r over the 64 lanes' slots, starting at a different
        // slot per row so that the 64 reads of one step fall on distinct banks
        for (int r = lane; r < rows_w; r += kWave) {
            float s = 0.0f;
            for (int j = 0; j < kWave; ++j) s += acc[r * kWave + ((j + r) & (kWave - 1))];
            atomicAdd(P.grad_w + r, s);
        }
    }
}

__global__ void zero_f32_kernel(float* p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0f;
}

template <int G, int F, bool DEEP>
hipError_t launch_tg(const TableGradParams& p, int blocks, int waves, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((table_grad_kernel<G, F, DEEP>), dim3(blocks), dim3(waves * kWave), lds, s, p);
    return hipGetLastError();
}

template <int G, int F>
hipError_t launch_tg_d(const TableGradParams& p, bool deep, int blocks, int waves, size_t lds, hipStream_t s) {
    return deep ? launch_tg<G, F, true>(p, blocks, waves, lds, s) : launch_tg<G, F, false>(p, blocks, waves, lds, s);
}

}  // namespace

// Wavefronts per workgroup and LDS bytes of the table-gradient kernel: each
// wavefront's G_w accumulator takes os_w * 4 * 64 floats (16 KiB at os_w 16),
// and a workgroup keeps within 64 KiB.
void table_grad_shape(int os_w, bool want_w, int* waves, size_t* lds_bytes) {
    const size_t per_wave = want_w ? (size_t)os_w * kSupportW * kWave * sizeof(float) : 0;
    int w = kWavesPerBlock;
    while (w > 1 && per_wave * (size_t)w > 65536) w /= 2;
    *waves = w;
    *lds_bytes = per_wave * (size_t)w;
}

hipError_t launch_table_grad(const TableGradParams& p, int grid_kind, int gcf_kind, bool deep, int blocks,
                             hipStream_t stream) {
    int waves = 0;
    size_t lds = 0;
    table_grad_shape(p.prob.os_w, p.grad_w != nullptr, &waves, &lds);
    switch (grid_kind * 3 + gcf_kind) {
        case kGridC64 * 3 + kGcfF32: return launch_tg_d<kGridC64, kGcfF32>(p, deep, blocks, waves, lds, stream);
        case kGridC64 * 3 + kGcfF16: return launch_tg_d<kGridC64, kGcfF16>(p, deep, blocks, waves, lds, stream);
        case kGridC64 * 3 + kGcfBF16: return launch_tg_d<kGridC64, kGcfBF16>(p, deep, blocks, waves, lds, stream);
        case kGridCBF16 * 3 + kGcfF32: return launch_tg_d<kGridCBF16, kGcfF32>(p, deep, blocks, waves, lds, stream);
        case kGridCBF16 * 3 + kGcfF16: return launch_tg_d<kGridCBF16, kGcfF16>(p, deep, blocks, waves, lds, stream);
        case kGridCBF16 * 3 + kGcfBF16: return launch_tg_d<kGridCBF16, kGcfBF16>(p, deep, blocks, waves, lds, stream);
        case kGridCF16 * 3 + kGcfF32: return launch_tg_d<kGridCF16, kGcfF32>(p, deep, blocks, waves, lds, stream);
        case kGridCF16 * 3 + kGcfF16: return launch_tg_d<kGridCF16, kGcfF16>(p, deep, blocks, waves, lds, stream);
        case kGridCF16 * 3 + kGcfBF16: return launch_tg_d<kGridCF16, kGcfBF16>(p, deep, blocks, waves, lds, stream);
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
