// Degridding for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc): the
// kernels of degrid_execute_noalloc and the device scratch they use.
//
// The scratch is one file-scope device array per GPU, `scratch`, of
// kNoAllocBytes bytes, holding
//   - the tile cursor (its own 128-byte line) and the tile count;
//   - the caller's visibility offsets, staged from the host ([S+1] int64);
//   - the first tile of every subgrid ([S+1] int64, a prefix sum of
//     ceil(N_s / n_b)).
// Host code never passes the array's name to a kernel: at a device's first
// call, hipGetSymbolAddress gives that device's copy's address, which is
// kept per device and used for every copy and launch. Every call on one GPU
// shares the array, so calls that overlap on one GPU race.
//
// Work: one tile is n_b consecutive visibilities of one subgrid, in input
// order (Section 2 gives each thread block N_b visibilities of a subgrid);
// a persistent grid claims tiles from the cursor and finds a tile's subgrid
// by binary search over the tile offsets. The gather is the degrid
// kernel's cache gather (gather_tile).
#include "dg_device.h"

#include <mutex>

namespace dg {
namespace {

constexpr size_t kNoAllocCursor = 0;      // uint32 tile cursor
constexpr size_t kNoAllocTiles = 128;     // int64 tile count
constexpr size_t kNoAllocOffsets = 256;   // int64 visibility offsets [S+1]
constexpr size_t kNoAllocTileOffsets = kNoAllocOffsets + sizeof(int64_t) * (kNoAllocMaxSubgrids + 1);
constexpr size_t kNoAllocUsed = kNoAllocTileOffsets + sizeof(int64_t) * (kNoAllocMaxSubgrids + 1);
static_assert(kNoAllocUsed <= kNoAllocBytes, "scratch layout exceeds the array");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

typedef const __attribute__((address_space(4))) int64_t* ConstI64Ptr;

constexpr int kSetupThreads = 1024;

// Tile offsets of every subgrid (exclusive prefix sum of ceil(N_s / n_b)),
// the tile count, the cursor reset to 0 and the caller's out-of-range count
// cleared. One workgroup; thread k scans a contiguous run of subgrids.
__global__ __launch_bounds__(kSetupThreads) void noalloc_setup_kernel(unsigned char* scr, int64_t n_sub, int nb,
                                                                      unsigned long long* oob_out) {
    const int64_t* off = reinterpret_cast<const int64_t*>(scr + kNoAllocOffsets);
    int64_t* toff = reinterpret_cast<int64_t*>(scr + kNoAllocTileOffsets);
    __shared__ int64_t part[kSetupThreads];
    const int64_t per = (n_sub + kSetupThreads - 1) / kSetupThreads;
    const int64_t s0 = (int64_t)threadIdx.x * per;
    const int64_t s1 = s0 + per < n_sub ? s0 + per : n_sub;
    int64_t sum = 0;
    for (int64_t s = s0; s < s1; ++s) sum += (off[s + 1] - off[s] + nb - 1) / nb;
    part[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int k = 0; k < kSetupThreads; ++k) {
            const int64_t x = part[k];
            part[k] = run;
            run += x;
        }
        toff[n_sub] = run;
        *reinterpret_cast<int64_t*>(scr + kNoAllocTiles) = run;
        *reinterpret_cast<uint32_t*>(scr + kNoAllocCursor) = 0u;
        if (oob_out) *oob_out = 0ull;
    }
    __syncthreads();
    int64_t run = part[threadIdx.x];
    for (int64_t s = s0; s < s1; ++s) {
        toff[s] = run;
        run += (off[s + 1] - off[s] + nb - 1) / nb;
    }
}

template <int G, int F, bool DEEP>
__global__ __launch_bounds__(kBlockThreads, 2) void degrid_noalloc_kernel(Problem pr, unsigned char* scr,
                                                                          int64_t n_sub, int nb,
                                                                          unsigned long long* oob_out) {
    using GT = GridTraits<G>;
    __shared__ float2 s_out[kWavesPerBlock][kMaxNb];
    const int lane = lane_id();
    const int wv = (int)(threadIdx.x / kWave);
    uint32_t* cursor = reinterpret_cast<uint32_t*>(scr + kNoAllocCursor);
    const ConstI64Ptr off = (ConstI64Ptr)uniform_u64((uint64_t)(scr + kNoAllocOffsets));
    const ConstI64Ptr toff = (ConstI64Ptr)uniform_u64((uint64_t)(scr + kNoAllocTileOffsets));
    const int64_t n_tiles = *(ConstI64Ptr)uniform_u64((uint64_t)(scr + kNoAllocTiles));
    const __amdgpu_buffer_rsrc_t rg = make_rsrc(pr.g_uv, pr.guv_bytes);
    const uint64_t g_w = uniform_u64((uint64_t)pr.g_w);
    const uint32_t lane_g = (uint32_t)lane * GcfTraits<F>::kBytes;
    const uint32_t lane_a = (uint32_t)(((lane >> 3) * pr.n_u + (lane & 7)) * pr.n_w) * GT::kElemBytes;
    uint32_t wave_oob = 0;
    int64_t s = 0;   // subgrid of the previous tile (tiles are claimed in increasing order)
    while (true) {
        uint32_t idx = 0;
        if (lane == 0) idx = atomicAdd(cursor, 1u);
        const int64_t t = (int64_t)(uint32_t)uniform((int)idx);
        if (t >= n_tiles) break;
        // subgrid of tile t: the last s with toff[s] <= t (empty subgrids
        // share their offset with the next one). The previous tile's
        // subgrid is tried first.
        if (!(toff[s] <= t && t < toff[s + 1])) {
            int64_t lo = 0, hi = n_sub;
            while (hi - lo > 1) {
                const int64_t mid = (lo + hi) >> 1;
                if (toff[mid] <= t) lo = mid; else hi = mid;
            }
            s = lo;
        }
        const int64_t beg = off[s] + (t - toff[s]) * nb;
        const int64_t lim = off[s + 1];
        const int count = (int)(beg + nb < lim ? nb : lim - beg);
        const int64_t vis = beg + lane;

        int32_t x0 = 0, y0 = 0, cell = 0, tab = 0, ow = 0;
        bool in_range = false;
        if (lane < count) {
            const double* c = pr.uvw + 3 * vis;
            in_range = coords_from(pr, c[0], c[1], c[2], cell, tab, ow, x0, y0);
        }
        if (!in_range) ow = 0;
        wave_oob += (uint32_t)__popcll(__ballot(lane < count && !in_range));

        const char* sub_base = static_cast<const char*>(pr.subgrids) + s * (int64_t)pr.sub_bytes;
        const __amdgpu_buffer_rsrc_t ra = make_rsrc(sub_base, pr.sub_bytes);
        // G_uv weights of the tile (block offset in the scalar offset; an
        // out-of-range visibility reads block 0 and is written as 0 below)
        const int g_off = in_range ? tab * (int)GcfTraits<F>::kBytes : 0;
        float gv[kMaxNb];
#pragma unroll
        for (int g0 = 0; g0 < kMaxNb; g0 += 8) {
            if (g0 < count) {
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    gv[g0 + k] = load_gcf_rsrc<F>(rg, lane_g, (uint32_t)__builtin_amdgcn_readlane(g_off, g0 + k));
            }
        }
        const int a_off = in_range ? cell * (int)GT::kElemBytes : (int)kOutOfRange;
        gather_tile<G, F, kMaxNb, false, 16, DEEP>(s_out[wv], count, a_off, ow, gv, ra, g_w, lane_a, nullptr);
        wave_lds_sync();
        if (lane < count) static_cast<float2*>(pr.vis)[vis] = in_range ? s_out[wv][lane] : make_float2(0.f, 0.f);
        wave_lds_sync();
    }
    if (oob_out && lane == 0 && wave_oob != 0u) atomicAdd(oob_out, (unsigned long long)wave_oob);
}

template <int G, int F>
hipError_t launch_main(const Problem& pr, bool deep, int blocks, unsigned char* scr, int64_t n_sub, int nb,
                       unsigned long long* oob_out, hipStream_t stream) {
    if (deep)
        hipLaunchKernelGGL((degrid_noalloc_kernel<G, F, true>), dim3(blocks), dim3(kBlockThreads), 0, stream, pr, scr,
                           n_sub, nb, oob_out);
    else
        hipLaunchKernelGGL((degrid_noalloc_kernel<G, F, false>), dim3(blocks), dim3(kBlockThreads), 0, stream, pr,
                           scr, n_sub, nb, oob_out);
    return hipGetLastError();
}

template <int G, int F>
hipError_t occupancy(bool deep, int* n) {
    return deep ? hipOccupancyMaxActiveBlocksPerMultiprocessor(n, degrid_noalloc_kernel<G, F, true>, kBlockThreads, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(n, degrid_noalloc_kernel<G, F, false>, kBlockThreads, 0);
}

hipError_t launch_main_any(const Problem& pr, int grid_kind, int gcf_kind, bool deep, int blocks,
                           unsigned char* scr, int64_t n_sub, int nb, unsigned long long* oob_out,
                           hipStream_t stream) {
#define DG_CALL(G, F) launch_main<G, F>(pr, deep, blocks, scr, n_sub, nb, oob_out, stream)
    switch (grid_kind * 3 + gcf_kind) {
        case kGridC64 * 3 + kGcfF32: return DG_CALL(kGridC64, kGcfF32);
        case kGridC64 * 3 + kGcfF16: return DG_CALL(kGridC64, kGcfF16);
        case kGridC64 * 3 + kGcfBF16: return DG_CALL(kGridC64, kGcfBF16);
        case kGridCBF16 * 3 + kGcfF32: return DG_CALL(kGridCBF16, kGcfF32);
        case kGridCBF16 * 3 + kGcfF16: return DG_CALL(kGridCBF16, kGcfF16);
        case kGridCBF16 * 3 + kGcfBF16: return DG_CALL(kGridCBF16, kGcfBF16);
        case kGridCF16 * 3 + kGcfF32: return DG_CALL(kGridCF16, kGcfF32);
        case kGridCF16 * 3 + kGcfF16: return DG_CALL(kGridCF16, kGcfF16);
        case kGridCF16 * 3 + kGcfBF16: return DG_CALL(kGridCF16, kGcfBF16);
        default: return hipErrorInvalidValue;
    }
#undef DG_CALL
}

hipError_t occupancy_any(int grid_kind, int gcf_kind, bool deep, int* n) {
#define DG_CALL(G, F) occupancy<G, F>(deep, n)
    switch (grid_kind * 3 + gcf_kind) {
        case kGridC64 * 3 + kGcfF32: return DG_CALL(kGridC64, kGcfF32);
        case kGridC64 * 3 + kGcfF16: return DG_CALL(kGridC64, kGcfF16);
        case kGridC64 * 3 + kGcfBF16: return DG_CALL(kGridC64, kGcfBF16);
        case kGridCBF16 * 3 + kGcfF32: return DG_CALL(kGridCBF16, kGcfF32);
        case kGridCBF16 * 3 + kGcfF16: return DG_CALL(kGridCBF16, kGcfF16);
        case kGridCBF16 * 3 + kGcfBF16: return DG_CALL(kGridCBF16, kGcfBF16);
        case kGridCF16 * 3 + kGcfF32: return DG_CALL(kGridCF16, kGcfF32);
        case kGridCF16 * 3 + kGcfF16: return DG_CALL(kGridCF16, kGcfF16);
        case kGridCF16 * 3 + kGcfBF16: return DG_CALL(kGridCF16, kGcfBF16);
        default: return hipErrorInvalidValue;
    }
#undef DG_CALL
}

// Per device: the address of this device's copy of `scratch` and the
// resident workgroups of each kernel instance, looked up once.
constexpr int kMaxDevices = 64;
struct DeviceState {
    unsigned char* scratch = nullptr;
    int n_cu = 0;
    int occ[9][2] = {};
};
std::mutex g_mutex;
DeviceState g_dev[kMaxDevices];

hipError_t device_state(int grid_kind, int gcf_kind, bool deep, unsigned char** scr, int* resident) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mutex);
    DeviceState& d = g_dev[dev];
    if (!d.scratch) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        e = hipDeviceGetAttribute(&d.n_cu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        d.scratch = static_cast<unsigned char*>(p);
    }
    int& occ = d.occ[grid_kind * 3 + gcf_kind][deep ? 1 : 0];
    if (occ == 0) {
        e = occupancy_any(grid_kind, gcf_kind, deep, &occ);
        if (e != hipSuccess) return e;
        if (occ < 1) occ = 1;
    }
    *scr = d.scratch;
    *resident = d.n_cu * occ;
    return hipSuccess;
}

}  // namespace

hipError_t launch_degrid_noalloc(const Problem& pr, int grid_kind, int gcf_kind, bool deep,
                                 const int64_t* offsets_host, int64_t n_sub, int nb, int64_t n_tiles,
                                 unsigned long long* oob_out, hipStream_t stream) {
    if (n_sub < 0 || n_sub > kNoAllocMaxSubgrids || nb < 1 || nb > kMaxNb) return hipErrorInvalidValue;
    unsigned char* scr = nullptr;
    int resident = 0;
    hipError_t e = device_state(grid_kind, gcf_kind, deep, &scr, &resident);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(scr + kNoAllocOffsets, offsets_host, sizeof(int64_t) * (size_t)(n_sub + 1),
                       hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(noalloc_setup_kernel, dim3(1), dim3(kSetupThreads), 0, stream, scr, n_sub, nb, oob_out);
    e = hipGetLastError();
    if (e != hipSuccess || n_tiles == 0) return e;
    const int64_t useful = (n_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    const int blocks = (int)(useful < resident ? useful : resident);
    return launch_main_any(pr, grid_kind, gcf_kind, deep, blocks, scr, n_sub, nb, oob_out, stream);
}

}  // namespace dg
