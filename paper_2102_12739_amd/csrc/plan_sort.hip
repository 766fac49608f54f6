// Plan-time work order: a stable sort of each subgrid's visibilities by the
// position along a Hilbert curve of the cell that holds (u, v).
//
// Tiles are cut from consecutive positions of the work order, so after this
// sort a tile holds visibilities that are close in the subgrid, and the
// tiles an XCD drains one after another cover neighbouring regions: the
// subgrid data a tile needs is then mostly in that XCD's L2 already. The sum
// each visibility receives does not depend on the order, so results are
// unchanged; only locality is.
#include "dg_internal.h"

#include <hipcub/hipcub.hpp>

namespace dg {
namespace {

// Position of cell (x, y) along the Hilbert curve of the 65536 x 65536
// grid: level by level from the top, the rank of the cell's quadrant along
// the curve, then the coordinates turned into the orientation of that
// quadrant's sub-curve. Consecutive positions are neighbouring cells, so a
// run of positions covers a compact region (a Z-order curve jumps between
// quadrants; on the paper-scale workload this order reads 2.6 % fewer HBM
// bytes and runs about 2 % faster, cold).
__device__ __forceinline__ uint32_t hilbert16(uint32_t x, uint32_t y) {
    uint32_t d = 0;
    for (uint32_t s = 1u << 15; s > 0; s >>= 1) {
        const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
        d += s * s * ((3u * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = 0xFFFFu - x;
                y = 0xFFFFu - y;
            }
            const uint32_t t = x;
            x = y;
            y = t;
        }
    }
    return d;
}

// key = subgrid << 32 | Hilbert position of (cell_u, cell_v); coordinates outside
// [0, 65536) or not finite go to the end of their subgrid.
__global__ void sort_keys_kernel(const double* uvw, const int64_t* offsets, int64_t n_sub, int64_t n_vis,
                                 uint64_t* keys, uint32_t* idx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_vis) return;
    int64_t lo = 0, hi = n_sub;   // offsets[lo] <= i < offsets[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (offsets[mid] <= i) lo = mid; else hi = mid;
    }
    const double u = uvw[3 * i], v = uvw[3 * i + 1];
    uint32_t code = 0xFFFFFFFFu;
    if (u >= 0.0 && u < 65536.0 && v >= 0.0 && v < 65536.0)
        code = hilbert16((uint32_t)u, (uint32_t)v);
    keys[i] = ((uint64_t)lo << 32) | code;
    idx[i] = (uint32_t)i;
}

}  // namespace

hipError_t sort_visibilities(const double* uvw, const int64_t* offsets_host, int64_t n_sub,
                             uint32_t* perm, hipStream_t stream) {
    const int64_t n = offsets_host[n_sub];
    if (n == 0) return hipSuccess;
    int end_bit = 32;
    while (end_bit < 64 && (int64_t(1) << (end_bit - 32)) < n_sub) ++end_bit;
    int64_t* d_off = nullptr;
    uint64_t *k_in = nullptr, *k_out = nullptr;
    uint32_t* v_in = nullptr;
    void* temp = nullptr;
    size_t temp_bytes = 0;
    hipError_t e = hipMalloc(&d_off, sizeof(int64_t) * (n_sub + 1));
    if (e == hipSuccess) e = hipMalloc(&k_in, sizeof(uint64_t) * n);
    if (e == hipSuccess) e = hipMalloc(&k_out, sizeof(uint64_t) * n);
    if (e == hipSuccess) e = hipMalloc(&v_in, sizeof(uint32_t) * n);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_off, offsets_host, sizeof(int64_t) * (n_sub + 1), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) {
        const int threads = 256;
        const int64_t blocks = (n + threads - 1) / threads;
        hipLaunchKernelGGL(sort_keys_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, uvw, d_off, n_sub,
                           n, k_in, v_in);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, k_in, k_out, v_in, perm, n, 0, end_bit, stream);
    if (e == hipSuccess) e = hipMalloc(&temp, temp_bytes);
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, k_in, k_out, v_in, perm, n, 0, end_bit, stream);
    const hipError_t es = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = es;
    if (temp) (void)hipFree(temp);
    if (v_in) (void)hipFree(v_in);
    if (k_out) (void)hipFree(k_out);
    if (k_in) (void)hipFree(k_in);
    if (d_off) (void)hipFree(d_off);
    return e;
}

}  // namespace dg
