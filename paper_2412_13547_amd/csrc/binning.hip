// Tile-Gaussian pair generation and per-tile ranges (stage (b)).
//
// The (tile id, depth) order of the pairs is produced in two steps that give
// exactly the permutation a stable sort of 64-bit (tile << 32 | depth bits)
// keys would: the Gaussians are first sorted by their 32-bit depth key
// (stable, so equal depths keep ascending index), pairs are emitted in that
// order, and the pairs are then stably sorted by tile id alone.  This moves
// uint32 instead of uint64 keys and sorts ceil(log2(tiles)) bits instead of
// 32 + ceil(log2(tiles)).
#include "common.hpp"

namespace tgs {
namespace {

constexpr int kEmitThreads = 256;

// One block per 256 consecutive Gaussians of the depth order.  The block's
// pairs form one contiguous output range; thread t writes pairs
// t, t + 256, ... of it, so stores are coalesced whatever the per-Gaussian
// counts are.  The owner of a pair is found by binary search over the 256
// output offsets kept in LDS.
__global__ void __launch_bounds__(kEmitThreads)
emit_pairs_kernel(const float4* __restrict__ rec, const uint32_t* __restrict__ order,
                  const uint64_t* __restrict__ offsets, int64_t n, Grid grid,
                  uint32_t* __restrict__ tiles, uint32_t* __restrict__ vals) {
    __shared__ uint64_t s_off[kEmitThreads + 1];
    __shared__ int s_xlo[kEmitThreads], s_ylo[kEmitThreads], s_w[kEmitThreads];
    __shared__ uint32_t s_id[kEmitThreads];
    const int tid = threadIdx.x;
    const int64_t k0 = int64_t(blockIdx.x) * kEmitThreads;
    const int64_t k = k0 + tid;
    if (k < n) {
        const uint32_t id = order[k];
        const float4 a = rec[3 * uint64_t(id)];
        const float4 c = rec[3 * uint64_t(id) + 2];
        const Rect r = tile_rect(a.x, a.y, __float_as_int(c.z), grid);
        s_off[tid] = offsets[k];
        s_xlo[tid] = r.xlo;
        s_ylo[tid] = r.ylo;
        s_w[tid] = r.xhi - r.xlo;
        s_id[tid] = id;
    } else {
        s_off[tid] = offsets[n];
        s_xlo[tid] = s_ylo[tid] = 0;
        s_w[tid] = 1;
        s_id[tid] = 0;
    }
    if (tid == 0) s_off[kEmitThreads] = offsets[k0 + kEmitThreads < n ? k0 + kEmitThreads : n];
    __syncthreads();
    const uint64_t p0 = s_off[0], p1 = s_off[kEmitThreads];
    for (uint64_t p = p0 + tid; p < p1; p += kEmitThreads) {
        int lo = 0, hi = kEmitThreads;          // largest lo with s_off[lo] <= p
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_off[mid] <= p) lo = mid; else hi = mid;
        }
        const uint32_t local = uint32_t(p - s_off[lo]);
        const uint32_t w = uint32_t(s_w[lo]);
        const uint32_t ty = uint32_t(s_ylo[lo]) + local / w;
        const uint32_t tx = uint32_t(s_xlo[lo]) + local % w;
        tiles[p] = ty * uint32_t(grid.gx) + tx;
        vals[p] = s_id[lo];
    }
}

__global__ void ranges_kernel(const uint32_t* __restrict__ tiles, uint64_t count,
                              uint32_t* __restrict__ ranges) {
    const uint64_t p = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= count) return;
    const uint32_t t = tiles[p];
    if (p == 0 || tiles[p - 1] != t) ranges[2 * uint64_t(t)] = uint32_t(p);
    if (p + 1 == count || tiles[p + 1] != t) ranges[2 * uint64_t(t) + 1] = uint32_t(p + 1);
}

}  // namespace

hipError_t launch_emit_pairs(const uint8_t* ws, const Layout& L, const uint32_t* order, int64_t n,
                             const Grid& grid, uint32_t* tiles, uint32_t* vals, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const auto* rec = reinterpret_cast<const float4*>(ws + L.records);
    const auto* off = reinterpret_cast<const uint64_t*>(ws + L.offsets);
    emit_pairs_kernel<<<dim3(unsigned((n + kEmitThreads - 1) / kEmitThreads)), dim3(kEmitThreads), 0,
                        s>>>(rec, order, off, n, grid, tiles, vals);
    return hipGetLastError();
}

hipError_t launch_ranges(const uint32_t* tiles, uint64_t count, uint32_t* ranges, int64_t num_tiles,
                         hipStream_t s) {
    hipError_t e = fill_u32(ranges, 0u, uint64_t(num_tiles) * 2, s);
    if (e != hipSuccess || count == 0) return e;
    ranges_kernel<<<dim3(unsigned((count + 255) / 256)), dim3(256), 0, s>>>(tiles, count, ranges);
    return hipGetLastError();
}

}  // namespace tgs
