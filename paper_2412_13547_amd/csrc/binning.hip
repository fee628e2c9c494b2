// Tile-Gaussian pairs in (tile id, depth) order and per-tile ranges (stage (b)).
//
// The order is the one a stable sort of 64-bit (tile << 32 | depth bits) keys
// produces, built without sorting 64-bit keys:
//   1. the Gaussians are sorted by their 32-bit depth key (stable, so equal
//      depths keep ascending index; ``radix_sort``);
//   2. row_counts: per chunk of 64 consecutive Gaussians of that order (one
//      wavefront) and per tile row, the number of pairs the chunk puts in the
//      row (a Gaussian covers the columns [xlo, xhi) of each of its rows);
//      an exclusive scan over (row, chunk) gives every chunk's first slot in
//      every row bucket, and the row starts;
//   3. emit_rows: every chunk writes, row by row, its pairs (column, Gaussian)
//      into the row buckets -- in depth order, each Gaussian's columns
//      ascending, with fully coalesced stores;
//   4. col_hist + col_scan + col_scatter: each row bucket is cut into slices
//      of kSlice pairs; a stable counting sort by column (LDS-staged,
//      wavefront ballots for ranks) moves each slice's pairs to their final
//      place.  Within a column the depth order of step 3 is kept, which is the
//      (tile, depth, index) order.  col_scan also writes every tile's
//      [start, end).
// Memory traffic per pair: 6 B written by the emission, 2 B read by the
// histogram, 6 B read and 4 B written by the scatter.
//
// The pair count is known only on the device (the scanned total).  Steps 3
// and 4 read it and write nothing when it exceeds the buffers' capacity, so
// the whole stage can be enqueued (or captured in a graph) without reading
// it back; col_scan then writes empty ranges and the rasterizer renders the
// background.
#include "common.hpp"
#include "wave.hpp"

namespace tgs {
namespace {

constexpr int kScatterThreads = 256;
constexpr int kScatterWaves = kScatterThreads / 64;
constexpr int kScatterRounds = kSlice / kScatterThreads;   // pairs per thread
constexpr int kScatterCols = kMaxCols / kScatterThreads;   // columns per thread in the scan
constexpr uint32_t kDirectCols = 8;   // widest row span written lane by lane

__device__ __forceinline__ int wave_min(int x) {
    for (int o = 32; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o));
    return x;
}

__device__ __forceinline__ int wave_max(int x) {
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o));
    return x;
}

// The tile rectangle of the Gaussian at depth position s (empty when culled,
// off-screen or s >= n).
__device__ __forceinline__ Rect rect_of(const float4* rec, const uint32_t* order, int64_t s,
                                        int64_t n, const Grid& grid, uint32_t& id) {
    Rect r{0, 0, 0, 0};
    id = 0;
    if (s < n) {
        id = order[s];
        const float4 a = rec[3 * uint64_t(id)];
        const int radius = __float_as_int(rec[3 * uint64_t(id) + 2].z);
        if (radius > 0) r = tile_rect(a.x, a.y, radius, grid);
        if (r.xhi <= r.xlo || r.yhi <= r.ylo) r = Rect{0, 0, 0, 0};
    }
    return r;
}

__global__ void __launch_bounds__(256)
row_counts_kernel(const float4* __restrict__ rec, const uint32_t* __restrict__ order, int64_t n,
                  Grid grid, uint32_t* __restrict__ rowtot, uint32_t nchunks) {
    const uint32_t chunk = (uint32_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    if (chunk >= nchunks) return;                      // wavefront-uniform
    const int lane = __lane_id();
    uint32_t id;
    const Rect r = rect_of(rec, order, int64_t(chunk) * 64 + lane, n, grid, id);
    const uint32_t w = uint32_t(r.xhi - r.xlo);
    const int ylo = wave_min(r.yhi > r.ylo ? r.ylo : grid.gy);
    const int yhi = wave_max(r.yhi);
    for (int ty = 0; ty < grid.gy; ++ty) {
        uint32_t tot = 0;
        if (ty >= ylo && ty < yhi) tot = wave_total((ty >= r.ylo && ty < r.yhi) ? w : 0u);
        if (lane == 0) rowtot[uint64_t(ty) * nchunks + chunk] = tot;
    }
}

// row_start[ty] = first pair of row ty; row_start[gy] = pair count.
// first_slice[ty] = first column-sort slice of row ty (prefix of ceil(len / kSlice)).
__global__ void __launch_bounds__(256)
row_setup_kernel(const uint32_t* __restrict__ rowscan, uint32_t nchunks, int gy,
                 uint32_t* __restrict__ row_start, uint32_t* __restrict__ first_slice) {
    __shared__ uint32_t carry;
    __shared__ uint32_t wsum[4];
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base <= gy; base += 256) {
        const int ty = base + threadIdx.x;
        uint32_t ns = 0;
        if (ty <= gy) {
            const uint32_t s0 = rowscan[uint64_t(ty) * nchunks];
            row_start[ty] = s0;
            if (ty < gy) ns = (rowscan[uint64_t(ty + 1) * nchunks] - s0 + kSlice - 1) / kSlice;
        }
        uint32_t tot;
        const uint32_t ex = wave_exclusive_sum(ns, tot);
        if (__lane_id() == 0) wsum[threadIdx.x >> 6] = tot;
        __syncthreads();
        uint32_t before = carry, all = 0;
        for (int w = 0; w < 4; ++w) {
            if (w < int(threadIdx.x >> 6)) before += wsum[w];
            all += wsum[w];
        }
        if (ty <= gy) first_slice[ty] = before + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry += all;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256)
emit_rows_kernel(const float4* __restrict__ rec, const uint32_t* __restrict__ order, int64_t n,
                 Grid grid, const uint32_t* __restrict__ rowscan, uint32_t nchunks,
                 uint32_t capacity, uint16_t* __restrict__ cols, uint32_t* __restrict__ vals) {
    __shared__ uint32_t s_pref[4][64];
    __shared__ int s_xlo[4][64];
    __shared__ uint32_t s_id[4][64];
    const uint32_t chunk = (uint32_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    if (chunk >= nchunks) return;                      // wavefront-uniform
    if (rowscan[uint64_t(grid.gy) * nchunks] > capacity) return;   // overflow: uniform
    const int lane = __lane_id(), wv = threadIdx.x >> 6;
    uint32_t id;
    const Rect r = rect_of(rec, order, int64_t(chunk) * 64 + lane, n, grid, id);
    const uint32_t w = uint32_t(r.xhi - r.xlo);
    s_xlo[wv][lane] = r.xlo;
    s_id[wv][lane] = id;
    const int ylo = wave_min(r.yhi > r.ylo ? r.ylo : grid.gy);
    const int yhi = wave_max(r.yhi);
    for (int r0 = ylo; r0 < yhi; r0 += 64) {
        // this chunk's segment [base, next) of rows r0 .. r0+63, one row per lane
        uint32_t my_base = 0, my_next = 0;
        if (r0 + lane < yhi) {
            const uint64_t at = uint64_t(r0 + lane) * nchunks + chunk;
            my_base = rowscan[at];
            my_next = rowscan[at + 1];
        }
        const int r1 = min(r0 + 64, yhi);
        for (int ty = r0; ty < r1; ++ty) {
            uint32_t tot;
            const uint32_t ex = wave_exclusive_sum((ty >= r.ylo && ty < r.yhi) ? w : 0u, tot);
            if (tot == 0) continue;                    // wavefront-uniform
            const uint32_t base = uint32_t(__builtin_amdgcn_readlane(int(my_base), ty - r0));
            const uint32_t next = uint32_t(__builtin_amdgcn_readlane(int(my_next), ty - r0));
            const uint32_t len = min(tot, next - base);    // never past this segment
            const uint32_t mine = (ty >= r.ylo && ty < r.yhi) ? w : 0u;
            const uint32_t wmax = uint32_t(wave_max(int(mine)));
            if (wmax <= kDirectCols) {
                // every lane writes its own (at most kDirectCols) pairs
                for (uint32_t c = 0; c < wmax; ++c) {
                    const uint32_t e = ex + c;
                    if (c < mine && e < len) {
                        cols[uint64_t(base) + e] = uint16_t(r.xlo + int(c));
                        vals[uint64_t(base) + e] = id;
                    }
                }
                continue;
            }
            // wide splats: the wavefront writes 64 consecutive pairs per round,
            // each lane finding its pair's Gaussian by binary search
            s_pref[wv][lane] = ex;
            for (uint32_t e = lane; e < len; e += 64) {
                int lo = 0, hi = 64;                   // largest lo with s_pref[lo] <= e
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_pref[wv][mid] <= e) lo = mid; else hi = mid;
                }
                cols[uint64_t(base) + e] = uint16_t(s_xlo[wv][lo] + int(e - s_pref[wv][lo]));
                vals[uint64_t(base) + e] = s_id[wv][lo];
            }
        }
    }
}

// Locate slice b: its row, index within the row and pair range.
struct Slice { int ty; uint32_t k, start, end; };

__device__ __forceinline__ bool find_slice(uint32_t b, const uint32_t* first_slice,
                                           const uint32_t* row_start, int gy, uint32_t capacity,
                                           Slice& s) {
    if (row_start[gy] > capacity || b >= first_slice[gy]) return false;
    int lo = 0, hi = gy;                                // largest lo with first_slice[lo] <= b
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (first_slice[mid] <= b) lo = mid; else hi = mid;
    }
    s.ty = lo;
    s.k = b - first_slice[lo];
    s.start = row_start[lo] + s.k * kSlice;
    s.end = min(s.start + uint32_t(kSlice), row_start[lo + 1]);
    return true;
}

// hist[b][tx]: pairs of slice b in column tx.
__global__ void __launch_bounds__(256)
col_hist_kernel(const uint16_t* __restrict__ cols, const uint32_t* __restrict__ first_slice,
                const uint32_t* __restrict__ row_start, Grid grid, uint32_t capacity,
                uint32_t* __restrict__ hist) {
    extern __shared__ uint32_t h[];
    Slice s;
    if (!find_slice(blockIdx.x, first_slice, row_start, grid.gy, capacity, s)) return;   // block-uniform
    for (int b = threadIdx.x; b < grid.gx; b += 256) h[b] = 0;
    __syncthreads();
    for (uint32_t i = s.start + threadIdx.x; i < s.end; i += 256) atomicAdd(&h[cols[i]], 1u);
    __syncthreads();
    const uint64_t base = uint64_t(blockIdx.x) * grid.gx;
    for (int b = threadIdx.x; b < grid.gx; b += 256) hist[base + b] = h[b];
}

// Block-wide exclusive scan (blockDim.x = NT, one value per thread).
template <int NT>
__device__ __forceinline__ uint32_t block_exclusive_sum(uint32_t x, uint32_t* s_w, uint32_t& total) {
    const int wv = threadIdx.x >> 6;
    uint32_t wt;
    const uint32_t ex = wave_exclusive_sum(x, wt);
    if (__lane_id() == 0) s_w[wv] = wt;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
    for (int w = 0; w < NT / 64; ++w) {
        if (w < wv) before += s_w[w];
        total += s_w[w];
    }
    __syncthreads();
    return before + ex;
}

// One block per tile row: turns hist[b][tx] into the first output slot of
// (slice b, column tx) -- order (row, column, slice) -- and writes the range
// of every tile of the row.  The slices of a column are split into
// segments of consecutive slices, one thread per (column, segment).
__global__ void __launch_bounds__(1024)
col_scan_kernel(uint32_t* __restrict__ hist, const uint32_t* __restrict__ first_slice,
                const uint32_t* __restrict__ row_start, Grid grid, uint32_t capacity,
                uint32_t* __restrict__ ranges) {
    __shared__ uint32_t s_seg[1024];
    __shared__ uint32_t s_start[kMaxCols];
    __shared__ uint32_t s_w[16];
    const int ty = blockIdx.x, t = threadIdx.x, gx = grid.gx;
    if (row_start[grid.gy] > capacity) {               // overflow: empty ranges, block-uniform
        if (t < gx) {
            const uint64_t tile = uint64_t(ty) * gx + t;
            ranges[2 * tile] = 0u;
            ranges[2 * tile + 1] = 0u;
        }
        return;
    }
    const uint32_t s0 = first_slice[ty], ns = first_slice[ty + 1] - s0;
    const int groups = max(1, 1024 / gx);
    const int tx = t % gx, g = t / gx;
    const bool act = g < groups;
    const uint32_t seg = (ns + groups - 1) / groups;
    const uint32_t k0 = act ? min(ns, uint32_t(g) * seg) : 0, k1 = act ? min(ns, k0 + seg) : 0;
    uint32_t sum = 0;
    for (uint32_t k = k0; k < k1; ++k) sum += hist[uint64_t(s0 + k) * gx + tx];
    s_seg[t] = sum;
    __syncthreads();
    // column totals; segment sums -> exclusive prefixes over segments
    uint32_t coltot = 0;
    if (t < gx) {
        for (int q = 0; q < groups; ++q) {
            const uint32_t v = s_seg[q * gx + t];
            s_seg[q * gx + t] = coltot;
            coltot += v;
        }
    }
    uint32_t all;
    const uint32_t ex = block_exclusive_sum<1024>(t < gx ? coltot : 0u, s_w, all);
    const uint32_t rs = row_start[ty];
    if (t < gx) {
        s_start[t] = rs + ex;
        const uint64_t tile = uint64_t(ty) * gx + t;
        ranges[2 * tile] = coltot > 0 ? rs + ex : 0u;
        ranges[2 * tile + 1] = coltot > 0 ? rs + ex + coltot : 0u;
    }
    __syncthreads();
    if (act) {
        uint32_t run = s_start[tx] + s_seg[t];
        for (uint32_t k = k0; k < k1; ++k) {
            const uint64_t at = uint64_t(s0 + k) * gx + tx;
            const uint32_t v = hist[at];
            hist[at] = run;
            run += v;
        }
    }
}

__global__ void __launch_bounds__(kScatterThreads)
col_scatter_kernel(const uint16_t* __restrict__ cols, const uint32_t* __restrict__ vals,
                   const uint32_t* __restrict__ first_slice, const uint32_t* __restrict__ row_start,
                   const uint32_t* __restrict__ hist, Grid grid, int col_bits,
                   uint32_t capacity, uint32_t* __restrict__ out) {
    constexpr int W = kScatterWaves, R = kScatterRounds, PER_WAVE = 64 * R;
    extern __shared__ uint32_t smem[];
    const int gx = grid.gx;
    uint32_t* s_val = smem;                              // [kSlice]
    uint32_t* s_wcnt = s_val + kSlice;                   // [W][gx]: counts, then wave prefixes
    uint32_t* s_start = s_wcnt + W * gx;                 // [gx]: first local slot of a column
    uint32_t* s_gbase = s_start + gx;                    // [gx]: first output slot of a column
    uint32_t* s_w = s_gbase + gx;                        // [W]
    uint16_t* s_col = reinterpret_cast<uint16_t*>(s_w + W);   // [kSlice]
    Slice s;
    if (!find_slice(blockIdx.x, first_slice, row_start, grid.gy, capacity, s)) return;   // block-uniform
    const int tid = threadIdx.x, lane = __lane_id(), wv = tid >> 6;
    const uint32_t count = s.end - s.start;
    for (int b = tid; b < W * gx; b += kScatterThreads) s_wcnt[b] = 0;
    // all loads first: R independent pairs per lane in flight
    uint32_t myv[R];
    uint32_t mycol[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t idx = uint32_t(wv * PER_WAVE + r * 64 + lane);
        const bool valid = idx < count;
        mycol[r] = valid ? uint32_t(cols[s.start + idx]) : 0u;
        myv[r] = valid ? vals[s.start + idx] : 0u;
    }
    __syncthreads();
    // ranks within the wavefront's PER_WAVE consecutive pairs, in input order
    uint32_t myrank[R];
    uint32_t* wc = s_wcnt + wv * gx;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t idx = uint32_t(wv * PER_WAVE + r * 64 + lane);
        const bool valid = idx < count;
        const uint32_t c = mycol[r];
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < col_bits; ++b) {
            const bool bit = (c >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t below = uint32_t(__popcll(peers & lanemask_lt()));
        const uint32_t before = valid ? wc[c] : 0u;
        myrank[r] = before + below;
        if (valid && below == 0) wc[c] = before + uint32_t(__popcll(peers));
    }
    __syncthreads();
    // per column: total over waves (wave counts become wave prefixes), then
    // the columns' local starts by a block scan (kScatterCols columns per thread)
    constexpr int CPT = kScatterCols;
    uint32_t tot[CPT];
    uint32_t mine = 0;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int c = CPT * tid + j;
        tot[j] = 0;
        if (c < gx) {
            uint32_t t = 0;
            for (int w = 0; w < W; ++w) {
                const uint32_t v = s_wcnt[w * gx + c];
                s_wcnt[w * gx + c] = t;
                t += v;
            }
            tot[j] = t;
        }
        mine += tot[j];
    }
    uint32_t all;
    uint32_t ex = block_exclusive_sum<kScatterThreads>(mine, s_w, all);
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int c = CPT * tid + j;
        if (c < gx) {
            s_start[c] = ex;
            s_gbase[c] = hist[uint64_t(blockIdx.x) * gx + c];
        }
        ex += tot[j];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t idx = uint32_t(wv * PER_WAVE + r * 64 + lane);
        if (idx < count) {
            const uint32_t c = mycol[r];
            const uint32_t pos = s_start[c] + s_wcnt[wv * gx + c] + myrank[r];
            s_val[pos] = myv[r];
            s_col[pos] = uint16_t(c);
        }
    }
    __syncthreads();
    for (uint32_t i = tid; i < count; i += kScatterThreads) {
        const uint32_t c = s_col[i];
        out[s_gbase[c] + (i - s_start[c])] = s_val[i];
    }
}

size_t scatter_lds_bytes(int gx) {
    return size_t(kSlice) * 4 + size_t(kScatterWaves * gx + 2 * gx + kScatterWaves) * 4 +
           size_t(kSlice) * 2;
}

}  // namespace

uint32_t bin_chunks(int64_t n) { return uint32_t((n + 63) / 64); }

uint64_t bin_max_slices(uint64_t pairs, int gy) { return pairs / kSlice + uint64_t(gy) + 1; }

hipError_t launch_row_counts(const uint8_t* ws, const Layout& L, const uint32_t* order, int64_t n,
                             const Grid& grid, hipStream_t s) {
    const uint32_t nchunks = bin_chunks(n);
    auto* rowtot = reinterpret_cast<uint32_t*>(const_cast<uint8_t*>(ws) + L.rowtot);
    if (nchunks > 0) {
        const auto* rec = reinterpret_cast<const float4*>(ws + L.records);
        row_counts_kernel<<<dim3((nchunks + 3) / 4), dim3(256), 0, s>>>(rec, order, n, grid, rowtot,
                                                                       nchunks);
    }
    return hipGetLastError();
}

hipError_t launch_row_setup(uint8_t* ws, const Layout& L, int64_t n, const Grid& grid,
                            hipStream_t s) {
    const uint32_t nchunks = bin_chunks(n);
    row_setup_kernel<<<1, 256, 0, s>>>(reinterpret_cast<const uint32_t*>(ws + L.rowtot),
                                       nchunks, grid.gy,
                                       reinterpret_cast<uint32_t*>(ws + L.row_start),
                                       reinterpret_cast<uint32_t*>(ws + L.first_slice));
    return hipGetLastError();
}

hipError_t launch_emit_rows(uint8_t* ws, const Layout& L, const uint32_t* order, int64_t n,
                            const Grid& grid, uint32_t capacity, hipStream_t s) {
    const uint32_t nchunks = bin_chunks(n);
    if (nchunks == 0) return hipSuccess;
    emit_rows_kernel<<<dim3((nchunks + 3) / 4), dim3(256), 0, s>>>(
        reinterpret_cast<const float4*>(ws + L.records), order, n, grid,
        reinterpret_cast<const uint32_t*>(ws + L.rowtot), nchunks, capacity,
        reinterpret_cast<uint16_t*>(ws + L.row_cols), reinterpret_cast<uint32_t*>(ws + L.row_vals));
    return hipGetLastError();
}

hipError_t prepare_binning_kernels() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&col_scatter_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               int(scatter_lds_bytes(kMaxCols)));
}

hipError_t launch_col_sort(uint8_t* ws, const Layout& L, const Grid& grid, uint64_t slices,
                           uint32_t capacity, hipStream_t s) {
    const auto* fs = reinterpret_cast<const uint32_t*>(ws + L.first_slice);
    const auto* rs = reinterpret_cast<const uint32_t*>(ws + L.row_start);
    auto* hist = reinterpret_cast<uint32_t*>(ws + L.col_hist);
    auto* ranges = reinterpret_cast<uint32_t*>(ws + L.ranges);
    if (slices > 0) {
        col_hist_kernel<<<dim3(unsigned(slices)), dim3(256), size_t(grid.gx) * 4, s>>>(
            reinterpret_cast<const uint16_t*>(ws + L.row_cols), fs, rs, grid, capacity, hist);
    }
    col_scan_kernel<<<dim3(unsigned(grid.gy)), dim3(1024), 0, s>>>(hist, fs, rs, grid, capacity,
                                                                  ranges);
    if (slices > 0) {
        int bits = 1;
        while ((1 << bits) < grid.gx) ++bits;
        // LDS above the default 64 KiB is enabled once by prepare_binning_kernels
        col_scatter_kernel<<<dim3(unsigned(slices)), dim3(kScatterThreads),
                             scatter_lds_bytes(grid.gx), s>>>(
            reinterpret_cast<const uint16_t*>(ws + L.row_cols),
            reinterpret_cast<const uint32_t*>(ws + L.row_vals), fs, rs, hist, grid, bits, capacity,
            reinterpret_cast<uint32_t*>(ws + L.pair_vals));
    }
    return hipGetLastError();
}

}  // namespace tgs
