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
//   4. col_hist + scan + col_scatter: each row bucket is cut into slices of
//      4096 pairs; a stable counting sort by column (LDS-staged, wavefront
//      ballots for ranks) moves each slice's pairs to their final place.
//      Within a column the depth order of step 3 is kept, which is the
//      (tile, depth, index) order.
//   5. tile_ranges: [start, end) of every tile straight from the column
//      histogram scan.
// Memory traffic: 6 B per pair written by the emission, 2 B read by the
// histogram, 6 B read and 4 B written by the scatter.
#include "common.hpp"

namespace tgs {
namespace {

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (uint64_t(1) << __lane_id()) - 1;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ int wave_min(int x) {
    for (int o = 32; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o));
    return x;
}

__device__ __forceinline__ int wave_max(int x) {
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o));
    return x;
}

__device__ __forceinline__ uint32_t wave_exclusive_sum(uint32_t x, uint32_t& total) {
    const int lane = __lane_id();
    uint32_t incl = x;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    total = __shfl(incl, 63);
    return incl - x;
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
        if (ty >= ylo && ty < yhi) tot = wave_sum((ty >= r.ylo && ty < r.yhi) ? w : 0u);
        if (lane == 0) rowtot[uint64_t(ty) * nchunks + chunk] = tot;
    }
}

// row_start[ty] = first pair of row ty; row_start[gy] = pair count.
// first_slice[ty] = first column-sort slice of row ty (prefix of ceil(len / kSlice)).
__global__ void __launch_bounds__(256)
row_setup_kernel(const uint32_t* __restrict__ rowscan, uint32_t nchunks, int gy,
                 uint32_t* __restrict__ row_start, uint32_t* __restrict__ first_slice) {
    __shared__ uint32_t carry;
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
        // block exclusive scan of ns
        __shared__ uint32_t wsum[4];
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
                 uint16_t* __restrict__ cols, uint32_t* __restrict__ vals) {
    __shared__ uint32_t s_pref[4][64];
    __shared__ int s_xlo[4][64];
    __shared__ uint32_t s_id[4][64];
    const uint32_t chunk = (uint32_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    if (chunk >= nchunks) return;                      // wavefront-uniform
    const int lane = __lane_id(), wv = threadIdx.x >> 6;
    uint32_t id;
    const Rect r = rect_of(rec, order, int64_t(chunk) * 64 + lane, n, grid, id);
    const uint32_t w = uint32_t(r.xhi - r.xlo);
    s_xlo[wv][lane] = r.xlo;
    s_id[wv][lane] = id;
    const int ylo = wave_min(r.yhi > r.ylo ? r.ylo : grid.gy);
    const int yhi = wave_max(r.yhi);
    for (int ty = ylo; ty < yhi; ++ty) {
        uint32_t tot;
        const uint32_t ex = wave_exclusive_sum((ty >= r.ylo && ty < r.yhi) ? w : 0u, tot);
        if (tot == 0) continue;                        // wavefront-uniform
        s_pref[wv][lane] = ex;
        const uint64_t base = rowscan[uint64_t(ty) * nchunks + chunk];
        for (uint32_t e = lane; e < tot; e += 64) {
            int lo = 0, hi = 64;                       // largest lo with s_pref[lo] <= e
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (s_pref[wv][mid] <= e) lo = mid; else hi = mid;
            }
            cols[base + e] = uint16_t(s_xlo[wv][lo] + int(e - s_pref[wv][lo]));
            vals[base + e] = s_id[wv][lo];
        }
    }
}

// Locate slice b: its row, index within the row and pair range.
struct Slice { int ty; uint32_t k, ns, start, end; };

__device__ __forceinline__ bool find_slice(uint32_t b, const uint32_t* first_slice,
                                           const uint32_t* row_start, int gy, Slice& s) {
    if (b >= first_slice[gy]) return false;
    int lo = 0, hi = gy;                                // largest lo with first_slice[lo] <= b
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (first_slice[mid] <= b) lo = mid; else hi = mid;
    }
    s.ty = lo;
    s.k = b - first_slice[lo];
    s.ns = first_slice[lo + 1] - first_slice[lo];
    s.start = row_start[lo] + s.k * kSlice;
    s.end = min(s.start + uint32_t(kSlice), row_start[lo + 1]);
    return true;
}

__global__ void __launch_bounds__(256)
col_hist_kernel(const uint16_t* __restrict__ cols, const uint32_t* __restrict__ first_slice,
                const uint32_t* __restrict__ row_start, Grid grid, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[kMaxCols];
    Slice s;
    if (!find_slice(blockIdx.x, first_slice, row_start, grid.gy, s)) return;   // block-uniform
    for (int b = threadIdx.x; b < grid.gx; b += 256) h[b] = 0;
    __syncthreads();
    for (uint32_t i = s.start + threadIdx.x; i < s.end; i += 256) atomicAdd(&h[cols[i]], 1u);
    __syncthreads();
    const uint64_t base = uint64_t(grid.gx) * first_slice[s.ty];
    for (int b = threadIdx.x; b < grid.gx; b += 256) hist[base + uint64_t(b) * s.ns + s.k] = h[b];
}

__global__ void __launch_bounds__(256)
col_scatter_kernel(const uint16_t* __restrict__ cols, const uint32_t* __restrict__ vals,
                   const uint32_t* __restrict__ first_slice, const uint32_t* __restrict__ row_start,
                   const uint32_t* __restrict__ hist, Grid grid, int col_bits,
                   uint32_t* __restrict__ out) {
    constexpr int W = 4, PER_WAVE = kSlice / W, ROUNDS = PER_WAVE / 64;
    __shared__ uint32_t s_wcnt[W][kMaxCols];   // per wave, then wave prefix
    __shared__ uint32_t s_start[kMaxCols];     // first local slot of each column
    __shared__ uint32_t s_gbase[kMaxCols];     // first output slot of each column
    __shared__ uint32_t s_val[kSlice];
    __shared__ uint16_t s_col[kSlice];
    __shared__ uint32_t s_part[256];
    Slice s;
    if (!find_slice(blockIdx.x, first_slice, row_start, grid.gy, s)) return;   // block-uniform
    const int tid = threadIdx.x, lane = __lane_id(), wv = tid >> 6;
    const int gx = grid.gx;
    const uint32_t count = s.end - s.start;
    for (int b = tid; b < gx; b += 256)
        for (int w = 0; w < W; ++w) s_wcnt[w][b] = 0;
    __syncthreads();
    uint32_t myv[ROUNDS], myrank[ROUNDS];
    uint16_t mycol[ROUNDS];
    // ranks within the wavefront's 1024 consecutive pairs, in input order
    for (int r = 0; r < ROUNDS; ++r) {
        const uint32_t idx = uint32_t(wv * PER_WAVE + r * 64 + lane);
        const bool valid = idx < count;
        const uint32_t c = valid ? cols[s.start + idx] : 0u;
        myv[r] = valid ? vals[s.start + idx] : 0u;
        mycol[r] = uint16_t(c);
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < col_bits; ++b) {
            const bool bit = (c >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t before = valid ? s_wcnt[wv][c] : 0u;
        myrank[r] = before + uint32_t(__popcll(peers & lanemask_lt()));
        if (valid && (peers & lanemask_lt()) == 0) s_wcnt[wv][c] = before + uint32_t(__popcll(peers));
    }
    __syncthreads();
    // per column: total, wave prefixes, and the local start (block scan over columns)
    constexpr int CPT = kMaxCols / 256;        // columns per thread
    uint32_t tot[CPT], run = 0;
    for (int j = 0; j < CPT; ++j) {
        const int b = tid * CPT + j;
        uint32_t t = 0;
        if (b < gx) {
            for (int w = 0; w < W; ++w) {
                const uint32_t c = s_wcnt[w][b];
                s_wcnt[w][b] = t;
                t += c;
            }
        }
        tot[j] = t;
        run += t;
    }
    s_part[tid] = run;
    __syncthreads();
    if (wv == 0) {                              // scan the 256 partial sums with one wavefront
        uint32_t v[4], sum = 0;
        for (int j = 0; j < 4; ++j) { v[j] = s_part[lane * 4 + j]; sum += v[j]; }
        uint32_t total;
        uint32_t ex = wave_exclusive_sum(sum, total);
        for (int j = 0; j < 4; ++j) { s_part[lane * 4 + j] = ex; ex += v[j]; }
    }
    __syncthreads();
    {
        uint32_t at = s_part[tid];
        const uint64_t hb = uint64_t(gx) * first_slice[s.ty];
        for (int j = 0; j < CPT; ++j) {
            const int b = tid * CPT + j;
            if (b < gx) {
                s_start[b] = at;
                s_gbase[b] = hist[hb + uint64_t(b) * s.ns + s.k];
            }
            at += tot[j];
        }
    }
    __syncthreads();
    for (int r = 0; r < ROUNDS; ++r) {
        const uint32_t idx = uint32_t(wv * PER_WAVE + r * 64 + lane);
        if (idx < count) {
            const uint32_t c = mycol[r];
            const uint32_t pos = s_start[c] + s_wcnt[wv][c] + myrank[r];
            s_val[pos] = myv[r];
            s_col[pos] = uint16_t(c);
        }
    }
    __syncthreads();
    for (uint32_t i = tid; i < count; i += 256) {
        const uint32_t c = s_col[i];
        out[s_gbase[c] + (i - s_start[c])] = s_val[i];
    }
}

__global__ void tile_ranges_kernel(const uint32_t* __restrict__ hist,
                                   const uint32_t* __restrict__ first_slice,
                                   const uint32_t* __restrict__ row_start, Grid grid,
                                   uint32_t* __restrict__ ranges) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= grid.num_tiles()) return;
    const int ty = int(t / grid.gx), tx = int(t % grid.gx);
    const uint32_t ns = first_slice[ty + 1] - first_slice[ty];
    uint32_t a = 0, b = 0;
    if (ns > 0) {
        const uint64_t hb = uint64_t(grid.gx) * first_slice[ty];
        a = hist[hb + uint64_t(tx) * ns];
        b = tx + 1 < grid.gx ? hist[hb + uint64_t(tx + 1) * ns] : row_start[ty + 1];
    }
    if (a == b) a = b = 0;
    ranges[2 * t] = a;
    ranges[2 * t + 1] = b;
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
                            const Grid& grid, hipStream_t s) {
    const uint32_t nchunks = bin_chunks(n);
    if (nchunks == 0) return hipSuccess;
    emit_rows_kernel<<<dim3((nchunks + 3) / 4), dim3(256), 0, s>>>(
        reinterpret_cast<const float4*>(ws + L.records), order, n, grid,
        reinterpret_cast<const uint32_t*>(ws + L.rowtot), nchunks,
        reinterpret_cast<uint16_t*>(ws + L.row_cols), reinterpret_cast<uint32_t*>(ws + L.row_vals));
    return hipGetLastError();
}

hipError_t launch_col_hist(uint8_t* ws, const Layout& L, const Grid& grid, uint64_t slices,
                           hipStream_t s) {
    if (slices == 0) return hipSuccess;
    col_hist_kernel<<<dim3(unsigned(slices)), dim3(256), 0, s>>>(
        reinterpret_cast<const uint16_t*>(ws + L.row_cols),
        reinterpret_cast<const uint32_t*>(ws + L.first_slice),
        reinterpret_cast<const uint32_t*>(ws + L.row_start), grid,
        reinterpret_cast<uint32_t*>(ws + L.col_hist));
    return hipGetLastError();
}

hipError_t launch_col_scatter(uint8_t* ws, const Layout& L, const Grid& grid, uint64_t slices,
                              hipStream_t s) {
    if (slices == 0) return hipSuccess;
    int bits = 1;
    while ((1 << bits) < grid.gx) ++bits;
    col_scatter_kernel<<<dim3(unsigned(slices)), dim3(256), 0, s>>>(
        reinterpret_cast<const uint16_t*>(ws + L.row_cols),
        reinterpret_cast<const uint32_t*>(ws + L.row_vals),
        reinterpret_cast<const uint32_t*>(ws + L.first_slice),
        reinterpret_cast<const uint32_t*>(ws + L.row_start),
        reinterpret_cast<const uint32_t*>(ws + L.col_hist), grid, bits,
        reinterpret_cast<uint32_t*>(ws + L.pair_vals));
    return hipGetLastError();
}

hipError_t launch_tile_ranges(uint8_t* ws, const Layout& L, const Grid& grid, hipStream_t s) {
    const int64_t nt = grid.num_tiles();
    if (nt == 0) return hipSuccess;
    tile_ranges_kernel<<<dim3(unsigned((nt + 255) / 256)), dim3(256), 0, s>>>(
        reinterpret_cast<const uint32_t*>(ws + L.col_hist),
        reinterpret_cast<const uint32_t*>(ws + L.first_slice),
        reinterpret_cast<const uint32_t*>(ws + L.row_start), grid,
        reinterpret_cast<uint32_t*>(ws + L.ranges));
    return hipGetLastError();
}

}  // namespace tgs
