// Tile-Gaussian pairs in (tile id, depth) order and per-tile ranges (stage (b)).
//
// The order is the one a stable sort of 64-bit (tile << 32 | depth bits) keys
// produces, built without sorting 64-bit keys and without ever writing the
// pairs in any order but the final one:
//   1. the Gaussians are sorted by their 32-bit depth key (stable, so equal
//      depths keep ascending index; ``radix_sort``);
//   2. count_kernel: per block of 256 consecutive Gaussians of that order and
//      per tile row, the number of *entries* (Gaussian x row: a Gaussian
//      covers the columns [xlo, xhi) of each row in [ylo, yhi)) and of pairs
//      the block puts in the row; exclusive scans over (row, block) give every
//      block's first entry and first pair in every row;
//   3. entry_kernel: every block writes, row by row, its entries (Gaussian,
//      first pair, columns) into the row's entry list -- in depth order --
//      with one block-wide scan per row, and marks where every column-sort
//      slice of kSlice pairs begins;
//   4. slice_hist + col_scan + slice_scatter: a stable counting sort by column
//      per slice.  The histogram comes from the slice's entries (two LDS
//      updates per entry, then a prefix over the columns); the scatter
//      expands the slice's entries into pairs in LDS, ranks them per column
//      with wavefront ballots and writes each pair once, to its final place.
//      Within a column the depth order of step 3 is kept, which is the
//      (tile, depth, index) order.  col_scan also writes every tile's
//      [start, end).
// Memory traffic per pair: the final 4 B write; per entry (about one per 15
// pairs at the benchmark scenes) 12 B written and read twice.
//
// The pair count is known only on the device (the scanned total).  Steps 3
// and 4 read it and write nothing when it exceeds the buffers' capacity, so
// the whole stage can be enqueued (or captured in a graph) without reading
// it back; col_scan then writes empty ranges and the rasterizer renders the
// background.  There are never more entries than pairs, so the entry arrays
// sized by the pair capacity cannot overflow either.
#include "common.hpp"
#include "wave.hpp"

namespace tgs {
namespace {

constexpr int kBinThreads = 256;                           // Gaussians per count/entry block
constexpr int kScatterThreads = 512;
constexpr int kScatterWaves = kScatterThreads / 64;
constexpr int kScatterRounds = kSlice / kScatterThreads;   // pairs per thread
constexpr int kScatterCols = kMaxCols / kScatterThreads;   // columns per thread in the scan
constexpr int kHistThreads = 256;
constexpr int kHistCols = kMaxCols / kHistThreads;

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

// Per block of kBinThreads depth positions and per row: entries and pairs.
// ecnt[r * nblk + blk], pcnt[r * nblk + blk] (row-major, so one flat scan
// gives the row starts and every block's offset inside every row).
__global__ void __launch_bounds__(kBinThreads)
count_kernel(const float4* __restrict__ rec, const uint32_t* __restrict__ order, int64_t n,
             Grid grid, uint32_t nblk, uint32_t* __restrict__ ecnt, uint32_t* __restrict__ pcnt) {
    extern __shared__ uint32_t lds[];
    const int gy = grid.gy;
    uint32_t* ce = lds;           // [gy]
    uint32_t* cp = lds + gy;      // [gy]
    for (int r = threadIdx.x; r < gy; r += kBinThreads) ce[r] = cp[r] = 0;
    __syncthreads();
    uint32_t id;
    const Rect rc = rect_of(rec, order, int64_t(blockIdx.x) * kBinThreads + threadIdx.x, n, grid, id);
    const uint32_t w = uint32_t(rc.xhi - rc.xlo);
    for (int r = rc.ylo; r < rc.yhi; ++r) {
        atomicAdd(&ce[r], 1u);
        atomicAdd(&cp[r], w);
    }
    __syncthreads();
    for (int r = threadIdx.x; r < gy; r += kBinThreads) {
        ecnt[uint64_t(r) * nblk + blockIdx.x] = ce[r];
        pcnt[uint64_t(r) * nblk + blockIdx.x] = cp[r];
    }
}

// row_start[r] = first pair of row r (row_start[gy] = pair count),
// erow[r] = first entry of row r, first_slice[r] = first column-sort slice
// of row r (prefix of ceil(pairs / kSlice)).
__global__ void __launch_bounds__(256)
row_setup_kernel(const uint32_t* __restrict__ escan, const uint32_t* __restrict__ pscan,
                 uint32_t nblk, int gy, uint32_t* __restrict__ row_start,
                 uint32_t* __restrict__ erow, uint32_t* __restrict__ first_slice) {
    __shared__ uint32_t carry;
    __shared__ uint32_t wsum[4];
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base <= gy; base += 256) {
        const int ty = base + threadIdx.x;
        uint32_t ns = 0;
        if (ty <= gy) {
            const uint32_t s0 = pscan[uint64_t(ty) * nblk];
            row_start[ty] = s0;
            erow[ty] = escan[uint64_t(ty) * nblk];
            if (ty < gy) ns = (pscan[uint64_t(ty + 1) * nblk] - s0 + kSlice - 1) / kSlice;
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

// Every block writes its entries row by row: ent_id (Gaussian), ent_pp
// (first pair of the entry), ent_x (xlo | xhi << 16).  One block scan per row
// ranks the block's entries and pairs at once (packed: pairs << 12 | 1; a
// block holds 256 entries and at most 256 * 1024 pairs of a row).  The entry
// that holds the first pair of a column-sort slice records itself in
// slice_entry.
__global__ void __launch_bounds__(kBinThreads)
entry_kernel(const float4* __restrict__ rec, const uint32_t* __restrict__ order, int64_t n,
             Grid grid, uint32_t nblk, const uint32_t* __restrict__ escan,
             const uint32_t* __restrict__ pscan, const uint32_t* __restrict__ row_start,
             const uint32_t* __restrict__ first_slice, uint32_t capacity,
             uint32_t* __restrict__ ent_id, uint32_t* __restrict__ ent_pp,
             uint32_t* __restrict__ ent_x, uint32_t* __restrict__ slice_entry,
             uint32_t* __restrict__ slice_row) {
    __shared__ uint32_t s_w[2][kBinThreads / 64];
    __shared__ int s_lim[2][kBinThreads / 64];
    if (row_start[grid.gy] > capacity) return;          // overflow: block-uniform
    const int wv = threadIdx.x >> 6;
    uint32_t id;
    const Rect rc = rect_of(rec, order, int64_t(blockIdx.x) * kBinThreads + threadIdx.x, n, grid, id);
    const uint32_t w = uint32_t(rc.xhi - rc.xlo);
    const uint32_t xpack = uint32_t(rc.xlo) | (uint32_t(rc.xhi) << 16);
    // rows the block touches
    const int lo = wave_min(rc.yhi > rc.ylo ? rc.ylo : grid.gy), hi = wave_max(rc.yhi);
    if (__lane_id() == 0) {
        s_lim[0][wv] = lo;
        s_lim[1][wv] = hi;
    }
    __syncthreads();
    int r0 = grid.gy, r1 = 0;
    for (int k = 0; k < kBinThreads / 64; ++k) {
        r0 = min(r0, s_lim[0][k]);
        r1 = max(r1, s_lim[1][k]);
    }
    for (int r = r0; r < r1; ++r) {
        const bool in = r >= rc.ylo && r < rc.yhi;
        // block exclusive scan of (w << 12 | 1); the wave totals alternate
        // between two buffers so one barrier per row suffices
        uint32_t wt;
        const uint32_t ex = wave_exclusive_sum(in ? (w << 12) | 1u : 0u, wt);
        uint32_t* sw = s_w[r & 1];
        if (__lane_id() == 0) sw[wv] = wt;
        __syncthreads();
        uint32_t before = 0;
        for (int k = 0; k < wv; ++k) before += sw[k];
        if (in) {
            const uint32_t rank = before + ex;
            const uint64_t at = uint64_t(r) * nblk + blockIdx.x;
            const uint32_t e = escan[at] + (rank & 0xFFFu);
            const uint32_t p = pscan[at] + (rank >> 12);
            ent_id[e] = id;
            ent_pp[e] = p;
            ent_x[e] = xpack;
            // slices of the row that begin inside [p, p + w)
            const uint32_t rel = p - row_start[r];
            const uint32_t k0 = (rel + kSlice - 1) / kSlice, k1 = (rel + w - 1) / kSlice;
            for (uint32_t k = k0; k <= k1; ++k) {
                slice_entry[first_slice[r] + k] = e;
                slice_row[first_slice[r] + k] = uint32_t(r);
            }
        }
    }
}

// Locate slice b: its row (recorded by entry_kernel), index within the row,
// pair range and the range of entries that may overlap it.
struct Slice { int ty; uint32_t k, start, end, e0, e1; };

__device__ __forceinline__ bool find_slice(uint32_t b, const uint32_t* first_slice,
                                           const uint32_t* row_start, const uint32_t* erow,
                                           const uint32_t* slice_entry, const uint32_t* slice_row,
                                           int gy, uint32_t capacity, Slice& s) {
    if (row_start[gy] > capacity || b >= first_slice[gy]) return false;
    const int lo = int(slice_row[b]);
    s.ty = lo;
    s.k = b - first_slice[lo];
    s.start = row_start[lo] + s.k * kSlice;
    s.end = min(s.start + uint32_t(kSlice), row_start[lo + 1]);
    s.e0 = slice_entry[b];
    // the next slice's first entry may straddle the boundary: include it
    s.e1 = b + 1 < first_slice[lo + 1] ? slice_entry[b + 1] + 1 : erow[lo + 1];
    return true;
}

// The columns [c0, c1) an entry contributes to the slice's pairs [a, b).
__device__ __forceinline__ bool clip_entry(uint32_t pp, uint32_t xpack, uint32_t a, uint32_t b,
                                           uint32_t& c0, uint32_t& c1, uint32_t& p0) {
    const uint32_t xlo = xpack & 0xFFFFu, xhi = xpack >> 16;
    const uint32_t lo = max(a, pp), hi = min(b, pp + (xhi - xlo));
    c0 = xlo + (lo - pp);
    c1 = xlo + (hi - pp);
    p0 = lo;
    return lo < hi;
}

// hist[b][tx]: pairs of slice b in column tx, from the slice's entries: +1 at
// the first column of each entry's part, -1 after its last, then a prefix.
__global__ void __launch_bounds__(kHistThreads)
slice_hist_kernel(const uint32_t* __restrict__ ent_pp, const uint32_t* __restrict__ ent_x,
                  const uint32_t* __restrict__ first_slice, const uint32_t* __restrict__ row_start,
                  const uint32_t* __restrict__ erow, const uint32_t* __restrict__ slice_entry,
                  const uint32_t* __restrict__ slice_row, Grid grid, uint32_t capacity,
                  uint32_t* __restrict__ hist) {
    __shared__ int32_t d[kMaxCols + 1];
    __shared__ uint32_t s_w[kHistThreads / 64];
    Slice s;
    if (!find_slice(blockIdx.x, first_slice, row_start, erow, slice_entry, slice_row, grid.gy,
                    capacity, s))
        return;                                         // block-uniform
    const int gx = grid.gx, tid = threadIdx.x;
    for (int c = tid; c <= gx; c += kHistThreads) d[c] = 0;
    __syncthreads();
    for (uint32_t e = s.e0 + tid; e < s.e1; e += kHistThreads) {
        uint32_t c0, c1, p0;
        if (clip_entry(ent_pp[e], ent_x[e], s.start, s.end, c0, c1, p0)) {
            atomicAdd(&d[c0], 1);
            atomicSub(&d[c1], 1);
        }
    }
    __syncthreads();
    // prefix over the columns, kHistCols per thread
    constexpr int CPT = kHistCols;
    int32_t v[CPT];
    int32_t mine = 0;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int c = CPT * tid + j;
        v[j] = c < gx ? d[c] : 0;
        mine += v[j];
    }
    uint32_t all;
    int32_t run = int32_t(block_exclusive_sum<kHistThreads>(uint32_t(mine), s_w, all));
    const uint64_t base = uint64_t(blockIdx.x) * gx;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int c = CPT * tid + j;
        run += v[j];
        if (c < gx) hist[base + c] = uint32_t(run);
    }
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

// Per slice: expand the entries into the slice's pairs (column, Gaussian) in
// LDS, rank them per column in input order, stage them by column in LDS and
// write each to its final slot.
__global__ void __launch_bounds__(kScatterThreads)
slice_scatter_kernel(const uint32_t* __restrict__ ent_id, const uint32_t* __restrict__ ent_pp,
                     const uint32_t* __restrict__ ent_x, const uint32_t* __restrict__ first_slice,
                     const uint32_t* __restrict__ row_start, const uint32_t* __restrict__ erow,
                     const uint32_t* __restrict__ slice_entry,
                     const uint32_t* __restrict__ slice_row, const uint32_t* __restrict__ hist,
                     Grid grid, int col_bits, uint32_t capacity, uint32_t* __restrict__ out) {
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
    if (!find_slice(blockIdx.x, first_slice, row_start, erow, slice_entry, slice_row, grid.gy,
                    capacity, s))
        return;                                         // block-uniform
    const int tid = threadIdx.x, lane = __lane_id(), wv = tid >> 6;
    const uint32_t count = s.end - s.start;
    constexpr int CPT = kScatterCols;
    // output bases of this thread's columns, loaded early
    uint32_t gbase[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int c = CPT * tid + j;
        gbase[j] = c < gx ? hist[uint64_t(blockIdx.x) * gx + c] : 0u;
    }
    for (int b = tid; b < W * gx; b += kScatterThreads) s_wcnt[b] = 0;
    // the slice's pairs, in row-bucket order, expanded from its entries
    for (uint32_t e = s.e0 + tid; e < s.e1; e += kScatterThreads) {
        uint32_t c0, c1, p0;
        if (clip_entry(ent_pp[e], ent_x[e], s.start, s.end, c0, c1, p0)) {
            const uint32_t id = ent_id[e];
            for (uint32_t c = c0, i = p0 - s.start; c < c1; ++c, ++i) {
                s_val[i] = id;
                s_col[i] = uint16_t(c);
            }
        }
    }
    __syncthreads();
    uint32_t myv[R];
    uint32_t mycol[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t idx = uint32_t(wv * PER_WAVE + r * 64 + lane);
        const bool valid = idx < count;
        mycol[r] = valid ? uint32_t(s_col[idx]) : 0u;
        myv[r] = valid ? s_val[idx] : 0u;
    }
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
            s_gbase[c] = gbase[j];
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

uint32_t bin_blocks(int64_t n) { return uint32_t((n + kBinThreads - 1) / kBinThreads); }

uint64_t bin_max_slices(uint64_t pairs, int gy) { return pairs / kSlice + uint64_t(gy) + 1; }

hipError_t launch_counts(const uint8_t* ws, const Layout& L, const uint32_t* order, int64_t n,
                         const Grid& grid, hipStream_t s) {
    const uint32_t nblk = bin_blocks(n);
    if (nblk > 0) {
        auto* w = const_cast<uint8_t*>(ws);
        count_kernel<<<dim3(nblk), dim3(kBinThreads), size_t(grid.gy) * 8, s>>>(
            reinterpret_cast<const float4*>(ws + L.records), order, n, grid, nblk,
            reinterpret_cast<uint32_t*>(w + L.ecnt), reinterpret_cast<uint32_t*>(w + L.pcnt));
    }
    return hipGetLastError();
}

hipError_t launch_row_setup(uint8_t* ws, const Layout& L, int64_t n, const Grid& grid,
                            hipStream_t s) {
    row_setup_kernel<<<1, 256, 0, s>>>(reinterpret_cast<const uint32_t*>(ws + L.ecnt),
                                       reinterpret_cast<const uint32_t*>(ws + L.pcnt), bin_blocks(n),
                                       grid.gy, reinterpret_cast<uint32_t*>(ws + L.row_start),
                                       reinterpret_cast<uint32_t*>(ws + L.erow),
                                       reinterpret_cast<uint32_t*>(ws + L.first_slice));
    return hipGetLastError();
}

hipError_t launch_entries(uint8_t* ws, const Layout& L, const uint32_t* order, int64_t n,
                          const Grid& grid, uint32_t capacity, hipStream_t s) {
    const uint32_t nblk = bin_blocks(n);
    if (nblk == 0) return hipSuccess;
    auto u32 = [&](uint64_t off) { return reinterpret_cast<uint32_t*>(ws + off); };
    entry_kernel<<<dim3(nblk), dim3(kBinThreads), 0, s>>>(
        reinterpret_cast<const float4*>(ws + L.records), order, n, grid, nblk, u32(L.ecnt),
        u32(L.pcnt), u32(L.row_start), u32(L.first_slice), capacity, u32(L.ent_id),
        u32(L.ent_pp), u32(L.ent_x), u32(L.slice_entry), u32(L.slice_row));
    return hipGetLastError();
}

hipError_t prepare_binning_kernels() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&slice_scatter_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               int(scatter_lds_bytes(kMaxCols)));
}

hipError_t launch_col_sort(uint8_t* ws, const Layout& L, const Grid& grid, uint64_t slices,
                           uint32_t capacity, hipStream_t s) {
    auto u32 = [&](uint64_t off) { return reinterpret_cast<uint32_t*>(ws + off); };
    const uint32_t* fs = u32(L.first_slice);
    const uint32_t* rs = u32(L.row_start);
    const uint32_t* er = u32(L.erow);
    const uint32_t* se = u32(L.slice_entry);
    const uint32_t* sr = u32(L.slice_row);
    uint32_t* hist = u32(L.col_hist);
    if (slices > 0) {
        slice_hist_kernel<<<dim3(unsigned(slices)), dim3(kHistThreads), 0, s>>>(
            u32(L.ent_pp), u32(L.ent_x), fs, rs, er, se, sr, grid, capacity, hist);
    }
    col_scan_kernel<<<dim3(unsigned(grid.gy)), dim3(1024), 0, s>>>(hist, fs, rs, grid, capacity,
                                                                  u32(L.ranges));
    if (slices > 0) {
        int bits = 1;
        while ((1 << bits) < grid.gx) ++bits;
        // LDS above the default 64 KiB is enabled once by prepare_binning_kernels
        slice_scatter_kernel<<<dim3(unsigned(slices)), dim3(kScatterThreads),
                               scatter_lds_bytes(grid.gx), s>>>(
            u32(L.ent_id), u32(L.ent_pp), u32(L.ent_x), fs, rs, er, se, sr, hist, grid, bits,
            capacity, u32(L.pair_vals));
    }
    return hipGetLastError();
}

}  // namespace tgs
