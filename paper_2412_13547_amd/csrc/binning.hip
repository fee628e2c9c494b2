// Tile-Gaussian pairs in (tile id, depth) order and per-tile ranges (stage (b)).
//
// The order is the one a stable sort of 64-bit (tile << 32 | depth bits) keys
// produces, built without sorting 64-bit keys and without ever writing the
// pairs in any order but the final one:
//   1. the Gaussians are sorted by their 32-bit depth key (stable, so equal
//      depths keep ascending index; ``radix_sort``);
//   2. count_kernel: per block of 1024 consecutive Gaussians of that order and
//      per tile row, the number of *entries* (Gaussian x row: a Gaussian
//      covers the columns [xlo, xhi) of each row in [ylo, yhi)) and of pairs
//      the block puts in the row; exclusive scans over (row, block) give every
//      block's first entry and first pair in every row;
//   3. entry_kernel: every block writes, row by row, its entries (Gaussian,
//      first pair, columns) into the row's entry list -- in depth order --
//      with one wavefront scan per row a wavefront touches (four Gaussians
//      per lane), and marks where every column-sort slice of kSlice pairs
//      begins;
//   4. slice_hist + col_scan + slice_scatter: a stable counting sort by column
//      per slice.  The histogram comes from the slice's entries (two LDS
//      updates per entry, then a prefix over the columns); the scatter
//      expands the slice's entries into pairs in LDS, appending each entry
//      to the runs of the columns it covers in depth order (no ranking),
//      and writes each pair once, to its final place.
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

#include <algorithm>

namespace tgs {
namespace {

constexpr int kBinThreads = 256;                           // threads per count/entry block
constexpr int kBinPer = 4;                                 // Gaussians per thread
constexpr int kBinGauss = kBinThreads * kBinPer;           // Gaussians per count/entry block
constexpr int kEntryBatch = 2;                             // 64-entry batches loaded at once
constexpr int kScatterWaves = 8;                           // wavefronts per scatter block
constexpr int kHistThreads = 256;
constexpr int kHistLoads = 4;                              // 64-entry batches loaded at once
constexpr int kColBatch = 16;                              // slices loaded together in col_scan

// Orders this wavefront's LDS accesses: what its lanes wrote is visible to
// all its lanes after this.
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int wave_min(int x) {
    for (int o = 32; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o));
    return x;
}

__device__ __forceinline__ int wave_max(int x) {
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o));
    return x;
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

// Per block of kBinGauss depth positions and per row: entries and pairs.
// ecnt[r * nblk + blk], pcnt[r * nblk + blk] (row-major, so one flat scan
// gives the row starts and every block's offset inside every row).  Each
// thread gathers kBinPer rectangles with all their loads in flight.
__global__ void __launch_bounds__(kBinThreads)
count_kernel(const uint2* __restrict__ rects, const uint32_t* __restrict__ order, int64_t n,
             const uint32_t* __restrict__ dcount, Grid grid, uint32_t nblk,
             uint32_t* __restrict__ ecnt, uint32_t* __restrict__ pcnt, uint2* __restrict__ srect) {
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t s_w[kBinThreads / 64];
    const int gy = grid.gy;
    const int tid = threadIdx.x;
    // difference arrays over the rows (+1 / +w at a Gaussian's first row,
    // -1 / -w after its last; modulo 2^32), then one prefix over the rows
    uint32_t* ce = lds;               // [gy + 1]
    uint32_t* cp = lds + (gy + 1);    // [gy + 1]
    for (int r = tid; r <= gy; r += kBinThreads) ce[r] = cp[r] = 0;
    // the ids first (the order holds n of them, m valid), then the rectangles
    const int64_t s0 = int64_t(blockIdx.x) * kBinGauss + tid;
    uint32_t id[kBinPer];
#pragma unroll
    for (int k = 0; k < kBinPer; ++k) {
        const int64_t s = s0 + int64_t(k) * kBinThreads;
        id[k] = s < n ? order[s] : 0u;
    }
    const int64_t m = dcount ? min(n, int64_t(*dcount)) : n;     // Gaussians in the order
    uint2 packed[kBinPer];
#pragma unroll
    for (int k = 0; k < kBinPer; ++k) {
        const int64_t s = s0 + int64_t(k) * kBinThreads;
        packed[k] = s < m ? rects[id[k]] : make_uint2(0u, 0u);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kBinPer; ++k) {
        const int64_t s = s0 + int64_t(k) * kBinThreads;
        if (s < n) srect[s] = packed[k];
        const Rect rc = unpack_rect(packed[k]);
        const uint32_t w = uint32_t(rc.xhi - rc.xlo);
        if (rc.ylo < rc.yhi) {
            atomicAdd(&ce[rc.ylo], 1u);
            atomicAdd(&cp[rc.ylo], w);
            atomicSub(&ce[rc.yhi], 1u);
            atomicSub(&cp[rc.yhi], w);
        }
    }
    __syncthreads();
    // thread t owns the consecutive rows [t * cpl, t * cpl + cpl)
    const int cpl = (gy + kBinThreads - 1) / kBinThreads;
    const int r0 = tid * cpl;
    uint32_t se = 0, sp = 0;
    for (int j = 0; j < cpl; ++j) {
        if (r0 + j < gy) {
            se += ce[r0 + j];
            sp += cp[r0 + j];
        }
    }
    uint32_t tot;
    uint32_t re = block_exclusive_sum<kBinThreads>(se, s_w, tot);
    uint32_t rp = block_exclusive_sum<kBinThreads>(sp, s_w, tot);
    for (int j = 0; j < cpl; ++j) {
        const int r = r0 + j;
        if (r < gy) {
            re += ce[r];
            rp += cp[r];
            ecnt[uint64_t(r) * nblk + blockIdx.x] = re;
            pcnt[uint64_t(r) * nblk + blockIdx.x] = rp;
        }
    }
}

// row_start[r] = first pair of row r (row_start[gy] = pair count),
// erow[r] = first entry of row r, first_slice[r] = first column-sort slice
// of row r (prefix of ceil(pairs / kSlice)); the last slice of a row ends at
// the row's last entry (slice_e1).
__global__ void __launch_bounds__(256)
row_setup_kernel(const uint32_t* __restrict__ escan, const uint32_t* __restrict__ pscan,
                 uint32_t nblk, int gy, uint32_t max_slices, uint32_t* __restrict__ row_start,
                 uint32_t* __restrict__ erow, uint32_t* __restrict__ first_slice,
                 uint32_t* __restrict__ slice_e1) {
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
        if (ty < gy && ns > 0 && before + ex + ns <= max_slices)
            slice_e1[before + ex + ns - 1] = escan[uint64_t(ty + 1) * nblk];
        __syncthreads();
        if (threadIdx.x == 0) carry += all;
        __syncthreads();
    }
}

// Every block writes its entries row by row: ent_id (Gaussian), ent_pp
// (first pair of the entry), ent_x (xlo | xhi << 16).  A Gaussian's rank in
// a row among the block's Gaussians counts entries and pairs at once
// (packed: pairs << 11 | 1; a block holds at most 1024 entries and 1024 *
// 1024 pairs of a row).  Lane l of wavefront w holds the kBinPer
// consecutive depth positions 256 w + 4 l .. 256 w + 4 l + 3 of the block,
// so a lane's sum followed by one wavefront scan ranks the wavefront's 256
// Gaussians in a row.  Per wavefront and row the packed totals come from
// difference arrays over the rows and a prefix, a prefix over the
// wavefronts gives each wavefront's first rank in every row, and then each
// wavefront walks its own rows with no barrier.  The entry that holds the
// first pair of a column-sort slice writes the slice's descriptor and
// closes the slice before it.
constexpr uint32_t kRankShift = 11;                        // pairs << 11 | entries
constexpr uint32_t kRankMask = (1u << kRankShift) - 1u;

__global__ void __launch_bounds__(kBinThreads)
entry_kernel(const uint2* __restrict__ srect, const uint32_t* __restrict__ order, int64_t n,
             const uint32_t* __restrict__ dcount, Grid grid, uint32_t nblk,
             const uint32_t* __restrict__ escan, const uint32_t* __restrict__ pscan,
             const uint32_t* __restrict__ row_start, const uint32_t* __restrict__ first_slice,
             uint32_t capacity, uint32_t* __restrict__ ent_id, uint32_t* __restrict__ ent_pp,
             uint32_t* __restrict__ ent_x, uint4* __restrict__ slice_desc,
             uint32_t* __restrict__ slice_e1) {
    constexpr int W = kBinThreads / 64;
    // per row: this block's first entry and pair, the row's first pair and
    // first slice (loaded once, so the row loop never waits on memory); per
    // wavefront and row: the packed count, then the wavefront's first rank
    extern __shared__ uint32_t s_row[];
    const int gy = grid.gy;
    uint32_t* s_e = s_row;
    uint32_t* s_p = s_row + (gy + 1);
    uint32_t* s_rs = s_row + 2 * (gy + 1);
    uint32_t* s_fs = s_row + 3 * (gy + 1);
    uint32_t* s_wr = s_row + 4 * (gy + 1);                  // [W][gy + 1]
    __shared__ uint32_t s_stage[W][3][kBinThreads];         // a row's entries per wavefront
    if (row_start[gy] > capacity) return;               // overflow: block-uniform
    for (int r = threadIdx.x; r <= gy; r += kBinThreads) {
        if (r < gy) {
            s_e[r] = escan[uint64_t(r) * nblk + blockIdx.x];
            s_p[r] = pscan[uint64_t(r) * nblk + blockIdx.x];
        }
        s_rs[r] = row_start[r];
        s_fs[r] = first_slice[r];
    }
    for (int i = threadIdx.x; i < W * (gy + 1); i += kBinThreads) s_wr[i] = 0;
    const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int lane = __lane_id();
    const int64_t s0 = int64_t(blockIdx.x) * kBinGauss + int64_t(threadIdx.x) * kBinPer;
    uint32_t id[kBinPer], xpack[kBinPer], unit[kBinPer];
    int ylo[kBinPer], yhi[kBinPer];
#pragma unroll
    for (int k = 0; k < kBinPer; ++k) {
        const int64_t s = s0 + k;
        id[k] = s < n ? order[s] : 0u;                       // (loaded before m arrives)
        const uint2 packed = s < n ? srect[s] : make_uint2(0u, 0u);
        const Rect rc = unpack_rect(packed);
        xpack[k] = packed.x;
        ylo[k] = rc.ylo;
        yhi[k] = rc.yhi;
        unit[k] = (uint32_t(rc.xhi - rc.xlo) << kRankShift) | 1u;
    }
    const int64_t m = dcount ? min(n, int64_t(*dcount)) : n;
#pragma unroll
    for (int k = 0; k < kBinPer; ++k)
        if (s0 + k >= m) id[k] = 0u;
    __syncthreads();
    // difference arrays of this wavefront's packed counts over the rows
    // (modulo 2^32; a wavefront's count of a row stays below 2048)
    uint32_t* wr = s_wr + wv * (gy + 1);
#pragma unroll
    for (int k = 0; k < kBinPer; ++k) {
        if (ylo[k] < yhi[k]) {
            atomicAdd(&wr[ylo[k]], unit[k]);
            atomicSub(&wr[yhi[k]], unit[k]);
        }
    }
    wave_sync_lds();
    // prefix over the rows: lane l owns the rows [l * cpl, l * cpl + cpl)
    const int cpl = (gy + 63) / 64;
    uint32_t sum = 0;
    for (int j = 0; j < cpl; ++j) {
        const int r = lane * cpl + j;
        if (r < gy) sum += wr[r];
    }
    uint32_t all;
    uint32_t run = wave_exclusive_sum(sum, all);
    for (int j = 0; j < cpl; ++j) {
        const int r = lane * cpl + j;
        if (r < gy) {
            run += wr[r];
            wr[r] = run;
        }
    }
    __syncthreads();
    // per row: the wavefronts' first ranks (exclusive prefix over them)
    for (int r = threadIdx.x; r < gy; r += kBinThreads) {
        uint32_t b = 0;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const uint32_t v = s_wr[k * (gy + 1) + r];
            s_wr[k * (gy + 1) + r] = b;
            b += v;
        }
    }
    __syncthreads();
    // this wavefront's rows
    int lo = gy, hi = 0;
#pragma unroll
    for (int k = 0; k < kBinPer; ++k) {
        if (ylo[k] < yhi[k]) {
            lo = min(lo, ylo[k]);
            hi = max(hi, yhi[k]);
        }
    }
    const int r0 = wave_min(lo), r1 = wave_max(hi);
    // per row: the wavefront's entries of the row are consecutive in the
    // row's list; they are staged in LDS by their index among them and
    // written with full-wavefront stores
    uint32_t* st_id = s_stage[wv][0];
    uint32_t* st_pp = s_stage[wv][1];
    uint32_t* st_x = s_stage[wv][2];
    for (int r = r0; r < r1; ++r) {
        uint32_t x[kBinPer], lsum = 0;
#pragma unroll
        for (int k = 0; k < kBinPer; ++k) {
            x[k] = (r >= ylo[k] && r < yhi[k]) ? unit[k] : 0u;
            lsum += x[k];
        }
        const uint32_t incl = wave_inclusive_sum(lsum);
        const uint32_t first = wr[r];                        // the wavefront's first rank
        const uint32_t cnt = uint32_t(__builtin_amdgcn_readlane(int(incl), 63)) & kRankMask;
        const uint32_t pbase = s_p[r];
        uint32_t rank = first + incl - lsum;
#pragma unroll
        for (int k = 0; k < kBinPer; ++k) {
            if (x[k] != 0u) {
                const uint32_t i = (rank & kRankMask) - (first & kRankMask);
                st_id[i] = id[k];
                st_pp[i] = pbase + (rank >> kRankShift);
                st_x[i] = xpack[k];
            }
            rank += x[k];
        }
        wave_sync_lds();
        const uint32_t e0 = s_e[r] + (first & kRankMask);
        const uint32_t rs = s_rs[r];
        for (uint32_t i = uint32_t(lane); i < cnt; i += 64u) {
            const uint32_t e = e0 + i;
            const uint32_t p = st_pp[i], xp = st_x[i];
            ent_id[e] = st_id[i];
            ent_pp[e] = p;
            ent_x[e] = xp;
            // slices of the row that begin inside [p, p + w): their
            // descriptors, and the end of the slice before each (entries
            // overlapping a slice boundary belong to both slices; row_setup
            // ends every row's last slice)
            const uint32_t w = (xp >> 16) - (xp & 0xFFFFu);
            const uint32_t rel = p - rs;
            const uint32_t k0 = (rel + kSlice - 1) / kSlice, k1 = (rel + w - 1) / kSlice;
            if (k0 <= k1) {
                const uint32_t re = s_rs[r + 1];
                const uint32_t fs = s_fs[r], ns = s_fs[r + 1] - fs;
                for (uint32_t q = k0; q <= k1; ++q) {
                    const uint32_t a = rs + q * kSlice;
                    slice_desc[fs + q] = make_uint4(e, a, min(a + uint32_t(kSlice), re),
                                                    uint32_t(r) | (q + 1 == ns ? 1u << 31 : 0u));
                    if (q > 0) slice_e1[fs + q - 1] = e + 1;
                }
            }
        }
        wave_sync_lds();                                     // stage read before the next row
    }
}

// Slice b: its row, pair range and the range of entries that may overlap it
// (the descriptor written by entry_kernel; e1 includes the entry that
// straddles into the next slice).  False when b is past the slices or the
// pairs overflowed the capacity.
struct Slice { int ty; bool last; uint32_t start, end, e0, e1; };

__device__ __forceinline__ bool find_slice(uint32_t b, const uint32_t* first_slice,
                                           const uint32_t* row_start, const uint4* slice_desc,
                                           const uint32_t* slice_e1, int gy, uint32_t capacity,
                                           Slice& s) {
    const uint32_t total = row_start[gy], nsl = first_slice[gy];
    const uint4 d = slice_desc[b];
    s.e1 = slice_e1[b];
    if (total > capacity || b >= nsl) return false;
    s.e0 = d.x;
    s.start = d.y;
    s.end = d.z;
    s.ty = int(d.w & 0x7FFFFFFFu);
    s.last = (d.w >> 31) != 0;
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
// One wavefront per slice (no block barriers), kHistThreads / 64 slices per
// block.
__global__ void __launch_bounds__(kHistThreads)
slice_hist_kernel(const uint32_t* __restrict__ ent_pp, const uint32_t* __restrict__ ent_x,
                  const uint32_t* __restrict__ first_slice, const uint32_t* __restrict__ row_start,
                  const uint4* __restrict__ slice_desc, const uint32_t* __restrict__ slice_e1,
                  Grid grid, uint32_t slices, uint32_t capacity, uint32_t* __restrict__ hist) {
    constexpr int W = kHistThreads / 64;
    __shared__ int32_t d_all[W][kMaxCols + 1];
    const int wv = int(threadIdx.x >> 6), lane = __lane_id();
    const uint32_t b = blockIdx.x * W + uint32_t(wv);
    Slice s;
    if (b >= slices ||                                  // past the launched slices
        !find_slice(b, first_slice, row_start, slice_desc, slice_e1, grid.gy, capacity, s))
        return;                                         // wavefront-uniform
    const int gx = grid.gx;
    int32_t* d = d_all[wv];
    for (int c = lane; c <= gx; c += 64) d[c] = 0;
    wave_sync_lds();
    // kHistLoads batches of 64 entries in flight at once
    for (uint32_t e0 = s.e0; e0 < s.e1; e0 += 64u * kHistLoads) {
        uint32_t pp[kHistLoads], xp[kHistLoads];
#pragma unroll
        for (int u = 0; u < kHistLoads; ++u) {
            const uint32_t e = e0 + 64u * uint32_t(u) + uint32_t(lane);
            pp[u] = e < s.e1 ? ent_pp[e] : 0u;
            xp[u] = e < s.e1 ? ent_x[e] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kHistLoads; ++u) {
            const uint32_t e = e0 + 64u * uint32_t(u) + uint32_t(lane);
            uint32_t c0, c1, p0;
            if (e < s.e1 && clip_entry(pp[u], xp[u], s.start, s.end, c0, c1, p0)) {
                atomicAdd(&d[c0], 1);
                atomicSub(&d[c1], 1);
            }
        }
    }
    wave_sync_lds();
    // prefix over the columns: each lane a chunk of consecutive columns
    const int cpl = (gx + 63) / 64;
    int32_t mine = 0;
    for (int j = 0; j < cpl; ++j) {
        const int c = lane * cpl + j;
        if (c < gx) mine += d[c];
    }
    uint32_t all;
    int32_t run = int32_t(wave_exclusive_sum(uint32_t(mine), all));
    for (int j = 0; j < cpl; ++j) {
        const int c = lane * cpl + j;
        if (c < gx) {
            run += d[c];
            d[c] = run;
        }
    }
    wave_sync_lds();
    const uint64_t base = uint64_t(b) * gx;
    for (int c = lane; c < gx; c += 64) hist[base + c] = uint32_t(d[c]);
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
    // kColBatch independent loads in flight per thread
    uint32_t sum = 0;
    for (uint32_t k = k0; k < k1; k += kColBatch) {
        uint32_t v[kColBatch];
#pragma unroll
        for (int q = 0; q < kColBatch; ++q)       // clamped: no branch between the loads
            v[q] = hist[uint64_t(s0 + min(k + q, k1 - 1)) * gx + tx];
#pragma unroll
        for (int q = 0; q < kColBatch; ++q) sum += k + q < k1 ? v[q] : 0u;
    }
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
        for (uint32_t k = k0; k < k1; k += kColBatch) {
            uint32_t v[kColBatch];
#pragma unroll
            for (int q = 0; q < kColBatch; ++q)
                v[q] = hist[uint64_t(s0 + min(k + q, k1 - 1)) * gx + tx];
#pragma unroll
            for (int q = 0; q < kColBatch; ++q) {
                if (k + q < k1) hist[uint64_t(s0 + k + q) * gx + tx] = run;
                run += v[q];
            }
        }
    }
}

// Per slice: a lane per column, one wavefront per (group of 64 columns,
// part of the slice's entries).  A wavefront walks its part's entries in
// depth order; an entry covering the lane's column appends the Gaussian to
// the column's run in LDS, so every run is in depth order without ranking.
// Runs are laid out in column order (local slot of column c = the slice's
// pairs in columns < c), the parts of a column one after the other: a
// part's first slot in a column follows the earlier parts' pairs there,
// counted from difference arrays (+1 at an entry's first column, -1 after
// its last) that the wavefronts fill before the walk.  For the walk, each
// batch of 64 entries held in registers is compacted (ballot + lane prefix)
// into a wavefront-private LDS list of the entries that touch the group;
// the wavefront then reads the list back entry by entry with uniform
// addresses (an LDS broadcast), so per covering entry the walk is a few
// vector instructions and one LDS write by the covered lanes.  A run's local
// and output slots advance together (across the parts of a column too), so
// beside each Gaussian the walk stores the column's constant (output slot -
// local slot).  At the end each wavefront copies a share of its group's runs
// out; a run's consecutive local slots go to consecutive output slots.
//
// The count of (slice b, column c) is base[b + 1][c] - base[b][c] for the
// bases col_scan wrote, or the tile's end minus base[b][c] for the row's last
// slice (an empty tile has end 0 and count 0).
struct ScatterShape {
    int groups, parts;
};

constexpr int kWalkUnroll = 4;                             // list entries read per walk step
constexpr int kListLen = 64 + kWalkUnroll;                 // a batch plus the padding

__host__ __device__ inline ScatterShape scatter_shape(int gx) {
    const int groups = (gx + 63) / 64;
    const int parts = groups >= kScatterWaves ? 1 : kScatterWaves / groups;
    return ScatterShape{groups, parts};
}

__global__ void __launch_bounds__(1024)
slice_scatter_kernel(const uint32_t* __restrict__ ent_id, const uint32_t* __restrict__ ent_pp,
                     const uint32_t* __restrict__ ent_x, const uint32_t* __restrict__ first_slice,
                     const uint32_t* __restrict__ row_start, const uint4* __restrict__ slice_desc,
                     const uint32_t* __restrict__ slice_e1, const uint32_t* __restrict__ base,
                     const uint32_t* __restrict__ ranges, Grid grid, uint32_t max_slices,
                     uint32_t capacity, uint32_t* __restrict__ out) {
    extern __shared__ uint32_t smem[];
    const int gx = grid.gx;
    const ScatterShape sh = scatter_shape(gx);
    const int waves = sh.groups * sh.parts;
    uint32_t* s_id = smem;                                         // [kSlice] Gaussian, then
                                                                   // [kSlice] output - local slot
    uint2* s_list = reinterpret_cast<uint2*>(smem + 2 * kSlice);   // [waves][kListLen] (Gaussian, lo | len << 16)
    int32_t* s_diff = reinterpret_cast<int32_t*>(s_list + kListLen * waves); // [waves][65]
    uint32_t* s_gtot = reinterpret_cast<uint32_t*>(s_diff + 65 * waves);  // [groups]
    const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6)), lane = __lane_id();
    const int g = w % sh.groups, p = w / sh.groups;
    const uint32_t b = blockIdx.x;
    const uint32_t cbeg = 64u * uint32_t(g), col = cbeg + uint32_t(lane);
    const bool col_ok = col < uint32_t(gx);
    // the slice and this column's bases (independent loads)
    uint32_t c_base = 0, c_next = 0;
    if (col_ok) {
        c_base = base[uint64_t(b) * gx + col];
        if (b + 1 < max_slices) c_next = base[uint64_t(b + 1) * gx + col];
    }
    Slice s;
    if (!find_slice(b, first_slice, row_start, slice_desc, slice_e1, grid.gy, capacity, s))
        return;                                                    // block-uniform
    // this part's entries [pe0, pe1)
    const uint32_t ne = s.e1 - s.e0, per = (ne + uint32_t(sh.parts) - 1) / uint32_t(sh.parts);
    const uint32_t pe0 = s.e0 + min(ne, uint32_t(p) * per);
    const uint32_t pe1 = s.e0 + min(ne, uint32_t(p + 1) * per);
    uint32_t pp[kEntryBatch], xp[kEntryBatch], id[kEntryBatch];
    auto load = [&](uint32_t e) {
#pragma unroll
        for (int j = 0; j < kEntryBatch; ++j) {
            const uint32_t ee = e + 64u * uint32_t(j) + uint32_t(lane);
            const bool ok = ee < pe1;
            pp[j] = ok ? ent_pp[ee] : 0u;
            xp[j] = ok ? ent_x[ee] : 0u;
            id[j] = ok ? ent_id[ee] : 0u;
        }
    };
    load(pe0);
    if (s.last && col_ok) {
        c_next = ranges[2 * (uint64_t(s.ty) * gx + col) + 1];
        if (c_next == 0) c_next = c_base;
    }
    const uint32_t cnt = col_ok ? c_next - c_base : 0u;
    for (int i = int(threadIdx.x); i < 65 * waves; i += int(blockDim.x)) s_diff[i] = 0;
    if (p == 0) {
        const uint32_t t = wave_total(cnt);
        if (lane == 0) s_gtot[g] = t;
    }
    __syncthreads();
    // the columns [lo, hi) of the group that entry j of the batch at e
    // covers in the slice (lo == hi: none)
    auto cover = [&](int j, uint32_t e, uint32_t& lo, uint32_t& hi) {
        const uint32_t ee = e + 64u * uint32_t(j) + uint32_t(lane);
        uint32_t c0 = 0, c1 = 0, p0;
        const bool in = ee < pe1 && clip_entry(pp[j], xp[j], s.start, s.end, c0, c1, p0);
        lo = max(c0, cbeg) - cbeg;
        hi = min(c1, cbeg + 64u);
        hi = in && hi > cbeg ? hi - cbeg : 0u;
        if (hi < lo) hi = lo;
    };
    // difference array of this wavefront's part over the group's columns;
    // when the part fits one load the spans are kept for the walk
    int32_t* diff = s_diff + 65 * w;
    constexpr uint32_t kBatch = 64u * kEntryBatch;
    uint32_t span[kEntryBatch];
    for (uint32_t e = pe0; e < pe1; e += kBatch) {
        if (e != pe0) load(e);
#pragma unroll
        for (int j = 0; j < kEntryBatch; ++j) {
            if (e + 64u * uint32_t(j) >= pe1) break;               // wave-uniform
            uint32_t lo, hi;
            cover(j, e, lo, hi);
            span[j] = lo | (hi << 16);
            if (lo < hi) {
                atomicAdd(&diff[lo], 1);
                atomicAdd(&diff[hi], -1);
            }
        }
    }
    __syncthreads();
    // first local slot and first output slot of the column in this part
    uint32_t before = 0;
    for (int h = 0; h < g; ++h) before += s_gtot[h];
    uint32_t gtot;
    uint32_t slot = before + wave_exclusive_sum(cnt, gtot);
    uint32_t dst = c_base;
    for (int q = 0; q < p; ++q) {
        const uint32_t c = wave_inclusive_sum(uint32_t(s_diff[65 * (q * sh.groups + g) + lane]));
        slot += c;
        dst += c;
    }
    // the walk: the entries covering part of the group, in depth order,
    // compacted per batch into this wavefront's list and read back with
    // uniform addresses; padding entries (len 0) cover no column
    uint32_t* pv = s_id + slot;                                    // next slot of the column
    const uint32_t kofs = dst - slot;
    uint2* list = s_list + kListLen * w;
    const bool reload = pe1 - pe0 > kBatch;
    for (uint32_t e = pe0; e < pe1; e += kBatch) {
        if (reload) load(e);
#pragma unroll
        for (int j = 0; j < kEntryBatch; ++j) {
            if (e + 64u * uint32_t(j) >= pe1) break;               // wave-uniform
            uint32_t lo, hi;
            if (reload) {
                cover(j, e, lo, hi);
            } else {
                lo = span[j] & 0xFFFFu;
                hi = span[j] >> 16;
            }
            const bool has = lo < hi;
            const uint64_t m = __ballot(has);
            const uint32_t pos = __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32),
                                                           __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
            const uint32_t cnt = uint32_t(__builtin_popcountll(m));
            if (has) list[pos] = make_uint2(id[j], lo | ((hi - lo) << 16));
            if (lane < kWalkUnroll) list[cnt + uint32_t(lane)] = make_uint2(0u, 0u);
            wave_sync_lds();
            for (uint32_t k = 0; k < cnt; k += kWalkUnroll) {
                uint2 v[kWalkUnroll];
#pragma unroll
                for (int u = 0; u < kWalkUnroll; ++u) v[u] = list[k + uint32_t(u)];
#pragma unroll
                for (int u = 0; u < kWalkUnroll; ++u) {
                    if (uint32_t(lane) - (v[u].y & 0xFFFFu) < (v[u].y >> 16)) {
                        pv[0] = v[u].x;
                        pv[kSlice] = kofs;
                        ++pv;
                    }
                }
            }
            wave_sync_lds();                                       // list read before it is rewritten
        }
    }
    __syncthreads();
    // a share of the group's runs, local slots [before, before + gtot) (the
    // counts of a consistent column sort keep them within kSlice)
    const uint32_t share = (gtot + uint32_t(sh.parts) - 1) / uint32_t(sh.parts);
    const uint32_t i0 = before + min(gtot, uint32_t(p) * share);
    const uint32_t i1 = min(before + min(gtot, uint32_t(p + 1) * share), uint32_t(kSlice));
    for (uint32_t i = i0 + uint32_t(lane); i < i1; i += 256u) {
        uint2 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t ii = i + 64u * uint32_t(q);
            v[q] = ii < i1 ? make_uint2(s_id[ii], s_id[kSlice + ii]) : make_uint2(0u, capacity - ii);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t o = i + 64u * uint32_t(q) + v[q].y;     // output slot
            if (o < capacity) out[o] = v[q].x;
        }
    }
}

size_t scatter_lds_bytes(int gx) {
    const ScatterShape sh = scatter_shape(gx);
    const size_t waves = size_t(sh.groups) * sh.parts;
    return size_t(kSlice) * 8 + waves * kListLen * 8 + waves * 65 * 4 + size_t(sh.groups) * 4;
}

// Dynamic LDS of the entry kernel for gy tile rows: four row tables and
// one row table per wavefront.
size_t entry_lds_bytes(int gy) { return size_t(gy + 1) * 4 * (4 + kBinThreads / 64); }

}  // namespace

uint32_t bin_blocks(int64_t n) { return uint32_t((n + kBinGauss - 1) / kBinGauss); }

uint64_t bin_max_slices(uint64_t pairs, int gy) { return pairs / kSlice + uint64_t(gy) + 1; }

hipError_t launch_counts(const uint8_t* ws, const Layout& L, const uint32_t* order, int64_t n,
                         const uint32_t* dcount, const Grid& grid, hipStream_t s) {
    const uint32_t nblk = bin_blocks(n);
    if (nblk > 0) {
        auto* w = const_cast<uint8_t*>(ws);
        count_kernel<<<dim3(nblk), dim3(kBinThreads), size_t(grid.gy + 1) * 8, s>>>(
            reinterpret_cast<const uint2*>(ws + L.rects), order, n, dcount, grid, nblk,
            reinterpret_cast<uint32_t*>(w + L.ecnt), reinterpret_cast<uint32_t*>(w + L.pcnt),
            reinterpret_cast<uint2*>(w + L.srect));
    }
    return hipGetLastError();
}

hipError_t launch_row_setup(uint8_t* ws, const Layout& L, int64_t n, const Grid& grid,
                            uint64_t max_slices, hipStream_t s) {
    auto u32 = [&](uint64_t off) { return reinterpret_cast<uint32_t*>(ws + off); };
    row_setup_kernel<<<1, 256, 0, s>>>(u32(L.ecnt), u32(L.pcnt), bin_blocks(n), grid.gy,
                                       uint32_t(std::min<uint64_t>(max_slices, 0xFFFFFFFFu)),
                                       u32(L.row_start), u32(L.erow), u32(L.first_slice),
                                       u32(L.slice_e1));
    return hipGetLastError();
}

hipError_t launch_entries(uint8_t* ws, const Layout& L, const uint32_t* order, int64_t n,
                          const uint32_t* dcount, const Grid& grid, uint32_t capacity,
                          hipStream_t s) {
    const uint32_t nblk = bin_blocks(n);
    if (nblk == 0) return hipSuccess;
    auto u32 = [&](uint64_t off) { return reinterpret_cast<uint32_t*>(ws + off); };
    entry_kernel<<<dim3(nblk), dim3(kBinThreads), entry_lds_bytes(grid.gy), s>>>(
        reinterpret_cast<const uint2*>(ws + L.srect), order, n, dcount, grid, nblk, u32(L.ecnt),
        u32(L.pcnt), u32(L.row_start), u32(L.first_slice), capacity, u32(L.ent_id),
        u32(L.ent_pp), u32(L.ent_x), reinterpret_cast<uint4*>(ws + L.slice_desc), u32(L.slice_e1));
    return hipGetLastError();
}

hipError_t prepare_binning_kernels() {
    size_t most = 0;
    for (int gx = 1; gx <= kMaxCols; gx += 64) most = std::max(most, scatter_lds_bytes(gx));
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&slice_scatter_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(most));
    if (e != hipSuccess) return e;
    // the row tables of the tallest grid the API accepts (4 kMaxCols rows)
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&entry_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               int(entry_lds_bytes(4 * kMaxCols)));
}

hipError_t launch_col_sort(uint8_t* ws, const Layout& L, const Grid& grid, uint64_t slices,
                           uint32_t capacity, hipStream_t s) {
    auto u32 = [&](uint64_t off) { return reinterpret_cast<uint32_t*>(ws + off); };
    const uint32_t* fs = u32(L.first_slice);
    const uint32_t* rs = u32(L.row_start);
    const auto* sd = reinterpret_cast<const uint4*>(ws + L.slice_desc);
    const uint32_t* e1 = u32(L.slice_e1);
    uint32_t* hist = u32(L.col_hist);
    if (slices > 0) {
        const uint64_t hist_blocks = (slices + kHistThreads / 64 - 1) / (kHistThreads / 64);
        slice_hist_kernel<<<dim3(unsigned(hist_blocks)), dim3(kHistThreads), 0, s>>>(
            u32(L.ent_pp), u32(L.ent_x), fs, rs, sd, e1, grid, uint32_t(slices), capacity, hist);
    }
    col_scan_kernel<<<dim3(unsigned(grid.gy)), dim3(1024), 0, s>>>(hist, fs, rs, grid, capacity,
                                                                  u32(L.ranges));
    if (slices > 0) {
        const ScatterShape sh = scatter_shape(grid.gx);
        const unsigned threads = 64u * unsigned(sh.groups * sh.parts);
        slice_scatter_kernel<<<dim3(unsigned(slices)), dim3(threads), scatter_lds_bytes(grid.gx),
                               s>>>(u32(L.ent_id), u32(L.ent_pp), u32(L.ent_x), fs, rs, sd, e1,
                                    hist, u32(L.ranges), grid, uint32_t(slices), capacity,
                                    u32(L.pair_vals));
    }
    return hipGetLastError();
}

}  // namespace tgs
