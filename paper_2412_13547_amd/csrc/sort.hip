// Device-wide primitives: exclusive scan and stable LSD radix sort of
// (uint32 key, uint32 value) pairs, written for wave64.
//
// Radix sort over 8-bit digits, least significant first: two set-up
// launches, then one launch per digit (a decoupled look-back over the tiles
// replaces a device-wide scan of per-tile counts in every pass):
//   1. a fill of the digit totals and tickets, then sort_hist: every block
//      counts the digits of all passes over its share of the keys (eight
//      LDS copies), adds its counts to the totals and clears part of the
//      look-back states.
//   2. sort_pass, per digit: a block takes the next tile of 4096 keys in
//      launch order (a ticket, so that every earlier tile's block has
//      started) and each digit's first output slot from a prefix over the
//      totals (the first pass's first tile also stores the number of pairs
//      kept).  It ranks the tile's keys among those of their digit, 1024 at
//      a time in input order (equal digits inside a wavefront ranked with
//      eight ballots, wavefronts ordered by a prefix over them per digit,
//      so equal keys keep their input order), publishes its count per digit
//      at once, sums the counts of the earlier tiles per digit by reading
//      their published states from the nearest back (a state that already
//      holds an inclusive prefix ends the walk) and publishes its own
//      inclusive prefix, while the other wavefronts order the tile by digit
//      in LDS; then it writes each digit's run to consecutive output slots.
// A published state is one word, flag << 30 | count, so a reader needs no
// ordering beyond the word itself; waits are bounded.
// The sort may drop every pair whose key equals a given value (it is
// neither counted nor written); the number of pairs kept is then on the
// device, and the passes after the first read it (their grids are sized for
// the input count; tiles past the kept count are empty).
#include "common.hpp"
#include "wave.hpp"

namespace tgs {
namespace {

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (uint64_t(1) << lane_id()) - 1;
}

// How a pass treats its input: the number of keys (the host bound, or the
// device count when given) and the dropped key, if any.
struct PassInput {
    uint64_t bound;
    const uint32_t* dcount;
    bool drop_on;
    uint32_t drop;
    __device__ uint64_t count() const { return dcount ? min(bound, uint64_t(*dcount)) : bound; }
    __device__ bool kept(uint32_t k) const { return !drop_on || k != drop; }
};

constexpr int kMaxPasses = 4;                          // 32-bit keys
constexpr int kHistBlocks = 256;                       // blocks of sort_hist
constexpr uint32_t kStateAgg = 1u << 30;               // the tile's own count
constexpr uint32_t kStateIncl = 2u << 30;              // the count of tiles [0, tile]
constexpr uint32_t kStateMask = (1u << 30) - 1u;
constexpr int kLookbackSpins = 1 << 17;                // bound on a wait for one state

// The sort's work area (uint32 words): per pass the total of every digit,
// the kept count, a ticket per pass, then the look-back states,
// [pass][tile][digit].
struct SortArea {
    uint32_t* total;      // [kMaxPasses][kRadixBuckets]
    uint32_t* kept;       // [1]
    uint32_t* tickets;    // [kMaxPasses]
    uint32_t* states;     // [kMaxPasses][tiles][kRadixBuckets]
};

constexpr uint64_t kAreaHead = kMaxPasses * kRadixBuckets + 8;   // totals, kept, tickets

__host__ __device__ inline SortArea sort_area(uint32_t* w) {
    SortArea a;
    a.total = w;
    a.kept = w + kMaxPasses * kRadixBuckets;
    a.tickets = a.kept + 1;
    a.states = w + kAreaHead;
    return a;
}

__global__ void __launch_bounds__(1024)
sort_hist(const uint32_t* __restrict__ keys, uint64_t count, int passes, bool drop_on,
          uint32_t drop, SortArea area, uint64_t state_words) {
    // eight copies (two wavefronts each): the top digits of depth keys
    // share a few values, and one copy would serialise their updates
    constexpr int kCopies = 8;
    __shared__ uint32_t hist[kCopies][kMaxPasses * kRadixBuckets];
    const uint32_t tid = threadIdx.x;
    uint32_t* mine = hist[(tid >> 6) & (kCopies - 1)];
    for (uint32_t i = tid; i < kCopies * kMaxPasses * kRadixBuckets; i += blockDim.x)
        (&hist[0][0])[i] = 0u;
    // the look-back states start empty (the totals and tickets were filled)
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + tid; i < state_words;
         i += uint64_t(gridDim.x) * blockDim.x)
        area.states[i] = 0u;
    __syncthreads();
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + tid; i < count;
         i += uint64_t(gridDim.x) * blockDim.x) {
        const uint32_t k = keys[i];
        if (drop_on && k == drop) continue;
        for (int p = 0; p < passes; ++p)
            atomicAdd(&mine[p * kRadixBuckets + ((k >> (p * kRadixBits)) & (kRadixBuckets - 1))], 1u);
    }
    __syncthreads();
    for (uint32_t i = tid; i < kMaxPasses * kRadixBuckets; i += blockDim.x) {
        uint32_t t = 0;
        for (int c = 0; c < kCopies; ++c) t += hist[c][i];
        if (t) atomicAdd(&area.total[i], t);
    }
}

// Forward declaration: block-wide exclusive scan (defined with the scans).
template <typename T, int NT, bool SAT = false>
__device__ __forceinline__ T block_exclusive_scan(T x, T& total);

constexpr int kScatterThreads = 1024;
constexpr int kScatterRounds = kSortTile / kScatterThreads;

constexpr int kLookbackWindow = 4;                   // states read at once

// One tile's state for digit d (the word at w), waiting while it is empty.
// A wait ends after kLookbackSpins reads: a tile's state is published right
// after its keys are ranked, by a block that started before the reader's,
// so the bound is never reached in a correct launch.
__device__ __forceinline__ uint32_t wait_state(const uint32_t* w, uint32_t v) {
    for (int spin = 0; v == 0u && spin < kLookbackSpins; ++spin) {
        __builtin_amdgcn_s_sleep(1);
        v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return v;
}

// The counts of the tiles before `tile` for digit d, from their states,
// nearest first, kLookbackWindow states per round trip; a state holding an
// inclusive prefix ends the walk.
__device__ __forceinline__ uint32_t look_back(const uint32_t* states, uint32_t tile, uint32_t d) {
    uint32_t sum = 0;
    for (int64_t t = int64_t(tile) - 1; t >= 0; t -= kLookbackWindow) {
        uint32_t v[kLookbackWindow];
#pragma unroll
        for (int q = 0; q < kLookbackWindow; ++q)
            v[q] = t - q >= 0 ? __hip_atomic_load(states + uint64_t(t - q) * kRadixBuckets + d,
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                              : kStateIncl;              // before the first tile: nothing
#pragma unroll
        for (int q = 0; q < kLookbackWindow; ++q) {
            const uint32_t x = t - q >= 0 ? wait_state(states + uint64_t(t - q) * kRadixBuckets + d, v[q])
                                          : kStateIncl;
            sum += x & kStateMask;
            if ((x & ~kStateMask) == kStateIncl) return sum;
        }
    }
    return sum;
}

__global__ void __launch_bounds__(kScatterThreads)
sort_pass(const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
          uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out, PassInput in,
          int pass, SortArea area, uint32_t tiles) {
    constexpr int W = kScatterThreads / 64;
    __shared__ uint32_t s_key[kSortTile], s_val[kSortTile];   // the tile, ordered by digit
    __shared__ uint32_t run[kRadixBuckets];       // keys of the digit ranked so far
    __shared__ uint32_t lstart[kRadixBuckets];    // first local slot per digit
    __shared__ uint32_t gbase[kRadixBuckets];     // first output slot per digit
    // per round: (round + 1) << 16 | count of the digit in the wavefront,
    // written by the digit's first lane; then the wavefront's first rank
    __shared__ uint32_t wcnt[W][kRadixBuckets];
    __shared__ uint32_t s_tile;
    const int tid = threadIdx.x, wave = tid >> 6;
    const int shift = pass * kRadixBits;
    if (tid == 0) s_tile = atomicAdd(&area.tickets[pass], 1u);
    if (tid < kRadixBuckets) run[tid] = 0u;
    for (int j = tid; j < W * kRadixBuckets; j += kScatterThreads) (&wcnt[0][0])[j] = 0u;
    __syncthreads();
    const uint32_t tile = s_tile;
    if (tile >= tiles) return;                                   // (more blocks than tiles)
    uint32_t* states = area.states + uint64_t(pass) * tiles * kRadixBuckets;
    uint32_t* mine = states + uint64_t(tile) * kRadixBuckets;
    const uint64_t count = in.count();
    const uint64_t base = uint64_t(tile) * kSortTile;
    if (base >= count) {                                         // empty tile, block-uniform
        if (tid < kRadixBuckets)
            __hip_atomic_store(mine + tid, kStateIncl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    // the tile's keys, all loads in flight at once
    uint32_t key[kScatterRounds], val[kScatterRounds], rk[kScatterRounds];
#pragma unroll
    for (int it = 0; it < kScatterRounds; ++it) {
        const uint64_t idx = base + uint64_t(it) * kScatterThreads + tid;
        key[it] = idx < count ? keys_in[idx] : 0u;
        val[it] = idx < count ? vals_in[idx] : 0u;
    }
    // the digits' first output slots: a prefix over the pass's totals
    uint32_t all;
    const uint32_t first = block_exclusive_scan<uint32_t, kScatterThreads>(
        tid < kRadixBuckets ? area.total[pass * kRadixBuckets + tid] : 0u, all);
    if (tid < kRadixBuckets) gbase[tid] = first;
    if (pass == 0 && tile == 0 && tid == 0) *area.kept = all;
    // rank every key among the tile's keys of its digit, in input order
#pragma unroll
    for (int it = 0; it < kScatterRounds; ++it) {
        const uint64_t idx = base + uint64_t(it) * kScatterThreads + tid;
        const uint32_t k = key[it];
        const bool valid = idx < count && in.kept(k);
        const uint32_t d = (k >> shift) & (kRadixBuckets - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = __popcll(peers & lanemask_lt());
        const uint32_t tag = uint32_t(it + 1) << 16;
        if (valid && rank == 0) wcnt[wave][d] = tag | uint32_t(__popcll(peers));
        __syncthreads();
        // per digit: the first rank of every wavefront this round
        if (tid < kRadixBuckets) {
            uint32_t acc = run[tid];
            for (int w = 0; w < W; ++w) {
                const uint32_t v = wcnt[w][tid];
                wcnt[w][tid] = acc;                   // < 4096: never carries a tag
                acc += (v >> 16) == uint32_t(it + 1) ? (v & 0xFFFFu) : 0u;
            }
            run[tid] = acc;
        }
        __syncthreads();
        rk[it] = valid ? wcnt[wave][d] + rank : 0u;
        __syncthreads();                              // wcnt is rewritten next round
    }
    // the tile's count per digit: published at once (the first tile's is
    // already inclusive), and its prefix gives each digit's local slots
    const uint32_t c = tid < kRadixBuckets ? run[tid] : 0u;
    if (tid < kRadixBuckets)
        __hip_atomic_store(mine + tid, (tile == 0 ? kStateIncl : kStateAgg) | c, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    uint32_t total;
    const uint32_t ls = block_exclusive_scan<uint32_t, kScatterThreads>(c, total);
    if (tid < kRadixBuckets) lstart[tid] = ls;
    __syncthreads();
    // the first four wavefronts sum the earlier tiles' counts per digit and
    // publish this tile's inclusive state while the others place their keys
    // by digit in LDS; then the four place theirs
    if (tid < kRadixBuckets) {
        const uint32_t before = tile == 0 ? 0u : look_back(states, tile, uint32_t(tid));
        if (tile > 0)
            __hip_atomic_store(mine + tid, kStateIncl | (before + c), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        gbase[tid] += before;
    }
#pragma unroll
    for (int it = 0; it < kScatterRounds; ++it) {
        const uint64_t idx = base + uint64_t(it) * kScatterThreads + tid;
        const uint32_t k = key[it];
        if (idx < count && in.kept(k)) {
            const uint32_t pos = lstart[(k >> shift) & (kRadixBuckets - 1)] + rk[it];
            s_key[pos] = k;
            s_val[pos] = val[it];
        }
    }
    __syncthreads();
    // out in local order: a digit's keys go to consecutive output slots, so
    // neighbouring threads write neighbouring addresses
    for (uint32_t j = tid; j < total; j += kScatterThreads) {
        const uint32_t k = s_key[j];
        const uint32_t d = (k >> shift) & (kRadixBuckets - 1);
        const uint32_t pos = gbase[d] + (j - lstart[d]);
        keys_out[pos] = k;
        vals_out[pos] = s_val[j];
    }
}

// ---- exclusive scan: reduce tiles, then scan each tile after the sums of the
// tiles before it ------------------------------------------------------------

template <typename In, typename Out>
__device__ __forceinline__ Out load_in(const In* in, const uint32_t* gather, uint64_t i) {
    return Out(gather ? in[gather[i]] : in[i]);
}

// a + b, or, with SAT, min(a + b, max of Out): saturating addition of
// non-negative values is associative, so a scan built from it equals the
// exact prefix sums wherever those fit and the maximum everywhere after.
template <bool SAT, typename T>
__device__ __forceinline__ T add(T a, T b) {
    if constexpr (SAT) {
        const T s = a + b;
        return s < a ? T(~T(0)) : s;
    } else {
        return a + b;
    }
}

template <typename In, typename Out, bool SAT>
__global__ void __launch_bounds__(kScanThreads)
scan_reduce(const In* __restrict__ in0, const In* __restrict__ in1,
            const uint32_t* __restrict__ gather, uint64_t count, Out* __restrict__ partials,
            uint64_t pstride) {
    // grid row y scans array y (in0 or in1), its tile sums at partials + y * pstride
    __shared__ Out wsum[kScanThreads / 64];
    const In* in = blockIdx.y ? in1 : in0;
    partials += blockIdx.y * pstride;
    const uint64_t base = uint64_t(blockIdx.x) * kScanTile;
    Out s = 0;
    for (int it = 0; it < kScanItems; ++it) {
        const uint64_t idx = base + uint64_t(it) * kScanThreads + threadIdx.x;
        if (idx < count) s = add<SAT>(s, load_in<In, Out>(in, gather, idx));
    }
    for (int o = 32; o > 0; o >>= 1) s = add<SAT>(s, Out(__shfl_xor(s, o)));
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        Out t = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) t = add<SAT>(t, wsum[w]);
        partials[blockIdx.x] = t;
    }
}

// Block-wide exclusive scan of one value per thread; returns the block total.
template <typename T, int NT, bool SAT>
__device__ __forceinline__ T block_exclusive_scan(T x, T& total) {
    __shared__ T wsum[NT / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T incl = x;
    for (int o = 1; o < 64; o <<= 1) {
        const T y = __shfl_up(incl, o);
        if (lane >= o) incl = add<SAT>(incl, y);
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    T before = 0;
    total = 0;
    for (int w = 0; w < NT / 64; ++w) {
        if (w < wave) before = add<SAT>(before, wsum[w]);
        total = add<SAT>(total, wsum[w]);
    }
    __syncthreads();
    if constexpr (SAT) {
        // the lane before's inclusive value (a saturated sum cannot be undone
        // by subtracting x)
        T excl = __shfl_up(incl, 1);
        if (lane == 0) excl = 0;
        return add<SAT>(before, excl);
    } else {
        return before + incl - x;
    }
}

template <typename In, typename Out, bool SAT>
__global__ void __launch_bounds__(kScanThreads)
scan_down(const In* in0, const In* in1, const uint32_t* __restrict__ gather, uint64_t count,
          const Out* __restrict__ partials, uint64_t pstride, Out* out0, Out* out1,
          bool write_total) {
    const In* in = blockIdx.y ? in1 : in0;
    Out* out = blockIdx.y ? out1 : out0;
    partials += blockIdx.y * pstride;
    // blocked arrangement: thread t owns items [t*16, t*16 + 16) of the tile
    const uint64_t base = uint64_t(blockIdx.x) * kScanTile + uint64_t(threadIdx.x) * kScanItems;
    Out v[kScanItems];
    Out s = 0;
    for (int it = 0; it < kScanItems; ++it) {
        const uint64_t idx = base + it;
        v[it] = idx < count ? load_in<In, Out>(in, gather, idx) : Out(0);
        s = add<SAT>(s, v[it]);
    }
    // the sums of the tiles before this one (a few hundred at most in use)
    Out before = 0;
    for (uint32_t b = threadIdx.x; b < blockIdx.x; b += kScanThreads)
        before = add<SAT>(before, partials[b]);
    Out carry;
    (void)block_exclusive_scan<Out, kScanThreads, SAT>(before, carry);
    Out total;
    Out run = add<SAT>(carry, block_exclusive_scan<Out, kScanThreads, SAT>(s, total));
    for (int it = 0; it < kScanItems; ++it) {
        const uint64_t idx = base + it;
        if (idx < count) out[idx] = run;
        run = add<SAT>(run, v[it]);
    }
    if (write_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
        out[count] = add<SAT>(carry, total);
}

// One or two arrays of the same length (in1/out1 null: one); the second
// array's tile sums follow the first's in partials.  With SAT the sums
// saturate at the largest Out (see add).
template <typename In, typename Out, bool SAT = false>
hipError_t exclusive_scan(const In* in, const uint32_t* gather, Out* out, uint64_t count,
                          Out* partials, bool write_total, hipStream_t s,
                          const In* in1 = nullptr, Out* out1 = nullptr) {
    const uint64_t nb = (count + kScanTile - 1) / kScanTile;
    if (nb == 0) return hipSuccess;
    const unsigned rows = in1 ? 2u : 1u;
    if (!in1) {
        in1 = in;
        out1 = out;
    }
    scan_reduce<In, Out, SAT><<<dim3(unsigned(nb), rows), dim3(kScanThreads), 0, s>>>(
        in, in1, gather, count, partials, nb);
    scan_down<In, Out, SAT><<<dim3(unsigned(nb), rows), dim3(kScanThreads), 0, s>>>(
        in, in1, gather, count, partials, nb, out, out1, write_total);
    return hipGetLastError();
}

// 16-byte stores over the aligned body, single words for the head and tail.
__global__ void fill_kernel(uint32_t* p, uint32_t value, uint64_t head, uint64_t n4,
                            uint64_t count) {
    const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n4) reinterpret_cast<uint4*>(p + head)[i] = make_uint4(value, value, value, value);
    if (i < head) p[i] = value;
    const uint64_t t = head + 4 * n4 + i;
    if (i < 4 && t < count) p[t] = value;
}

}  // namespace

hipError_t fill_u32(uint32_t* p, uint32_t value, uint64_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    const uint64_t mis = (reinterpret_cast<uintptr_t>(p) / 4) % 4;
    const uint64_t head = std::min<uint64_t>(count, mis == 0 ? 0 : 4 - mis);
    const uint64_t n4 = (count - head) / 4;
    const uint64_t threads = std::max<uint64_t>(n4, 4);
    fill_kernel<<<dim3(unsigned((threads + 255) / 256)), dim3(256), 0, s>>>(p, value, head, n4,
                                                                              count);
    return hipGetLastError();
}

uint64_t scan_partials_elems(uint64_t count) { return (count + kScanTile - 1) / kScanTile + 1; }

uint64_t radix_counts_elems(uint64_t count) {
    const uint64_t tiles = (count + kSortTile - 1) / kSortTile;
    return kAreaHead + uint64_t(kMaxPasses) * tiles * kRadixBuckets;
}

int radix_sort_passes(int bits) { return (bits + kRadixBits - 1) / kRadixBits; }

hipError_t exclusive_scan_u32_pair(const uint32_t* in0, uint32_t* out0, const uint32_t* in1,
                                   uint32_t* out1, uint64_t count, uint64_t* partials,
                                   bool write_total, hipStream_t s) {
    if (count == 0) {
        if (!write_total) return hipSuccess;
        hipError_t e = fill_u32(out0, 0u, 1, s);
        return e != hipSuccess ? e : fill_u32(out1, 0u, 1, s);
    }
    return exclusive_scan<uint32_t, uint32_t, true>(in0, nullptr, out0, count,
                                                    reinterpret_cast<uint32_t*>(partials),
                                                    write_total, s, in1, out1);
}

hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, uint64_t count,
                              uint64_t* partials, bool write_total, hipStream_t s) {
    if (count == 0) return write_total ? fill_u32(out, 0u, 1, s) : hipSuccess;
    return exclusive_scan<uint32_t, uint32_t>(in, nullptr, out, count,
                                              reinterpret_cast<uint32_t*>(partials), write_total, s);
}

hipError_t radix_sort(uint32_t* const keys[2], uint32_t* const vals[2], uint64_t count, int bits,
                      uint32_t* counts, uint64_t* partials, int* result, hipStream_t s,
                      bool drop_on, uint32_t drop) {
    (void)partials;
    int cur = 0;
    const SortArea area = sort_area(counts);
    if (count == 0) {
        *result = 0;
        return fill_u32(area.kept, 0u, 1, s);
    }
    const uint64_t tiles = (count + kSortTile - 1) / kSortTile;
    const int passes = std::min(radix_sort_passes(bits), kMaxPasses);
    const uint64_t state_words = uint64_t(passes) * tiles * kRadixBuckets;
    const unsigned hblocks =
        unsigned(std::min<uint64_t>(kHistBlocks, std::max<uint64_t>(1, (count + 4095) / 4096)));
    hipError_t e = fill_u32(area.total, 0u, kAreaHead, s);     // totals, kept, tickets
    if (e != hipSuccess) return e;
    sort_hist<<<dim3(hblocks), dim3(1024), 0, s>>>(keys[0], count, passes, drop_on, drop, area,
                                                   state_words);
    for (int p = 0; p < passes; ++p) {
        PassInput in{count, nullptr, drop_on && p == 0, drop};
        if (drop_on && p > 0) in.dcount = area.kept;
        sort_pass<<<dim3(unsigned(tiles)), dim3(kScatterThreads), 0, s>>>(
            keys[cur], vals[cur], keys[1 - cur], vals[1 - cur], in, p, area, uint32_t(tiles));
        cur = 1 - cur;
    }
    *result = cur;
    return hipGetLastError();
}

uint64_t radix_kept_offset(uint64_t count) {
    (void)count;
    return uint64_t(kMaxPasses) * kRadixBuckets;
}

}  // namespace tgs
