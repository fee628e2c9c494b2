// Device-wide primitives: exclusive scan and stable LSD radix sort of
// (uint32 key, uint32 value) pairs, written for wave64.
//
// Radix sort, per 8-bit digit pass:
//   1. digit_counts : each block counts the digits of its 4096 keys in LDS
//                     (one private histogram per wavefront, then summed) and
//                     stores them digit-major, counts[digit][block];
//   2. exclusive scan of counts -> first output slot of (digit, block), and
//      the total after the last entry;
//   3. scatter      : the block sorts its tile by digit in LDS, walking its
//                     keys in input order 1024 at a time (equal digits inside
//                     a wavefront ranked with eight ballots, wavefronts
//                     ordered by a prefix over them per digit, so equal keys
//                     keep their input order), then writes each digit's run
//                     to consecutive output slots.
// The first pass may drop every pair whose key equals a given value (it is
// neither counted nor written); the scanned total is then the number of
// pairs kept, and the later passes read it on the device (their grids are
// sized for the input count; tiles past the kept count are empty).
#include "common.hpp"

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

__global__ void __launch_bounds__(kSortThreads)
digit_counts(const uint32_t* __restrict__ keys, PassInput in, int shift,
             uint32_t* __restrict__ counts, uint32_t nblocks) {
    __shared__ uint32_t hist[kSortThreads / 64][kRadixBuckets];
    const uint64_t count = in.count();
    const int tid = threadIdx.x, wave = tid >> 6;
    if (uint64_t(blockIdx.x) * kSortTile >= count) {             // empty tile, block-uniform
        counts[uint64_t(tid) * nblocks + blockIdx.x] = 0u;
        return;
    }
    for (int w = 0; w < kSortThreads / 64; ++w) hist[w][tid] = 0;
    __syncthreads();
    const uint64_t base = uint64_t(blockIdx.x) * kSortTile;
#pragma unroll 4
    for (int it = 0; it < kSortItems; ++it) {
        const uint64_t idx = base + uint64_t(it) * kSortThreads + tid;
        if (idx < count) {
            const uint32_t k = keys[idx];
            if (in.kept(k)) atomicAdd(&hist[wave][(k >> shift) & (kRadixBuckets - 1)], 1u);
        }
    }
    __syncthreads();
    uint32_t s = 0;
    for (int w = 0; w < kSortThreads / 64; ++w) s += hist[w][tid];
    counts[uint64_t(tid) * nblocks + blockIdx.x] = s;
}

// Forward declaration: block-wide exclusive scan (defined with the scans).
template <typename T, int NT, bool SAT = false>
__device__ __forceinline__ T block_exclusive_scan(T x, T& total);

constexpr int kScatterThreads = 1024;
constexpr int kScatterRounds = kSortTile / kScatterThreads;

__global__ void __launch_bounds__(kScatterThreads)
digit_scatter(const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
              uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out, PassInput in,
              int shift, const uint32_t* __restrict__ offsets, uint32_t nblocks) {
    constexpr int W = kScatterThreads / 64;
    __shared__ uint32_t s_key[kSortTile], s_val[kSortTile];   // the tile, ordered by digit
    __shared__ uint32_t run[kRadixBuckets];       // next local slot per digit
    __shared__ uint32_t lstart[kRadixBuckets];    // first local slot per digit
    __shared__ uint32_t gbase[kRadixBuckets];     // first output slot per digit
    // per round: (round + 1) << 16 | count of the digit in the wavefront,
    // written by the digit's first lane; then the wavefront's first local slot
    __shared__ uint32_t wcnt[W][kRadixBuckets];
    const uint64_t count = in.count();
    const uint64_t base = uint64_t(blockIdx.x) * kSortTile;
    if (base >= count) return;                                   // empty tile, block-uniform
    const int tid = threadIdx.x, wave = tid >> 6;
    // the tile's keys, all loads in flight at once
    uint32_t key[kScatterRounds], val[kScatterRounds];
#pragma unroll
    for (int it = 0; it < kScatterRounds; ++it) {
        const uint64_t idx = base + uint64_t(it) * kScatterThreads + tid;
        key[it] = idx < count ? keys_in[idx] : 0u;
        val[it] = idx < count ? vals_in[idx] : 0u;
    }
    // this block's count of digit tid (difference of consecutive scanned
    // counts; the scan ends with the total) -> its first local slot; and its
    // first output slot
    uint32_t off = 0, nxt = 0;
    if (tid < kRadixBuckets) {
        const uint64_t i = uint64_t(tid) * nblocks + blockIdx.x;
        off = offsets[i];
        nxt = offsets[i + 1];
    }
    uint32_t total;
    const uint32_t ls = block_exclusive_scan<uint32_t, kScatterThreads>(nxt - off, total);
    if (tid < kRadixBuckets) {
        lstart[tid] = ls;
        run[tid] = ls;
        gbase[tid] = off;
    }
    for (int j = tid; j < W * kRadixBuckets; j += kScatterThreads) (&wcnt[0][0])[j] = 0u;
    __syncthreads();
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
        // per digit: the first local slot of every wavefront this round
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
        if (valid) {
            const uint32_t pos = wcnt[wave][d] + rank;
            s_key[pos] = k;
            s_val[pos] = val[it];
        }
        __syncthreads();
    }
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
    return uint64_t(kRadixBuckets) * ((count + kSortTile - 1) / kSortTile) + 1;
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
    int cur = 0;
    const uint64_t nb = (count + kSortTile - 1) / kSortTile;
    const int passes = radix_sort_passes(bits);
    // the scanned total (kept pairs) sits after the nb * buckets counts
    const uint32_t* kept = counts + nb * kRadixBuckets;
    if (count == 0) {
        *result = 0;
        return fill_u32(counts, 0u, 1, s);
    }
    for (int p = 0; p < passes; ++p) {
        const int shift = p * kRadixBits;
        PassInput in{count, nullptr, drop_on && p == 0, drop};
        if (drop_on && p > 0) in.dcount = kept;
        digit_counts<<<dim3(unsigned(nb)), dim3(kSortThreads), 0, s>>>(keys[cur], in, shift, counts,
                                                                        uint32_t(nb));
        // digit counts fit in uint32; the scan writes the total after them
        hipError_t e = exclusive_scan<uint32_t, uint32_t>(
            counts, nullptr, counts, nb * kRadixBuckets, reinterpret_cast<uint32_t*>(partials),
            true, s);
        if (e != hipSuccess) return e;
        digit_scatter<<<dim3(unsigned(nb)), dim3(kScatterThreads), 0, s>>>(
            keys[cur], vals[cur], keys[1 - cur], vals[1 - cur], in, shift, counts, uint32_t(nb));
        cur = 1 - cur;
    }
    *result = cur;
    return hipGetLastError();
}

uint64_t radix_kept_offset(uint64_t count) {
    return uint64_t(kRadixBuckets) * ((count + kSortTile - 1) / kSortTile);
}

}  // namespace tgs
