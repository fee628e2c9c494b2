// Densification selection from the accumulated statistics of Sec. 4.3.
//
// A Gaussian is a candidate when its mean positional-gradient norm reaches
// tau_pos, or -- only in densification events where the appearance branch is
// active -- its mean appearance-gradient norm reaches tau_col.  Means are the
// accumulated sums divided by the number of views that saw the Gaussian.
// With a budget K >= 0 (the convergence-aware schedule of Sec. 4.2 gives the
// number of Gaussians that may still be added), only the K candidates with
// the largest score max(pos / tau_pos, col / tau_col) are kept, ties in
// ascending index: a stable radix sort of the complemented float bits of the
// scores (non-candidates carry the largest key and sort last).
#include "common.hpp"
#include "wave.hpp"

namespace tgs {
namespace {

constexpr uint32_t kNotSelected = 0xFFFFFFFFu;

__global__ void __launch_bounds__(256)
densify_score_kernel(int64_t n, const float* __restrict__ pos, const float* __restrict__ col,
                     const int32_t* __restrict__ count, float tau_pos, float tau_col, int color,
                     uint8_t* __restrict__ selected, uint32_t* __restrict__ keys,
                     uint32_t* __restrict__ vals, uint32_t* __restrict__ n_candidates) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    bool cand = false;
    if (i < n) {
        const int32_t c = count[i];
        float score = 0.0f;
        if (c > 0) {
            const float fc = float(c);
            const float ap = pos[i] / fc;
            const float sp = ap / tau_pos;
            cand = ap >= tau_pos;
            score = sp;
            if (color) {
                const float ac = col[i] / fc;
                cand = cand || ac >= tau_col;
                score = fmaxf(score, ac / tau_col);
            }
        }
        selected[i] = cand ? 1 : 0;
        if (keys) {
            keys[i] = cand ? ~__float_as_uint(score) : kNotSelected;
            vals[i] = uint32_t(i);
        }
    }
    const uint64_t b = __ballot(cand);
    if (__lane_id() == 0 && b) atomicAdd(n_candidates, uint32_t(__popcll(b)));
}

// After the sort: keep the first min(K, candidates) entries of the order.
__global__ void __launch_bounds__(256)
densify_budget_kernel(int64_t n, const uint32_t* __restrict__ keys,
                      const uint32_t* __restrict__ vals, uint64_t budget,
                      const uint32_t* __restrict__ n_candidates, uint8_t* __restrict__ selected,
                      uint32_t* __restrict__ n_selected) {
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t keep = min(uint64_t(*n_candidates), budget);
    if (j < n) selected[vals[j]] = (uint64_t(j) < keep && keys[j] != kNotSelected) ? 1 : 0;
    if (j == 0) *n_selected = uint32_t(keep);
}

__global__ void copy_count_kernel(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

}  // namespace

uint64_t densify_workspace_bytes(int64_t n) {
    const uint64_t un = uint64_t(n);
    const uint64_t pairs = 4 * align_up(un * 4, 256);                 // keys and values, twice
    const uint64_t counts = align_up(radix_counts_elems(un) * 4, 256);
    const uint64_t partials = align_up(scan_partials_elems(radix_counts_elems(un)) * 8, 256);
    return 256 + pairs + counts + partials;
}

hipError_t launch_densify(int64_t n, const float* pos, const float* col, const int32_t* count,
                          float tau_pos, float tau_col, int color, int64_t budget,
                          uint8_t* selected, uint32_t* n_selected, uint8_t* ws, hipStream_t s) {
    // workspace: [candidate count | pad] keys[2] vals[2] radix counts, scan partials
    auto* n_cand = reinterpret_cast<uint32_t*>(ws);
    const uint64_t un = uint64_t(n);
    uint8_t* p = ws + 256;
    uint32_t* keys[2];
    uint32_t* vals[2];
    for (int b = 0; b < 2; ++b) {
        keys[b] = reinterpret_cast<uint32_t*>(p);
        p += align_up(un * 4, 256);
        vals[b] = reinterpret_cast<uint32_t*>(p);
        p += align_up(un * 4, 256);
    }
    auto* counts = reinterpret_cast<uint32_t*>(p);
    p += align_up(radix_counts_elems(un) * 4, 256);
    auto* partials = reinterpret_cast<uint64_t*>(p);
    hipError_t e = fill_u32(n_cand, 0u, 1, s);
    if (e != hipSuccess) return e;
    const bool capped = budget >= 0;
    const unsigned blocks = unsigned((un + 255) / 256);
    if (n > 0) {
        densify_score_kernel<<<blocks, 256, 0, s>>>(n, pos, col, count, tau_pos, tau_col, color,
                                                    selected, capped ? keys[0] : nullptr,
                                                    capped ? vals[0] : nullptr, n_cand);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (!capped || n == 0) {
        copy_count_kernel<<<1, 64, 0, s>>>(n_cand, n_selected);
        return hipGetLastError();
    }
    int res = 0;
    if ((e = radix_sort(keys, vals, un, 32, counts, partials, &res, s)) != hipSuccess) return e;
    densify_budget_kernel<<<blocks, 256, 0, s>>>(n, keys[res], vals[res], uint64_t(budget), n_cand,
                                                 selected, n_selected);
    return hipGetLastError();
}

}  // namespace tgs
