// Dilated compositing, forward and backward (stages (c) and (d1)), and the
// L1 loss gradient.
//
// One workgroup per tile of a DOWNSAMPLED image (Sec. 4.1: pairs live in the
// downsampled grid; each downsampled pixel is blended at its full-resolution
// position d i + o, so no thread is spent on an unrendered pixel).  One launch
// covers the tiles of up to kMaxViews views (a view table passed by value):
// workgroups are laid out view after view, so a batch of views of uneven size
// is balanced by the hardware dispatcher like one big image, and within a
// view they take the tiles heaviest first (the schedule below).  16x16 and 8x8
// tiles give one pixel per thread, 32x32 tiles a 2x2 block per thread.  The
// tile's list is staged through LDS B splat records at a time; every pixel
// walks it front to back (Sec. 3 Eq. 2).
//
// The backward replays the forward walk in the same order with the same
// arithmetic (one shared inline routine), so it takes bit-identical skip and
// stop decisions and needs no per-pixel state from the forward: the colour
// still to come behind entry k is image - (colour accumulated up to k).
#include "common.hpp"
#include "wave.hpp"

namespace tgs {
namespace {

constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

// Splat constants as staged in LDS.  The conic is pre-scaled so that the
// exponent comes out in base 2 with no extra multiply:
//   qa = -A log2(e) / 2,  qb = -B log2(e),  qc = -C log2(e) / 2,
//   log2(e) * power = dx (qa dx + qb dy) + qc dy dy,   dx = u - X, dy = v - Y.
// ga = (u, v, qa, qb), gb = (qc, o, r, g).
__device__ __forceinline__ void stage_conic(const float4 r0, const float4 r1, float4& ga,
                                            float4& gb) {
    constexpr float kHalf = -0.5f * kLog2e, kFull = -kLog2e;
    ga = make_float4(r0.x, r0.y, r0.z * kHalf, r0.w * kFull);
    gb = make_float4(r1.x * kHalf, r1.y, r1.z, r1.w);
}

// alpha = min(0.99, o 2^(log2e power)); false if the entry is skipped
// (power > 0 or alpha < 1/255; o G >= 1/255 is the same test since
// 0.99 > 1/255).  G, alpha and the partial t = qb dy are
// computed either way (branch-free callers select on the result).  Forward
// and backward evaluate exactly these operations (explicit FMAs, no
// contraction elsewhere), so they take bit-identical decisions.
// The two halves: the exponent, then the test on it.
__device__ __forceinline__ float splat_exponent(const float4 ga, const float4 gb, float X,
                                                float Y, float& dx, float& dy, float& t) {
    dx = ga.x - X;
    dy = ga.y - Y;
    t = ga.w * dy;
    return fmaf(dx, fmaf(ga.z, dx, t), (gb.x * dy) * dy);
}

__device__ __forceinline__ bool splat_test(const float4 gb, float p2, float& G, float& raw,
                                           float& alpha) {
    G = __builtin_amdgcn_exp2f(p2);
    raw = gb.y * G;
    alpha = __builtin_amdgcn_fmed3f(raw, 0.0f, kAlphaMax);   // min(0.99, raw) for raw >= 0
    return p2 <= 0.0f && raw >= kAlphaMin;
}

// Exponent below which o 2^p2 < 1/255 for certain: log2(1/255 / o) less a
// margin (1/64 in log2, i.e. 1.1 % of alpha) far above the rounding of the
// exponential, the product and this logarithm.  An entry whose exponent is
// below it at every live pixel of a wavefront is skipped by the whole
// wavefront: it would be skipped by each pixel anyway (o <= 0 gives NaN or
// +inf here, and no exponent passes).
constexpr float kSkipMargin = 1.0f / 64.0f;
__device__ __forceinline__ float skip_threshold(float o) {
    return log2f(kAlphaMin / o) - kSkipMargin;
}

// Launch shape (the work split): a T x T tile is covered by (T/PX) x (T/PY)
// threads owning PX x PY pixels each (PPT = PX PY = 1, 2 or 4); each LDS
// read of a splat then serves PPT pixels.
// Each wavefront covers an 8 x 8 block of threads, so its pixels form a
// compact square whose walks end at similar depths (a wavefront iterates
// until its last pixel saturates).
template <int T, int PPT>
struct Shape {
    static constexpr int PX = PPT >= 2 ? 2 : 1, PY = PPT == 4 ? 2 : 1, NP = PX * PY;
    static constexpr int TX = T / PX, TY = T / PY, NT = TX * TY;   // threads
    static_assert(TX % 8 == 0 && TY % 8 == 0, "threads must tile into 8 x 8 wavefronts");
    // thread -> (column, row) of its first pixel within the tile
    __device__ static int px(int tid) { return ((tid >> 6) % (TX / 8) * 8 + (tid & 7)) * PX; }
    __device__ static int py(int tid) { return ((tid >> 6) / (TX / 8) * 8 + ((tid >> 3) & 7)) * PY; }
};

// The pixel rectangles of a tile's wavefronts, in full-resolution coordinates
// of their pixel centres (pixels past the image edge included): wavefront w
// covers x in [x0 + w_x step, x0 + w_x step + span], w_x = w mod (TX / 8),
// and likewise in y.
template <class S>
struct WaveRects {
    static constexpr int NW = S::NT / 64, WX = S::TX / 8;
    float x0, y0, stepx, stepy, spanx, spany;
    __device__ void init(const Grid& g, int tx, int ty, int T) {
        auto u = [](float x) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))); };
        x0 = u(float(g.stride * tx * T + g.off_x));
        y0 = u(float(g.stride * ty * T + g.off_y));
        stepx = float(g.stride * 8 * S::PX);
        stepy = float(g.stride * 8 * S::PY);
        spanx = float(g.stride * (8 * S::PX - 1));
        spany = float(g.stride * (8 * S::PY - 1));
    }
};

// Bit w set when the splat's exponent may reach thr somewhere on wavefront
// w's rectangle: the maximum of the (negative definite) quadratic form over
// the rectangle -- 0 if it holds the centre, else the largest of the four
// edge maxima -- plus a margin (1/32 in log2 and a relative bound on the
// rounding of the form's terms) against thr.  A clear bit is a promise that
// no pixel of the wavefront passes the per-pixel test, so the wavefront
// skips the entry without evaluating it; a form that is not negative
// definite sets every bit.
template <class S>
__device__ __forceinline__ uint32_t wave_mask(const float4 ga, float qc, float thr,
                                              const WaveRects<S>& wr) {
    constexpr int NW = WaveRects<S>::NW;
    constexpr uint32_t kAll = NW >= 32 ? 0xFFFFFFFFu : (1u << NW) - 1u;
    const float u = ga.x, v = ga.y, qa = ga.z, qb = ga.w;
    if (!(qa < 0.0f && qc < 0.0f && 4.0f * qa * qc > qb * qb)) return kAll;
    const float ka = -qb / (2.0f * qa);      // maximising dx on a line dy = e: ka e
    const float kc = -qb / (2.0f * qc);      // maximising dy on a line dx = d: kc d
    auto f = [&](float d, float e) { return fmaf(d, fmaf(qa, d, qb * e), (qc * e) * e); };
    uint32_t mask = 0;
#pragma unroll 1
    for (int w = 0; w < NW; ++w) {
        const float xa = wr.x0 + float(w % WaveRects<S>::WX) * wr.stepx;
        const float ya = wr.y0 + float(w / WaveRects<S>::WX) * wr.stepy;
        const float d0 = u - (xa + wr.spanx), d1 = u - xa;       // d0 <= d1
        const float e0 = v - (ya + wr.spany), e1 = v - ya;
        float m;
        if (d0 <= 0.0f && d1 >= 0.0f && e0 <= 0.0f && e1 >= 0.0f) {
            m = 0.0f;
        } else {
            m = f(d0, fminf(fmaxf(kc * d0, e0), e1));
            m = fmaxf(m, f(d1, fminf(fmaxf(kc * d1, e0), e1)));
            m = fmaxf(m, f(fminf(fmaxf(ka * e0, d0), d1), e0));
            m = fmaxf(m, f(fminf(fmaxf(ka * e1, d0), d1), e1));
            const float dm = fmaxf(-d0, d1), em = fmaxf(-e0, e1);
            const float mag = fmaf(-qa * dm, dm, fmaf(fabsf(qb) * dm, em, (-qc * em) * em));
            m += 1.0f / 32.0f + 4e-6f * mag;
        }
        if (m >= thr) mask |= 1u << w;
    }
    return mask;
}

// Which view workgroup b works on, and its index within the view: the
// views' workgroups are laid out one view after the other (the index is the
// tile itself unless the view carries a tile order).
__device__ __forceinline__ bool locate(const RasterViews& vt, uint32_t b, int& v, int64_t& tile) {
    if (b >= vt.first_block[vt.count]) return false;
    v = 0;
    while (b >= vt.first_block[v + 1]) ++v;
    tile = int64_t(b - vt.first_block[v]);
    return true;
}

// Clamp a tile's range to the pairs that exist: a view whose binning
// overflowed its capacity reports a pair count above it and renders nothing.
// The bounds are made wave-uniform (scalar registers).
__device__ __forceinline__ void tile_range(const RasterView& rv, int64_t tile, uint32_t& start,
                                           uint32_t& end) {
    const uint32_t pc = *rv.pair_count;
    const uint32_t lim = pc <= rv.capacity ? pc : 0u;
    const uint32_t e = min(rv.ranges[2 * tile + 1], lim);
    const uint32_t s = min(rv.ranges[2 * tile], e);
    start = uint32_t(__builtin_amdgcn_readfirstlane(int(s)));
    end = uint32_t(__builtin_amdgcn_readfirstlane(int(e)));
}

// a + b after exchanging the upper 32 lanes of a with the lower 32 of b:
// lanes 0-31 get a[i] + a[i+32], lanes 32-63 get b[i-32] + b[i].
__device__ __forceinline__ float swap32_add(float a, float b) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                    false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// The same between rows of 16 lanes: rows 0 and 2 get a[row] + a[row + 1],
// rows 1 and 3 get b[row - 1] + b[row].
__device__ __forceinline__ float swap16_add(float a, float b) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                    false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Sums of 9 per-lane values over the wavefront.  Eight of them go through a
// transposing butterfly -- each exchange halves the values a lane keeps: the
// upper half-wave keeps values 4-7, the odd rows keep the upper two of the
// remaining four, the upper 8 lanes of a row the second one -- and end with
// a sum over the 8 lanes of each octet (row mirror, half mirror, quad swaps),
// so lane 8c (c = 0..7) holds the total of value c.  Value 8 is summed over
// all lanes the same way and lane 1 keeps it.  Returns the value this lane
// owns and its index (or -1).
__device__ __forceinline__ float wave_sum9(const float* v, int& comp) {
    const int lane = __lane_id();
    const bool h16 = lane & 16, h8 = lane & 8;
    float w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = swap32_add(v[k], v[k + 4]);
    const float x0 = swap16_add(w[0], w[2]);
    const float x1 = swap16_add(w[1], w[3]);
    const float send = h8 ? x0 : x1;
    float y = (h8 ? x1 : x0) + dpp_f<kDppRowMirror>(send);
    y += dpp_f<kDppRowHalfMirror>(y);
    y += dpp_f<kDppQuadXor2>(y);
    y += dpp_f<kDppQuadXor1>(y);
    float z = swap32_add(v[8], v[8]);
    z = swap16_add(z, z);
    z += dpp_f<kDppRowMirror>(z);
    z += dpp_f<kDppRowHalfMirror>(z);
    z += dpp_f<kDppQuadXor2>(z);
    z += dpp_f<kDppQuadXor1>(z);
    comp = -1;
    if ((lane & 7) == 0) comp = ((lane & 32) ? 4 : 0) + (h16 ? 2 : 0) + (h8 ? 1 : 0);
    if (lane == 1) {
        comp = 8;
        y = z;
    }
    return y;
}

// Calls entry(e), in order, for the entries e < cnt of an LDS batch whose
// wavefront mask has this wavefront's bit, while live() holds on some lane:
// each 64 entries' bits become one ballot, and the wavefront visits the set
// bits only, so an entry its rectangle cannot reach costs nothing.  Entries
// after every pixel has stopped change nothing, so leaving early keeps the
// result.
template <class L, class F>
__device__ __forceinline__ void for_wave_entries(const uint32_t* s_m, int cnt, int wave, L&& live,
                                                 F&& entry) {
    for (int c = 0; c < cnt; c += 64) {
        const int q = c + __lane_id();
        uint64_t m = __ballot(q < cnt && ((s_m[q] >> wave) & 1u));
        while (m != 0 && __ballot(live()) != 0) {
            const int e = c + int(__builtin_ctzll(m));
            m &= m - 1;
            entry(e);
        }
    }
}

// Every pixel's final transmittance and the 1-based index of its last
// blended entry go to the workspace for the backward.  COUNTS adds the
// per-pixel counters n_eval, n_blend and n_tested.
//
// A pixel's state is its transmittance with a sign: positive while it
// still takes entries, negated (the magnitude kept) once it has stopped or
// when it lies outside the image.  Live transmittance never drops below
// the floor kTMin > 0, so the sign is never ambiguous, and no per-pixel
// flag has to be carried from entry to entry.
template <int T, int PPT, int BATCH, bool COUNTS>
__global__ void __launch_bounds__((Shape<T, PPT>::NT)) raster_fwd_kernel(RasterViews vt) {
    using S = Shape<T, PPT>;
    __shared__ float4 s_a[BATCH], s_b[BATCH];
    // blue, at the stride of s_a and s_b so one address serves all three
    __shared__ float4 s_c[BATCH];
    __shared__ uint32_t s_m[BATCH];                              // wavefronts that look at it
    int v;
    int64_t tile;
    if (!locate(vt, blockIdx.x, v, tile)) return;                // block-uniform
    const RasterView& rv = vt.v[v];
    const Grid& grid = rv.grid;
    if (rv.order)                                                // heaviest tiles first
        tile = __builtin_amdgcn_readfirstlane(
            int(min(rv.order[tile], uint32_t(grid.num_tiles() - 1))));
    const int tid = threadIdx.x;
    const int tx = int(tile % grid.gx), ty = int(tile / grid.gx);
    const int i0 = tx * T + S::px(tid), j0 = ty * T + S::py(tid);
    uint32_t start, end;
    tile_range(rv, tile, start, end);
    WaveRects<S> wr;
    wr.init(grid, tx, ty, T);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    float X[S::NP], Y[S::NP], Ts[S::NP], c0[S::NP], c1[S::NP], c2[S::NP];
    uint32_t last[S::NP], neval[S::NP], nblend[S::NP], ntest[S::NP];
#pragma unroll
    for (int k = 0; k < S::NP; ++k) {
        const int i = i0 + k % S::PX, j = j0 + k / S::PX;
        X[k] = float(grid.stride * i + grid.off_x);
        Y[k] = float(grid.stride * j + grid.off_y);
        Ts[k] = i < grid.w_ds && j < grid.h_ds ? 1.0f : -1.0f;
        c0[k] = c1[k] = c2[k] = 0.0f;
        last[k] = 0;
        nblend[k] = 0;
        ntest[k] = 0;
        neval[k] = end - start;
    }
    auto live = [&]() {
        bool l = false;
#pragma unroll
        for (int k = 0; k < S::NP; ++k) l = l || Ts[k] > 0.0f;
        return l;
    };
    uint32_t base = start;
    for (; base < end; base += BATCH) {
        if (__syncthreads_count(live()) == 0) break;
        const int cnt = min(BATCH, int(end - base));
        for (int q = tid; q < cnt; q += S::NT) {
            const uint32_t id = rv.vals[base + q];
            const float4* r = rv.rec + 3 * uint64_t(id);
            const float4 r1 = r[1];
            float4 ga, gb;
            stage_conic(r[0], r1, ga, gb);
            const float thr = skip_threshold(r1.y);
            s_a[q] = ga;
            s_b[q] = gb;
            s_c[q] = make_float4(r[2].x, 0.0f, 0.0f, 0.0f);
            s_m[q] = wave_mask<S>(ga, gb.x, thr, wr);
        }
        __syncthreads();
        // branch-free per entry: a skipped entry adds exactly 0 and leaves T
        // (entries no pixel of the wavefront can reach are not visited)
        auto entry = [&](int e) {
            bool any = false;
            if constexpr (COUNTS) {
#pragma unroll
                for (int k = 0; k < S::NP; ++k) ntest[k] += Ts[k] > 0.0f ? 1u : 0u;
            }
            const float4 a = s_a[e], b = s_b[e];
            const float bb = s_c[e].x;
            float dx[S::NP], dy[S::NP], t[S::NP], p2[S::NP];
#pragma unroll
            for (int k = 0; k < S::NP; ++k) p2[k] = splat_exponent(a, b, X[k], Y[k], dx[k], dy[k], t[k]);
#pragma unroll
            for (int k = 0; k < S::NP; ++k) {
                float G, raw, alpha;
                const bool hit = splat_test(b, p2[k], G, raw, alpha) && Ts[k] > 0.0f;
                const float w0 = alpha * Ts[k];
                // T after this entry below the floor: the pixel stops here;
                // otherwise it blends (one comparison: stop implies hit)
                const bool stop = hit && Ts[k] - w0 < kTMin;
                const bool blend = hit != stop;
                const float w = blend ? w0 : 0.0f;
                c0[k] = fmaf(b.z, w, c0[k]);
                c1[k] = fmaf(b.w, w, c1[k]);
                c2[k] = fmaf(bb, w, c2[k]);
                const float tn = Ts[k] - w;           // Ts itself when not blending
                Ts[k] = stop ? -tn : tn;
                const uint32_t pos = base - start + uint32_t(e) + 1;
                last[k] = blend ? pos : last[k];
                any = any || blend;
                if constexpr (COUNTS) {
                    nblend[k] += blend ? 1u : 0u;
                    neval[k] = stop ? pos : neval[k];
                }
            }
            return __ballot(any) != 0;
        };
        // the same walk as for_wave_entries, also collecting per 64 entries
        // the bits of those some pixel of this wavefront blended: they are
        // all the backward has to visit
        for (int c = 0; c < cnt; c += 64) {
            const int q = c + __lane_id();
            uint64_t m = __ballot(q < cnt && ((s_m[q] >> wave) & 1u));
            uint64_t bm = 0;
            while (m != 0 && __ballot(live()) != 0) {
                const int j = int(__builtin_ctzll(m));
                m &= m - 1;
                if (entry(c + j)) bm |= uint64_t(1) << j;
            }
            if (__lane_id() == 0)                    // entry base + c is chunk (base - start + c) / 64
                rv.bits[uint64_t(wave) * rv.bits_stride + (start >> 6) + uint64_t(tile) +
                        (base - start + uint32_t(c)) / 64u] = bm;
        }
    }
    // the tile's weight for the backward's schedule; the work split the
    // blend bits were written with (one workgroup of the view records it)
    if (rv.work && tid == 0) rv.work[tile] = min(base, end) - start;
    if (tid == 0 && blockIdx.x == vt.first_block[v]) *rv.fwd_split = uint32_t(PPT);
    const uint64_t pix = uint64_t(grid.w_ds) * grid.h_ds;
#pragma unroll
    for (int k = 0; k < S::NP; ++k) {
        const int i = i0 + k % S::PX, j = j0 + k / S::PX;
        if (!(i < grid.w_ds && j < grid.h_ds)) continue;
        const uint64_t p = uint64_t(j) * grid.w_ds + i;
        const float Tr = fabsf(Ts[k]);
        if (rv.image) {
            rv.image[p] = fmaf(Tr, rv.bg[0], c0[k]);
            rv.image[pix + p] = fmaf(Tr, rv.bg[1], c1[k]);
            rv.image[2 * pix + p] = fmaf(Tr, rv.bg[2], c2[k]);
        }
        // what the backward starts from
        rv.ws_tfinal[p] = Tr;
        rv.ws_last[p] = last[k];
        if (rv.t_final) rv.t_final[p] = Tr;
        if (rv.last_contrib) rv.last_contrib[p] = last[k];
        if constexpr (COUNTS) {
            if (rv.n_eval) rv.n_eval[p] = neval[k];
            if (rv.n_blend) rv.n_blend[p] = nblend[k];
            if (rv.n_tested) rv.n_tested[p] = ntest[k];
        }
    }
}

// Calls entry(e), from the last to the first, for the entries e < cnt of an
// LDS batch that some pixel of this wavefront blended in the forward: the
// blend bits, one word per 64 entries from word `chunk` on (the batch
// starts at a multiple of 64 entries of the tile's list).  Without usable
// bits (a forward with another work split has another wavefront
// partition) every entry is visited; each pixel still decides its own.
template <class F>
__device__ __forceinline__ void for_blended_entries_reverse(const unsigned long long* bits,
                                                            bool use_bits, uint64_t chunk, int cnt,
                                                            F&& entry) {
    for (int c = ((cnt - 1) >> 6) << 6; c >= 0; c -= 64) {
        uint64_t m = use_bits ? uint64_t(bits[chunk + uint64_t(c >> 6)]) : ~uint64_t(0);
        if (cnt - c < 64) m &= (uint64_t(1) << (cnt - c)) - 1;
        while (m != 0) {
            const int hb = 63 - __builtin_clzll(m);
            m ^= uint64_t(1) << hb;
            entry(c + hb);
        }
    }
}

// The blend backward: each pixel walks its list back to front, from the
// last entry it blended (ws_last) down to the first, starting from its
// final transmittance (ws_tfinal); both were left by the forward, and so
// were the blend bits, by which a wavefront visits only the entries some
// of its pixels blended.  With
// T_k the transmittance in front of entry k and B_k the colour behind it
// seen through it (the blended colours of the later entries and the
// background, composited from the back):
//   T_k = T_{k+1} / (1 - alpha_k),
//   dC/dalpha_k = T_k (c_k - B_k),   B_{k-1} = alpha_k c_k + (1 - alpha_k) B_k,
// B starting at the background.  Only the gradient-weighted S_k = sum_c
// dL/dC_c B_k,c is needed, updated by the same convex combination, so every
// quantity keeps its relative precision however small T gets (the colour
// behind is never formed as a difference of the whole pixel colour and a
// prefix).  The skip decisions (alpha < 1/255, exponent > 0) are the
// forward's inline routine; an entry is blended iff it passes them and lies
// before the pixel's last blended entry.
//
// Per blended entry the lane's contribution to the nine sums, as moments
// that the wave reduces first; the splat's constants and the constant
// factors of each component (ln 2 for u and v, -1/2, -1, -1/2 for A, B, C)
// are applied once per wave to the reduced sums:
//   dL/du = ln2 (qa2 Sx + qb Sy),  dL/dv = ln2 (qc2 Sy + qb Sx),
//   Sx = sum dp dx,  Sy = sum dp dy,
//   dL/dA = -1/2 sum dp dx^2,  dL/dB = -sum dp dx dy,  dL/dC = -1/2 sum dp dy^2,
// with dp = dL/dpower, qa2 = 2 qa, qc2 = 2 qc.
template <int T, int PPT, int BATCH>
__global__ void __launch_bounds__((Shape<T, PPT>::NT)) raster_bwd_kernel(RasterViews vt) {
    using S = Shape<T, PPT>;
    __shared__ float4 s_a[BATCH], s_b[BATCH], s_c[BATCH];
    __shared__ uint32_t s_id[BATCH];
    __shared__ uint32_t s_end;                                   // entries the tile walks
    // multi-wavefront tiles add their wavefronts' sums in LDS and flush each
    // batch with one set of global atomics per entry
    constexpr bool kBlockSum = S::NT > 64;
    __shared__ float s_g[kBlockSum ? BATCH * kGrad2d : 1];
    int v;
    int64_t tile;
    if (!locate(vt, blockIdx.x, v, tile)) return;                // block-uniform
    const RasterView& rv = vt.v[v];
    const Grid& grid = rv.grid;
    if (rv.order)                                                // heaviest tiles first
        tile = __builtin_amdgcn_readfirstlane(
            int(min(rv.order[tile], uint32_t(grid.num_tiles() - 1))));
    const int tid = threadIdx.x;
    const int tx = int(tile % grid.gx), ty = int(tile / grid.gx);
    const int i0 = tx * T + S::px(tid), j0 = ty * T + S::py(tid);
    uint32_t start, end;
    tile_range(rv, tile, start, end);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const unsigned long long* wbits = rv.bits + uint64_t(wave) * rv.bits_stride;
    // the bits describe this launch's wavefronts only if the forward used the
    // same work split
    const bool use_bits = __builtin_amdgcn_readfirstlane(int(*rv.fwd_split)) == PPT;
    const uint64_t pix = uint64_t(grid.w_ds) * grid.h_ds;
    // per pixel: the transmittance behind the current entry (T_final at the
    // start), the gradient-weighted colour behind it (the background at the
    // start), dL/dC and the 1-based index of the last blended entry
    float X[S::NP], Y[S::NP], Ts[S::NP], Sb[S::NP];
    float g0[S::NP], g1[S::NP], g2[S::NP];
    uint32_t last[S::NP];
    uint32_t lmax = 0;
#pragma unroll
    for (int k = 0; k < S::NP; ++k) {
        const int i = i0 + k % S::PX, j = j0 + k / S::PX;
        const bool in = i < grid.w_ds && j < grid.h_ds;
        X[k] = float(grid.stride * i + grid.off_x);
        Y[k] = float(grid.stride * j + grid.off_y);
        Ts[k] = 1.0f;
        g0[k] = g1[k] = g2[k] = 0.0f;
        last[k] = 0;
        if (in) {
            const uint64_t p = uint64_t(j) * grid.w_ds + i;
            g0[k] = rv.dL[p];
            g1[k] = rv.dL[pix + p];
            g2[k] = rv.dL[2 * pix + p];
            Ts[k] = rv.ws_tfinal[p];
            last[k] = min(rv.ws_last[p], end - start);
        }
        Sb[k] = fmaf(g2[k], rv.bg[2], fmaf(g1[k], rv.bg[1], g0[k] * rv.bg[0]));
        lmax = max(lmax, last[k]);
    }
    // entries [0, wend) hold every blend of this wavefront's pixels, [0, s_end)
    // those of the tile
    for (int o = 32; o > 0; o >>= 1) lmax = max(lmax, uint32_t(__shfl_xor(int(lmax), o)));
    const uint32_t wend = uint32_t(__builtin_amdgcn_readfirstlane(int(lmax)));
    if (S::NT > 64) {
        if (tid == 0) s_end = 0;
        __syncthreads();
        if (__lane_id() == 0) atomicMax(&s_end, wend);
        __syncthreads();
    }
    const uint32_t tend = S::NT > 64 ? uint32_t(__builtin_amdgcn_readfirstlane(int(s_end))) : wend;
    // factor of the component this lane owns after wave_sum9
    const int lane = __lane_id();
    const int own = (lane & 7) == 0 ? (lane >> 3) : (lane == 1 ? 8 : -1);
    const float scale = own == 0 || own == 1 ? kLn2
                        : own == 2 || own == 4 ? -0.5f
                        : own == 3 ? -1.0f : 1.0f;
    // batches of the list from the back, starting at multiples of BATCH
    const int top = int(tend) == 0 ? -1 : (int(tend) - 1) / BATCH * BATCH;
    for (int lo = top; lo >= 0; lo -= BATCH) {
        const int cnt = min(BATCH, int(tend) - lo);
        if (lo != top) __syncthreads();                          // the previous batch is done
        for (int q = tid; q < cnt; q += S::NT) {
            const uint32_t id = rv.vals[start + uint32_t(lo + q)];
            const float4* r = rv.rec + 3 * uint64_t(id);
            float4 ga, gb;
            stage_conic(r[0], r[1], ga, gb);
            s_a[q] = ga;
            s_b[q] = gb;
            s_c[q] = make_float4(r[2].x, ga.z + ga.z, gb.x + gb.x, 0.0f);
            s_id[q] = id;
        }
        if constexpr (kBlockSum)
            for (int q = tid; q < cnt * kGrad2d; q += S::NT) s_g[q] = 0.0f;
        __syncthreads();
        auto entry = [&](int e) {
            const float4 a = s_a[e], b = s_b[e];
            const float4 c = s_c[e];                  // (b, qa2, qc2, unused)
            const uint32_t pos = uint32_t(lo + e);    // 0-based position in the list
            // the forward's skip decisions; blended iff also before the last blend
            float dx[S::NP], dy[S::NP], t[S::NP], p2[S::NP], G[S::NP], raw[S::NP], alpha[S::NP];
            bool blend[S::NP];
#pragma unroll
            for (int k = 0; k < S::NP; ++k) p2[k] = splat_exponent(a, b, X[k], Y[k], dx[k], dy[k], t[k]);
            bool lane_any = false;                    // a pixel of this lane blends it
#pragma unroll
            for (int k = 0; k < S::NP; ++k) {
                blend[k] = splat_test(b, p2[k], G[k], raw[k], alpha[k]) && pos < last[k];
                lane_any = lane_any || blend[k];
            }
            if (__ballot(lane_any) == 0) return;      // no pixel of the wavefront blends it
            float gv[kGrad2d];
            // ab = alpha where the pixel blends the entry, 0 elsewhere: then
            // w, the S update, dp and the G term vanish by themselves (T is
            // kept by a select, so it never picks up the rounding of a
            // reciprocal of 1).  The lane's pixels are summed with FMAs.
#pragma unroll
            for (int k = 0; k < S::NP; ++k) {
                const float ab = blend[k] ? alpha[k] : 0.0f;
                const float inv = __builtin_amdgcn_rcpf(1.0f - ab);
                const float T0 = blend[k] ? Ts[k] * inv : Ts[k];    // in front of the entry
                const float w = ab * T0;
                // dL/dalpha = T0 (sum_c dL/dC_c rgb_c - S)
                const float gcol = fmaf(g2[k], c.x, fmaf(g1[k], b.w, g0[k] * b.z));
                const float diff = gcol - Sb[k];
                const float dal = T0 * diff;
                Sb[k] = fmaf(ab, diff, Sb[k]);
                // no gradient through the 0.99 clamp
                const bool live = blend[k] && !(raw[k] > kAlphaMax);
                const float dp = (live ? alpha[k] : 0.0f) * dal;
                const float Gl = live ? G[k] : 0.0f;
                const float pdx = dp * dx[k], pdy = dp * dy[k];
                if (k == 0) {
                    gv[0] = pdx;
                    gv[1] = pdy;
                    gv[2] = pdx * dx[k];
                    gv[3] = pdx * dy[k];
                    gv[4] = pdy * dy[k];
                    gv[5] = Gl * dal;
                    gv[6] = w * g0[k];
                    gv[7] = w * g1[k];
                    gv[8] = w * g2[k];
                } else {
                    gv[0] += pdx;
                    gv[1] += pdy;
                    gv[2] = fmaf(pdx, dx[k], gv[2]);
                    gv[3] = fmaf(pdx, dy[k], gv[3]);
                    gv[4] = fmaf(pdy, dy[k], gv[4]);
                    gv[5] = fmaf(Gl, dal, gv[5]);
                    gv[6] = fmaf(w, g0[k], gv[6]);
                    gv[7] = fmaf(w, g1[k], gv[7]);
                    gv[8] = fmaf(w, g2[k], gv[8]);
                }
                Ts[k] = T0;
            }
            int comp;
            float sum = wave_sum9(gv, comp);
            // lanes 0 and 8 hold Sx and Sy: exchange them (rotation by 8
            // within a row of 16 lanes) to form the u and v components
            const float other = dpp_f<kDppRowRor8>(sum);
            if (comp == 0) sum = fmaf(c.y, sum, a.w * other);
            if (comp == 1) sum = fmaf(c.z, sum, a.w * other);
            if (comp >= 0 && sum != 0.0f) {
                if constexpr (kBlockSum) atomicAdd(&s_g[e * kGrad2d + comp], sum * scale);
                else atomicAdd(&rv.g2d[uint64_t(s_id[e]) * kGrad2d + comp], sum * scale);
            }
        };
        // entries at or past this wavefront's last blend change nothing
        const int wcnt = min(cnt, max(0, int(wend) - lo));
        for_blended_entries_reverse(wbits, use_bits, (start >> 6) + uint64_t(tile) + uint64_t(lo / 64),
                                    wcnt, entry);
        if constexpr (kBlockSum) {
            __syncthreads();
            for (int q = tid; q < cnt * kGrad2d; q += S::NT) {
                const float g = s_g[q];
                if (g != 0.0f)
                    atomicAdd(&rv.g2d[uint64_t(s_id[q / kGrad2d]) * kGrad2d + q % kGrad2d], g);
            }
        }
    }
}

// L1 photometric loss of the rendered pixels against the full-resolution
// pixels they are rendered at (Sec. 4.1, Fig. 2: supervision from the
// corresponding high-resolution pixels; Sec. 4.2 names the L1 loss) and its
// gradient, for a table of views in one launch.  A view's blocks walk rows of its strided image
// (the rows of a pixel phase), so the image and dL accesses are contiguous;
// one double atomic per block adds the block's share of the view's loss (a
// bounded number of atomics on one address).
constexpr uint32_t kL1MaxBlocks = 2048;

__global__ void __launch_bounds__(256) l1_grad_kernel(L1Views vt) {
    __shared__ double wsum[4];
    int v = 0;
    while (v + 1 < vt.count && blockIdx.x >= vt.first_block[v + 1]) ++v;   // block-uniform
    const L1View& lv = vt.v[v];
    const Grid& grid = lv.grid;
    const uint32_t lb = blockIdx.x - vt.first_block[v];
    const uint32_t nb = vt.first_block[v + 1] - vt.first_block[v];
    const uint32_t w = uint32_t(grid.w_ds), h = uint32_t(grid.h_ds);
    const uint64_t pix = uint64_t(w) * h;
    const uint64_t full = uint64_t(grid.width) * grid.height;
    const float inv = 1.0f / float(3 * pix);
    double s = 0.0;
    for (uint32_t j = lb; j < h; j += nb) {
        const uint64_t Y = uint64_t(grid.stride) * j + grid.off_y;
        const float* trow = lv.target + Y * grid.width + grid.off_x;
        // four pixels per thread and pass, every load issued before the
        // first use
        constexpr int kU = 4;
        for (uint32_t i0 = threadIdx.x; i0 < w; i0 += kU * blockDim.x) {
            float im[kU][3], tg[kU][3];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const uint32_t i = i0 + uint32_t(u) * blockDim.x;
                const uint64_t p = uint64_t(j) * w + i;
                const uint64_t X = uint64_t(grid.stride) * i;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    im[u][c] = i < w ? lv.image[c * pix + p] : 0.0f;
                    tg[u][c] = i < w ? trow[c * full + X] : 0.0f;
                }
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const uint32_t i = i0 + uint32_t(u) * blockDim.x;
                if (i >= w) continue;
                const uint64_t p = uint64_t(j) * w + i;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float diff = im[u][c] - tg[u][c];
                    const float sg = diff > 0.0f ? 1.0f : (diff < 0.0f ? -1.0f : 0.0f);
                    lv.dL[c * pix + p] = sg * inv;
                    s += fabs(double(diff));
                }
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0 && lv.loss) {
        atomicAdd(lv.loss, (wsum[0] + wsum[1] + wsum[2] + wsum[3]) / double(3 * pix));
    }
}

// The views' losses to zero before the atomics (a fill kernel, so the step
// stays capturable without memset nodes).
__global__ void l1_zero_kernel(L1Views vt) {
    const int v = int(threadIdx.x);
    if (v < vt.count && vt.v[v].loss) *vt.v[v].loss = 0.0;
}

bool wants_counts(const RasterViews& vt) {
    for (int k = 0; k < vt.count; ++k)
        if (vt.v[k].n_eval || vt.v[k].n_blend || vt.v[k].n_tested)
            return true;
    return false;
}

// The rasterizers' schedule.  A view's tiles carry very different work
// (the entries walked before every pixel stops: up to 3x the mean at the
// 4K scene), and in row-major order the heavy tiles of the image centre
// end up unevenly on the SIMDs: the last ones finish 40-50 % after the
// mean.  The dispatcher starts workgroups in index order as slots free up,
// so the tiles of each view are handed out heaviest first by the entries a
// forward walked in them (longest-processing-time-first list scheduling):
// the backward by those of its own forward, the forward by those the
// previous forward on the same workspace left (the same view at another
// phase, or the same camera at its previous visit).  A counting sort over
// 256 weight buckets (exact below 32, then eight per power of two), one
// block per view.  Any weights give a permutation of the tiles: they
// decide the order only, never what is rendered.
constexpr int kOrderBuckets = 256;

__device__ __forceinline__ uint32_t weight_bucket(uint32_t w) {
    if (w < 32u) return w;
    const uint32_t e = 31u - uint32_t(__builtin_clz(w));         // 5 .. 31
    return 32u + (e - 5u) * 8u + ((w >> (e - 3u)) & 7u);         // < 248
}

__global__ void __launch_bounds__(1024) tile_order_kernel(RasterViews vt) {
    __shared__ uint32_t s_cur[kOrderBuckets];
    const RasterView& rv = vt.v[blockIdx.x];
    if (!rv.order || !rv.work) return;                           // block-uniform
    const uint32_t nt = uint32_t(rv.grid.num_tiles());
    const uint32_t tid = threadIdx.x;
    for (uint32_t k = tid; k < kOrderBuckets; k += blockDim.x) s_cur[k] = 0;
    __syncthreads();
    for (uint32_t t = tid; t < nt; t += blockDim.x) atomicAdd(&s_cur[weight_bucket(rv.work[t])], 1u);
    __syncthreads();
    // first slot of every bucket, heaviest bucket first: lane l holds
    // buckets 255 - 4l .. 252 - 4l
    if (tid < 64) {
        uint32_t c[4], sum = 0, total;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            c[q] = s_cur[kOrderBuckets - 1 - 4 * int(tid) - q];
            sum += c[q];
        }
        uint32_t run = wave_exclusive_sum(sum, total);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            s_cur[kOrderBuckets - 1 - 4 * int(tid) - q] = run;
            run += c[q];
        }
    }
    __syncthreads();
    for (uint32_t t = tid; t < nt; t += blockDim.x) {
        const uint32_t pos = atomicAdd(&s_cur[weight_bucket(rv.work[t])], 1u);
        if (pos < nt) rv.order[pos] = t;                         // (weights changed under us)
    }
}

template <int T, int PPT, int B>
void launch_both(bool fwd, const RasterViews& vt, hipStream_t s) {
    const dim3 grid(vt.first_block[vt.count]), block(Shape<T, PPT>::NT);
    if (!fwd) {
        tile_order_kernel<<<dim3(unsigned(vt.count)), dim3(1024), 0, s>>>(vt);
        raster_bwd_kernel<T, PPT, B><<<grid, block, 0, s>>>(vt);
    } else if (wants_counts(vt)) {
        tile_order_kernel<<<dim3(unsigned(vt.count)), dim3(1024), 0, s>>>(vt);
        raster_fwd_kernel<T, PPT, B, true><<<grid, block, 0, s>>>(vt);
    } else {
        tile_order_kernel<<<dim3(unsigned(vt.count)), dim3(1024), 0, s>>>(vt);
        raster_fwd_kernel<T, PPT, B, false><<<grid, block, 0, s>>>(vt);
    }
}

template <int T, int PPT>
void launch_batch(bool fwd, int batch, const RasterViews& vt, hipStream_t s) {
    if (batch == 64) launch_both<T, PPT, 64>(fwd, vt, s);
    else if (batch == 128) launch_both<T, PPT, 128>(fwd, vt, s);
    else launch_both<T, PPT, 256>(fwd, vt, s);
}

// Work splits compiled per tile size: T = 8 one pixel per thread (a single
// wavefront); T = 16 one, two or four; T = 32 two or four.
hipError_t launch_raster(bool fwd, int tile, int ppt, int batch, const RasterViews& vt,
                         hipStream_t s) {
    if (vt.count == 0 || vt.first_block[vt.count] == 0) return hipSuccess;
    if (tile == 8) {
        launch_batch<8, 1>(fwd, batch, vt, s);
    } else if (tile == 32) {
        if (ppt == 2) launch_batch<32, 2>(fwd, batch, vt, s);
        else launch_batch<32, 4>(fwd, batch, vt, s);
    } else {
        if (ppt == 2) launch_batch<16, 2>(fwd, batch, vt, s);
        else if (ppt == 4) launch_batch<16, 4>(fwd, batch, vt, s);
        else launch_batch<16, 1>(fwd, batch, vt, s);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_raster_fwd(int tile, int ppt, int batch, const RasterViews& vt, hipStream_t s) {
    return launch_raster(true, tile, ppt, batch, vt, s);
}

hipError_t launch_raster_bwd(int tile, int ppt, int batch, const RasterViews& vt, hipStream_t s) {
    return launch_raster(false, tile, ppt, batch, vt, s);
}

hipError_t launch_l1_grad(L1Views& vt, hipStream_t s) {
    uint32_t blocks = 0;
    for (int k = 0; k < vt.count; ++k) {
        vt.first_block[k] = blocks;
        const Grid& g = vt.v[k].grid;
        const uint64_t pix = uint64_t(g.w_ds) * g.h_ds;
        blocks += pix == 0 ? 0u : uint32_t(std::min<uint64_t>(uint64_t(g.h_ds), kL1MaxBlocks));
    }
    vt.first_block[vt.count] = blocks;
    if (vt.count == 0) return hipSuccess;
    l1_zero_kernel<<<1, 64, 0, s>>>(vt);
    if (blocks > 0) l1_grad_kernel<<<dim3(blocks), dim3(256), 0, s>>>(vt);
    return hipGetLastError();
}

}  // namespace tgs
