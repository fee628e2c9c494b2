// Dilated compositing, forward and backward (stages (c) and (d1)), and the
// L1 loss gradient.
//
// One workgroup per tile of a DOWNSAMPLED image (Sec. 4.1: pairs live in the
// downsampled grid; each downsampled pixel is blended at its full-resolution
// position d i + o, so no thread is spent on an unrendered pixel).  One launch
// covers the tiles of up to kMaxViews views (a view table passed by value):
// workgroups are laid out view after view, so a batch of views of uneven size
// is balanced by the hardware dispatcher like one big image.  16x16 and 8x8
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

// alpha = min(0.99, o exp(p)), p = -1/2 (A dx^2 + C dy^2) - B dx dy; false if
// the entry is skipped (p > 0 or alpha < 1/255).  ga = (u, v, A, B),
// gb = (C, o, r, g).  G and alpha are computed either way (branch-free
// callers select on the result).  Compiled without FP contraction: forward
// and backward evaluate exactly the same operations.
__device__ __forceinline__ bool splat_alpha(const float4 ga, const float4 gb, float X, float Y,
                                            float& dx, float& dy, float& G, float& alpha) {
    dx = ga.x - X;
    dy = ga.y - Y;
    const float power = -0.5f * (ga.z * dx * dx + gb.x * dy * dy) - ga.w * dx * dy;
    G = __builtin_amdgcn_exp2f(power * kLog2e);
    alpha = fminf(kAlphaMax, gb.y * G);
    return power <= 0.0f && alpha >= kAlphaMin;
}

// Launch shape: a T x T tile is covered by (T/P) x (T/P) threads owning P x P
// pixels each; B splat records are staged per LDS round.
template <int T, int B_>
struct Shape {
    static constexpr int P = T == 32 ? 2 : 1, NP = P * P;
    static constexpr int TX = T / P, NT = TX * TX;   // threads
    static constexpr int B = B_;
};

// Which view and tile workgroup b works on.
__device__ __forceinline__ bool locate(const RasterViews& vt, uint32_t b, int& v, int64_t& tile) {
    if (b >= vt.first_block[vt.count]) return false;
    v = 0;
    while (b >= vt.first_block[v + 1]) ++v;
    tile = int64_t(b - vt.first_block[v]);
    return true;
}

// Clamp a tile's range to the pairs that exist: a view whose binning
// overflowed its capacity reports a pair count above it and renders nothing.
__device__ __forceinline__ void tile_range(const RasterView& rv, int64_t tile, uint32_t& start,
                                           uint32_t& end) {
    const uint32_t pc = *rv.pair_count;
    const uint32_t lim = pc <= rv.capacity ? pc : 0u;
    end = min(rv.ranges[2 * tile + 1], lim);
    start = min(rv.ranges[2 * tile], end);
}

// Stage records [base, base + cnt) of the list into LDS (all threads).
template <int NT, int B>
__device__ __forceinline__ void stage(const RasterView& rv, uint32_t base, int cnt, float4* s_a,
                                      float4* s_b, float* s_c, uint32_t* s_id) {
    for (int q = threadIdx.x; q < cnt; q += NT) {
        const uint32_t id = rv.vals[base + q];
        if (s_id) s_id[q] = id;
        s_a[q] = rv.rec[3 * uint64_t(id)];
        s_b[q] = rv.rec[3 * uint64_t(id) + 1];
        s_c[q] = rv.rec[3 * uint64_t(id) + 2].x;
    }
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

template <int T, int BATCH>
__global__ void __launch_bounds__((Shape<T, BATCH>::NT)) raster_fwd_kernel(RasterViews vt) {
    using S = Shape<T, BATCH>;
    __shared__ float4 s_a[BATCH], s_b[BATCH];
    __shared__ float s_c[BATCH];
    int v;
    int64_t tile;
    if (!locate(vt, blockIdx.x, v, tile)) return;                // block-uniform
    const RasterView& rv = vt.v[v];
    const Grid& grid = rv.grid;
    const int tid = threadIdx.x;
    const int tx = int(tile % grid.gx), ty = int(tile / grid.gx);
    const int i0 = tx * T + (tid % S::TX) * S::P, j0 = ty * T + (tid / S::TX) * S::P;
    uint32_t start, end;
    tile_range(rv, tile, start, end);
    float X[S::NP], Y[S::NP], Tr[S::NP], c0[S::NP], c1[S::NP], c2[S::NP];
    uint32_t last[S::NP], neval[S::NP], nblend[S::NP];
    bool done[S::NP];
    bool alive = false;
#pragma unroll
    for (int k = 0; k < S::NP; ++k) {
        const int i = i0 + k % S::P, j = j0 + k / S::P;
        done[k] = !(i < grid.w_ds && j < grid.h_ds);
        alive |= !done[k];
        X[k] = float(grid.stride * i + grid.off_x);
        Y[k] = float(grid.stride * j + grid.off_y);
        Tr[k] = 1.0f;
        c0[k] = c1[k] = c2[k] = 0.0f;
        last[k] = 0;
        nblend[k] = 0;
        neval[k] = end - start;
    }
    for (uint32_t base = start; base < end; base += BATCH) {
        if (__syncthreads_count(alive) == 0) break;
        const int cnt = min(BATCH, int(end - base));
        stage<S::NT, BATCH>(rv, base, cnt, s_a, s_b, s_c, nullptr);
        __syncthreads();
        // branch-free per entry: a skipped entry adds exactly 0 and leaves T
        for (int e = 0; e < cnt; ++e) {
            if (__ballot(alive) == 0) break;           // the whole wavefront has stopped
            const float4 a = s_a[e], b = s_b[e];
            const float bb = s_c[e];
            const uint32_t pos = base - start + uint32_t(e) + 1;
            alive = false;
#pragma unroll
            for (int k = 0; k < S::NP; ++k) {
                float dx, dy, G, alpha;
                const bool hit = splat_alpha(a, b, X[k], Y[k], dx, dy, G, alpha) && !done[k];
                const float Tn = Tr[k] * (1.0f - alpha);
                const bool stop = hit && Tn < kTMin;
                const bool blend = hit && !stop;
                const float w = blend ? alpha * Tr[k] : 0.0f;
                c0[k] += b.z * w;
                c1[k] += b.w * w;
                c2[k] += bb * w;
                Tr[k] = blend ? Tn : Tr[k];
                last[k] = blend ? pos : last[k];
                nblend[k] += blend ? 1u : 0u;
                neval[k] = stop ? pos : neval[k];
                done[k] = done[k] || stop;
                alive = alive || !done[k];
            }
        }
    }
    const uint64_t pix = uint64_t(grid.w_ds) * grid.h_ds;
#pragma unroll
    for (int k = 0; k < S::NP; ++k) {
        const int i = i0 + k % S::P, j = j0 + k / S::P;
        if (!(i < grid.w_ds && j < grid.h_ds)) continue;
        const uint64_t p = uint64_t(j) * grid.w_ds + i;
        rv.image[p] = c0[k] + Tr[k] * rv.bg[0];
        rv.image[pix + p] = c1[k] + Tr[k] * rv.bg[1];
        rv.image[2 * pix + p] = c2[k] + Tr[k] * rv.bg[2];
        if (rv.t_final) rv.t_final[p] = Tr[k];
        if (rv.last_contrib) rv.last_contrib[p] = last[k];
        if (rv.n_eval) rv.n_eval[p] = neval[k];
        if (rv.n_blend) rv.n_blend[p] = nblend[k];
    }
}

template <int T, int BATCH>
__global__ void __launch_bounds__((Shape<T, BATCH>::NT)) raster_bwd_kernel(RasterViews vt) {
    using S = Shape<T, BATCH>;
    __shared__ float4 s_a[BATCH], s_b[BATCH];
    __shared__ float s_c[BATCH];
    __shared__ uint32_t s_id[BATCH];
    int v;
    int64_t tile;
    if (!locate(vt, blockIdx.x, v, tile)) return;                // block-uniform
    const RasterView& rv = vt.v[v];
    const Grid& grid = rv.grid;
    const int tid = threadIdx.x;
    const int tx = int(tile % grid.gx), ty = int(tile / grid.gx);
    const int i0 = tx * T + (tid % S::TX) * S::P, j0 = ty * T + (tid / S::TX) * S::P;
    uint32_t start, end;
    tile_range(rv, tile, start, end);
    const uint64_t pix = uint64_t(grid.w_ds) * grid.h_ds;
    float X[S::NP], Y[S::NP], Tr[S::NP], p0[S::NP], p1[S::NP], p2[S::NP];
    float g0[S::NP], g1[S::NP], g2[S::NP], im0[S::NP], im1[S::NP], im2[S::NP];
    bool done[S::NP];
    bool alive = false;
#pragma unroll
    for (int k = 0; k < S::NP; ++k) {
        const int i = i0 + k % S::P, j = j0 + k / S::P;
        const bool in = i < grid.w_ds && j < grid.h_ds;
        done[k] = !in;
        alive |= in;
        X[k] = float(grid.stride * i + grid.off_x);
        Y[k] = float(grid.stride * j + grid.off_y);
        Tr[k] = 1.0f;
        p0[k] = p1[k] = p2[k] = 0.0f;
        g0[k] = g1[k] = g2[k] = im0[k] = im1[k] = im2[k] = 0.0f;
        if (in) {
            const uint64_t p = uint64_t(j) * grid.w_ds + i;
            g0[k] = rv.dL[p];
            g1[k] = rv.dL[pix + p];
            g2[k] = rv.dL[2 * pix + p];
            im0[k] = rv.image[p];
            im1[k] = rv.image[pix + p];
            im2[k] = rv.image[2 * pix + p];
        }
    }
    for (uint32_t base = start; base < end; base += BATCH) {
        if (__syncthreads_count(alive) == 0) break;
        const int cnt = min(BATCH, int(end - base));
        stage<S::NT, BATCH>(rv, base, cnt, s_a, s_b, s_c, s_id);
        __syncthreads();
        for (int e = 0; e < cnt; ++e) {
            if (__ballot(alive) == 0) break;          // the whole wavefront has stopped
            const float4 a = s_a[e], b = s_b[e];
            const float bb = s_c[e];
            // decisions, exactly as in the forward
            float dx[S::NP], dy[S::NP], G[S::NP], alpha[S::NP];
            bool blend[S::NP];
            bool any = false;
            alive = false;
#pragma unroll
            for (int k = 0; k < S::NP; ++k) {
                const bool hit = splat_alpha(a, b, X[k], Y[k], dx[k], dy[k], G[k], alpha[k]) && !done[k];
                const bool stop = hit && Tr[k] * (1.0f - alpha[k]) < kTMin;
                blend[k] = hit && !stop;
                any = any || blend[k];
                done[k] = done[k] || stop;
                alive = alive || !done[k];
            }
            if (__ballot(any) == 0) continue;          // no pixel of the wavefront blends it
            float gv[kGrad2d];
#pragma unroll
            for (int c = 0; c < kGrad2d; ++c) gv[c] = 0.0f;
#pragma unroll
            for (int k = 0; k < S::NP; ++k) {
                const float T0 = Tr[k];
                const float w = blend[k] ? alpha[k] * T0 : 0.0f;
                p0[k] += b.z * w;
                p1[k] += b.w * w;
                p2[k] += bb * w;
                gv[6] += w * g0[k];
                gv[7] += w * g1[k];
                gv[8] += w * g2[k];
                // d image / d alpha = rgb T - (colour behind) / (1 - alpha)
                const float inv = __builtin_amdgcn_rcpf(1.0f - alpha[k]);
                const float dal = g0[k] * (b.z * T0 - (im0[k] - p0[k]) * inv) +
                                  g1[k] * (b.w * T0 - (im1[k] - p1[k]) * inv) +
                                  g2[k] * (bb * T0 - (im2[k] - p2[k]) * inv);
                // no gradient through the 0.99 clamp
                const bool live = blend[k] && !(b.y * G[k] > kAlphaMax);
                const float dp = live ? alpha[k] * dal : 0.0f;
                gv[5] += live ? G[k] * dal : 0.0f;
                gv[0] -= dp * (a.z * dx[k] + a.w * dy[k]);
                gv[1] -= dp * (b.x * dy[k] + a.w * dx[k]);
                gv[2] -= 0.5f * dp * dx[k] * dx[k];
                gv[3] -= dp * dx[k] * dy[k];
                gv[4] -= 0.5f * dp * dy[k] * dy[k];
                Tr[k] = blend[k] ? T0 * (1.0f - alpha[k]) : T0;
            }
            int comp;
            const float s = wave_sum9(gv, comp);
            if (comp >= 0 && s != 0.0f) atomicAdd(&rv.g2d[uint64_t(s_id[e]) * kGrad2d + comp], s);
        }
    }
}

__global__ void __launch_bounds__(256)
l1_grad_kernel(Grid grid, const float* __restrict__ image, const float* __restrict__ target,
               float* __restrict__ dL, double* __restrict__ loss) {
    __shared__ double wsum[4];
    const uint64_t pix = uint64_t(grid.w_ds) * grid.h_ds;
    const uint64_t p = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (p < pix) {
        const int i = int(p % uint64_t(grid.w_ds)), j = int(p / uint64_t(grid.w_ds));
        const uint64_t X = uint64_t(grid.stride) * i + grid.off_x;
        const uint64_t Y = uint64_t(grid.stride) * j + grid.off_y;
        const uint64_t full = uint64_t(grid.width) * grid.height;
        const float inv = 1.0f / float(3 * pix);
        for (int c = 0; c < 3; ++c) {
            const float diff = image[c * pix + p] - target[c * full + Y * grid.width + X];
            const float sg = diff > 0.0f ? 1.0f : (diff < 0.0f ? -1.0f : 0.0f);
            dL[c * pix + p] = sg * inv;
            s += fabs(double(diff));
        }
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0 && loss) {
        atomicAdd(loss, (wsum[0] + wsum[1] + wsum[2] + wsum[3]) / double(3 * pix));
    }
}

template <int T, int B>
void launch_both(bool fwd, const RasterViews& vt, hipStream_t s) {
    const dim3 grid(vt.first_block[vt.count]), block(Shape<T, B>::NT);
    if (fwd) raster_fwd_kernel<T, B><<<grid, block, 0, s>>>(vt);
    else raster_bwd_kernel<T, B><<<grid, block, 0, s>>>(vt);
}

template <int T>
void launch_tile(bool fwd, int batch, const RasterViews& vt, hipStream_t s) {
    if (batch == 64) launch_both<T, 64>(fwd, vt, s);
    else if (batch == 128) launch_both<T, 128>(fwd, vt, s);
    else launch_both<T, 256>(fwd, vt, s);
}

hipError_t launch_raster(bool fwd, int tile, int batch, const RasterViews& vt, hipStream_t s) {
    if (vt.count == 0 || vt.first_block[vt.count] == 0) return hipSuccess;
    if (tile == 8) launch_tile<8>(fwd, batch, vt, s);
    else if (tile == 32) launch_tile<32>(fwd, batch, vt, s);
    else launch_tile<16>(fwd, batch, vt, s);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_raster_fwd(int tile, int batch, const RasterViews& vt, hipStream_t s) {
    return launch_raster(true, tile, batch, vt, s);
}

hipError_t launch_raster_bwd(int tile, int batch, const RasterViews& vt, hipStream_t s) {
    return launch_raster(false, tile, batch, vt, s);
}

hipError_t launch_l1_grad(const Grid& grid, const float* image, const float* target,
                          float* dL_dimage, double* loss, hipStream_t s) {
    const uint64_t pix = uint64_t(grid.w_ds) * grid.h_ds;
    if (loss) {
        hipError_t e = fill_u32(reinterpret_cast<uint32_t*>(loss), 0u, 2, s);
        if (e != hipSuccess) return e;
    }
    if (pix == 0) return hipSuccess;
    l1_grad_kernel<<<dim3(unsigned((pix + 255) / 256)), dim3(256), 0, s>>>(grid, image, target,
                                                                           dL_dimage, loss);
    return hipGetLastError();
}

}  // namespace tgs
