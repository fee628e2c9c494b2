// Dilated compositing, forward and backward (stages (c) and (d1)), and the
// L1 loss gradient.
//
// One workgroup per tile of the DOWNSAMPLED image (Sec. 4.1: pairs live in
// the downsampled grid; each downsampled pixel is blended at its
// full-resolution position d i + o, so no thread is spent on an unrendered
// pixel).  Threads own 1, 2 or 4 pixels of the tile (launch knob): with more
// pixels per thread the splat records staged in LDS, and the per-splat
// gradient reduction of the backward, are shared by several pixels.  Every
// pixel walks its tile's list front to back (Sec. 3 Eq. 2).
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
constexpr int kXcds = 8;

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

// Tile of workgroup b.  order 0: tile = b.  order 1: the tile grid is cut
// into 2x2 quads; quad q goes to XCD q mod 8 (workgroup b runs on XCD b mod 8)
// and the 4 tiles of a quad are consecutive workgroups of that XCD, so they
// run together and share splat records in its L2, while neighbouring quads
// spread the expensive parts of the image over all XCDs.
__device__ __forceinline__ int64_t tile_of_block(uint32_t b, const Grid& g, int order) {
    if (order == 0) return b;
    const int qx_n = (g.gx + 1) / 2;
    const uint32_t xcd = b % kXcds, local = b / kXcds;
    const int64_t q = int64_t(local / 4) * kXcds + xcd;
    const int r = int(local % 4);
    const int qy = int(q / qx_n), qx = int(q % qx_n);
    const int tx = 2 * qx + (r & 1), ty = 2 * qy + (r >> 1);
    if (tx >= g.gx || ty >= g.gy) return g.num_tiles();          // no tile: exit
    return int64_t(ty) * g.gx + tx;
}

__host__ inline uint32_t blocks_for_tiles(const Grid& g, int order) {
    if (order == 0) return uint32_t(g.num_tiles());
    const int64_t quads = int64_t((g.gx + 1) / 2) * ((g.gy + 1) / 2);
    return uint32_t(((quads + kXcds - 1) / kXcds) * kXcds * 4);
}

// Launch shape: a T x T tile is covered by (T/PX) x (T/PY) threads owning
// PX x PY pixels each.
template <int T, int PX_, int PY_>
struct Shape {
    static constexpr int PX = PX_, PY = PY_, NP = PX * PY;
    static constexpr int TX = T / PX, TY = T / PY, NT = TX * TY;   // threads
    static constexpr int BATCH = NT < 256 ? NT : 256;
};

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

template <int T, int PX, int PY>
__global__ void __launch_bounds__((Shape<T, PX, PY>::NT))
raster_fwd_kernel(Grid grid, int order, float bg0, float bg1, float bg2,
                  const float4* __restrict__ rec, const uint32_t* __restrict__ ranges,
                  const uint32_t* __restrict__ vals, uint32_t pair_count,
                  float* __restrict__ image, float* __restrict__ t_final,
                  uint32_t* __restrict__ last_contrib, uint32_t* __restrict__ n_eval,
                  uint32_t* __restrict__ n_blend) {
    using S = Shape<T, PX, PY>;
    __shared__ float4 s_a[S::BATCH], s_b[S::BATCH];
    __shared__ float s_c[S::BATCH];
    const int64_t tile = tile_of_block(blockIdx.x, grid, order);
    if (tile >= grid.num_tiles()) return;                      // block-uniform
    const int tid = threadIdx.x;
    const int tx = int(tile % grid.gx), ty = int(tile / grid.gx);
    const int i0 = tx * T + (tid % S::TX) * S::PX, j0 = ty * T + (tid / S::TX) * S::PY;
    // ranges come from the sort of this state; clamping them to the pair
    // count keeps every list read inside the pair buffer
    const uint32_t end = min(ranges[2 * tile + 1], pair_count);
    const uint32_t start = min(ranges[2 * tile], end);
    float X[S::NP], Y[S::NP], Tr[S::NP], c0[S::NP], c1[S::NP], c2[S::NP];
    uint32_t last[S::NP], neval[S::NP], nblend[S::NP];
    bool done[S::NP];
    bool alive = false;
#pragma unroll
    for (int k = 0; k < S::NP; ++k) {
        const int i = i0 + k % S::PX, j = j0 + k / S::PX;
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
    for (uint32_t base = start; base < end; base += S::BATCH) {
        if (__syncthreads_count(alive) == 0) break;
        if (tid < S::BATCH && base + tid < end) {
            const uint64_t id = vals[base + tid];
            s_a[tid] = rec[3 * id];
            s_b[tid] = rec[3 * id + 1];
            s_c[tid] = rec[3 * id + 2].x;
        }
        __syncthreads();
        const int cnt = min(S::BATCH, int(end - base));
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
        const int i = i0 + k % S::PX, j = j0 + k / S::PX;
        if (!(i < grid.w_ds && j < grid.h_ds)) continue;
        const uint64_t p = uint64_t(j) * grid.w_ds + i;
        image[p] = c0[k] + Tr[k] * bg0;
        image[pix + p] = c1[k] + Tr[k] * bg1;
        image[2 * pix + p] = c2[k] + Tr[k] * bg2;
        if (t_final) t_final[p] = Tr[k];
        if (last_contrib) last_contrib[p] = last[k];
        if (n_eval) n_eval[p] = neval[k];
        if (n_blend) n_blend[p] = nblend[k];
    }
}

template <int T, int PX, int PY>
__global__ void __launch_bounds__((Shape<T, PX, PY>::NT))
raster_bwd_kernel(Grid grid, int order, const float4* __restrict__ rec,
                  const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ vals,
                  uint32_t pair_count, const float* __restrict__ image,
                  const float* __restrict__ dL_dimage, float* __restrict__ grad2d) {
    using S = Shape<T, PX, PY>;
    __shared__ float4 s_a[S::BATCH], s_b[S::BATCH];
    __shared__ float s_c[S::BATCH];
    __shared__ uint32_t s_id[S::BATCH];
    const int64_t tile = tile_of_block(blockIdx.x, grid, order);
    if (tile >= grid.num_tiles()) return;                      // block-uniform
    const int tid = threadIdx.x;
    const int tx = int(tile % grid.gx), ty = int(tile / grid.gx);
    const int i0 = tx * T + (tid % S::TX) * S::PX, j0 = ty * T + (tid / S::TX) * S::PY;
    const uint32_t end = min(ranges[2 * tile + 1], pair_count);
    const uint32_t start = min(ranges[2 * tile], end);
    const uint64_t pix = uint64_t(grid.w_ds) * grid.h_ds;
    float X[S::NP], Y[S::NP], Tr[S::NP], p0[S::NP], p1[S::NP], p2[S::NP];
    float g0[S::NP], g1[S::NP], g2[S::NP], im0[S::NP], im1[S::NP], im2[S::NP];
    bool done[S::NP];
    bool alive = false;
#pragma unroll
    for (int k = 0; k < S::NP; ++k) {
        const int i = i0 + k % S::PX, j = j0 + k / S::PX;
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
            g0[k] = dL_dimage[p];
            g1[k] = dL_dimage[pix + p];
            g2[k] = dL_dimage[2 * pix + p];
            im0[k] = image[p];
            im1[k] = image[pix + p];
            im2[k] = image[2 * pix + p];
        }
    }
    for (uint32_t base = start; base < end; base += S::BATCH) {
        if (__syncthreads_count(alive) == 0) break;
        if (tid < S::BATCH && base + tid < end) {
            const uint32_t id = vals[base + tid];
            s_id[tid] = id;
            s_a[tid] = rec[3 * uint64_t(id)];
            s_b[tid] = rec[3 * uint64_t(id) + 1];
            s_c[tid] = rec[3 * uint64_t(id) + 2].x;
        }
        __syncthreads();
        const int cnt = min(S::BATCH, int(end - base));
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
            if (comp >= 0 && s != 0.0f) atomicAdd(&grad2d[uint64_t(s_id[e]) * kGrad2d + comp], s);
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

template <int T, int PX, int PY>
void fwd_launch(const Grid& grid, int order, const float bg[3], const float4* rec,
                const uint32_t* ranges, const uint32_t* vals, uint32_t pc, float* image,
                float* t_final, uint32_t* last, uint32_t* neval, uint32_t* nblend, hipStream_t s) {
    raster_fwd_kernel<T, PX, PY><<<dim3(blocks_for_tiles(grid, order)),
                                   dim3(Shape<T, PX, PY>::NT), 0, s>>>(
        grid, order, bg[0], bg[1], bg[2], rec, ranges, vals, pc, image, t_final, last, neval,
        nblend);
}

template <int T, int PX, int PY>
void bwd_launch(const Grid& grid, int order, const float4* rec, const uint32_t* ranges,
                const uint32_t* vals, uint32_t pc, const float* image, const float* dL,
                float* g2d, hipStream_t s) {
    raster_bwd_kernel<T, PX, PY><<<dim3(blocks_for_tiles(grid, order)),
                                   dim3(Shape<T, PX, PY>::NT), 0, s>>>(
        grid, order, rec, ranges, vals, pc, image, dL, g2d);
}

}  // namespace

hipError_t launch_raster_fwd(const Grid& grid, const RasterTuning& tune, const float bg[3],
                             const uint8_t* ws, const Layout& L, const uint32_t* pair_vals,
                             uint32_t pair_count, float* image, float* t_final,
                             uint32_t* last_contrib, uint32_t* n_eval, uint32_t* n_blend,
                             hipStream_t s) {
    const auto* rec = reinterpret_cast<const float4*>(ws + L.records);
    const auto* ranges = reinterpret_cast<const uint32_t*>(ws + L.ranges);
    if (grid.num_tiles() == 0) return hipSuccess;
    const int o = tune.order;
#define TGS_FWD(T, PX, PY) fwd_launch<T, PX, PY>(grid, o, bg, rec, ranges, pair_vals, pair_count, \
                                                image, t_final, last_contrib, n_eval, n_blend, s)
    if (grid.tile == 8) TGS_FWD(8, 1, 1);
    else if (grid.tile == 32) { if (tune.ppt == 2) TGS_FWD(32, 2, 1); else TGS_FWD(32, 2, 2); }
    else if (tune.ppt == 1) TGS_FWD(16, 1, 1);
    else if (tune.ppt == 2) TGS_FWD(16, 2, 1);
    else TGS_FWD(16, 2, 2);
#undef TGS_FWD
    return hipGetLastError();
}

hipError_t launch_raster_bwd(const Grid& grid, const RasterTuning& tune, const uint8_t* ws,
                             const Layout& L, const uint32_t* pair_vals, uint32_t pair_count,
                             const float* image, const float* dL_dimage, float* grad2d,
                             hipStream_t s) {
    const auto* rec = reinterpret_cast<const float4*>(ws + L.records);
    const auto* ranges = reinterpret_cast<const uint32_t*>(ws + L.ranges);
    if (grid.num_tiles() == 0) return hipSuccess;
    const int o = tune.order;
#define TGS_BWD(T, PX, PY) bwd_launch<T, PX, PY>(grid, o, rec, ranges, pair_vals, pair_count, \
                                                image, dL_dimage, grad2d, s)
    if (grid.tile == 8) TGS_BWD(8, 1, 1);
    else if (grid.tile == 32) { if (tune.ppt == 2) TGS_BWD(32, 2, 1); else TGS_BWD(32, 2, 2); }
    else if (tune.ppt == 1) TGS_BWD(16, 1, 1);
    else if (tune.ppt == 2) TGS_BWD(16, 2, 1);
    else TGS_BWD(16, 2, 2);
#undef TGS_BWD
    return hipGetLastError();
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
