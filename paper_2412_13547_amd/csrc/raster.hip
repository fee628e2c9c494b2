// Dilated compositing, forward and backward (stages (c) and (d1)), and the
// L1 loss gradient.
//
// One workgroup per tile of the DOWNSAMPLED image, one thread per rendered
// pixel (Sec. 4.1: pairs live in the downsampled grid, blending happens at
// the full-resolution position d i + o of each downsampled pixel, so no
// thread is masked off for an unrendered pixel).  The tile's list is staged
// through LDS in batches of up to 256 splat records; every thread then walks
// the batch front to back (Sec. 3 Eq. 2).
//
// The backward replays the forward walk in the same order with the same
// arithmetic (one shared inline routine), so it takes bit-identical skip and
// stop decisions and needs no per-pixel state from the forward: the colour
// still to come behind entry k is image - (colour accumulated up to k).
#include "common.hpp"

namespace tgs {
namespace {

constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;
constexpr float kLog2e = 1.4426950408889634f;

// alpha = min(0.99, o exp(p)), p = -1/2 (A dx^2 + C dy^2) - B dx dy; false if
// the entry is skipped (p > 0 or alpha < 1/255).  ga = (u, v, A, B),
// gb = (C, o, r, g).  Compiled without FP contraction: forward and backward
// evaluate exactly the same operations.
__device__ __forceinline__ bool splat_alpha(const float4 ga, const float4 gb, float X, float Y,
                                            float& dx, float& dy, float& G, float& alpha) {
    dx = ga.x - X;
    dy = ga.y - Y;
    const float power = -0.5f * (ga.z * dx * dx + gb.x * dy * dy) - ga.w * dx * dy;
    if (power > 0.0f) return false;
    G = __builtin_amdgcn_exp2f(power * kLog2e);
    alpha = fminf(kAlphaMax, gb.y * G);
    return alpha >= kAlphaMin;
}

__device__ __forceinline__ float wave_sum(float x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

template <int T>
__global__ void __launch_bounds__(T * T)
raster_fwd_kernel(Grid grid, float bg0, float bg1, float bg2, const float4* __restrict__ rec,
                  const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ vals,
                  uint32_t pair_count, float* __restrict__ image, float* __restrict__ t_final,
                  uint32_t* __restrict__ last_contrib, uint32_t* __restrict__ n_eval) {
    constexpr int NT = T * T;
    constexpr int BATCH = NT < 256 ? NT : 256;
    __shared__ float4 s_a[BATCH], s_b[BATCH];
    __shared__ float s_c[BATCH];
    const int tid = threadIdx.x;
    const uint32_t tile = blockIdx.x;
    const int tx = int(tile % uint32_t(grid.gx)), ty = int(tile / uint32_t(grid.gx));
    const int i = tx * T + (tid % T), j = ty * T + (tid / T);
    const bool inside = i < grid.w_ds && j < grid.h_ds;
    const float X = float(grid.stride * i + grid.off_x);
    const float Y = float(grid.stride * j + grid.off_y);
    // ranges come from the sort of this state; clamping them to the pair
    // count keeps every list read inside the pair buffer
    const uint32_t end = min(ranges[2 * tile + 1], pair_count);
    const uint32_t start = min(ranges[2 * tile], end);
    bool done = !inside;
    float Tr = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    uint32_t last = 0, neval = end - start;
    for (uint32_t base = start; base < end; base += BATCH) {
        if (__syncthreads_count(!done) == 0) break;
        if (tid < BATCH && base + tid < end) {
            const uint64_t id = vals[base + tid];
            s_a[tid] = rec[3 * id];
            s_b[tid] = rec[3 * id + 1];
            s_c[tid] = rec[3 * id + 2].x;
        }
        __syncthreads();
        const int cnt = min(BATCH, int(end - base));
        for (int e = 0; e < cnt && !done; ++e) {
            const float4 a = s_a[e], b = s_b[e];
            float dx, dy, G, alpha;
            if (!splat_alpha(a, b, X, Y, dx, dy, G, alpha)) continue;
            const float Tn = Tr * (1.0f - alpha);
            if (Tn < kTMin) {
                done = true;
                neval = base - start + uint32_t(e) + 1;
                break;
            }
            const float w = alpha * Tr;
            c0 += b.z * w;
            c1 += b.w * w;
            c2 += s_c[e] * w;
            Tr = Tn;
            last = base - start + uint32_t(e) + 1;
        }
    }
    if (inside) {
        const uint64_t pix = uint64_t(grid.w_ds) * grid.h_ds;
        const uint64_t p = uint64_t(j) * grid.w_ds + i;
        image[p] = c0 + Tr * bg0;
        image[pix + p] = c1 + Tr * bg1;
        image[2 * pix + p] = c2 + Tr * bg2;
        if (t_final) t_final[p] = Tr;
        if (last_contrib) last_contrib[p] = last;
        if (n_eval) n_eval[p] = neval;
    }
}

template <int T>
__global__ void __launch_bounds__(T * T)
raster_bwd_kernel(Grid grid, const float4* __restrict__ rec, const uint32_t* __restrict__ ranges,
                  const uint32_t* __restrict__ vals, uint32_t pair_count,
                  const float* __restrict__ image, const float* __restrict__ dL_dimage,
                  float* __restrict__ grad2d) {
    constexpr int NT = T * T;
    constexpr int BATCH = NT < 256 ? NT : 256;
    __shared__ float4 s_a[BATCH], s_b[BATCH];
    __shared__ float s_c[BATCH];
    __shared__ uint32_t s_id[BATCH];
    __shared__ float s_g[BATCH * kGrad2d];
    const int tid = threadIdx.x;
    const uint32_t tile = blockIdx.x;
    const int tx = int(tile % uint32_t(grid.gx)), ty = int(tile / uint32_t(grid.gx));
    const int i = tx * T + (tid % T), j = ty * T + (tid / T);
    const bool inside = i < grid.w_ds && j < grid.h_ds;
    const float X = float(grid.stride * i + grid.off_x);
    const float Y = float(grid.stride * j + grid.off_y);
    // ranges come from the sort of this state; clamping them to the pair
    // count keeps every list read inside the pair buffer
    const uint32_t end = min(ranges[2 * tile + 1], pair_count);
    const uint32_t start = min(ranges[2 * tile], end);
    float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f, im0 = 0.0f, im1 = 0.0f, im2 = 0.0f;
    if (inside) {
        const uint64_t pix = uint64_t(grid.w_ds) * grid.h_ds;
        const uint64_t p = uint64_t(j) * grid.w_ds + i;
        g0 = dL_dimage[p];
        g1 = dL_dimage[pix + p];
        g2 = dL_dimage[2 * pix + p];
        im0 = image[p];
        im1 = image[pix + p];
        im2 = image[2 * pix + p];
    }
    for (int k = tid; k < BATCH * kGrad2d; k += NT) s_g[k] = 0.0f;
    bool done = !inside;
    float Tr = 1.0f, p0 = 0.0f, p1 = 0.0f, p2 = 0.0f;
    const int lane = tid & 63;
    for (uint32_t base = start; base < end; base += BATCH) {
        if (__syncthreads_count(!done) == 0) break;
        if (tid < BATCH && base + tid < end) {
            const uint32_t id = vals[base + tid];
            s_id[tid] = id;
            s_a[tid] = rec[3 * uint64_t(id)];
            s_b[tid] = rec[3 * uint64_t(id) + 1];
            s_c[tid] = rec[3 * uint64_t(id) + 2].x;
        }
        __syncthreads();
        const int cnt = min(BATCH, int(end - base));
        for (int e = 0; e < cnt; ++e) {
            if (__ballot(!done) == 0) break;      // the whole wavefront has stopped
            float gv[kGrad2d];
            for (int c = 0; c < kGrad2d; ++c) gv[c] = 0.0f;
            bool contrib = false;
            if (!done) {
                const float4 a = s_a[e], b = s_b[e];
                float dx, dy, G, alpha;
                if (splat_alpha(a, b, X, Y, dx, dy, G, alpha)) {
                    const float Tn = Tr * (1.0f - alpha);
                    if (Tn < kTMin) {
                        done = true;
                    } else {
                        contrib = true;
                        const float bb = s_c[e];
                        const float w = alpha * Tr;
                        p0 += b.z * w;
                        p1 += b.w * w;
                        p2 += bb * w;
                        gv[6] = w * g0;
                        gv[7] = w * g1;
                        gv[8] = w * g2;
                        const float inv = 1.0f / (1.0f - alpha);
                        const float dal = g0 * (b.z * Tr - (im0 - p0) * inv) +
                                          g1 * (b.w * Tr - (im1 - p1) * inv) +
                                          g2 * (bb * Tr - (im2 - p2) * inv);
                        // no gradient through the 0.99 clamp
                        const bool clamped = b.y * G > kAlphaMax;
                        const float dp = clamped ? 0.0f : alpha * dal;
                        gv[5] = clamped ? 0.0f : G * dal;
                        gv[0] = -dp * (a.z * dx + a.w * dy);
                        gv[1] = -dp * (b.x * dy + a.w * dx);
                        gv[2] = -0.5f * dp * dx * dx;
                        gv[3] = -dp * dx * dy;
                        gv[4] = -0.5f * dp * dy * dy;
                        Tr = Tn;
                    }
                }
            }
            if (__ballot(contrib) != 0) {
                for (int c = 0; c < kGrad2d; ++c) {
                    const float s = wave_sum(gv[c]);
                    if (lane == 0) atomicAdd(&s_g[e * kGrad2d + c], s);
                }
            }
        }
        __syncthreads();
        for (int k = tid; k < cnt * kGrad2d; k += NT) {
            const float v = s_g[k];
            if (v != 0.0f) atomicAdd(&grad2d[uint64_t(s_id[k / kGrad2d]) * kGrad2d + k % kGrad2d], v);
            s_g[k] = 0.0f;
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

}  // namespace

hipError_t launch_raster_fwd(const Grid& grid, const float bg[3], const uint8_t* ws,
                             const Layout& L, const uint32_t* pair_vals, uint32_t pair_count,
                             float* image,
                             float* t_final, uint32_t* last_contrib, uint32_t* n_eval,
                             hipStream_t s) {
    const auto* rec = reinterpret_cast<const float4*>(ws + L.records);
    const auto* ranges = reinterpret_cast<const uint32_t*>(ws + L.ranges);
    const dim3 nb(unsigned(grid.num_tiles()));
    if (grid.num_tiles() == 0) return hipSuccess;
    switch (grid.tile) {
        case 8:
            raster_fwd_kernel<8><<<nb, dim3(64), 0, s>>>(grid, bg[0], bg[1], bg[2], rec, ranges,
                                                         pair_vals, pair_count, image, t_final, last_contrib, n_eval);
            break;
        case 32:
            raster_fwd_kernel<32><<<nb, dim3(1024), 0, s>>>(grid, bg[0], bg[1], bg[2], rec, ranges,
                                                            pair_vals, pair_count, image, t_final, last_contrib, n_eval);
            break;
        default:
            raster_fwd_kernel<16><<<nb, dim3(256), 0, s>>>(grid, bg[0], bg[1], bg[2], rec, ranges,
                                                           pair_vals, pair_count, image, t_final, last_contrib, n_eval);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_raster_bwd(const Grid& grid, const float bg[3], const uint8_t* ws,
                             const Layout& L, const uint32_t* pair_vals, uint32_t pair_count,
                             const float* image,
                             const float* dL_dimage, float* grad2d, hipStream_t s) {
    (void)bg;   // the background enters through image = C + T_final bg
    const auto* rec = reinterpret_cast<const float4*>(ws + L.records);
    const auto* ranges = reinterpret_cast<const uint32_t*>(ws + L.ranges);
    const dim3 nb(unsigned(grid.num_tiles()));
    if (grid.num_tiles() == 0) return hipSuccess;
    switch (grid.tile) {
        case 8:
            raster_bwd_kernel<8><<<nb, dim3(64), 0, s>>>(grid, rec, ranges, pair_vals, pair_count, image, dL_dimage, grad2d);
            break;
        case 32:
            raster_bwd_kernel<32><<<nb, dim3(1024), 0, s>>>(grid, rec, ranges, pair_vals, pair_count, image, dL_dimage, grad2d);
            break;
        default:
            raster_bwd_kernel<16><<<nb, dim3(256), 0, s>>>(grid, rec, ranges, pair_vals, pair_count, image, dL_dimage, grad2d);
            break;
    }
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
