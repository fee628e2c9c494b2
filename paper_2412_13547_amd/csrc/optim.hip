// Fused Adam step over the structure-of-arrays parameter groups (the
// optimiser that follows stage (d2) in a fitting iteration; Adam as in the
// 3DGS training recipe the paper builds on, Tab. 2).
//
// Per element, with step t (1-based) and the standard bias corrections:
//   m <- b1 m + (1 - b1) g
//   v <- b2 v + (1 - b2) g^2
//   p <- p - (lr / (1 - b1^t)) m / (sqrt(v) / sqrt(1 - b2^t) + eps)
// One pass reads p, g, m, v and writes p, m, v: 28 bytes per element, so the
// kernel is HBM-bound; it streams float4 vectors with a grid-stride loop.
//
// The step counter lives in device memory: a one-thread prologue increments
// it and writes the two bias-correction factors (computed in double) next to
// it, so a captured graph replays correct steps without host involvement.
#include "common.hpp"

namespace tgs {
namespace {

struct AdamCoeffs {
    uint32_t step;
    uint32_t pad;
    float inv_bc1;        // 1 / (1 - b1^t)
    float inv_sqrt_bc2;   // 1 / sqrt(1 - b2^t)
};

__global__ void adam_prologue_kernel(AdamCoeffs* c, double b1, double b2) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const uint32_t t = c->step + 1u;
        c->step = t;
        c->inv_bc1 = float(1.0 / (1.0 - pow(b1, double(t))));
        c->inv_sqrt_bc2 = float(1.0 / sqrt(1.0 - pow(b2, double(t))));
    }
}

__device__ __forceinline__ void adam_one(float& p, float g, float& m, float& v, float b1, float b2,
                                         float a, float isb2, float eps) {
    m = b1 * m + (1.0f - b1) * g;
    v = b2 * v + (1.0f - b2) * (g * g);
    p = p - a * m / (sqrtf(v) * isb2 + eps);
}

__global__ void __launch_bounds__(256)
adam_kernel(AdamGroups groups, const AdamCoeffs* __restrict__ c, float b1, float b2, float eps) {
    const float isb2 = c->inv_sqrt_bc2;
    const float ibc1 = c->inv_bc1;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (int k = 0; k < groups.count; ++k) {
        const AdamGroup& G = groups.g[k];
        const float a = G.lr * ibc1;
        const uint64_t n = uint64_t(G.count);
        const uint64_t n4 = G.vec4 ? n / 4 : 0;
        float4* p4 = reinterpret_cast<float4*>(G.param);
        const float4* g4 = reinterpret_cast<const float4*>(G.grad);
        float4* m4 = reinterpret_cast<float4*>(G.exp_avg);
        float4* v4 = reinterpret_cast<float4*>(G.exp_avg_sq);
        for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n4; i += stride) {
            float4 p = p4[i], m = m4[i], v = v4[i];
            const float4 g = g4[i];
            adam_one(p.x, g.x, m.x, v.x, b1, b2, a, isb2, eps);
            adam_one(p.y, g.y, m.y, v.y, b1, b2, a, isb2, eps);
            adam_one(p.z, g.z, m.z, v.z, b1, b2, a, isb2, eps);
            adam_one(p.w, g.w, m.w, v.w, b1, b2, a, isb2, eps);
            p4[i] = p;
            m4[i] = m;
            v4[i] = v;
        }
        for (uint64_t i = 4 * n4 + uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
             i += stride) {
            float p = G.param[i], m = G.exp_avg[i], v = G.exp_avg_sq[i];
            adam_one(p, G.grad[i], m, v, b1, b2, a, isb2, eps);
            G.param[i] = p;
            G.exp_avg[i] = m;
            G.exp_avg_sq[i] = v;
        }
    }
}

}  // namespace

hipError_t launch_adam(const AdamGroups& groups, void* coeffs, float b1, float b2, float eps,
                       hipStream_t s) {
    auto* c = static_cast<AdamCoeffs*>(coeffs);
    adam_prologue_kernel<<<1, 64, 0, s>>>(c, double(b1), double(b2));
    uint64_t total = 0;
    for (int k = 0; k < groups.count; ++k) total += uint64_t(groups.g[k].count);
    // enough workgroups to fill the chip several times over, no more
    uint64_t blocks = (total / 4 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) blocks = 1;
    adam_kernel<<<dim3(unsigned(blocks)), dim3(256), 0, s>>>(groups, c, b1, b2, eps);
    return hipGetLastError();
}

}  // namespace tgs
