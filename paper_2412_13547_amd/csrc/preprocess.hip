// Per-Gaussian preprocess, forward and backward (stage (a) and (d2)).
//
// Forward (Sec. 3 Eq. 1, Sec. 4.1): view transform, near cull,
// Sigma = R S S^T R^T, EWA projection with the full-resolution focal length
// plus a 0.3 px^2 low-pass, conic, 3-sigma radius, SH colour, and the tiles
// of the downsampled grid the splat's box overlaps (Eq. 3-4).
// Backward: the chain rule from dL/d(u, v, A, B, C, o, r, g, b) to the
// parameters, and the densification statistics of Sec. 4.3.
//
// One thread per Gaussian; parameters are read structure-of-arrays so that
// every load instruction of a wavefront touches 64 consecutive floats.  Both
// kernels serve a table of views (cameras and dilation patterns): the
// forward reads the parameters once and writes every view's records, the
// backward sums the parameter gradients of every view before writing them.
#include "common.hpp"

namespace tgs {
namespace {

// Real SH basis (Condon-Shortley phase, m = -l..l), Cartesian form on the
// unit sphere.  Constants are the closed forms in the comments.
constexpr int kPrepThreads = 256;              // threads per block of the preprocess kernels

constexpr float kC0 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
constexpr float kC1 = 0.4886025119029199f;    // sqrt(3/(4 pi))
constexpr float kC2a = 1.0925484305920792f;   // sqrt(15/(4 pi))
constexpr float kC2b = 0.31539156525252005f;  // sqrt(5/(16 pi))
constexpr float kC2c = 0.5462742152960396f;   // sqrt(15/(16 pi))
constexpr float kC3a = 0.5900435899266435f;   // sqrt(35/(32 pi))
constexpr float kC3b = 2.890611442640554f;    // sqrt(105/(4 pi))
constexpr float kC3c = 0.4570457994644658f;   // sqrt(21/(32 pi))
constexpr float kC3d = 0.3731763325901154f;   // sqrt(7/(16 pi))
constexpr float kC3e = 1.445305721320277f;    // sqrt(105/(16 pi))

template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
    Y[0] = kC0;
    if constexpr (DEG >= 1) {
        Y[1] = -kC1 * y;
        Y[2] = kC1 * z;
        Y[3] = -kC1 * x;
    }
    if constexpr (DEG >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = kC2a * (x * y);
        Y[5] = -kC2a * (y * z);
        Y[6] = kC2b * (3.0f * zz - 1.0f);
        Y[7] = -kC2a * (x * z);
        Y[8] = kC2c * (xx - yy);
        if constexpr (DEG >= 3) {
            Y[9] = -kC3a * (y * (3.0f * xx - yy));
            Y[10] = kC3b * (x * y * z);
            Y[11] = -kC3c * (y * (5.0f * zz - 1.0f));
            Y[12] = kC3d * (z * (5.0f * zz - 3.0f));
            Y[13] = -kC3c * (x * (5.0f * zz - 1.0f));
            Y[14] = kC3e * (z * (xx - yy));
            Y[15] = -kC3a * (x * (xx - 3.0f * yy));
        }
    }
}

// sum_k w[k] * grad Y_k(x, y, z)  (gradient in R^3 of the polynomial forms)
template <int DEG>
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, const float* w,
                                              float& gx, float& gy, float& gz) {
    gx = gy = gz = 0.0f;
    if constexpr (DEG >= 1) {
        gy += -kC1 * w[1];
        gz += kC1 * w[2];
        gx += -kC1 * w[3];
    }
    if constexpr (DEG >= 2) {
        gx += kC2a * y * w[4];
        gy += kC2a * x * w[4];
        gy += -kC2a * z * w[5];
        gz += -kC2a * y * w[5];
        gz += kC2b * 6.0f * z * w[6];
        gx += -kC2a * z * w[7];
        gz += -kC2a * x * w[7];
        gx += kC2c * 2.0f * x * w[8];
        gy += -kC2c * 2.0f * y * w[8];
        if constexpr (DEG >= 3) {
            const float xx = x * x, yy = y * y, zz = z * z;
            gx += -kC3a * 6.0f * x * y * w[9];
            gy += -kC3a * 3.0f * (xx - yy) * w[9];
            gx += kC3b * y * z * w[10];
            gy += kC3b * x * z * w[10];
            gz += kC3b * x * y * w[10];
            gy += -kC3c * (5.0f * zz - 1.0f) * w[11];
            gz += -kC3c * 10.0f * y * z * w[11];
            gz += kC3d * (15.0f * zz - 3.0f) * w[12];
            gx += -kC3c * (5.0f * zz - 1.0f) * w[13];
            gz += -kC3c * 10.0f * x * z * w[13];
            gx += kC3e * 2.0f * x * z * w[14];
            gy += -kC3e * 2.0f * y * z * w[14];
            gz += kC3e * (xx - yy) * w[14];
            gx += -kC3a * 3.0f * (xx - yy) * w[15];
            gy += kC3a * 6.0f * x * y * w[15];
        }
    }
}

// Rotation matrix (row-major) of the normalised quaternion (w, x, y, z).
__device__ __forceinline__ void quat_to_rot(float w, float x, float y, float z, float* R) {
    R[0] = 1.0f - 2.0f * (y * y + z * z);
    R[1] = 2.0f * (x * y - w * z);
    R[2] = 2.0f * (x * z + w * y);
    R[3] = 2.0f * (x * y + w * z);
    R[4] = 1.0f - 2.0f * (x * x + z * z);
    R[5] = 2.0f * (y * z - w * x);
    R[6] = 2.0f * (x * z - w * y);
    R[7] = 2.0f * (y * z + w * x);
    R[8] = 1.0f - 2.0f * (x * x + y * y);
}

struct Proj {
    float tx, ty, tz;
    float u, v;
    float cxr, cyr;      // FoV-guarded x/z, y/z
    bool fovx, fovy;
    float Tm[6];         // J R, 2x3 row-major
    float Sig[6];        // 3D covariance (xx, xy, xz, yy, yz, zz)
    float M[9];          // R_q diag(s)
    float Rq[9];
    float qn[4];         // normalised quaternion
    float qlen;
    float a, b, c;       // low-passed 2D covariance
};

// Everything of the forward up to the conic that the backward re-derives.
__device__ __forceinline__ bool project(const CamDev& cam, const float m[3], const float s[3],
                                        const float q[4], Proj& p) {
    p.tx = cam.R[0] * m[0] + cam.R[1] * m[1] + cam.R[2] * m[2] + cam.t[0];
    p.ty = cam.R[3] * m[0] + cam.R[4] * m[1] + cam.R[5] * m[2] + cam.t[1];
    p.tz = cam.R[6] * m[0] + cam.R[7] * m[1] + cam.R[8] * m[2] + cam.t[2];
    if (!(p.tz > cam.near_z)) return false;
    p.u = cam.fx * p.tx / p.tz + cam.cx;
    p.v = cam.fy * p.ty / p.tz + cam.cy;
    const float limx = kFovGuard * float(cam.width) / (2.0f * cam.fx);
    const float limy = kFovGuard * float(cam.height) / (2.0f * cam.fy);
    const float rx = p.tx / p.tz, ry = p.ty / p.tz;
    p.fovx = rx < -limx || rx > limx;
    p.fovy = ry < -limy || ry > limy;
    p.cxr = fminf(fmaxf(rx, -limx), limx);
    p.cyr = fminf(fmaxf(ry, -limy), limy);
    const float j00 = cam.fx / p.tz, j02 = -cam.fx * p.cxr / p.tz;
    const float j11 = cam.fy / p.tz, j12 = -cam.fy * p.cyr / p.tz;
    for (int k = 0; k < 3; ++k) {
        p.Tm[k] = j00 * cam.R[k] + j02 * cam.R[6 + k];
        p.Tm[3 + k] = j11 * cam.R[3 + k] + j12 * cam.R[6 + k];
    }
    p.qlen = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!(p.qlen > 0.0f)) return false;
    for (int k = 0; k < 4; ++k) p.qn[k] = q[k] / p.qlen;
    quat_to_rot(p.qn[0], p.qn[1], p.qn[2], p.qn[3], p.Rq);
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) p.M[r * 3 + k] = p.Rq[r * 3 + k] * s[k];
    // Sigma = M M^T
    p.Sig[0] = p.M[0] * p.M[0] + p.M[1] * p.M[1] + p.M[2] * p.M[2];
    p.Sig[1] = p.M[0] * p.M[3] + p.M[1] * p.M[4] + p.M[2] * p.M[5];
    p.Sig[2] = p.M[0] * p.M[6] + p.M[1] * p.M[7] + p.M[2] * p.M[8];
    p.Sig[3] = p.M[3] * p.M[3] + p.M[4] * p.M[4] + p.M[5] * p.M[5];
    p.Sig[4] = p.M[3] * p.M[6] + p.M[4] * p.M[7] + p.M[5] * p.M[8];
    p.Sig[5] = p.M[6] * p.M[6] + p.M[7] * p.M[7] + p.M[8] * p.M[8];
    // cov2 = Tm Sigma Tm^T
    float TS[6];
    for (int r = 0; r < 2; ++r) {
        const float* t = p.Tm + 3 * r;
        TS[3 * r + 0] = t[0] * p.Sig[0] + t[1] * p.Sig[1] + t[2] * p.Sig[2];
        TS[3 * r + 1] = t[0] * p.Sig[1] + t[1] * p.Sig[3] + t[2] * p.Sig[4];
        TS[3 * r + 2] = t[0] * p.Sig[2] + t[1] * p.Sig[4] + t[2] * p.Sig[5];
    }
    p.a = TS[0] * p.Tm[0] + TS[1] * p.Tm[1] + TS[2] * p.Tm[2] + kLowPass;
    p.b = TS[0] * p.Tm[3] + TS[1] * p.Tm[4] + TS[2] * p.Tm[5];
    p.c = TS[3] * p.Tm[3] + TS[4] * p.Tm[4] + TS[5] * p.Tm[5] + kLowPass;
    return true;
}

__device__ __forceinline__ bool finite_all(const float* x, int k) {
    bool ok = true;
    for (int i = 0; i < k; ++i) ok = ok && isfinite(x[i]);
    return ok;
}

// The record of one Gaussian in one view and its packed tile rectangle
// (empty when culled or off the grid); returns the tiles it overlaps.  With
// JAC, jac receives d(sum_k sh_k,c Y_k)/d dir_a at 3c + a (zero when culled),
// the only use the backward makes of the SH coefficients besides the basis.
template <int DEG, bool JAC>
__device__ __forceinline__ uint32_t preprocess_one(const CamDev& cam, const Grid& grid, bool ok,
                                                   const float m[3], const float s[3],
                                                   const float q[4], float op, const float* sh,
                                                   float4 out[3], uint2& rect, float jac[9]) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    Proj p;
    ok = ok && project(cam, m, s, q, p);
    float det = 0.0f;
    if (ok) {
        det = p.a * p.c - p.b * p.b;
        ok = det > 0.0f;
    }
    int radius = 0;
    if (ok) {
        const float hd = 0.5f * (p.a - p.c);
        const float lam = 0.5f * (p.a + p.c) + sqrtf(hd * hd + p.b * p.b);
        radius = int(ceilf(3.0f * sqrtf(lam)));
        ok = radius > 0;
    }
    rect = make_uint2(0u, 0u);
    if constexpr (JAC)
        for (int k = 0; k < 9; ++k) jac[k] = 0.0f;
    if (!ok) {
        out[0] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        out[1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        out[2] = make_float4(0.0f, 0.0f, __int_as_float(0), __uint_as_float(kCulled));
        return 0;
    }
    const float A = p.c / det, B = -p.b / det, C = p.a / det;
    // colour
    float dx = m[0] - cam.campos[0], dy = m[1] - cam.campos[1], dz = m[2] - cam.campos[2];
    const float len = sqrtf(dx * dx + dy * dy + dz * dz);
    dx /= len; dy /= len; dz /= len;
    float Y[16];
    sh_basis<DEG>(dx, dy, dz, Y);
    float rgb[3];
    uint32_t flags = (p.fovx ? kFovX : 0u) | (p.fovy ? kFovY : 0u);
    for (int c = 0; c < 3; ++c) {
        float acc = 0.0f;
        for (int k = 0; k < K; ++k) acc += sh[k * 3 + c] * Y[k];
        acc += 0.5f;
        if (acc < 0.0f) flags |= (1u << c);
        rgb[c] = fmaxf(acc, 0.0f);
    }
    if constexpr (JAC && DEG >= 1) {
        for (int c = 0; c < 3; ++c) {
            float w[K];
            for (int k = 0; k < K; ++k) w[k] = sh[k * 3 + c];
            sh_basis_grad<DEG>(dx, dy, dz, w, jac[3 * c], jac[3 * c + 1], jac[3 * c + 2]);
        }
    }
    out[0] = make_float4(p.u, p.v, A, B);
    out[1] = make_float4(C, op, rgb[0], rgb[1]);
    out[2] = make_float4(rgb[2], p.tz, __int_as_float(radius), __uint_as_float(flags));
    const Rect rc = tile_rect(p.u, p.v, radius, grid);
    const uint32_t nt = uint32_t(rc.xhi - rc.xlo) * uint32_t(rc.yhi - rc.ylo);
    if (nt > 0) rect = pack_rect(rc);
    return nt;
}

// One thread per Gaussian: the parameters are read once and the record of
// every view of the table is written.
template <int DEG, bool MULTI>
__global__ void __launch_bounds__(256) preprocess_fwd_kernel(tgs_gaussians g, PrepViews views) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const int64_t n = g.n;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float m[3], s[3], q[4], sh[K * 3];
    for (int k = 0; k < 3; ++k) m[k] = g.means[k * n + i];
    for (int k = 0; k < 3; ++k) s[k] = g.scales[k * n + i];
    for (int k = 0; k < 4; ++k) q[k] = g.quats[k * n + i];
    const float op = g.opacities[i];
    for (int k = 0; k < K * 3; ++k) sh[k] = g.sh[k * n + i];
    const bool ok = finite_all(m, 3) && finite_all(s, 3) && finite_all(q, 4) && isfinite(op) &&
                    finite_all(sh, K * 3);
    const int nv = MULTI ? views.count : 1;
    for (int v = 0; v < nv; ++v) {
        const PrepView& pv = views.v[v];
        if (!ok && pv.nonfinite) atomicAdd(pv.nonfinite, 1u);      // rare: diagnostics only
        float4 r[3];
        uint2 rect;
        float jac[9];
        const uint32_t nt = preprocess_one<DEG, !MULTI>(pv.cam, pv.grid, ok, m, s, q, op, sh, r,
                                                        rect, jac);
        float4* dst = reinterpret_cast<float4*>(pv.rec + i);
        dst[0] = r[0];
        dst[1] = r[1];
        dst[2] = r[2];
        // what the backward reads instead of the record and the tile count
        // (every forward), and in place of the SH coefficients (one view)
        float* jr = jac_rows(pv, n);
        if constexpr (!MULTI && DEG >= 1)
            for (int k = 0; k < 9; ++k) jr[k * n + i] = jac[k];
        jr[9 * n + i] = __uint_as_float(__float_as_uint(r[2].w) | (nt > 0 ? kHasTiles : 0u));
        pv.touched[i] = nt;
        pv.rects[i] = rect;
        pv.depth_key[i] = nt > 0 ? __float_as_uint(r[2].y) : 0xFFFFFFFFu;
        pv.depth_val[i] = uint32_t(i);
    }
}

// Parameter gradients of Gaussian i in one view, written to (dm, ds, dq);
// gr = dL/d(u, v, A, B, C, o, r, g, b).  The colour's gradient in the view
// direction comes from the forward's Jacobian rows jac ([9][n]) when given,
// else from the SH coefficients sh_g ([K*3][n]); the coefficients'
// gradients are added to dsh_acc (ACC: this thread's column of an LDS
// array [K*3][kPrepThreads]) or written to dsh_g (single view, zero where
// !vis: every lane stores, so each store of the wavefront covers whole
// cache lines).  `reload` (zero) offsets the coefficient reads.
template <int DEG, bool ACC>
__device__ __forceinline__ void preprocess_grad_one(const CamDev& cam, const float m[3],
                                                    const float s[3], const float q[4],
                                                    const float* sh_g, const float* jac,
                                                    float* dsh_g, int64_t n,
                                                    int64_t i, uint32_t flags,
                                                    const float gr[kGrad2d], float dm_out[3],
                                                    float ds_out[3], float dq_out[4],
                                                    float* dsh_acc, bool vis = true,
                                                    int64_t reload = 0) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const float gu = gr[0], gv = gr[1], gA = gr[2], gB = gr[3], gC = gr[4];
    float dm[3] = {0.0f, 0.0f, 0.0f};

    // ---- colour: rgb = max(sum_k sh_k Y_k(dir) + 0.5, 0), dir = (m - campos)/|.|
    {
        float dx = m[0] - cam.campos[0], dy = m[1] - cam.campos[1], dz = m[2] - cam.campos[2];
        const float len = sqrtf(dx * dx + dy * dy + dz * dz);
        dx /= len; dy /= len; dz /= len;
        float Y[16];
        sh_basis<DEG>(dx, dy, dz, Y);
        float graw[3];
        for (int c = 0; c < 3; ++c) graw[c] = (flags & (1u << c)) ? 0.0f : gr[6 + c];
        float gdx = 0.0f, gdy = 0.0f, gdz = 0.0f;
        if (jac) {
            for (int k = 0; k < K; ++k) {
                for (int c = 0; c < 3; ++c) {
                    const float d = Y[k] * graw[c];
                    if constexpr (ACC) dsh_acc[(k * 3 + c) * kPrepThreads] += d;
                    else dsh_g[(k * 3 + c) * n + i] = vis ? d : 0.0f;
                }
            }
            if constexpr (DEG >= 1) {
                // a Gaussian the view does not see skips the reads (result unused)
                for (int c = 0; c < 3; ++c) {
                    gdx += (vis ? jac[(3 * c) * n + i] : 0.0f) * graw[c];
                    gdy += (vis ? jac[(3 * c + 1) * n + i] : 0.0f) * graw[c];
                    gdz += (vis ? jac[(3 * c + 2) * n + i] : 0.0f) * graw[c];
                }
            }
        } else {
            float w[16];
            for (int k = 0; k < K; ++k) {
                float acc = 0.0f;
                for (int c = 0; c < 3; ++c) {
                    const float d = Y[k] * graw[c];
                    if constexpr (ACC) dsh_acc[(k * 3 + c) * kPrepThreads] += d;
                    else dsh_g[(k * 3 + c) * n + i] = vis ? d : 0.0f;
                    // a Gaussian the view does not see skips the read (result unused)
                    acc += (vis ? sh_g[(k * 3 + c) * n + i + reload] : 0.0f) * graw[c];
                }
                w[k] = acc;
            }
            sh_basis_grad<DEG>(dx, dy, dz, w, gdx, gdy, gdz);
        }
        // through the normalisation of dir
        const float dot = gdx * dx + gdy * dy + gdz * dz;
        dm[0] += (gdx - dx * dot) / len;
        dm[1] += (gdy - dy * dot) / len;
        dm[2] += (gdz - dz * dot) / len;
    }

    // the projection, after the colour so that their registers do not overlap
    Proj p;
    if constexpr (!ACC) p = Proj{};      // lanes the view does not see compute too (and discard)
    project(cam, m, s, q, p);

    // ---- conic (A, B, C) = (c, -b, a) / det  ->  (a, b, c)
    const float a = p.a, b = p.b, c = p.c;
    const float det = a * c - b * b;
    const float id2 = 1.0f / (det * det);
    const float da = (-c * c * gA + b * c * gB - b * b * gC) * id2;
    const float db = (2.0f * b * c * gA - (a * c + b * b) * gB + 2.0f * a * b * gC) * id2;
    const float dc = (-b * b * gA + a * b * gB - a * a * gC) * id2;
    // cov2 = Tm Sigma Tm^T with dcov2 = [[da, db/2], [db/2, dc]]
    const float D[4] = {da, 0.5f * db, 0.5f * db, dc};
    // dSigma = Tm^T D Tm (3x3 symmetric, full storage)
    float DT[6];   // D Tm, 2x3
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k) DT[3 * r + k] = D[2 * r] * p.Tm[k] + D[2 * r + 1] * p.Tm[3 + k];
    float dS[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) dS[3 * r + k] = p.Tm[r] * DT[k] + p.Tm[3 + r] * DT[3 + k];
    // dTm = 2 D Tm Sigma
    const float S9[9] = {p.Sig[0], p.Sig[1], p.Sig[2], p.Sig[1], p.Sig[3],
                         p.Sig[4], p.Sig[2], p.Sig[4], p.Sig[5]};
    float dTm[6];
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k)
            dTm[3 * r + k] = 2.0f * (DT[3 * r] * S9[k] + DT[3 * r + 1] * S9[3 + k] +
                                     DT[3 * r + 2] * S9[6 + k]);
    // Tm = J R  ->  dJ = dTm R^T (only the non-zero entries of J matter)
    const float dJ00 = dTm[0] * cam.R[0] + dTm[1] * cam.R[1] + dTm[2] * cam.R[2];
    const float dJ02 = dTm[0] * cam.R[6] + dTm[1] * cam.R[7] + dTm[2] * cam.R[8];
    const float dJ11 = dTm[3] * cam.R[3] + dTm[4] * cam.R[4] + dTm[5] * cam.R[5];
    const float dJ12 = dTm[3] * cam.R[6] + dTm[4] * cam.R[7] + dTm[5] * cam.R[8];
    const float tz = p.tz, iz = 1.0f / tz, iz2 = iz * iz;
    float dtx = 0.0f, dty = 0.0f, dtz = 0.0f;
    // J00 = fx/tz, J11 = fy/tz
    dtz += -cam.fx * iz2 * dJ00 - cam.fy * iz2 * dJ11;
    // J02 = -fx cxr / tz, cxr = clamp(tx / tz)
    dtz += cam.fx * p.cxr * iz2 * dJ02;
    if (!p.fovx) {
        const float dcx = -cam.fx * iz * dJ02;
        dtx += dcx * iz;
        dtz += -dcx * p.tx * iz2;
    }
    dtz += cam.fy * p.cyr * iz2 * dJ12;
    if (!p.fovy) {
        const float dcy = -cam.fy * iz * dJ12;
        dty += dcy * iz;
        dtz += -dcy * p.ty * iz2;
    }
    // u = fx tx/tz + cx, v = fy ty/tz + cy
    dtx += gu * cam.fx * iz;
    dty += gv * cam.fy * iz;
    dtz += -(gu * cam.fx * p.tx + gv * cam.fy * p.ty) * iz2;
    // t = R m + t0
    dm[0] += cam.R[0] * dtx + cam.R[3] * dty + cam.R[6] * dtz;
    dm[1] += cam.R[1] * dtx + cam.R[4] * dty + cam.R[7] * dtz;
    dm[2] += cam.R[2] * dtx + cam.R[5] * dty + cam.R[8] * dtz;

    // ---- Sigma = M M^T, M = Rq diag(s): dM = 2 dSigma M
    float dM[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k)
            dM[3 * r + k] = 2.0f * (dS[3 * r] * p.M[k] + dS[3 * r + 1] * p.M[3 + k] +
                                    dS[3 * r + 2] * p.M[6 + k]);
    float ds[3], dR[9];
    for (int k = 0; k < 3; ++k) {
        ds[k] = dM[k] * p.Rq[k] + dM[3 + k] * p.Rq[3 + k] + dM[6 + k] * p.Rq[6 + k];
        for (int r = 0; r < 3; ++r) dR[3 * r + k] = dM[3 * r + k] * s[k];
    }
    const float w = p.qn[0], x = p.qn[1], y = p.qn[2], z = p.qn[3];
    float dq[4];
    dq[0] = 2.0f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = 2.0f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0f * x * dR[4] - w * dR[5] +
                    z * dR[6] + w * dR[7] - 2.0f * x * dR[8]);
    dq[2] = 2.0f * (-2.0f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] -
                    w * dR[6] + z * dR[7] - 2.0f * y * dR[8]);
    dq[3] = 2.0f * (-2.0f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.0f * z * dR[4] +
                    y * dR[5] + x * dR[6] + y * dR[7]);
    // through q / |q|
    const float qd = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
    for (int k = 0; k < 4; ++k) dq_out[k] = (dq[k] - p.qn[k] * qd) / p.qlen;
    for (int k = 0; k < 3; ++k) ds_out[k] = ds[k];
    for (int k = 0; k < 3; ++k) dm_out[k] = dm[k];
}

// One thread per Gaussian, one view.  Gaussians the view does not see get
// zeros; they run the same arithmetic (on whatever their parameters give)
// and select zero at the stores, so every store instruction covers the
// whole wavefront.
template <int DEG>
__global__ void __launch_bounds__(kPrepThreads) preprocess_bwd_kernel(
    tgs_gaussians g, PrepViews views, tgs_grads out, float* __restrict__ pos_stat,
    float* __restrict__ col_stat, uint8_t* __restrict__ visible) {
    const int64_t n = g.n;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int K = (DEG + 1) * (DEG + 1);
    const int kc = g.sh_coeffs;
    const PrepView& pv = views.v[0];
    // the forward's flags word; after a one-view forward its Jacobian rows
    // replace the SH coefficients
    const bool use_jac = pv.nonfinite && *jac_current(pv) != 0u;
    const float* jr = jac_rows(pv, n);
    const uint32_t flags = __float_as_uint(jr[9 * n + i]);
    const bool vis = (flags & kHasTiles) && !(flags & kCulled);
    float gr[kGrad2d];
    for (int k = 0; k < kGrad2d; ++k) gr[k] = vis ? pv.g2d[i * kGrad2d + k] : 0.0f;
    // parameters only of Gaussians the view sees: the others' gradients and
    // statistics are zero, and their lanes' results are discarded
    float m[3], s[3], q[4];
    for (int k = 0; k < 3; ++k) m[k] = vis ? g.means[k * n + i] : 0.0f;
    for (int k = 0; k < 3; ++k) s[k] = vis ? g.scales[k * n + i] : 1.0f;
    for (int k = 0; k < 4; ++k) q[k] = vis ? g.quats[k * n + i] : 1.0f;
    float dm[3], ds[3], dq[4];
    preprocess_grad_one<DEG, false>(pv.cam, m, s, q, g.sh, use_jac ? jr : nullptr, out.sh, n,
                                    i, flags, gr, dm, ds, dq, nullptr, vis);
    for (int k = K * 3; k < kc * 3; ++k) out.sh[k * n + i] = 0.0f;
    for (int k = 0; k < 4; ++k) out.quats[k * n + i] = vis ? dq[k] : 0.0f;
    for (int k = 0; k < 3; ++k) out.scales[k * n + i] = vis ? ds[k] : 0.0f;
    for (int k = 0; k < 3; ++k) out.means[k * n + i] = vis ? dm[k] : 0.0f;
    out.opacities[i] = gr[5];
    if (pos_stat) {
        const float px = gr[0] * (0.5f * float(pv.cam.width));
        const float py = gr[1] * (0.5f * float(pv.cam.height));
        pos_stat[i] = sqrtf(px * px + py * py);
    }
    if (col_stat) col_stat[i] = sqrtf(gr[6] * gr[6] + gr[7] * gr[7] + gr[8] * gr[8]);
    if (visible) visible[i] = vis ? 1 : 0;
}

// One thread per Gaussian, several views: the gradients of every view are
// summed in registers (in view order) and written once.
template <int DEG>
__global__ void __launch_bounds__(kPrepThreads) preprocess_bwd_multi_kernel(
    tgs_gaussians g, PrepViews views, tgs_grads out, float* __restrict__ pos_stat,
    float* __restrict__ col_stat, uint8_t* __restrict__ visible) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const int64_t n = g.n;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int kc = g.sh_coeffs;
    float dm[3] = {0.0f, 0.0f, 0.0f}, ds[3] = {0.0f, 0.0f, 0.0f};
    float dq[4] = {0.0f, 0.0f, 0.0f, 0.0f}, dop = 0.0f;
    // the SH gradients summed over the views, in LDS (a column per thread):
    // in registers they left room for one wavefront per SIMD
    __shared__ float s_dsh[K * 3][kPrepThreads];
    float* dsh = &s_dsh[0][threadIdx.x];
    for (int k = 0; k < K * 3; ++k) dsh[k * kPrepThreads] = 0.0f;
    float pos = 0.0f, col = 0.0f;
    uint32_t nvis = 0;
    float m[3], s[3], q[4];
    for (int k = 0; k < 3; ++k) m[k] = g.means[k * n + i];
    for (int k = 0; k < 3; ++k) s[k] = g.scales[k * n + i];
    for (int k = 0; k < 4; ++k) q[k] = g.quats[k * n + i];
    for (int v = 0; v < views.count; ++v) {
        const PrepView& pv = views.v[v];
        const uint32_t flags = __float_as_uint(jac_rows(pv, n)[9 * n + i]);   // the forward's
        if (!((flags & kHasTiles) && !(flags & kCulled))) {
            // this view's own statistics, when asked for: zero where unseen
            if (pv.pos_out) pv.pos_out[i] = 0.0f;
            if (pv.col_out) pv.col_out[i] = 0.0f;
            if (pv.vis_out) pv.vis_out[i] = 0;
            continue;
        }
        float gr[kGrad2d];
        for (int k = 0; k < kGrad2d; ++k) gr[k] = pv.g2d[i * kGrad2d + k];
        float vm[3], vs[3], vq[4];
        // v >> 30 is 0 for every view, but not a constant: the coefficients
        // are read again for each view (from the caches) instead of being
        // held in 48 registers across the loop, which would leave room for
        // only two wavefronts per SIMD
        preprocess_grad_one<DEG, true>(pv.cam, m, s, q, g.sh, nullptr, nullptr, n, i, flags, gr,
                                       vm, vs, vq, dsh, true, int64_t(v >> 30));
        for (int k = 0; k < 3; ++k) dm[k] += vm[k];
        for (int k = 0; k < 3; ++k) ds[k] += vs[k];
        for (int k = 0; k < 4; ++k) dq[k] += vq[k];
        dop += gr[5];
        const float px = gr[0] * (0.5f * float(pv.cam.width));
        const float py = gr[1] * (0.5f * float(pv.cam.height));
        const float vpos = sqrtf(px * px + py * py);
        const float vcol = sqrtf(gr[6] * gr[6] + gr[7] * gr[7] + gr[8] * gr[8]);
        pos += vpos;
        col += vcol;
        ++nvis;
        if (pv.pos_out) pv.pos_out[i] = vpos;
        if (pv.col_out) pv.col_out[i] = vcol;
        if (pv.vis_out) pv.vis_out[i] = 1;
    }
    for (int k = 0; k < 3; ++k) out.means[k * n + i] = dm[k];
    for (int k = 0; k < 3; ++k) out.scales[k * n + i] = ds[k];
    for (int k = 0; k < 4; ++k) out.quats[k * n + i] = dq[k];
    out.opacities[i] = dop;
    for (int k = 0; k < K * 3; ++k) out.sh[k * n + i] = dsh[k * kPrepThreads];
    for (int k = K * 3; k < kc * 3; ++k) out.sh[k * n + i] = 0.0f;
    if (pos_stat) pos_stat[i] = pos;
    if (col_stat) col_stat[i] = col;
    if (visible) visible[i] = uint8_t(nvis);
}

template <bool MULTI>
void launch_fwd(const tgs_gaussians& g, const PrepViews& views, hipStream_t s) {
    const dim3 block(256), nb(unsigned((g.n + 255) / 256));
    switch (g.sh_degree) {
        case 0: preprocess_fwd_kernel<0, MULTI><<<nb, block, 0, s>>>(g, views); break;
        case 1: preprocess_fwd_kernel<1, MULTI><<<nb, block, 0, s>>>(g, views); break;
        case 2: preprocess_fwd_kernel<2, MULTI><<<nb, block, 0, s>>>(g, views); break;
        default: preprocess_fwd_kernel<3, MULTI><<<nb, block, 0, s>>>(g, views); break;
    }
}

template <bool MULTI>
void launch_bwd(const tgs_gaussians& g, const PrepViews& views, const tgs_grads& out,
                float* pos_stat, float* col_stat, uint8_t* visible, hipStream_t s) {
    const dim3 block(kPrepThreads), nb(unsigned((g.n + kPrepThreads - 1) / kPrepThreads));
#define TGS_BWD(D)                                                                                 \
    if (MULTI) preprocess_bwd_multi_kernel<D><<<nb, block, 0, s>>>(g, views, out, pos_stat, col_stat, visible); \
    else preprocess_bwd_kernel<D><<<nb, block, 0, s>>>(g, views, out, pos_stat, col_stat, visible)
    switch (g.sh_degree) {
        case 0: TGS_BWD(0); break;
        case 1: TGS_BWD(1); break;
        case 2: TGS_BWD(2); break;
        default: TGS_BWD(3); break;
    }
#undef TGS_BWD
}

}  // namespace

// The views' non-finite counters to zero before the forward's atomics (one
// small launch, so a captured step needs no memset node).
__global__ void zero_nonfinite_kernel(PrepViews views) {
    const int v = int(threadIdx.x);
    if (v < views.count && views.v[v].nonfinite) *views.v[v].nonfinite = 0u;
    // a one-view launch writes the backward's Jacobian rows (every launch the flags word)
    if (v < views.count && views.v[v].nonfinite) *jac_current(views.v[v]) = views.count == 1 ? 1u : 0u;
}

hipError_t launch_preprocess_fwd(const tgs_gaussians& g, const PrepViews& views, hipStream_t s) {
    if (views.count == 0) return hipSuccess;
    zero_nonfinite_kernel<<<1, 64, 0, s>>>(views);
    if (g.n == 0) return hipGetLastError();
    if (views.count == 1) launch_fwd<false>(g, views, s);
    else launch_fwd<true>(g, views, s);
    return hipGetLastError();
}

hipError_t launch_preprocess_bwd(const tgs_gaussians& g, const PrepViews& views,
                                 const tgs_grads& out, float* pos_stat, float* col_stat,
                                 uint8_t* visible, hipStream_t s) {
    if (g.n == 0) return hipSuccess;
    bool per_view = false;
    for (int v = 0; v < views.count; ++v)
        per_view = per_view || views.v[v].pos_out || views.v[v].col_out || views.v[v].vis_out;
    if (views.count == 1 && !per_view) launch_bwd<false>(g, views, out, pos_stat, col_stat, visible, s);
    else launch_bwd<true>(g, views, out, pos_stat, col_stat, visible, s);
    return hipGetLastError();
}

}  // namespace tgs
