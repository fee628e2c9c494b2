// C ABI of libtgs: argument validation, workspace layout and the order of
// the stages.  All validation happens before the first HIP call, so every
// error path can be exercised on a machine without a GPU.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "common.hpp"

struct tgs_context {
    int device;
    uint64_t* pinned;   // host-pinned readback of the tile-row starts
};

namespace {
constexpr size_t kPinnedBytes = 4 * (tgs::kMaxCols * 4 + 8);   // row starts of the tallest grid
}

namespace {

thread_local std::string g_error;

tgs_status fail(tgs_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return s;
}

tgs_status hip_fail(hipError_t e, const char* what) {
    return fail(TGS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define TGS_HIP(call)                                            \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return hip_fail(e_, #call);        \
    } while (0)

bool finitef(float x) { return std::isfinite(x); }

tgs_status check_camera(const tgs_camera* cam) {
    if (!cam) return fail(TGS_ERR_INVALID_ARG, "camera is NULL");
    if (cam->width <= 0 || cam->height <= 0)
        return fail(TGS_ERR_INVALID_ARG, "camera size %dx%d must be positive", cam->width, cam->height);
    if (!(cam->fx > 0) || !(cam->fy > 0) || !finitef(cam->fx) || !finitef(cam->fy))
        return fail(TGS_ERR_INVALID_ARG, "focal lengths must be positive and finite");
    if (!finitef(cam->cx) || !finitef(cam->cy) || !finitef(cam->near_z))
        return fail(TGS_ERR_INVALID_ARG, "principal point and near_z must be finite");
    for (int k = 0; k < 12; ++k)
        if (!finitef(cam->world_to_cam[k])) return fail(TGS_ERR_INVALID_ARG, "world_to_cam is not finite");
    return TGS_OK;
}

tgs_status check_dilation(const tgs_dilation* dil, const tgs_camera* cam) {
    if (!dil) return fail(TGS_ERR_INVALID_ARG, "dilation is NULL");
    if (dil->stride < 1) return fail(TGS_ERR_INVALID_ARG, "dilation stride %d < 1", dil->stride);
    if (dil->off_x < 0 || dil->off_x >= dil->stride || dil->off_y < 0 || dil->off_y >= dil->stride)
        return fail(TGS_ERR_INVALID_ARG, "offsets (%d, %d) must lie in [0, %d)", dil->off_x, dil->off_y,
                    dil->stride);
    if (dil->off_x >= cam->width || dil->off_y >= cam->height)
        return fail(TGS_ERR_INVALID_ARG, "offsets lie outside the image");
    return TGS_OK;
}

tgs_status check_options(const tgs_options* opt) {
    if (!opt) return fail(TGS_ERR_INVALID_ARG, "options is NULL");
    if (opt->tile != 8 && opt->tile != 16 && opt->tile != 32)
        return fail(TGS_ERR_INVALID_ARG, "tile %d must be 8, 16 or 32", opt->tile);
    if (opt->reserved != 0 || opt->flags != 0)
        return fail(TGS_ERR_INVALID_ARG, "reserved option fields must be 0");
    for (int c = 0; c < 3; ++c)
        if (!finitef(opt->bg[c])) return fail(TGS_ERR_INVALID_ARG, "background is not finite");
    return TGS_OK;
}

tgs_status check_gaussians(const tgs_gaussians* g) {
    if (!g) return fail(TGS_ERR_INVALID_ARG, "gaussians is NULL");
    if (g->n < 0) return fail(TGS_ERR_INVALID_ARG, "n = %lld < 0", (long long)g->n);
    if (g->n > int64_t(UINT32_MAX) - 1) return fail(TGS_ERR_UNSUPPORTED, "n exceeds 2^32 - 2");
    if (g->sh_degree < 0 || g->sh_degree > 3)
        return fail(TGS_ERR_INVALID_ARG, "sh_degree %d must be in [0, 3]", g->sh_degree);
    const int need = (g->sh_degree + 1) * (g->sh_degree + 1);
    if (g->sh_coeffs < need || g->sh_coeffs > 16)
        return fail(TGS_ERR_INVALID_ARG, "sh_coeffs %d must be in [%d, 16]", g->sh_coeffs, need);
    if (g->n > 0 && (!g->means || !g->scales || !g->quats || !g->opacities || !g->sh))
        return fail(TGS_ERR_INVALID_ARG, "a parameter pointer is NULL");
    return TGS_OK;
}

tgs_status check_grid(const tgs::Grid& g) {
    if (g.gx > tgs::kMaxCols || g.gy > 4 * tgs::kMaxCols)
        return fail(TGS_ERR_UNSUPPORTED, "tile grid %dx%d exceeds %dx%d", g.gx, g.gy, tgs::kMaxCols,
                    4 * tgs::kMaxCols);
    return TGS_OK;
}

tgs_status check_common(const tgs_camera* cam, const tgs_dilation* dil, const tgs_options* opt) {
    tgs_status s = check_camera(cam);
    if (s == TGS_OK) s = check_dilation(dil, cam);
    if (s == TGS_OK && opt) s = check_options(opt);
    if (s == TGS_OK && opt) s = check_grid(tgs::make_grid(*cam, *dil, opt->tile));
    return s;
}

tgs_status check_state(const tgs_state* st, int64_t n, const tgs::Grid& grid, tgs::Layout* L) {
    if (!st) return fail(TGS_ERR_INVALID_ARG, "state is NULL");
    if (!st->workspace) return fail(TGS_ERR_INVALID_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(st->workspace) % 256 != 0)
        return fail(TGS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    *L = tgs::make_layout(n, st->pair_capacity, grid);
    if (st->workspace_bytes < L->total)
        return fail(TGS_ERR_INVALID_ARG, "workspace of %llu bytes < %llu required",
                    (unsigned long long)st->workspace_bytes, (unsigned long long)L->total);
    return TGS_OK;
}

int key_bits_for(int64_t num_tiles) {
    int b = 1;
    while ((int64_t(1) << b) < num_tiles) ++b;
    return b;
}

// The raster stages read ranges and pair values written by tgs_bin_sort for
// the same tile grid; refuse a state that was not binned (or was binned for
// another grid) instead of reading stale indices.
tgs_status check_binned(const tgs_state* st, const tgs::Layout& L, const tgs::Grid& grid) {
    if (st->key_bits == 0 || st->key_bits != uint32_t(key_bits_for(grid.num_tiles())))
        return fail(TGS_ERR_INVALID_ARG, "state has not been binned for this tile grid");
    if (st->pair_count > st->pair_capacity)
        return fail(TGS_ERR_CAPACITY, "state holds %llu pairs, capacity %llu",
                    (unsigned long long)st->pair_count, (unsigned long long)st->pair_capacity);
    if (st->off_pair_vals != L.pair_vals)
        return fail(TGS_ERR_INVALID_ARG, "state offsets do not match its layout");
    return TGS_OK;
}

void publish_offsets(tgs_state* st, const tgs::Layout& L, int depth_buf) {
    st->off_records = L.records;
    st->off_tiles_touched = L.tiles_touched;
    st->off_depth_order = L.depth_val[depth_buf];
    st->off_pair_vals = L.pair_vals;
    st->off_ranges = L.ranges;
    st->off_grad2d = L.grad2d;
}

tgs_status use_device(tgs_context* ctx) {
    if (!ctx) return fail(TGS_ERR_INVALID_ARG, "context is NULL");
    TGS_HIP(hipSetDevice(ctx->device));
    return TGS_OK;
}

}  // namespace

namespace tgs {

Grid make_grid(const tgs_camera& cam, const tgs_dilation& dil, int tile) {
    Grid g;
    g.width = cam.width;
    g.height = cam.height;
    g.stride = dil.stride;
    g.off_x = dil.off_x;
    g.off_y = dil.off_y;
    g.tile = tile;
    g.w_ds = (cam.width - dil.off_x + dil.stride - 1) / dil.stride;
    g.h_ds = (cam.height - dil.off_y + dil.stride - 1) / dil.stride;
    g.gx = (g.w_ds + tile - 1) / tile;
    g.gy = (g.h_ds + tile - 1) / tile;
    return g;
}

Layout make_layout(int64_t n, uint64_t cap, const Grid& grid) {
    Layout L{};
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    const uint64_t un = uint64_t(n);
    const uint64_t gy = uint64_t(grid.gy), gx = uint64_t(grid.gx);
    const uint64_t rowtot = gy * bin_chunks(n) + 1;
    const uint64_t hist = gx * bin_max_slices(cap, grid.gy);
    L.records = take(un * kRecordBytes);
    L.tiles_touched = take(un * 4);
    for (int b = 0; b < 2; ++b) L.depth_key[b] = take(un * 4);
    for (int b = 0; b < 2; ++b) L.depth_val[b] = take(un * 4);
    L.rowtot = take(rowtot * 4);
    L.row_start = take((gy + 1) * 4);
    L.first_slice = take((gy + 1) * 4);
    L.row_cols = take(cap * 2);
    L.row_vals = take(cap * 4);
    L.pair_vals = take(cap * 4);
    L.col_hist = take(hist * 4);
    L.ranges = take(uint64_t(grid.num_tiles()) * 8);
    L.grad2d = take(un * kGrad2d * 4);
    L.sort_counts = take(radix_counts_elems(un) * 4);
    uint64_t most = radix_counts_elems(un);
    if (rowtot > most) most = rowtot;
    if (hist > most) most = hist;
    L.scan_partials = take(scan_partials_elems(most) * 8);
    L.total = o;
    return L;
}

RasterTuning raster_tuning() {
    static const RasterTuning t = [] {
        RasterTuning r;
        if (const char* e = std::getenv("TGS_RASTER_PPT")) {
            const int v = std::atoi(e);
            if (v == 1 || v == 2 || v == 4) r.ppt = v;
        }
        if (const char* e = std::getenv("TGS_TILE_ORDER")) {
            const int v = std::atoi(e);
            if (v == 0 || v == 1) r.order = v;
        }
        return r;
    }();
    return t;
}

CamDev make_cam(const tgs_camera& c) {
    CamDev d{};
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) d.R[3 * r + k] = c.world_to_cam[4 * r + k];
        d.t[r] = c.world_to_cam[4 * r + 3];
    }
    for (int k = 0; k < 3; ++k) {
        double s = 0;
        for (int r = 0; r < 3; ++r) s -= double(d.R[3 * r + k]) * double(d.t[r]);
        d.campos[k] = float(s);
    }
    d.fx = c.fx;
    d.fy = c.fy;
    d.cx = c.cx;
    d.cy = c.cy;
    d.near_z = c.near_z;
    d.width = c.width;
    d.height = c.height;
    return d;
}

}  // namespace tgs

extern "C" {

const char* tgs_status_str(tgs_status s) {
    switch (s) {
        case TGS_OK: return "ok";
        case TGS_ERR_INVALID_ARG: return "invalid argument";
        case TGS_ERR_CAPACITY: return "pair capacity exceeded";
        case TGS_ERR_HIP: return "HIP runtime error";
        case TGS_ERR_NO_DEVICE: return "no such device";
        case TGS_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* tgs_last_error(void) { return g_error.c_str(); }

const char* tgs_version(void) { return "tgs 0.1 gfx950"; }

tgs_status tgs_create(int device, tgs_context** out) {
    if (!out) return fail(TGS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return fail(TGS_ERR_NO_DEVICE, "device %d not available (%d devices)", device, count);
    TGS_HIP(hipSetDevice(device));
    auto* ctx = new (std::nothrow) tgs_context{device, nullptr};
    if (!ctx) return fail(TGS_ERR_HIP, "out of host memory");
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&ctx->pinned), kPinnedBytes,
                                 hipHostMallocDefault);
    if (e != hipSuccess) {
        delete ctx;
        return hip_fail(e, "hipHostMalloc");
    }
    *out = ctx;
    return TGS_OK;
}

void tgs_destroy(tgs_context* ctx) {
    if (!ctx) return;
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
}

tgs_status tgs_query_sizes(int64_t n, const tgs_camera* cam, const tgs_dilation* dil,
                           const tgs_options* opt, uint64_t pair_capacity, tgs_sizes* out) {
    if (!out) return fail(TGS_ERR_INVALID_ARG, "out is NULL");
    if (n < 0) return fail(TGS_ERR_INVALID_ARG, "n < 0");
    tgs_status s = check_common(cam, dil, opt);
    if (s != TGS_OK) return s;
    if (!opt) return fail(TGS_ERR_INVALID_ARG, "options is NULL");
    if (pair_capacity > uint64_t(UINT32_MAX))
        return fail(TGS_ERR_UNSUPPORTED, "pair capacity above 2^32 - 1");
    const tgs::Grid g = tgs::make_grid(*cam, *dil, opt->tile);
    if ((s = check_grid(g)) != TGS_OK) return s;
    const tgs::Layout L = tgs::make_layout(n, pair_capacity, g);
    out->w_ds = g.w_ds;
    out->h_ds = g.h_ds;
    out->grid_x = g.gx;
    out->grid_y = g.gy;
    out->num_tiles = g.num_tiles();
    out->pixels = int64_t(g.w_ds) * g.h_ds;
    out->pair_capacity = pair_capacity;
    out->workspace_bytes = L.total;
    return TGS_OK;
}

tgs_status tgs_preprocess_fwd(tgs_context* ctx, const tgs_gaussians* g, const tgs_camera* cam,
                              const tgs_dilation* dil, const tgs_options* opt, tgs_state* st,
                              void* stream) {
    tgs_status s = check_gaussians(g);
    if (s == TGS_OK) s = check_common(cam, dil, opt);
    if (s == TGS_OK && !opt) s = fail(TGS_ERR_INVALID_ARG, "options is NULL");
    if (s != TGS_OK) return s;
    const tgs::Grid grid = tgs::make_grid(*cam, *dil, opt->tile);
    tgs::Layout L;
    if ((s = check_state(st, g->n, grid, &L)) != TGS_OK) return s;
    if ((s = use_device(ctx)) != TGS_OK) return s;
    auto* ws = static_cast<uint8_t*>(st->workspace);
    TGS_HIP(tgs::launch_preprocess_fwd(*g, tgs::make_cam(*cam), grid, ws, L,
                                       static_cast<hipStream_t>(stream)));
    st->pair_count = 0;
    st->key_bits = 0;     // not binned yet
    publish_offsets(st, L, 0);
    return TGS_OK;
}

tgs_status tgs_bin_sort(tgs_context* ctx, const tgs_gaussians* g, const tgs_camera* cam,
                        const tgs_dilation* dil, const tgs_options* opt, tgs_state* st,
                        void* stream) {
    tgs_status s = check_gaussians(g);
    if (s == TGS_OK) s = check_common(cam, dil, opt);
    if (s == TGS_OK && !opt) s = fail(TGS_ERR_INVALID_ARG, "options is NULL");
    if (s != TGS_OK) return s;
    const tgs::Grid grid = tgs::make_grid(*cam, *dil, opt->tile);
    tgs::Layout L;
    if ((s = check_state(st, g->n, grid, &L)) != TGS_OK) return s;
    if ((s = use_device(ctx)) != TGS_OK) return s;
    auto* ws = static_cast<uint8_t*>(st->workspace);
    auto strm = static_cast<hipStream_t>(stream);
    const int64_t n = g->n;
    auto u32 = [&](uint64_t off) { return reinterpret_cast<uint32_t*>(ws + off); };
    auto* partials = reinterpret_cast<uint64_t*>(ws + L.scan_partials);

    // 1. Gaussians by depth key (stable; culled and off-screen ones last)
    uint32_t* dkeys[2] = {u32(L.depth_key[0]), u32(L.depth_key[1])};
    uint32_t* dvals[2] = {u32(L.depth_val[0]), u32(L.depth_val[1])};
    int dres = 0;
    TGS_HIP(tgs::radix_sort(dkeys, dvals, uint64_t(n), 32, u32(L.sort_counts), partials, &dres, strm));
    const uint32_t* order = dvals[dres];
    // 2. pairs per (tile row, chunk of the depth order); scan -> row buckets
    const uint64_t nrow = uint64_t(grid.gy) * tgs::bin_chunks(n);
    TGS_HIP(tgs::launch_row_counts(ws, L, order, n, grid, strm));
    TGS_HIP(tgs::exclusive_scan_u32(u32(L.rowtot), u32(L.rowtot), nrow, partials, true, strm));
    TGS_HIP(tgs::launch_row_setup(ws, L, n, grid, strm));
    // 3. row starts (and the pair count) back to the host
    TGS_HIP(hipMemcpyAsync(ctx->pinned, u32(L.row_start), (uint64_t(grid.gy) + 1) * 4,
                           hipMemcpyDeviceToHost, strm));
    TGS_HIP(hipStreamSynchronize(strm));
    const uint32_t* rs = reinterpret_cast<const uint32_t*>(ctx->pinned);
    const uint64_t P = rs[grid.gy];
    uint64_t slices = 0;
    for (int ty = 0; ty < grid.gy; ++ty) slices += (uint64_t(rs[ty + 1] - rs[ty]) + tgs::kSlice - 1) / tgs::kSlice;
    st->pair_count = P;
    st->key_bits = 0;
    publish_offsets(st, L, dres);
    if (P > st->pair_capacity)
        return fail(TGS_ERR_CAPACITY, "%llu pairs needed, capacity %llu", (unsigned long long)P,
                    (unsigned long long)st->pair_capacity);
    // 4. emit into row buckets, then a stable counting sort by column per row,
    //    which also yields the per-tile ranges
    TGS_HIP(tgs::launch_emit_rows(ws, L, order, n, grid, strm));
    TGS_HIP(tgs::launch_col_sort(ws, L, grid, slices, strm));
    st->key_bits = uint32_t(key_bits_for(grid.num_tiles()));   // marks the state as binned
    return TGS_OK;
}

tgs_status tgs_raster_fwd(tgs_context* ctx, const tgs_camera* cam, const tgs_dilation* dil,
                          const tgs_options* opt, const tgs_state* st, int64_t n, float* image,
                          float* t_final, uint32_t* last_contrib, uint32_t* n_eval,
                          uint32_t* n_blend, void* stream) {
    tgs_status s = check_common(cam, dil, opt);
    if (s == TGS_OK && !opt) s = fail(TGS_ERR_INVALID_ARG, "options is NULL");
    if (s != TGS_OK) return s;
    if (n < 0) return fail(TGS_ERR_INVALID_ARG, "n < 0");
    const tgs::Grid grid = tgs::make_grid(*cam, *dil, opt->tile);
    if (!image) return fail(TGS_ERR_INVALID_ARG, "image is NULL");
    tgs::Layout L;
    if ((s = check_state(st, n, grid, &L)) != TGS_OK) return s;
    if ((s = check_binned(st, L, grid)) != TGS_OK) return s;
    if ((s = use_device(ctx)) != TGS_OK) return s;
    auto* ws = static_cast<uint8_t*>(st->workspace);
    TGS_HIP(tgs::launch_raster_fwd(grid, tgs::raster_tuning(), opt->bg, ws, L,
                                   reinterpret_cast<const uint32_t*>(ws + st->off_pair_vals),
                                   uint32_t(st->pair_count), image, t_final, last_contrib, n_eval,
                                   n_blend, static_cast<hipStream_t>(stream)));
    return TGS_OK;
}

tgs_status tgs_forward(tgs_context* ctx, const tgs_gaussians* g, const tgs_camera* cam,
                       const tgs_dilation* dil, const tgs_options* opt, tgs_state* st, float* image,
                       void* stream) {
    if (!image) return fail(TGS_ERR_INVALID_ARG, "image is NULL");
    tgs_status s = tgs_preprocess_fwd(ctx, g, cam, dil, opt, st, stream);
    if (s == TGS_OK) s = tgs_bin_sort(ctx, g, cam, dil, opt, st, stream);
    if (s == TGS_OK)
        s = tgs_raster_fwd(ctx, cam, dil, opt, st, g->n, image, nullptr, nullptr, nullptr, nullptr,
                           stream);
    return s;
}

tgs_status tgs_l1_grad(tgs_context* ctx, const tgs_camera* cam, const tgs_dilation* dil,
                       const float* image, const float* target, float* dL_dimage, double* loss,
                       void* stream) {
    tgs_status s = check_common(cam, dil, nullptr);
    if (s != TGS_OK) return s;
    if (!image || !target || !dL_dimage) return fail(TGS_ERR_INVALID_ARG, "a buffer is NULL");
    if ((s = use_device(ctx)) != TGS_OK) return s;
    const tgs::Grid grid = tgs::make_grid(*cam, *dil, 16);
    TGS_HIP(tgs::launch_l1_grad(grid, image, target, dL_dimage, loss,
                                static_cast<hipStream_t>(stream)));
    return TGS_OK;
}

tgs_status tgs_raster_bwd(tgs_context* ctx, const tgs_camera* cam, const tgs_dilation* dil,
                          const tgs_options* opt, const tgs_state* st, int64_t n,
                          const float* image, const float* dL_dimage, void* stream) {
    tgs_status s = check_common(cam, dil, opt);
    if (s == TGS_OK && !opt) s = fail(TGS_ERR_INVALID_ARG, "options is NULL");
    if (s != TGS_OK) return s;
    if (n < 0) return fail(TGS_ERR_INVALID_ARG, "n < 0");
    if (!image || !dL_dimage) return fail(TGS_ERR_INVALID_ARG, "image or dL_dimage is NULL");
    const tgs::Grid grid = tgs::make_grid(*cam, *dil, opt->tile);
    tgs::Layout L;
    if ((s = check_state(st, n, grid, &L)) != TGS_OK) return s;
    if ((s = check_binned(st, L, grid)) != TGS_OK) return s;
    if ((s = use_device(ctx)) != TGS_OK) return s;
    auto* ws = static_cast<uint8_t*>(st->workspace);
    auto strm = static_cast<hipStream_t>(stream);
    auto* g2d = reinterpret_cast<float*>(ws + L.grad2d);
    TGS_HIP(tgs::fill_u32(reinterpret_cast<uint32_t*>(g2d), 0u, uint64_t(n) * tgs::kGrad2d, strm));
    TGS_HIP(tgs::launch_raster_bwd(grid, tgs::raster_tuning(), ws, L,
                                   reinterpret_cast<const uint32_t*>(ws + st->off_pair_vals),
                                   uint32_t(st->pair_count), image, dL_dimage, g2d, strm));
    return TGS_OK;
}

tgs_status tgs_preprocess_bwd(tgs_context* ctx, const tgs_gaussians* g, const tgs_camera* cam,
                              const tgs_dilation* dil, const tgs_options* opt, const tgs_state* st,
                              const tgs_grads* out, float* pos_stat, float* col_stat,
                              uint8_t* visible, void* stream) {
    tgs_status s = check_gaussians(g);
    if (s == TGS_OK) s = check_common(cam, dil, opt);
    if (s == TGS_OK && !opt) s = fail(TGS_ERR_INVALID_ARG, "options is NULL");
    if (s != TGS_OK) return s;
    if (!out || (g->n > 0 && (!out->means || !out->scales || !out->quats || !out->opacities || !out->sh)))
        return fail(TGS_ERR_INVALID_ARG, "a gradient pointer is NULL");
    const tgs::Grid grid = tgs::make_grid(*cam, *dil, opt->tile);
    tgs::Layout L;
    if ((s = check_state(st, g->n, grid, &L)) != TGS_OK) return s;
    if ((s = use_device(ctx)) != TGS_OK) return s;
    TGS_HIP(tgs::launch_preprocess_bwd(*g, tgs::make_cam(*cam),
                                       static_cast<const uint8_t*>(st->workspace), L, *out, pos_stat,
                                       col_stat, visible, static_cast<hipStream_t>(stream)));
    return TGS_OK;
}

tgs_status tgs_backward(tgs_context* ctx, const tgs_gaussians* g, const tgs_camera* cam,
                        const tgs_dilation* dil, const tgs_options* opt, const tgs_state* st,
                        const float* image, const float* dL_dimage, const tgs_grads* out,
                        float* pos_stat, float* col_stat, uint8_t* visible, void* stream) {
    tgs_status s = check_gaussians(g);
    if (s != TGS_OK) return s;
    s = tgs_raster_bwd(ctx, cam, dil, opt, st, g->n, image, dL_dimage, stream);
    if (s == TGS_OK)
        s = tgs_preprocess_bwd(ctx, g, cam, dil, opt, st, out, pos_stat, col_stat, visible, stream);
    return s;
}

}  // extern "C"
