// C ABI of libtgs: argument validation, workspace layout and the order of
// the stages.  All validation happens before the first HIP call, so every
// error path can be exercised on a machine without a GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "common.hpp"

namespace {
constexpr size_t kPinnedBytes = 4 * (tgs::kMaxCols * 4 + 8);   // row starts of the tallest grid
// Streams beside the caller's on which the batched binning runs views
// concurrently (forked from and joined into the caller's stream).
constexpr int kAuxStreams = 3;
// The device pair count is a saturating uint32 (UINT32_MAX means "2^32 - 1
// pairs or more"); a capacity below it tells an overflow from a fit.
constexpr uint64_t kSaturated = UINT32_MAX;
constexpr uint64_t kMaxPairCapacity = TGS_MAX_PAIR_CAPACITY;
static_assert(kMaxPairCapacity == kSaturated - 1, "capacity limit below the saturated count");
}

// The workspace of tgs_forward_static: a device array every GPU the library
// runs on holds once, for the whole process.  Host code never uses its name
// as an address (that is a host-side stand-in); tgs_create looks up the
// device address of this GPU's copy and keeps it in the context.
static __device__ __align__(256) uint8_t scratch[TGS_STATIC_SCRATCH_BYTES];

struct tgs_context {
    int device;
    void* scratch;      // device address of this GPU's static scratch array
    uint64_t* pinned;   // host-pinned readback of the tile-row starts
    hipStream_t aux[kAuxStreams];
    hipEvent_t fork;
    hipEvent_t join[kAuxStreams];
};

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

bool is_finite(float x) { return std::isfinite(x); }

tgs_status check_camera(const tgs_camera* cam) {
    if (!cam) return fail(TGS_ERR_INVALID_ARG, "camera is NULL");
    if (cam->width <= 0 || cam->height <= 0)
        return fail(TGS_ERR_INVALID_ARG, "camera size %dx%d must be positive", cam->width, cam->height);
    if (!(cam->fx > 0) || !(cam->fy > 0) || !is_finite(cam->fx) || !is_finite(cam->fy))
        return fail(TGS_ERR_INVALID_ARG, "focal lengths must be positive and finite");
    if (!is_finite(cam->cx) || !is_finite(cam->cy))
        return fail(TGS_ERR_INVALID_ARG, "principal point must be finite");
    // depth keys are float bits (their integer order is the depth order only
    // for positive depths) and the projection divides by the depth
    if (!(cam->near_z > 0.0f) || !is_finite(cam->near_z))
        return fail(TGS_ERR_INVALID_ARG, "near_z must be positive and finite");
    for (int k = 0; k < 12; ++k)
        if (!is_finite(cam->world_to_cam[k])) return fail(TGS_ERR_INVALID_ARG, "world_to_cam is not finite");
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
    if (opt->lds_batch != 0 && opt->lds_batch != 64 && opt->lds_batch != 128 &&
        opt->lds_batch != 256)
        return fail(TGS_ERR_INVALID_ARG, "lds_batch %d must be 0, 64, 128 or 256", opt->lds_batch);
    const int ppt = opt->pixels_per_thread;
    const bool ppt_ok = ppt == 0 || (opt->tile == 8 && ppt == 1) ||
                        (opt->tile == 16 && (ppt == 1 || ppt == 2 || ppt == 4)) ||
                        (opt->tile == 32 && (ppt == 2 || ppt == 4));
    if (!ppt_ok)
        return fail(TGS_ERR_INVALID_ARG,
                    "pixels_per_thread %d not available for tile %d (8: 1; 16: 1, 2, 4; 32: 2, 4)",
                    ppt, opt->tile);
    if ((opt->flags & ~uint32_t(TGS_SYNC_CHECK)) != 0)
        return fail(TGS_ERR_INVALID_ARG, "option flags 0x%x: only TGS_SYNC_CHECK is defined",
                    opt->flags);
    for (int c = 0; c < 3; ++c)
        if (!is_finite(opt->bg[c])) return fail(TGS_ERR_INVALID_ARG, "background is not finite");
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
    if (st->pair_capacity > kMaxPairCapacity)
        return fail(TGS_ERR_UNSUPPORTED, "pair capacity above 2^32 - 2");
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
// another grid) instead of reading stale indices.  A batched bin leaves the
// count on the device (pending), where the kernels check it themselves.
tgs_status check_binned(const tgs_state* st, const tgs::Layout& L, const tgs::Grid& grid,
                        bool allow_pending) {
    if (st->key_bits == 0 || st->key_bits != uint32_t(key_bits_for(grid.num_tiles())))
        return fail(TGS_ERR_INVALID_ARG, "state has not been binned for this tile grid");
    if (st->pair_count == TGS_PAIR_COUNT_PENDING) {
        if (!allow_pending)
            return fail(TGS_ERR_INVALID_ARG, "pair count pending: call tgs_pair_counts first");
    } else if (st->pair_count > st->pair_capacity)
        return fail(TGS_ERR_CAPACITY, "state holds %llu pairs, capacity %llu",
                    (unsigned long long)st->pair_count, (unsigned long long)st->pair_capacity);
    if (st->off_pair_vals != L.pair_vals)
        return fail(TGS_ERR_INVALID_ARG, "state offsets do not match its layout");
    return TGS_OK;
}

void publish_offsets(tgs_state* st, const tgs::Layout& L, const tgs::Grid& grid, int64_t n,
                     const uint32_t* depth_order, const uint8_t* ws) {
    st->off_pair_count = L.row_start + 4 * uint64_t(grid.gy);
    st->off_records = L.records;
    st->off_tiles_touched = L.tiles_touched;
    st->off_depth_order = uint64_t(reinterpret_cast<const uint8_t*>(depth_order) - ws);
    st->off_depth_count = L.sort_counts + 4 * tgs::radix_kept_offset(uint64_t(n));
    st->off_pair_vals = L.pair_vals;
    st->off_ranges = L.ranges;
    st->off_grad2d = L.grad2d;
    st->off_tile_work = L.tile_work;
    st->off_t_final = L.pix_tfinal;
    st->off_last_contrib = L.pix_last;
    st->off_nonfinite_count = L.nonfinite;
}

tgs_status use_device(tgs_context* ctx) {
    if (!ctx) return fail(TGS_ERR_INVALID_ARG, "context is NULL");
    TGS_HIP(hipSetDevice(ctx->device));
    return TGS_OK;
}

// The table entry of one view for the preprocess kernels.
tgs::PrepView prep_view(const tgs_camera& cam, const tgs::Grid& grid, uint8_t* ws,
                        const tgs::Layout& L) {
    tgs::PrepView v{};
    v.cam = tgs::make_cam(cam);
    v.grid = grid;
    v.rec = reinterpret_cast<tgs_record*>(ws + L.records);
    v.touched = reinterpret_cast<uint32_t*>(ws + L.tiles_touched);
    v.rects = reinterpret_cast<uint2*>(ws + L.rects);
    v.depth_key = reinterpret_cast<uint32_t*>(ws + L.depth_key[0]);
    v.depth_val = reinterpret_cast<uint32_t*>(ws + L.depth_val[0]);
    v.g2d = reinterpret_cast<const float*>(ws + L.grad2d);
    v.nonfinite = reinterpret_cast<uint32_t*>(ws + L.nonfinite);
    return v;
}

// The table entry of one binned view for the raster kernels.
tgs::RasterView raster_view(const tgs::Grid& grid, const tgs_options& opt, const tgs_state& st,
                            const tgs::Layout& L) {
    auto* ws = static_cast<uint8_t*>(st.workspace);
    tgs::RasterView v{};
    v.grid = grid;
    v.capacity = uint32_t(st.pair_capacity);
    for (int c = 0; c < 3; ++c) v.bg[c] = opt.bg[c];
    v.rec = reinterpret_cast<const float4*>(ws + L.records);
    v.ranges = reinterpret_cast<const uint32_t*>(ws + L.ranges);
    v.vals = reinterpret_cast<const uint32_t*>(ws + L.pair_vals);
    v.pair_count = reinterpret_cast<const uint32_t*>(ws + L.row_start) + grid.gy;
    v.g2d = reinterpret_cast<float*>(ws + L.grad2d);
    v.work = reinterpret_cast<uint32_t*>(ws + L.tile_work);
    v.order = reinterpret_cast<uint32_t*>(ws + L.tile_order);
    v.ws_tfinal = reinterpret_cast<float*>(ws + L.pix_tfinal);
    v.ws_last = reinterpret_cast<uint32_t*>(ws + L.pix_last);
    v.bits = reinterpret_cast<unsigned long long*>(ws + L.blend_bits);
    v.bits_stride = tgs::blend_words(st.pair_capacity, grid.num_tiles());
    v.fwd_split = reinterpret_cast<uint32_t*>(ws + L.fwd_split);
    return v;
}

void add_raster_view(tgs::RasterViews& t, const tgs::RasterView& v) {
    if (t.count == 0) t.first_block[0] = 0;
    t.v[t.count] = v;
    t.first_block[t.count + 1] = t.first_block[t.count] + uint32_t(v.grid.num_tiles());
    ++t.count;
}

int lds_batch_of(const tgs_options& opt) {
    return opt.lds_batch ? opt.lds_batch : tgs::default_lds_batch(opt.tile);
}

int ppt_of(const tgs_options& opt, int64_t tiles) {
    return opt.pixels_per_thread ? opt.pixels_per_thread
                                 : tgs::default_pixels_per_thread(opt.tile, tiles);
}

// Depth sort and the pair counts per (tile row, chunk), up to the row starts
// and the device pair count.  Returns the depth-sort result buffer and the
// device count of the Gaussians it holds.
tgs_status enqueue_counts(uint8_t* ws, const tgs::Layout& L, const tgs::Grid& grid, int64_t n,
                          uint64_t max_slices, hipStream_t strm, int* dres,
                          const uint32_t** order, const uint32_t** dcount) {
    auto u32 = [&](uint64_t off) { return reinterpret_cast<uint32_t*>(ws + off); };
    auto* partials = reinterpret_cast<uint64_t*>(ws + L.scan_partials);
    // the Gaussians with tiles sorted by depth key (stable, so equal keys
    // keep index order); culled and off-grid ones (key 0xFFFFFFFF) are left
    // out, their number stays on the device
    uint32_t* dkeys[2] = {u32(L.depth_key[0]), u32(L.depth_key[1])};
    uint32_t* dvals[2] = {u32(L.depth_val[0]), u32(L.depth_val[1])};
    TGS_HIP(tgs::radix_sort(dkeys, dvals, uint64_t(n), 32, u32(L.sort_counts), partials, dres, strm,
                            true, 0xFFFFFFFFu));
    const uint32_t* kept = u32(L.sort_counts) + tgs::radix_kept_offset(uint64_t(n));
    *order = dvals[*dres];
    *dcount = kept;
    // entries and pairs per (tile row, block of the depth order); scans ->
    // every block's place in every row
    const uint64_t nrow = uint64_t(grid.gy) * tgs::bin_blocks(n);
    TGS_HIP(tgs::launch_counts(ws, L, *order, n, kept, grid, strm));
    TGS_HIP(tgs::exclusive_scan_u32_pair(u32(L.ecnt), u32(L.ecnt), u32(L.pcnt), u32(L.pcnt), nrow,
                                         partials, true, strm));
    TGS_HIP(tgs::launch_row_setup(ws, L, n, grid, max_slices, strm));
    return TGS_OK;
}

// Entries into row buckets, then a stable counting sort by column per slice
// of every row, which writes the pairs and the per-tile ranges.  `slices`
// bounds the column-sort slices from above; the kernels skip all work when
// the device pair count exceeds the capacity.
tgs_status enqueue_emit(uint8_t* ws, const tgs::Layout& L, const tgs::Grid& grid, int64_t n,
                        const uint32_t* order, const uint32_t* dcount, uint64_t slices,
                        uint32_t capacity, hipStream_t strm) {
    TGS_HIP(tgs::launch_entries(ws, L, order, n, dcount, grid, capacity, strm));
    TGS_HIP(tgs::launch_col_sort(ws, L, grid, slices, capacity, strm));
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
    const uint64_t table = gy * bin_blocks(n) + 1;
    const uint64_t slices = bin_max_slices(cap, grid.gy);
    const uint64_t hist = gx * slices;
    L.records = take(un * kRecordBytes);
    L.tiles_touched = take(un * 4);
    L.jac = take(un * kJacWords * 4);     // directly after the tile counts (jac_rows)
    L.rects = take(un * 8);
    L.srect = take(un * 8);
    for (int b = 0; b < 2; ++b) L.depth_key[b] = take(un * 4);
    for (int b = 0; b < 2; ++b) L.depth_val[b] = take(un * 4);
    L.ecnt = take(table * 4);
    L.pcnt = take(table * 4);
    L.row_start = take((gy + 1) * 4);
    L.erow = take((gy + 1) * 4);
    L.first_slice = take((gy + 1) * 4);
    L.slice_desc = take(slices * 16);
    L.slice_e1 = take(slices * 4);
    L.ent_id = take(cap * 4);
    L.ent_pp = take(cap * 4);
    L.ent_x = take(cap * 4);
    L.pair_vals = take(cap * 4);
    L.col_hist = take(hist * 4);
    L.ranges = take(uint64_t(grid.num_tiles()) * 8);
    L.tile_work = take(uint64_t(grid.num_tiles()) * 4);
    L.tile_order = take(uint64_t(grid.num_tiles()) * 4);
    L.pix_tfinal = take(uint64_t(grid.w_ds) * uint64_t(grid.h_ds) * 4);
    L.pix_last = take(uint64_t(grid.w_ds) * uint64_t(grid.h_ds) * 4);
    L.nonfinite = take(8);                // the counter, then whether jac is current
    L.fwd_split = take(4);
    L.blend_bits = take(uint64_t(max_tile_waves(grid.tile)) * blend_words(cap, grid.num_tiles()) * 8);
    L.grad2d = take(un * kGrad2d * 4);
    L.sort_counts = take(radix_counts_elems(un) * 4);
    // the row tables' device-wide scan (two arrays: 8 bytes per tile sum)
    L.scan_partials = take(scan_partials_elems(table) * 8);
    L.total = o;
    return L;
}

// Fastest settings measured by the launch autotuner on a batch of 12 views
// (2M Gaussians) and at the 4K dilated scene (3M Gaussians, stride 2).
int default_lds_batch(int tile) { return tile == 8 ? 128 : tile == 16 ? 64 : 256; }

int default_pixels_per_thread(int tile) { return tile == 8 ? 1 : 4; }

int default_pixels_per_thread(int tile, int64_t tiles) {
    if (tile == 8) return 1;
    // wavefronts per tile at 4 pixels per thread: 1 (T = 16), 4 (T = 32)
    const int64_t waves = tile == 16 ? tiles : 4 * tiles;
    if (tile == 32) return waves >= 6144 ? 4 : 2;
    return waves >= 6144 ? 4 : waves >= 3072 ? 2 : 1;
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
    TGS_HIP(tgs::prepare_binning_kernels());
    auto* ctx = new (std::nothrow) tgs_context{};
    if (!ctx) return fail(TGS_ERR_HIP, "out of host memory");
    ctx->device = device;
    // this device's copy of the static scratch array (device current)
    hipError_t e = hipGetSymbolAddress(&ctx->scratch, HIP_SYMBOL(scratch));
    const char* what = "hipGetSymbolAddress";
    if (e == hipSuccess) {
        what = "hipHostMalloc";
        e = hipHostMalloc(reinterpret_cast<void**>(&ctx->pinned), kPinnedBytes,
                          hipHostMallocDefault);
    }
    // default-priority streams, not synchronising with the null stream
    for (int a = 0; a < kAuxStreams && e == hipSuccess; ++a) {
        what = "hipStreamCreateWithFlags";
        e = hipStreamCreateWithFlags(&ctx->aux[a], hipStreamNonBlocking);
        if (e == hipSuccess) {
            what = "hipEventCreateWithFlags";
            e = hipEventCreateWithFlags(&ctx->join[a], hipEventDisableTiming);
        }
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming);
    if (e != hipSuccess) {
        tgs_destroy(ctx);
        return hip_fail(e, what);
    }
    *out = ctx;
    return TGS_OK;
}

void tgs_destroy(tgs_context* ctx) {
    if (!ctx) return;
    for (int a = 0; a < kAuxStreams; ++a) {
        if (ctx->aux[a]) (void)hipStreamDestroy(ctx->aux[a]);
        if (ctx->join[a]) (void)hipEventDestroy(ctx->join[a]);
    }
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
}

tgs_status tgs_default_launch(int32_t tile, int32_t* lds_batch, int32_t* pixels_per_thread) {
    if (!lds_batch || !pixels_per_thread) return fail(TGS_ERR_INVALID_ARG, "output is NULL");
    if (tile != 8 && tile != 16 && tile != 32) return fail(TGS_ERR_INVALID_ARG, "tile must be 8, 16 or 32");
    *lds_batch = tgs::default_lds_batch(tile);
    *pixels_per_thread = tgs::default_pixels_per_thread(tile);
    return TGS_OK;
}

tgs_status tgs_query_sizes(int64_t n, const tgs_camera* cam, const tgs_dilation* dil,
                           const tgs_options* opt, uint64_t pair_capacity, tgs_sizes* out) {
    if (!out) return fail(TGS_ERR_INVALID_ARG, "out is NULL");
    if (n < 0) return fail(TGS_ERR_INVALID_ARG, "n < 0");
    tgs_status s = check_common(cam, dil, opt);
    if (s != TGS_OK) return s;
    if (!opt) return fail(TGS_ERR_INVALID_ARG, "options is NULL");
    if (pair_capacity > kMaxPairCapacity)
        return fail(TGS_ERR_UNSUPPORTED, "pair capacity above 2^32 - 2");
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
    tgs::PrepViews t{};
    t.count = 1;
    t.v[0] = prep_view(*cam, grid, static_cast<uint8_t*>(st->workspace), L);
    TGS_HIP(tgs::launch_preprocess_fwd(*g, t, static_cast<hipStream_t>(stream)));
    st->pair_count = 0;
    st->key_bits = 0;     // not binned yet
    auto* ws = static_cast<uint8_t*>(st->workspace);
    publish_offsets(st, L, grid, g->n, reinterpret_cast<const uint32_t*>(ws + L.depth_val[0]), ws);
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
    int dres = 0;
    const uint32_t* order = nullptr;
    const uint32_t* dcount = nullptr;
    const uint64_t max_slices = tgs::bin_max_slices(st->pair_capacity, grid.gy);
    if ((s = enqueue_counts(ws, L, grid, g->n, max_slices, strm, &dres, &order, &dcount)) != TGS_OK)
        return s;
    uint64_t slices = max_slices;
    st->key_bits = 0;
    if (opt->flags & TGS_SYNC_CHECK) {
        // row starts (and the pair count) back to the host: a capacity
        // error can be reported now, and the column sort is launched with
        // exactly as many slices as there are
        TGS_HIP(hipMemcpyAsync(ctx->pinned, ws + L.row_start, (uint64_t(grid.gy) + 1) * 4,
                               hipMemcpyDeviceToHost, strm));
        TGS_HIP(hipStreamSynchronize(strm));
        const uint32_t* rs = reinterpret_cast<const uint32_t*>(ctx->pinned);
        const uint64_t P = rs[grid.gy];
        st->pair_count = P;
        publish_offsets(st, L, grid, g->n, order, ws);
        if (P >= kSaturated)
            return fail(TGS_ERR_UNSUPPORTED, "2^32 - 1 or more pairs in one view");
        if (P > st->pair_capacity)
            return fail(TGS_ERR_CAPACITY, "%llu pairs needed, capacity %llu",
                        (unsigned long long)P, (unsigned long long)st->pair_capacity);
        slices = 0;
        for (int ty = 0; ty < grid.gy; ++ty)
            slices += (uint64_t(rs[ty + 1] - rs[ty]) + tgs::kSlice - 1) / tgs::kSlice;
    } else {
        // asynchronous: the count stays on the device; the emission and the
        // column sort are launched for the capacity's bound of slices and do
        // nothing when the count exceeds the capacity (the view then renders
        // the background); tgs_pair_counts reads the count later
        st->pair_count = TGS_PAIR_COUNT_PENDING;
        publish_offsets(st, L, grid, g->n, order, ws);
    }
    if ((s = enqueue_emit(ws, L, grid, g->n, order, dcount, slices, uint32_t(st->pair_capacity),
                          strm)) != TGS_OK)
        return s;
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
    tgs::Layout L;
    if ((s = check_state(st, n, grid, &L)) != TGS_OK) return s;
    if ((s = check_binned(st, L, grid, true)) != TGS_OK) return s;
    if ((s = use_device(ctx)) != TGS_OK) return s;
    tgs::RasterView v = raster_view(grid, *opt, *st, L);
    v.image = image;
    v.t_final = t_final;
    v.last_contrib = last_contrib;
    v.n_eval = n_eval;
    v.n_blend = n_blend;
    tgs::RasterViews t{};
    add_raster_view(t, v);
    TGS_HIP(tgs::launch_raster_fwd(opt->tile, ppt_of(*opt, grid.num_tiles()), lds_batch_of(*opt), t,
                                   static_cast<hipStream_t>(stream)));
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

tgs_status tgs_forward_static(tgs_context* ctx, const tgs_gaussians* g, const tgs_camera* cam,
                              const tgs_dilation* dil, const tgs_options* opt,
                              uint64_t pair_capacity, float* image, void* stream) {
    tgs_status s = check_gaussians(g);
    if (s == TGS_OK) s = check_common(cam, dil, opt);
    if (s == TGS_OK && !opt) s = fail(TGS_ERR_INVALID_ARG, "options is NULL");
    if (s != TGS_OK) return s;
    if (!image) return fail(TGS_ERR_INVALID_ARG, "image is NULL");
    if (pair_capacity == 0 || pair_capacity > kMaxPairCapacity)
        return fail(TGS_ERR_UNSUPPORTED, "pair_capacity %llu outside [1, %llu]",
                    (unsigned long long)pair_capacity, (unsigned long long)kMaxPairCapacity);
    const tgs::Grid grid = tgs::make_grid(*cam, *dil, opt->tile);
    const tgs::Layout L = tgs::make_layout(g->n, pair_capacity, grid);
    if (L.total > TGS_STATIC_SCRATCH_BYTES)
        return fail(TGS_ERR_UNSUPPORTED,
                    "%lld Gaussians, a %d x %d tile grid and %llu pairs need %llu bytes of "
                    "workspace, above the static scratch of %llu bytes",
                    (long long)g->n, grid.gx, grid.gy, (unsigned long long)pair_capacity,
                    (unsigned long long)L.total, (unsigned long long)TGS_STATIC_SCRATCH_BYTES);
    if (!ctx) return fail(TGS_ERR_INVALID_ARG, "context is NULL");
    if (!ctx->scratch) return fail(TGS_ERR_HIP, "the static scratch was not set up");
    // the same stages as tgs_forward on a state whose workspace is this
    // GPU's scratch; nothing in it has to start at zero (every stage writes
    // what it reads later in the call)
    tgs_state st{};
    st.workspace = ctx->scratch;
    st.workspace_bytes = TGS_STATIC_SCRATCH_BYTES;
    st.pair_capacity = pair_capacity;
    return tgs_forward(ctx, g, cam, dil, opt, &st, image, stream);
}

tgs_status tgs_l1_grad(tgs_context* ctx, const tgs_camera* cam, const tgs_dilation* dil,
                       const float* image, const float* target, float* dL_dimage, double* loss,
                       void* stream) {
    tgs_status s = check_common(cam, dil, nullptr);
    if (s != TGS_OK) return s;
    if (!image || !target || !dL_dimage) return fail(TGS_ERR_INVALID_ARG, "a buffer is NULL");
    if ((s = use_device(ctx)) != TGS_OK) return s;
    tgs::L1Views lt{};
    lt.count = 1;
    lt.v[0] = tgs::L1View{tgs::make_grid(*cam, *dil, 16), image, target, dL_dimage, loss};
    TGS_HIP(tgs::launch_l1_grad(lt, static_cast<hipStream_t>(stream)));
    return TGS_OK;
}

tgs_status tgs_raster_bwd(tgs_context* ctx, const tgs_camera* cam, const tgs_dilation* dil,
                          const tgs_options* opt, const tgs_state* st, int64_t n,
                          const float* dL_dimage, void* stream) {
    tgs_status s = check_common(cam, dil, opt);
    if (s == TGS_OK && !opt) s = fail(TGS_ERR_INVALID_ARG, "options is NULL");
    if (s != TGS_OK) return s;
    if (n < 0) return fail(TGS_ERR_INVALID_ARG, "n < 0");
    if (!dL_dimage) return fail(TGS_ERR_INVALID_ARG, "dL_dimage is NULL");
    const tgs::Grid grid = tgs::make_grid(*cam, *dil, opt->tile);
    tgs::Layout L;
    if ((s = check_state(st, n, grid, &L)) != TGS_OK) return s;
    if ((s = check_binned(st, L, grid, true)) != TGS_OK) return s;
    if ((s = use_device(ctx)) != TGS_OK) return s;
    auto strm = static_cast<hipStream_t>(stream);
    tgs::RasterView v = raster_view(grid, *opt, *st, L);
    v.dL = dL_dimage;
    TGS_HIP(tgs::fill_u32(reinterpret_cast<uint32_t*>(v.g2d), 0u, uint64_t(n) * tgs::kGrad2d, strm));
    tgs::RasterViews t{};
    add_raster_view(t, v);
    TGS_HIP(tgs::launch_raster_bwd(opt->tile, ppt_of(*opt, grid.num_tiles()), lds_batch_of(*opt), t,
                                   strm));
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
    tgs::PrepViews t{};
    t.count = 1;
    t.v[0] = prep_view(*cam, grid, static_cast<uint8_t*>(st->workspace), L);
    TGS_HIP(tgs::launch_preprocess_bwd(*g, t, *out, pos_stat, col_stat, visible,
                                       static_cast<hipStream_t>(stream)));
    return TGS_OK;
}

tgs_status tgs_backward(tgs_context* ctx, const tgs_gaussians* g, const tgs_camera* cam,
                        const tgs_dilation* dil, const tgs_options* opt, const tgs_state* st,
                        const float* dL_dimage, const tgs_grads* out, float* pos_stat,
                        float* col_stat, uint8_t* visible, void* stream) {
    tgs_status s = check_gaussians(g);
    if (s != TGS_OK) return s;
    s = tgs_raster_bwd(ctx, cam, dil, opt, st, g->n, dL_dimage, stream);
    if (s == TGS_OK)
        s = tgs_preprocess_bwd(ctx, g, cam, dil, opt, st, out, pos_stat, col_stat, visible, stream);
    return s;
}

// ---- batched views

namespace {

// Validation shared by the batched calls; fills the grids and layouts.
tgs_status check_views(int64_t n, int32_t views, const tgs_camera* cams, const tgs_dilation* dils,
                       const tgs_options* opt, const tgs_state* states, tgs::Grid* grids,
                       tgs::Layout* Ls) {
    if (n < 0) return fail(TGS_ERR_INVALID_ARG, "n < 0");
    if (views < 1 || views > TGS_MAX_VIEWS)
        return fail(TGS_ERR_INVALID_ARG, "views = %d must be in [1, %d]", views, TGS_MAX_VIEWS);
    if (!cams || !dils || !states) return fail(TGS_ERR_INVALID_ARG, "a per-view array is NULL");
    tgs_status s = check_options(opt);
    if (s != TGS_OK) return s;
    for (int v = 0; v < views; ++v) {
        if ((s = check_common(&cams[v], &dils[v], opt)) != TGS_OK)
            return fail(s, "view %d: %s", v, g_error.c_str());
        grids[v] = tgs::make_grid(cams[v], dils[v], opt->tile);
        if ((s = check_state(&states[v], n, grids[v], &Ls[v])) != TGS_OK)
            return fail(s, "view %d: %s", v, g_error.c_str());
        if (states[v].pair_capacity > kMaxPairCapacity)
            return fail(TGS_ERR_UNSUPPORTED, "view %d: pair capacity above 2^32 - 2", v);
    }
    // workspaces must be disjoint: the views are processed concurrently
    for (int a = 0; a < views; ++a) {
        const auto a0 = reinterpret_cast<uintptr_t>(states[a].workspace);
        for (int b = a + 1; b < views; ++b) {
            const auto b0 = reinterpret_cast<uintptr_t>(states[b].workspace);
            if (a0 < b0 + Ls[b].total && b0 < a0 + Ls[a].total)
                return fail(TGS_ERR_INVALID_ARG, "workspaces of views %d and %d overlap", a, b);
        }
    }
    return TGS_OK;
}

tgs_status check_binned_views(int32_t views, const tgs_state* states, const tgs::Grid* grids,
                              const tgs::Layout* Ls) {
    for (int v = 0; v < views; ++v) {
        tgs_status s = check_binned(&states[v], Ls[v], grids[v], true);
        if (s != TGS_OK) return fail(s, "view %d: %s", v, g_error.c_str());
    }
    return TGS_OK;
}

tgs_status check_io(int32_t views, const tgs_view_io* io, bool need_dL) {
    if (!io) return fail(TGS_ERR_INVALID_ARG, "io is NULL");
    for (int v = 0; v < views; ++v) {
        if (!need_dL && !io[v].image) return fail(TGS_ERR_INVALID_ARG, "view %d: image is NULL", v);
        if (need_dL && !io[v].dL_dimage)
            return fail(TGS_ERR_INVALID_ARG, "view %d: dL_dimage is NULL", v);
    }
    return TGS_OK;
}

tgs_status check_grads(const tgs_gaussians* g, const tgs_grads* out) {
    if (!out || (g->n > 0 && (!out->means || !out->scales || !out->quats || !out->opacities || !out->sh)))
        return fail(TGS_ERR_INVALID_ARG, "a gradient pointer is NULL");
    return TGS_OK;
}

#define TGS_CHECK(expr)                      \
    do {                                     \
        tgs_status s_ = (expr);              \
        if (s_ != TGS_OK) return s_;         \
    } while (0)

}  // namespace

tgs_status tgs_batch_preprocess_fwd(tgs_context* ctx, const tgs_gaussians* g, int32_t views,
                                    const tgs_camera* cams, const tgs_dilation* dils,
                                    const tgs_options* opt, tgs_state* states, void* stream) {
    tgs::Grid grids[TGS_MAX_VIEWS];
    tgs::Layout Ls[TGS_MAX_VIEWS];
    TGS_CHECK(check_gaussians(g));
    TGS_CHECK(check_views(g->n, views, cams, dils, opt, states, grids, Ls));
    TGS_CHECK(use_device(ctx));
    tgs::PrepViews pt{};
    pt.count = views;
    for (int v = 0; v < views; ++v)
        pt.v[v] = prep_view(cams[v], grids[v], static_cast<uint8_t*>(states[v].workspace), Ls[v]);
    TGS_HIP(tgs::launch_preprocess_fwd(*g, pt, static_cast<hipStream_t>(stream)));
    for (int v = 0; v < views; ++v) {
        states[v].pair_count = 0;
        states[v].key_bits = 0;
        auto* ws = static_cast<uint8_t*>(states[v].workspace);
        publish_offsets(&states[v], Ls[v], grids[v], g->n,
                        reinterpret_cast<const uint32_t*>(ws + Ls[v].depth_val[0]), ws);
    }
    return TGS_OK;
}

tgs_status tgs_batch_bin_sort(tgs_context* ctx, const tgs_gaussians* g, int32_t views,
                              const tgs_camera* cams, const tgs_dilation* dils,
                              const tgs_options* opt, tgs_state* states, void* stream) {
    tgs::Grid grids[TGS_MAX_VIEWS];
    tgs::Layout Ls[TGS_MAX_VIEWS];
    TGS_CHECK(check_gaussians(g));
    TGS_CHECK(check_views(g->n, views, cams, dils, opt, states, grids, Ls));
    TGS_CHECK(use_device(ctx));
    auto strm = static_cast<hipStream_t>(stream);
    // the views' binning chains are independent (each view has its own
    // workspace): spread them over the caller's stream and the auxiliary
    // streams, largest first onto the least loaded chain, forked from and
    // joined back into the caller's stream (a captured graph gets parallel
    // branches)
    const int chains = views > 1 ? std::min(views, kAuxStreams + 1) : 1;
    hipStream_t chain_stream[kAuxStreams + 1] = {strm};
    for (int a = 0; a + 1 < chains; ++a) chain_stream[a + 1] = ctx->aux[a];
    int chain_of[TGS_MAX_VIEWS];
    {
        uint64_t load[kAuxStreams + 1] = {};
        int idx[TGS_MAX_VIEWS];
        for (int v = 0; v < views; ++v) idx[v] = v;
        std::sort(idx, idx + views, [&](int a, int b) {
            return states[a].pair_capacity > states[b].pair_capacity;
        });
        for (int k = 0; k < views; ++k) {
            int best = 0;
            for (int c = 1; c < chains; ++c)
                if (load[c] < load[best]) best = c;
            chain_of[idx[k]] = best;
            load[best] += states[idx[k]].pair_capacity + uint64_t(g->n);
        }
    }
    if (chains > 1) {
        TGS_HIP(hipEventRecord(ctx->fork, strm));
        for (int c = 1; c < chains; ++c) TGS_HIP(hipStreamWaitEvent(chain_stream[c], ctx->fork, 0));
    }
    tgs_status status = TGS_OK;
    for (int v = 0; v < views && status == TGS_OK; ++v) {
        tgs_state& st = states[v];
        auto* ws = static_cast<uint8_t*>(st.workspace);
        const uint32_t cap = uint32_t(st.pair_capacity);
        int dres = 0;
        const uint32_t* order = nullptr;
        const uint32_t* dcount = nullptr;
        const uint64_t max_slices = tgs::bin_max_slices(cap, grids[v].gy);
        const hipStream_t vs = chain_stream[chain_of[v]];
        status = enqueue_counts(ws, Ls[v], grids[v], g->n, max_slices, vs, &dres, &order, &dcount);
        if (status == TGS_OK)
            status = enqueue_emit(ws, Ls[v], grids[v], g->n, order, dcount, max_slices, cap, vs);
        if (status == TGS_OK) publish_offsets(&st, Ls[v], grids[v], g->n, order, ws);
        st.pair_count = TGS_PAIR_COUNT_PENDING;
        st.key_bits = uint32_t(key_bits_for(grids[v].num_tiles()));
    }
    // join every chain, also after an error, so no stream is left forked
    for (int c = 1; c < chains; ++c) {
        TGS_HIP(hipEventRecord(ctx->join[c - 1], chain_stream[c]));
        TGS_HIP(hipStreamWaitEvent(strm, ctx->join[c - 1], 0));
    }
    return status;
}

tgs_status tgs_batch_raster_fwd(tgs_context* ctx, int64_t n, int32_t views, const tgs_camera* cams,
                                const tgs_dilation* dils, const tgs_options* opt,
                                const tgs_state* states, const tgs_view_io* io, void* stream) {
    tgs::Grid grids[TGS_MAX_VIEWS];
    tgs::Layout Ls[TGS_MAX_VIEWS];
    TGS_CHECK(check_views(n, views, cams, dils, opt, states, grids, Ls));
    TGS_CHECK(check_io(views, io, false));
    TGS_CHECK(check_binned_views(views, states, grids, Ls));
    TGS_CHECK(use_device(ctx));
    tgs::RasterViews rt{};
    for (int v = 0; v < views; ++v) {
        tgs::RasterView rv = raster_view(grids[v], *opt, states[v], Ls[v]);
        rv.image = io[v].image;
        rv.t_final = io[v].t_final;
        rv.last_contrib = io[v].last_contrib;
        rv.n_eval = io[v].n_eval;
        rv.n_blend = io[v].n_blend;
        rv.n_tested = io[v].n_tested;
        add_raster_view(rt, rv);
    }
    TGS_HIP(tgs::launch_raster_fwd(opt->tile, ppt_of(*opt, rt.first_block[rt.count]), lds_batch_of(*opt), rt,
                                   static_cast<hipStream_t>(stream)));
    return TGS_OK;
}

tgs_status tgs_batch_forward(tgs_context* ctx, const tgs_gaussians* g, int32_t views,
                             const tgs_camera* cams, const tgs_dilation* dils,
                             const tgs_options* opt, tgs_state* states, const tgs_view_io* io,
                             void* stream) {
    tgs::Grid grids[TGS_MAX_VIEWS];
    tgs::Layout Ls[TGS_MAX_VIEWS];
    TGS_CHECK(check_gaussians(g));
    TGS_CHECK(check_views(g->n, views, cams, dils, opt, states, grids, Ls));
    TGS_CHECK(check_io(views, io, false));
    TGS_CHECK(tgs_batch_preprocess_fwd(ctx, g, views, cams, dils, opt, states, stream));
    TGS_CHECK(tgs_batch_bin_sort(ctx, g, views, cams, dils, opt, states, stream));
    return tgs_batch_raster_fwd(ctx, g->n, views, cams, dils, opt, states, io, stream);
}

tgs_status tgs_batch_l1_grad(tgs_context* ctx, int32_t views, const tgs_camera* cams,
                             const tgs_dilation* dils, const tgs_view_io* io, double* loss,
                             void* stream) {
    if (views < 1 || views > TGS_MAX_VIEWS)
        return fail(TGS_ERR_INVALID_ARG, "views = %d must be in [1, %d]", views, TGS_MAX_VIEWS);
    if (!cams || !dils || !io) return fail(TGS_ERR_INVALID_ARG, "a per-view array is NULL");
    tgs_status s;
    for (int v = 0; v < views; ++v) {
        if ((s = check_common(&cams[v], &dils[v], nullptr)) != TGS_OK)
            return fail(s, "view %d: %s", v, g_error.c_str());
        if (!io[v].image || !io[v].target || !io[v].dL_dimage)
            return fail(TGS_ERR_INVALID_ARG, "view %d: a buffer is NULL", v);
    }
    TGS_CHECK(use_device(ctx));
    auto strm = static_cast<hipStream_t>(stream);
    tgs::L1Views lt{};
    lt.count = views;
    for (int v = 0; v < views; ++v)
        lt.v[v] = tgs::L1View{tgs::make_grid(cams[v], dils[v], 16), io[v].image, io[v].target,
                              io[v].dL_dimage, loss ? loss + v : nullptr};
    TGS_HIP(tgs::launch_l1_grad(lt, strm));
    return TGS_OK;
}

tgs_status tgs_batch_raster_bwd(tgs_context* ctx, int64_t n, int32_t views, const tgs_camera* cams,
                                const tgs_dilation* dils, const tgs_options* opt,
                                const tgs_state* states, const tgs_view_io* io, void* stream) {
    tgs::Grid grids[TGS_MAX_VIEWS];
    tgs::Layout Ls[TGS_MAX_VIEWS];
    TGS_CHECK(check_views(n, views, cams, dils, opt, states, grids, Ls));
    TGS_CHECK(check_io(views, io, true));
    TGS_CHECK(check_binned_views(views, states, grids, Ls));
    TGS_CHECK(use_device(ctx));
    auto strm = static_cast<hipStream_t>(stream);
    tgs::RasterViews rt{};
    for (int v = 0; v < views; ++v) {
        tgs::RasterView rv = raster_view(grids[v], *opt, states[v], Ls[v]);
        rv.dL = io[v].dL_dimage;
        TGS_HIP(tgs::fill_u32(reinterpret_cast<uint32_t*>(rv.g2d), 0u, uint64_t(n) * tgs::kGrad2d, strm));
        add_raster_view(rt, rv);
    }
    TGS_HIP(tgs::launch_raster_bwd(opt->tile, ppt_of(*opt, rt.first_block[rt.count]), lds_batch_of(*opt), rt,
                                   strm));
    return TGS_OK;
}

tgs_status tgs_batch_preprocess_bwd(tgs_context* ctx, const tgs_gaussians* g, int32_t views,
                                    const tgs_camera* cams, const tgs_dilation* dils,
                                    const tgs_options* opt, const tgs_state* states,
                                    const tgs_view_io* io, const tgs_grads* out, float* pos_stat,
                                    float* col_stat, uint8_t* visible, void* stream) {
    tgs::Grid grids[TGS_MAX_VIEWS];
    tgs::Layout Ls[TGS_MAX_VIEWS];
    TGS_CHECK(check_gaussians(g));
    TGS_CHECK(check_views(g->n, views, cams, dils, opt, states, grids, Ls));
    TGS_CHECK(check_grads(g, out));
    TGS_CHECK(use_device(ctx));
    tgs::PrepViews pt{};
    pt.count = views;
    for (int v = 0; v < views; ++v) {
        pt.v[v] = prep_view(cams[v], grids[v], static_cast<uint8_t*>(states[v].workspace), Ls[v]);
        if (io) {
            pt.v[v].pos_out = io[v].pos_stat;
            pt.v[v].col_out = io[v].col_stat;
            pt.v[v].vis_out = io[v].visible;
        }
    }
    TGS_HIP(tgs::launch_preprocess_bwd(*g, pt, *out, pos_stat, col_stat, visible,
                                       static_cast<hipStream_t>(stream)));
    return TGS_OK;
}

tgs_status tgs_batch_backward(tgs_context* ctx, const tgs_gaussians* g, int32_t views,
                              const tgs_camera* cams, const tgs_dilation* dils,
                              const tgs_options* opt, const tgs_state* states,
                              const tgs_view_io* io, const tgs_grads* out, float* pos_stat,
                              float* col_stat, uint8_t* visible, void* stream) {
    tgs::Grid grids[TGS_MAX_VIEWS];
    tgs::Layout Ls[TGS_MAX_VIEWS];
    TGS_CHECK(check_gaussians(g));
    TGS_CHECK(check_views(g->n, views, cams, dils, opt, states, grids, Ls));
    TGS_CHECK(check_grads(g, out));
    TGS_CHECK(check_io(views, io, true));
    TGS_CHECK(check_binned_views(views, states, grids, Ls));
    TGS_CHECK(tgs_batch_raster_bwd(ctx, g->n, views, cams, dils, opt, states, io, stream));
    return tgs_batch_preprocess_bwd(ctx, g, views, cams, dils, opt, states, io, out, pos_stat,
                                    col_stat, visible, stream);
}

tgs_status tgs_pair_counts(tgs_context* ctx, int32_t views, tgs_state* states, void* stream) {
    if (views < 1 || views > TGS_MAX_VIEWS)
        return fail(TGS_ERR_INVALID_ARG, "views = %d must be in [1, %d]", views, TGS_MAX_VIEWS);
    if (!states) return fail(TGS_ERR_INVALID_ARG, "states is NULL");
    for (int v = 0; v < views; ++v) {
        const tgs_state& st = states[v];
        if (!st.workspace || st.key_bits == 0 || st.off_pair_count + 4 > st.workspace_bytes)
            return fail(TGS_ERR_INVALID_ARG, "view %d has not been binned", v);
    }
    tgs_status s = use_device(ctx);
    if (s != TGS_OK) return s;
    auto strm = static_cast<hipStream_t>(stream);
    auto* pin = reinterpret_cast<uint32_t*>(ctx->pinned);
    for (int v = 0; v < views; ++v)
        TGS_HIP(hipMemcpyAsync(pin + v, static_cast<uint8_t*>(states[v].workspace) + states[v].off_pair_count,
                               4, hipMemcpyDeviceToHost, strm));
    TGS_HIP(hipStreamSynchronize(strm));
    int over = -1, huge = -1;
    for (int v = 0; v < views; ++v) {
        states[v].pair_count = pin[v];
        if (pin[v] > states[v].pair_capacity && over < 0) over = v;
        if (pin[v] >= kSaturated && huge < 0) huge = v;
    }
    if (huge >= 0)
        return fail(TGS_ERR_UNSUPPORTED, "view %d: 2^32 - 1 or more pairs in one view", huge);
    if (over >= 0)
        return fail(TGS_ERR_CAPACITY, "view %d: %llu pairs needed, capacity %llu", over,
                    (unsigned long long)states[over].pair_count,
                    (unsigned long long)states[over].pair_capacity);
    return TGS_OK;
}

tgs_status tgs_adam_step(tgs_context* ctx, const tgs_adam_group* groups, int32_t n_groups,
                         float beta1, float beta2, float eps, void* state, void* stream) {
    if (!groups) return fail(TGS_ERR_INVALID_ARG, "groups is NULL");
    if (n_groups < 1 || n_groups > TGS_MAX_ADAM_GROUPS)
        return fail(TGS_ERR_INVALID_ARG, "n_groups = %d must be in [1, %d]", n_groups,
                    TGS_MAX_ADAM_GROUPS);
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f))
        return fail(TGS_ERR_INVALID_ARG, "betas must lie in [0, 1)");
    if (!(eps > 0.0f) || !is_finite(eps)) return fail(TGS_ERR_INVALID_ARG, "eps must be positive");
    if (!state || reinterpret_cast<uintptr_t>(state) % 16 != 0)
        return fail(TGS_ERR_INVALID_ARG, "state must be a 16-byte aligned device buffer");
    tgs::AdamGroups t{};
    t.count = n_groups;
    for (int k = 0; k < n_groups; ++k) {
        const tgs_adam_group& G = groups[k];
        if (G.count < 0) return fail(TGS_ERR_INVALID_ARG, "group %d: count < 0", k);
        if (!(G.lr >= 0.0f) || !is_finite(G.lr))
            return fail(TGS_ERR_INVALID_ARG, "group %d: lr must be finite and >= 0", k);
        if (G.count > 0 && (!G.param || !G.grad || !G.exp_avg || !G.exp_avg_sq))
            return fail(TGS_ERR_INVALID_ARG, "group %d: a pointer is NULL", k);
        auto al = [](const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; };
        t.g[k] = tgs::AdamGroup{G.param, G.grad, G.exp_avg, G.exp_avg_sq, G.count, G.lr,
                                al(G.param) && al(G.grad) && al(G.exp_avg) && al(G.exp_avg_sq)};
    }
    TGS_CHECK(use_device(ctx));
    TGS_HIP(tgs::launch_adam(t, state, beta1, beta2, eps, static_cast<hipStream_t>(stream)));
    return TGS_OK;
}

tgs_status tgs_densify_query(int64_t n, uint64_t* workspace_bytes) {
    if (!workspace_bytes) return fail(TGS_ERR_INVALID_ARG, "workspace_bytes is NULL");
    if (n < 0) return fail(TGS_ERR_INVALID_ARG, "n < 0");
    if (n > int64_t(UINT32_MAX) - 1) return fail(TGS_ERR_UNSUPPORTED, "n exceeds 2^32 - 2");
    *workspace_bytes = tgs::densify_workspace_bytes(n);
    return TGS_OK;
}

tgs_status tgs_densify_select(tgs_context* ctx, int64_t n, const float* pos_sum,
                              const float* col_sum, const int32_t* count, float tau_pos,
                              float tau_col, int32_t color_active, int64_t budget,
                              uint8_t* selected, uint32_t* n_selected, void* workspace,
                              uint64_t workspace_bytes, void* stream) {
    if (n < 0) return fail(TGS_ERR_INVALID_ARG, "n < 0");
    if (n > int64_t(UINT32_MAX) - 1) return fail(TGS_ERR_UNSUPPORTED, "n exceeds 2^32 - 2");
    if (n > 0 && (!pos_sum || !count || !selected || (color_active && !col_sum)))
        return fail(TGS_ERR_INVALID_ARG, "a statistics or output pointer is NULL");
    if (!n_selected) return fail(TGS_ERR_INVALID_ARG, "n_selected is NULL");
    if (!(tau_pos > 0.0f) || !is_finite(tau_pos))
        return fail(TGS_ERR_INVALID_ARG, "tau_pos must be positive and finite");
    if (color_active && (!(tau_col > 0.0f) || !is_finite(tau_col)))
        return fail(TGS_ERR_INVALID_ARG, "tau_col must be positive and finite");
    if (budget < -1) return fail(TGS_ERR_INVALID_ARG, "budget must be >= -1");
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(TGS_ERR_INVALID_ARG, "workspace must be a 256-byte aligned device buffer");
    if (workspace_bytes < tgs::densify_workspace_bytes(n))
        return fail(TGS_ERR_INVALID_ARG, "workspace of %llu bytes < %llu required",
                    (unsigned long long)workspace_bytes,
                    (unsigned long long)tgs::densify_workspace_bytes(n));
    TGS_CHECK(use_device(ctx));
    TGS_HIP(tgs::launch_densify(n, pos_sum, col_sum, count, tau_pos, tau_col, color_active ? 1 : 0,
                                budget, selected, n_selected, static_cast<uint8_t*>(workspace),
                                static_cast<hipStream_t>(stream)));
    return TGS_OK;
}

}  // extern "C"
