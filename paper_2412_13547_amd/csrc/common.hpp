// Internal declarations shared by the HIP kernels and the C ABI of libtgs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "tgs.h"

namespace tgs {

constexpr float kNearDefault = 0.2f;
constexpr float kLowPass = 0.3f;       // px^2 added to the 2D covariance diagonal
constexpr float kFovGuard = 1.3f;      // x/z, y/z clamp, in units of W/(2 fx), H/(2 fy)
constexpr int kRecordBytes = 48;       // sizeof(tgs_record)
constexpr int kGrad2d = 9;             // dL/d(u, v, A, B, C, o, r, g, b)

// radix sort / scan tiling
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;   // keys per block and pass
constexpr int kRadixBits = 8;
constexpr int kRadixBuckets = 1 << kRadixBits;
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;
// binning: pairs per column-sort slice, and the widest tile grid supported
constexpr int kSlice = 4096;
constexpr int kMaxCols = 1024;

enum RecordFlags : uint32_t {
    kClampR = 1u, kClampG = 2u, kClampB = 4u, kCulled = 8u, kFovX = 16u, kFovY = 32u,
    kHasTiles = 64u           // only in the backward's flags word (Layout::jac)
};
constexpr int kJacWords = 10;   // Layout::jac: d rgb / d dir (3 x 3), then the flags word

struct Grid {
    int width, height;        // full resolution
    int stride, off_x, off_y;
    int tile;
    int w_ds, h_ds, gx, gy;
    __host__ __device__ int64_t num_tiles() const { return int64_t(gx) * gy; }
};

Grid make_grid(const tgs_camera& cam, const tgs_dilation& dil, int tile);

// Byte offsets of the sub-buffers of one view's workspace.
struct Layout {
    uint64_t records, tiles_touched;
    uint64_t rects;            // uint2[n], tile rectangle per Gaussian (packed, empty if culled)
    uint64_t srect;            // uint2[n], the same in depth order
    uint64_t depth_key[2], depth_val[2];
    uint64_t ecnt;             // uint32[gy * blocks + 1], entries per (row, block), then scanned
    uint64_t pcnt;             // uint32[gy * blocks + 1], pairs per (row, block), then scanned
    uint64_t row_start;        // uint32[gy + 1], first pair of every row
    uint64_t erow;             // uint32[gy + 1], first entry of every row
    uint64_t first_slice;      // uint32[gy + 1]
    uint64_t slice_desc;       // uint4[max_slices]: first entry, first pair, end pair,
                               //   tile row | last-slice-of-row << 31
    uint64_t slice_e1;         // uint32[max_slices], one past the slice's last entry
    uint64_t ent_id;           // uint32[capacity], Gaussian of each entry (row-bucketed)
    uint64_t ent_pp;           // uint32[capacity], first pair of each entry
    uint64_t ent_x;            // uint32[capacity], xlo | xhi << 16 of each entry
    uint64_t pair_vals;        // uint32[capacity], Gaussian of each pair, final order
    uint64_t col_hist;         // uint32[gx * max_slices], column histograms, then scanned
    uint64_t ranges;           // uint32[num_tiles][2]
    uint64_t tile_work;        // uint32[num_tiles], entries the forward walked per tile
    uint64_t tile_order;       // uint32[num_tiles], the backward's tile per workgroup
    uint64_t pix_tfinal;       // float[h_ds][w_ds], transmittance after each pixel's walk
    uint64_t pix_last;         // uint32[h_ds][w_ds], 1-based index of each pixel's last
                               //   blended list entry (0: none)
    uint64_t fwd_split;        // uint32: pixels per thread of the last forward
    uint64_t nonfinite;        // uint32: Gaussians the last preprocess culled for a
                               //   non-finite parameter (diagnostics)
    uint64_t jac;              // float[kJacWords][n]: d rgb_c / d dir_a at row 3c + a
                               //   (SH degree >= 1), written by a one-view preprocess
                               //   (the word after nonfinite is 1 when the last one
                               //   wrote them); row 9 the record's flags | kHasTiles as a
                               //   word, written by every preprocess.  It follows
                               //   tiles_touched directly (jac_rows)
    uint64_t blend_bits;       // uint64[max_tile_waves(T)][blend_words(capacity, tiles)]:
                               //   per wavefront slot of a tile and per 64 list entries
                               //   of the tile, the entries some pixel of that wavefront
                               //   blended (written by the forward)
    uint64_t grad2d;           // float[n][9]
    uint64_t sort_counts;      // uint32, radix digit counts, then the number of Gaussians
                               //   with tiles (at radix_kept_offset(n))
    uint64_t scan_partials;    // uint64, scan block sums
    uint64_t total;
};

Layout make_layout(int64_t n, uint64_t pair_capacity, const Grid& grid);

// Wavefronts of a tile of every work split of a tile size (T = 8: 1; T = 16:
// up to 4; T = 32: up to 8), and the 64-bit words of one wavefront slot's
// blend bits.  Chunk c (entries [64 c, 64 c + 64) of the list) of the tile
// whose pairs start at s has word floor(s / 64) + tile + c: every (tile,
// chunk) owns a word of its own, so the forward writes them without
// atomics or clearing.
inline int max_tile_waves(int tile) { return tile == 8 ? 1 : tile == 16 ? 4 : 8; }
inline uint64_t blend_words(uint64_t capacity, int64_t tiles) {
    return (capacity + 63) / 64 + uint64_t(tiles) + 1;
}

// Device kernel launchers (stream-ordered, no synchronisation).
struct CamDev {
    float R[9], t[3];
    float campos[3];          // -R^T t, camera centre in world space
    float fx, fy, cx, cy;
    float near_z;
    int width, height;
};
CamDev make_cam(const tgs_camera& c);

// Views of one launch.  Kernels that serve several views at once take a
// table of up to kMaxViews views by value (kernel arguments stay well below
// the 4 KiB argument segment).
constexpr int kMaxViews = 16;

// One view of the per-Gaussian preprocess.
struct PrepView {
    CamDev cam;
    Grid grid;
    tgs_record* rec;          // forward out / backward in
    uint32_t* touched;        // forward out / backward in
    uint2* rects;             // forward out: packed tile rectangle (pack_rect)
    uint32_t* depth_key;      // forward out
    uint32_t* depth_val;      // forward out
    const float* g2d;         // backward in
    uint32_t* nonfinite;      // forward out: count of Gaussians culled for non-finite input
    float* pos_out;           // backward, optional: this view's positional statistic
    float* col_out;           // backward, optional: this view's appearance statistic
    uint8_t* vis_out;         // backward, optional: 1 where this view sees the Gaussian
};

// Layout::jac of a view of n Gaussians (it follows the tile counts, whose
// size rounds up to the 256-byte alignment of the workspace's arrays), and
// the word beside the non-finite counter that says whether it is current.
__host__ __device__ inline float* jac_rows(const PrepView& v, int64_t n) {
    return reinterpret_cast<float*>(v.touched + ((n + 63) / 64) * 64);
}
__host__ __device__ inline uint32_t* jac_current(const PrepView& v) { return v.nonfinite + 1; }
struct PrepViews {
    int count;
    PrepView v[kMaxViews];
};
static_assert(sizeof(PrepViews) <= 3584, "preprocess view table too large for kernel arguments");

// Zeroes every view's non-finite counter, then the per-Gaussian preprocess.
hipError_t launch_preprocess_fwd(const tgs_gaussians& g, const PrepViews& views, hipStream_t s);
// Gradients summed over the views; statistics summed over the views where the
// Gaussian is visible, visible = number of such views.
hipError_t launch_preprocess_bwd(const tgs_gaussians& g, const PrepViews& views,
                                 const tgs_grads& out, float* pos_stat, float* col_stat,
                                 uint8_t* visible, hipStream_t s);

// Stable LSD radix sort of (key, value) uint32 pairs on bits [0, bits).
// Returns the index (0 or 1) of the buffer pair holding the result.  With
// drop_on, the pairs whose key equals drop are left out; the number of pairs
// kept is then counts[radix_kept_offset(count)] on the device (the result
// holds that many).  counts needs radix_counts_elems(count) entries.
int radix_sort_passes(int bits);
hipError_t radix_sort(uint32_t* const keys[2], uint32_t* const vals[2], uint64_t count, int bits,
                      uint32_t* counts, uint64_t* partials, int* result, hipStream_t s,
                      bool drop_on = false, uint32_t drop = 0u);
uint64_t radix_counts_elems(uint64_t count);
uint64_t radix_kept_offset(uint64_t count);

// Exclusive scan of uint32 (in may equal out); with write_total, out[count]
// receives the total (out then has count + 1 entries).
hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, uint64_t count,
                              uint64_t* partials, bool write_total, hipStream_t s);
// The same for two arrays of one length in the same launches (partials needs
// room for both arrays' tile sums).
hipError_t exclusive_scan_u32_pair(const uint32_t* in0, uint32_t* out0, const uint32_t* in1,
                                   uint32_t* out1, uint64_t count, uint64_t* partials,
                                   bool write_total, hipStream_t s);
uint64_t scan_partials_elems(uint64_t count);

// binning (binning.hip).  The pair count lives on the device (row_start[gy]);
// the entry emission and the column sort do nothing when it exceeds
// `capacity` (and the column sort then writes empty ranges), so the stage
// can be enqueued without reading the count back.
uint32_t bin_blocks(int64_t n);
uint64_t bin_max_slices(uint64_t pairs, int gy);
// `order` holds the Gaussians with tiles in depth order; their number is
// min(n, *dcount) when dcount is given (device), n otherwise.
hipError_t launch_counts(const uint8_t* ws, const Layout& L, const uint32_t* order, int64_t n,
                         const uint32_t* dcount, const Grid& grid, hipStream_t s);
hipError_t launch_row_setup(uint8_t* ws, const Layout& L, int64_t n, const Grid& grid,
                            uint64_t max_slices, hipStream_t s);
hipError_t launch_entries(uint8_t* ws, const Layout& L, const uint32_t* order, int64_t n,
                          const uint32_t* dcount, const Grid& grid, uint32_t capacity,
                          hipStream_t s);
// Stable counting sort of every row bucket by column, and the tile ranges;
// `slices` bounds the number of column-sort slices from above.
hipError_t launch_col_sort(uint8_t* ws, const Layout& L, const Grid& grid, uint64_t slices,
                           uint32_t capacity, hipStream_t s);
// One-time kernel attributes (the column scatter of the widest grid needs
// more than 64 KiB of LDS).
hipError_t prepare_binning_kernels();

// One view of a raster launch.
struct RasterView {
    Grid grid;
    uint32_t capacity;        // pairs the view's buffers hold
    float bg[3];
    const float4* rec;        // tgs_record[n] as 3 float4
    const uint32_t* ranges;   // [num_tiles][2]
    const uint32_t* vals;     // pair values in (tile, depth, index) order
    const uint32_t* pair_count;   // device: pairs binned; above capacity = overflow
    float* image;             // forward out (may be null)
    float* ws_tfinal;         // forward out / backward in: per-pixel final transmittance
    uint32_t* ws_last;        // forward out / backward in: per-pixel last blended entry
    float* t_final;           // forward, optional copy of ws_tfinal for the caller
    uint32_t* last_contrib;   // forward, optional copy of ws_last for the caller
    uint32_t* n_eval;         // forward, optional
    uint32_t* n_blend;        // forward, optional
    uint32_t* n_tested;       // forward, optional: entries evaluated pixel by pixel
    const float* dL;          // backward in
    float* g2d;               // backward out (accumulated; zero it first)
    uint32_t* work;           // forward out, optional: entries walked per tile
    uint32_t* order;          // backward, optional: the tile of each workgroup, a
                              //   permutation of the tiles written before the walk
    unsigned long long* bits; // forward out / backward in: blend bits,
                              //   bits_stride words per wavefront slot
    uint64_t bits_stride;
    uint32_t* fwd_split;      // forward out / backward in: the work split (pixels per
                              //   thread) the bits were written with
};
struct RasterViews {
    int count;
    uint32_t first_block[kMaxViews + 1];   // workgroups of views [0, v): prefix of tile counts
    RasterView v[kMaxViews];
};
static_assert(sizeof(RasterViews) <= 3584, "raster view table too large for kernel arguments");

// Defaults of the launch options of a tile size: splat records per LDS round
// (64, 128 or 256) and pixels per thread (T = 8: 1; T = 16: 1, 2, 4;
// T = 32: 2, 4).  Results do not depend on either.
int default_lds_batch(int tile);
int default_pixels_per_thread(int tile);
// The default work split of a launch over `tiles` tiles (all its views'):
// fewer pixels per thread, hence more wavefronts per tile, when the tiles
// alone would leave SIMDs idle (measured at 1080p-4K, strides 1-4).
int default_pixels_per_thread(int tile, int64_t tiles);
hipError_t launch_raster_fwd(int tile, int ppt, int lds_batch, const RasterViews& views,
                             hipStream_t s);
hipError_t launch_raster_bwd(int tile, int ppt, int lds_batch, const RasterViews& views,
                             hipStream_t s);
// L1 loss and gradient of a table of views in one launch (loss may be null).
struct L1View {
    Grid grid;
    const float* image;
    const float* target;
    float* dL;
    double* loss;
};
struct L1Views {
    int count;
    uint32_t first_block[kMaxViews + 1];   // filled by launch_l1_grad
    L1View v[kMaxViews];
};
static_assert(sizeof(L1Views) <= 3584, "L1 view table too large for kernel arguments");
hipError_t launch_l1_grad(L1Views& views, hipStream_t s);

// Fused Adam (optim.hip): a table of parameter groups, the step counter and
// bias corrections in a small device buffer.
constexpr int kMaxAdamGroups = 8;
struct AdamGroup {
    float* param;
    const float* grad;
    float* exp_avg;
    float* exp_avg_sq;
    int64_t count;
    float lr;
    int vec4;                 // all four arrays 16-byte aligned
};
struct AdamGroups {
    int count;
    AdamGroup g[kMaxAdamGroups];
};
hipError_t launch_adam(const AdamGroups& groups, void* coeffs, float b1, float b2, float eps,
                       hipStream_t s);

// Densification selection (densify.hip).
uint64_t densify_workspace_bytes(int64_t n);
hipError_t launch_densify(int64_t n, const float* pos, const float* col, const int32_t* count,
                          float tau_pos, float tau_col, int color, int64_t budget,
                          uint8_t* selected, uint32_t* n_selected, uint8_t* ws, hipStream_t s);

hipError_t fill_u32(uint32_t* p, uint32_t value, uint64_t count, hipStream_t s);

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// Downsampled tile rectangle [xlo, xhi) x [ylo, yhi) of a splat centred at
// full-resolution (u, v) with integer radius r (Sec. 4.1 Eq. 3-4, read as the
// inverse of Eq. 5): u_ds = (u - (d-1)/2) / d, r_ds = r / d, and the tiles
// holding a downsampled pixel in [u_ds - r_ds, u_ds + r_ds].  Evaluated in
// IEEE double in a fixed order so every stage gets the same integers.
struct Rect { int xlo, xhi, ylo, yhi; };

// A rectangle in 8 bytes: (xlo | xhi << 16, ylo | yhi << 16); grids are far
// below 65536 tiles a side.
__host__ __device__ inline uint2 pack_rect(const Rect& r) {
    return make_uint2(uint32_t(r.xlo) | (uint32_t(r.xhi) << 16),
                      uint32_t(r.ylo) | (uint32_t(r.yhi) << 16));
}
__host__ __device__ inline Rect unpack_rect(uint2 p) {
    return Rect{int(p.x & 0xFFFFu), int(p.x >> 16), int(p.y & 0xFFFFu), int(p.y >> 16)};
}
__host__ __device__ inline Rect tile_rect(float u, float v, int radius, const Grid& g) {
    const double d = double(g.stride), T = double(g.tile);
    const double half = 0.5 * double(g.stride - 1);
    const double ud = (double(u) - half) / d;
    const double vd = (double(v) - half) / d;
    const double rd = double(radius) / d;
    const double gx = double(g.gx), gy = double(g.gy);
    Rect r;
    r.xlo = int(fmin(fmax(floor((ud - rd) / T), 0.0), gx));
    r.xhi = int(fmin(fmax(floor((ud + rd) / T) + 1.0, 0.0), gx));
    r.ylo = int(fmin(fmax(floor((vd - rd) / T), 0.0), gy));
    r.yhi = int(fmin(fmax(floor((vd + rd) / T) + 1.0, 0.0), gy));
    return r;
}

}  // namespace tgs
