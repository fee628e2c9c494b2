/*
 * tgs.h - C ABI of libtgs, the dilated differentiable Gaussian-splat rasterizer
 * for AMD Instinct MI355X (gfx950).
 *
 * The operation is the hot path of one fitting iteration of Turbo-GS
 * (arXiv 2412.13547): Gaussian parameters (Sec. 3, Eq. 1 and the SH colour
 * model), a pinhole camera with its ORIGINAL focal length (Sec. 4.1) and a
 * dilation pattern (stride d, offsets o_x, o_y; Sec. 4.1 and Fig. 2) go in;
 * the downsampled image of that pattern (Sec. 4.1, Eq. 3-5) and the
 * gradients of a loss with respect to every Gaussian attribute, with the
 * per-Gaussian densification statistics of Sec. 4.3, come out.
 *
 * Conventions shared by every call
 *  - Pointers named "device" point to HIP device memory; everything else is
 *    host memory.  The caller allocates every device buffer and keeps
 *    ownership; the library never frees caller memory.
 *  - All float data is IEEE float32, structure-of-arrays:
 *      means[3][n], scales[3][n] (positive, already exponentiated),
 *      quats[4][n] (w, x, y, z; normalised inside), opacities[n] (in [0,1],
 *      already passed through a sigmoid), sh[sh_coeffs][3][n].
 *    Images are planar: image[3][H_ds][W_ds], row-major per channel.
 *  - The dilated image of (d, o_x, o_y) has W_ds = ceil((W - o_x) / d),
 *    H_ds = ceil((H - o_y) / d) pixels; downsampled pixel (i, j) is rendered
 *    at full-resolution pixel (d i + o_x, d j + o_y), whose centre is at those
 *    integer coordinates.
 *  - Device work is enqueued on the given stream and calls return before it
 *    finishes; no call synchronises except tgs_pair_counts and, when the
 *    caller opts in with TGS_SYNC_CHECK in tgs_options.flags, tgs_bin_sort /
 *    tgs_forward (see tgs_bin_sort).  Without that flag a whole fitting step,
 *    single-view or batched, can be captured in one HIP graph.
 *  - Arguments are validated on the host before any HIP call; a failing call
 *    has enqueued nothing.  No C++ exception crosses this interface.
 *    tgs_last_error() returns a thread-local description of the last failure.
 *  - Not thread-safe per context: calls that share a context or a workspace
 *    must be ordered by the caller.
 */
#ifndef TGS_H
#define TGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tgs_status {
    TGS_OK = 0,
    TGS_ERR_INVALID_ARG = 1, /* a pointer, size or option is out of range      */
    TGS_ERR_CAPACITY = 2,    /* the workspace holds fewer pairs than required  */
    TGS_ERR_HIP = 3,         /* a HIP runtime call failed                      */
    TGS_ERR_NO_DEVICE = 4,   /* no HIP device with the requested ordinal       */
    TGS_ERR_UNSUPPORTED = 5  /* a valid request the library does not implement */
} tgs_status;

/* Pinhole camera, OpenCV axes (x right, y down, z forward). */
typedef struct tgs_camera {
    int32_t width, height;   /* full-resolution image size in pixels (> 0)     */
    float fx, fy, cx, cy;    /* focal lengths and principal point, full-res px */
    float world_to_cam[12];  /* row-major 3x4 [R | t]: x_cam = R x_world + t    */
    float near_z;            /* Gaussians with camera depth <= near_z are culled;
                                positive and finite (else TGS_ERR_INVALID_ARG) */
} tgs_camera;

/* Dilation pattern of Sec. 4.1: stride d >= 1, 0 <= off_x, off_y < d.
 * d = 1, offsets 0 is the plain full-resolution renderer. */
typedef struct tgs_dilation {
    int32_t stride, off_x, off_y;
} tgs_dilation;

typedef struct tgs_gaussians {
    int64_t n;               /* number of Gaussians, >= 0                        */
    int32_t sh_degree;       /* active SH degree, 0..3                            */
    int32_t sh_coeffs;       /* coefficients allocated per channel, >= (deg+1)^2  */
    const float* means;      /* device [3][n]                                     */
    const float* scales;     /* device [3][n]                                     */
    const float* quats;      /* device [4][n]                                     */
    const float* opacities;  /* device [n]                                        */
    const float* sh;         /* device [sh_coeffs][3][n]                          */
} tgs_gaussians;

typedef struct tgs_options {
    int32_t tile;            /* tile edge T in downsampled pixels: 8, 16 or 32.
                                The paper fixes 16 (Sec. 4.1); T changes which
                                Gaussians a pixel considers, hence the result.  */
    int32_t lds_batch;       /* splat records staged in LDS per round by the
                                rasterizer: 64, 128 or 256, or 0 for the default
                                of the tile size.  Speed only; results do not
                                depend on it.                                    */
    int32_t pixels_per_thread; /* rasterizer work split: 1, 2 or 4 pixels per
                                thread (tile 8: 1; tile 16: 1, 2, 4; tile 32:
                                2, 4), or 0 for the default of the tile size.
                                Speed only; results do not depend on it.        */
    float bg[3];             /* background colour added with the final T         */
    uint32_t flags;          /* 0 or TGS_SYNC_CHECK; other bits are invalid      */
} tgs_options;

/* tgs_options.flags: tgs_bin_sort (and tgs_forward) read the pair count back
 * (one stream synchronisation) and report TGS_ERR_CAPACITY at once.  Without
 * it the count stays on the device (see tgs_bin_sort). */
#define TGS_SYNC_CHECK 1u

/* Pair capacity limit of one view: the device pair count is a saturating
 * uint32, so 2^32 - 1 or more pairs in one view cannot be represented; such a
 * view is reported as TGS_ERR_UNSUPPORTED (it renders the background). */
#define TGS_MAX_PAIR_CAPACITY 4294967294ull

/* Gradients, same layout as the parameters; every array is overwritten. */
typedef struct tgs_grads {
    float* means;            /* device [3][n]          */
    float* scales;           /* device [3][n]          */
    float* quats;            /* device [4][n]          */
    float* opacities;        /* device [n]             */
    float* sh;               /* device [sh_coeffs][3][n]; rows >= (deg+1)^2 are 0 */
} tgs_grads;

/* Sizes of one view, filled by tgs_query_sizes (host only).  The tile grid
 * may be at most 1024 tiles wide and 4096 tall (TGS_ERR_UNSUPPORTED). */
typedef struct tgs_sizes {
    int32_t w_ds, h_ds;      /* downsampled image size                           */
    int32_t grid_x, grid_y;  /* tile grid of the downsampled image               */
    int64_t num_tiles;
    int64_t pixels;          /* w_ds * h_ds                                      */
    uint64_t pair_capacity;  /* capacity the workspace size below is for        */
    uint64_t workspace_bytes;
} tgs_sizes;

/* Device layout of the per-Gaussian record written by the preprocess and read
 * by the other stages (48 bytes, 16-byte aligned):
 *   u, v      splat centre in full-resolution pixels
 *   A, B, C   conic: inverse of the low-passed 2D covariance
 *   opacity   the Gaussian's opacity
 *   r, g, b   colour after the clamp at 0
 *   z         camera-space depth
 *   radius    ceil(3 sqrt(lambda_max)) in full-resolution pixels, 0 if culled
 *   flags     bit 0..2: colour channel clamped; bit 3: culled;
 *             bit 4 / 5: x / y FoV guard active                              */
typedef struct tgs_record {
    float u, v, A, B;
    float C, opacity, r, g;
    float b, z;
    int32_t radius;
    uint32_t flags;
} tgs_record;

/* Per-view state inside a caller-allocated workspace.  The caller sets the
 * three input fields; tgs_forward / tgs_bin_sort fill the rest.  The byte
 * offsets locate results inside the workspace for inspection. */
typedef struct tgs_state {
    void* workspace;             /* in: device, >= tgs_sizes.workspace_bytes, 256-aligned */
    uint64_t workspace_bytes;    /* in */
    uint64_t pair_capacity;      /* in: the capacity passed to tgs_query_sizes           */
    uint64_t pair_count;         /* out: tile-Gaussian pairs of the last bin/sort        */
    uint32_t key_bits;           /* out: tile-id bits sorted                             */
    uint32_t reserved;
    uint64_t off_records;        /* out: tgs_record[n]                                    */
    uint64_t off_tiles_touched;  /* out: uint32[n], ds tiles each Gaussian overlaps       */
    uint64_t off_depth_order;    /* out: uint32[n]; its first m entries are the ids of the
                                         m Gaussians with tiles, sorted by depth key (equal
                                         keys by id); the rest is unspecified            */
    uint64_t off_pair_vals;      /* out: uint32[pair_count], Gaussian id of each pair in
                                         (tile, depth, index) order                      */
    uint64_t off_ranges;         /* out: uint32[num_tiles][2], [start, end) per tile      */
    uint64_t off_grad2d;         /* out: float[n][9], dL/d(u,v,A,B,C,o,r,g,b) (backward)  */
    uint64_t off_pair_count;     /* out: uint32, the pair count on the device; above
                                         pair_capacity when a batched bin/sort overflowed */
    uint64_t off_depth_count;    /* out: uint32 on the device, m of off_depth_order;
                                         valid once a bin/sort of this state has run     */
    uint64_t off_tile_work;      /* out: uint32[num_tiles], the entries the last forward
                                         walked in each tile (at most the tile's pairs).
                                         The backward takes the tiles heaviest first by
                                         them, and so does the next forward on this
                                         workspace before it overwrites them.  Any values
                                         give the same results: they only order the work */
    uint64_t off_t_final;        /* out: float[H_ds][W_ds], every pixel's transmittance
                                         after its walk, written by the last forward      */
    uint64_t off_last_contrib;   /* out: uint32[H_ds][W_ds], 1-based index of every
                                         pixel's last blended list entry (0: none), written
                                         by the last forward; with off_t_final, what the
                                         backward reads                                  */
    uint64_t off_nonfinite_count;/* out: uint32 on the device, the Gaussians the last
                                         preprocess culled because a parameter was not
                                         finite (diagnostics)                            */
} tgs_state;

/* st->pair_count after a batched bin/sort, until tgs_pair_counts reads the
 * device count back. */
#define TGS_PAIR_COUNT_PENDING UINT64_MAX

/* Most views of one batched call. */
#define TGS_MAX_VIEWS 16

/* Per-view device buffers of the batched calls. */
typedef struct tgs_view_io {
    float* image;            /* [3][H_ds][W_ds]; written by the forward (the backward does not
                                read it)                                                    */
    float* t_final;          /* optional [H_ds][W_ds] float, as tgs_raster_fwd               */
    uint32_t* last_contrib;  /* optional [H_ds][W_ds]                                        */
    uint32_t* n_eval;        /* optional [H_ds][W_ds]                                        */
    uint32_t* n_blend;       /* optional [H_ds][W_ds]                                        */
    const float* target;     /* [3][H][W] full-resolution target (tgs_batch_l1_grad)         */
    float* dL_dimage;        /* [3][H_ds][W_ds]; written by tgs_batch_l1_grad, read by the
                                backward                                                    */
    uint32_t* n_tested;      /* optional [H_ds][W_ds]: of the entries the pixel examined, those
                                its wavefront evaluated pixel by pixel (the others it skipped
                                on a bound over its 8 x 8 pixel block); a measure of the
                                rasterizer's work, not of the method's result              */
    float* pos_stat;         /* optional [n]: this view's positional statistic (Sec. 4.3),
                                written by the batched preprocess backward                  */
    float* col_stat;         /* optional [n]: this view's appearance statistic               */
    uint8_t* visible;        /* optional [n]: 1 where this view sees the Gaussian            */
} tgs_view_io;

typedef struct tgs_context tgs_context;

const char* tgs_status_str(tgs_status s);
/* Thread-local text of the last failure in this thread ("" if none). */
const char* tgs_last_error(void);
/* Library version string. */
const char* tgs_version(void);

/* Create a context bound to HIP device `device`.  Returns TGS_ERR_NO_DEVICE
 * when the device does not exist.  The context owns a small pinned host
 * buffer; release with tgs_destroy. */
tgs_status tgs_create(int device, tgs_context** out);
void tgs_destroy(tgs_context* ctx);

/* Host only, no device needed.  Sizes of one view: downsampled image, tile
 * grid (Sec. 4.1: T x T tiles of the downsampled image) and the workspace
 * bytes needed for n Gaussians and up to pair_capacity tile-Gaussian pairs. */
tgs_status tgs_query_sizes(int64_t n, const tgs_camera* cam, const tgs_dilation* dil,
                           const tgs_options* opt, uint64_t pair_capacity, tgs_sizes* out);

/* Host only, no device needed.  The rasterizer launch a tile size gets when
 * tgs_options leaves lds_batch and pixels_per_thread at 0: the LDS batch and
 * pixels per thread written to *lds_batch and *pixels_per_thread, for a
 * launch of many tiles.  A launch whose tiles (all its views') would leave
 * SIMDs idle gets fewer pixels per thread: at T = 16, 2 below 6144 tiles and
 * 1 below 3072; at T = 32, 2 below 1536.  Results do not depend on it.
 * Returns TGS_ERR_INVALID_ARG for a tile other than 8, 16 or 32 or a NULL
 * output. */
tgs_status tgs_default_launch(int32_t tile, int32_t* lds_batch, int32_t* pixels_per_thread);

/* Stage (a), Sec. 3 and Sec. 4.1: per Gaussian, view transform, near cull,
 * Sigma = R S S^T R^T, EWA projection with the full-resolution focal length
 * plus a 0.3 px^2 low-pass, conic, radius, SH colour, and the number of
 * tiles of the DOWNSAMPLED grid its box [u_ds +- r/d] x [v_ds +- r/d]
 * overlaps, with u_ds = (u - (d-1)/2) / d (Eq. 3-4 read as the inverse of
 * Eq. 5).  Writes records and tiles_touched into the workspace, and for
 * tgs_preprocess_bwd the colour's Jacobian in the view direction (the
 * coefficients' only other use in the backward). */
tgs_status tgs_preprocess_fwd(tgs_context* ctx, const tgs_gaussians* g, const tgs_camera* cam,
                              const tgs_dilation* dil, const tgs_options* opt, tgs_state* st,
                              void* stream);

/* Stage (b), Sec. 4.1 and Sec. 3 ("sorted by depth ... tile-based
 * rasterizer"): one pair per (Gaussian, overlapped tile), sorted by the key
 * (tile id, float32 depth bits), equal keys in ascending Gaussian index, and
 * the [start, end) range of every tile.  Requires tgs_preprocess_fwd on the
 * same state.
 * Default (opt->flags without TGS_SYNC_CHECK): asynchronous.  The pair count
 * stays on the device (st->off_pair_count) and st->pair_count is set to
 * TGS_PAIR_COUNT_PENDING; when the count exceeds pair_capacity no pair is
 * written, every tile range is empty (the raster stages render the
 * background and backpropagate zero), and tgs_pair_counts later reports
 * TGS_ERR_CAPACITY with the required count.
 * With TGS_SYNC_CHECK: the count is read back to the host (one stream
 * synchronisation) into st->pair_count; if it exceeds pair_capacity nothing
 * more is enqueued and TGS_ERR_CAPACITY is returned.
 * Either way 2^32 - 1 or more pairs give TGS_ERR_UNSUPPORTED (at once, or
 * from tgs_pair_counts); pair_capacity above TGS_MAX_PAIR_CAPACITY is
 * TGS_ERR_UNSUPPORTED. */
tgs_status tgs_bin_sort(tgs_context* ctx, const tgs_gaussians* g, const tgs_camera* cam,
                        const tgs_dilation* dil, const tgs_options* opt, tgs_state* st,
                        void* stream);

/* Stage (c), Sec. 3 Eq. 2 on the dilated pixels of Sec. 4.1 (Eq. 5, Fig. 2):
 * each downsampled pixel walks its tile's list front to back with
 * alpha = min(0.99, o exp(-1/2 d^T Sigma^-1 d)), skips alpha < 1/255, stops
 * before the entry that would take T below 1e-4, and outputs C + T bg.
 * image: device [3][H_ds][W_ds], or NULL to write only the per-pixel state
 * the backward reads.  That state -- every pixel's final transmittance and
 * the 1-based index of its last blended list entry -- always goes to the
 * workspace (st->off_t_final, st->off_last_contrib).  Optional (may be NULL)
 * device outputs per downsampled pixel: t_final float and last_contrib
 * uint32 (copies of that state), n_eval uint32 (entries examined, stop
 * included), n_blend uint32 (entries blended). */
tgs_status tgs_raster_fwd(tgs_context* ctx, const tgs_camera* cam, const tgs_dilation* dil,
                          const tgs_options* opt, const tgs_state* st, int64_t n, float* image,
                          float* t_final, uint32_t* last_contrib, uint32_t* n_eval,
                          uint32_t* n_blend, void* stream);

/* Stages (a)-(c) in order.  Same arguments and outputs as the three calls. */
tgs_status tgs_forward(tgs_context* ctx, const tgs_gaussians* g, const tgs_camera* cam,
                       const tgs_dilation* dil, const tgs_options* opt, tgs_state* st,
                       float* image, void* stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid it): tgs_forward without a
 * caller workspace.  Every intermediate lives in a static device array of
 * TGS_STATIC_SCRATCH_BYTES bytes that each GPU the library runs on holds
 * from the library's load to the end of the process; the call allocates
 * nothing.  The caller passes the Gaussians, camera, dilation, options and
 * the image [3][H_ds][W_ds] (device) and chooses pair_capacity.  A request
 * whose workspace (n Gaussians, the tile grid, pair_capacity pairs; the
 * bytes tgs_query_sizes reports) exceeds the array returns
 * TGS_ERR_UNSUPPORTED before any device work.  Pairs beyond pair_capacity
 * behave as in tgs_bin_sort: asynchronous by default (the image is the
 * background), or TGS_ERR_CAPACITY with TGS_SYNC_CHECK in opt->flags.
 * All calls on one GPU share its array and the array keeps the last call's
 * contents: calls that overlap on one GPU (other streams, other threads)
 * race, and no state survives for a backward. */
#define TGS_STATIC_SCRATCH_BYTES (64ull << 20)
tgs_status tgs_forward_static(tgs_context* ctx, const tgs_gaussians* g, const tgs_camera* cam,
                              const tgs_dilation* dil, const tgs_options* opt,
                              uint64_t pair_capacity, float* image, void* stream);

/* L1 photometric loss of Sec. 4.1 / Fig. 2: each rendered pixel against the
 * full-resolution target pixel it was rendered at.  L = mean over rendered
 * pixels and channels of |image - target|; dL_dimage = sign(.) / (3 W_ds H_ds)
 * with sign(0) = 0.  target: device [3][H][W]; dL_dimage: device
 * [3][H_ds][W_ds]; loss: device double[1], overwritten (may be NULL). */
tgs_status tgs_l1_grad(tgs_context* ctx, const tgs_camera* cam, const tgs_dilation* dil,
                       const float* image, const float* target, float* dL_dimage, double* loss,
                       void* stream);

/* Stage (d1): the derivative of the forward (Sec. 3 Eq. 2; the paper's
 * backward follows prior work) with respect to every splat's
 * (u, v, A, B, C, o, r, g, b), summed over the rendered pixels, into the
 * workspace's float[n][9] grad2d.  Every pixel walks its list back to front
 * from the last entry it blended, starting from the final transmittance;
 * both come from the last tgs_raster_fwd on this state (which must be the
 * forward being differentiated).  The transmittance in front of each entry
 * is recovered by division and the colour behind it accumulated from the
 * back, so every quantity keeps its relative precision however deep the
 * entry lies.  dL_dimage: device [3][H_ds][W_ds]. */
tgs_status tgs_raster_bwd(tgs_context* ctx, const tgs_camera* cam, const tgs_dilation* dil,
                          const tgs_options* opt, const tgs_state* st, int64_t n,
                          const float* dL_dimage, void* stream);

/* Stage (d2): chain rule from grad2d to the parameters, and the
 * densification statistics of Sec. 4.3: pos_stat = ||(dL/du W/2, dL/dv H/2)||
 * (view-space positional gradient in NDC units of the full-resolution image),
 * col_stat = ||dL/d(r,g,b)|| (appearance gradient), visible = 1 where the
 * Gaussian overlapped at least one tile.  pos_stat, col_stat: device float[n];
 * visible: device uint8[n]; each may be NULL.  Reads the records of the
 * last preprocess on this state; after tgs_preprocess_fwd it takes the
 * colour term from the Jacobian that call stored, after a batched
 * preprocess of several views from the SH coefficients. */
tgs_status tgs_preprocess_bwd(tgs_context* ctx, const tgs_gaussians* g, const tgs_camera* cam,
                              const tgs_dilation* dil, const tgs_options* opt, const tgs_state* st,
                              const tgs_grads* out, float* pos_stat, float* col_stat,
                              uint8_t* visible, void* stream);

/* Stages (d1) and (d2) in order. */
tgs_status tgs_backward(tgs_context* ctx, const tgs_gaussians* g, const tgs_camera* cam,
                        const tgs_dilation* dil, const tgs_options* opt, const tgs_state* st,
                        const float* dL_dimage, const tgs_grads* out, float* pos_stat,
                        float* col_stat, uint8_t* visible, void* stream);

/* ---- Batched views (several cameras and dilation patterns, one Gaussian set).
 *
 * The views of one call share the Gaussians, the tile size, the LDS batch
 * and the background; each has its own camera, dilation pattern and state
 * (workspace), and the workspaces must not overlap.  1 <= views <=
 * TGS_MAX_VIEWS.  Each call enqueues a fixed sequence of kernels and never
 * reads back from the device, so the sequence can be captured in a graph and
 * replayed.  The preprocess forward and backward and the rasterizer forward
 * and backward are single launches covering every view; tile/Gaussian
 * binning runs per view.  A failing call has enqueued nothing, except the
 * composite tgs_batch_forward / tgs_batch_backward, whose arguments are all
 * checked first as well.  Results of each view are those of the single-view
 * calls on the same camera and pattern, up to the order of float additions
 * in the summed gradients.
 *
 * Pair capacity: every view's binning writes its pair count to the device
 * and, when the count exceeds the view's pair_capacity, emits no pair and
 * renders the background with zero gradients.  tgs_pair_counts reads the
 * counts back and reports TGS_ERR_CAPACITY; the caller then grows the
 * workspaces and repeats the step. */

/* Stage (a) for every view: one launch that reads the parameters once and
 * writes every view's records and tiles_touched (as tgs_preprocess_fwd). */
tgs_status tgs_batch_preprocess_fwd(tgs_context* ctx, const tgs_gaussians* g, int32_t views,
                                    const tgs_camera* cams, const tgs_dilation* dils,
                                    const tgs_options* opt, tgs_state* states, void* stream);

/* Stage (b) for every view (as tgs_bin_sort, without the readback): the
 * pair count stays on the device and a view whose pairs exceed its capacity
 * gets empty ranges.  Sets states[v].pair_count to TGS_PAIR_COUNT_PENDING.
 * The views are binned concurrently on streams the context owns, forked from
 * and joined back into `stream` (under graph capture: parallel branches of
 * the graph); calls of this function on one context must not overlap. */
tgs_status tgs_batch_bin_sort(tgs_context* ctx, const tgs_gaussians* g, int32_t views,
                              const tgs_camera* cams, const tgs_dilation* dils,
                              const tgs_options* opt, tgs_state* states, void* stream);

/* Stage (c) for every view: one launch over the tiles of all views (as
 * tgs_raster_fwd; outputs in io[v], image required). */
tgs_status tgs_batch_raster_fwd(tgs_context* ctx, int64_t n, int32_t views,
                                const tgs_camera* cams, const tgs_dilation* dils,
                                const tgs_options* opt, const tgs_state* states,
                                const tgs_view_io* io, void* stream);

/* Stages (a)-(c) for every view, the three calls above in order. */
tgs_status tgs_batch_forward(tgs_context* ctx, const tgs_gaussians* g, int32_t views,
                             const tgs_camera* cams, const tgs_dilation* dils,
                             const tgs_options* opt, tgs_state* states, const tgs_view_io* io,
                             void* stream);

/* The L1 loss and its gradient (as tgs_l1_grad) for every view: reads
 * io[v].image and io[v].target, writes io[v].dL_dimage.  loss: device
 * double[views], overwritten (may be NULL). */
tgs_status tgs_batch_l1_grad(tgs_context* ctx, int32_t views, const tgs_camera* cams,
                             const tgs_dilation* dils, const tgs_view_io* io, double* loss,
                             void* stream);

/* Stage (d1) for every view: one launch over the tiles of all views, from
 * io[v].dL_dimage and the per-pixel state of each view's last forward into
 * each view's grad2d (as tgs_raster_bwd). */
tgs_status tgs_batch_raster_bwd(tgs_context* ctx, int64_t n, int32_t views,
                                const tgs_camera* cams, const tgs_dilation* dils,
                                const tgs_options* opt, const tgs_state* states,
                                const tgs_view_io* io, void* stream);

/* Stage (d2) for every view: one launch that sums the parameter gradients
 * over the views (the Gaussians are shared, so the gradient of the summed
 * loss is the sum).  The statistics of Sec. 4.3 are summed over the views
 * where the Gaussian is visible and visible[i] counts those views.  Each of
 * pos_stat, col_stat, visible may be NULL.  io may be NULL; where it is not,
 * io[v].pos_stat / col_stat / visible (each optional) receive view v's own
 * statistics (as tgs_preprocess_bwd of that view alone would write them). */
tgs_status tgs_batch_preprocess_bwd(tgs_context* ctx, const tgs_gaussians* g, int32_t views,
                                    const tgs_camera* cams, const tgs_dilation* dils,
                                    const tgs_options* opt, const tgs_state* states,
                                    const tgs_view_io* io, const tgs_grads* out, float* pos_stat,
                                    float* col_stat, uint8_t* visible, void* stream);

/* Stages (d1)-(d2) for every view, the two calls above in order. */
tgs_status tgs_batch_backward(tgs_context* ctx, const tgs_gaussians* g, int32_t views,
                              const tgs_camera* cams, const tgs_dilation* dils,
                              const tgs_options* opt, const tgs_state* states,
                              const tgs_view_io* io, const tgs_grads* out, float* pos_stat,
                              float* col_stat, uint8_t* visible, void* stream);

/* Reads the device pair count of every state back (one stream
 * synchronisation) into states[v].pair_count, after a batched or an
 * asynchronous single-view bin/sort.  Returns TGS_ERR_CAPACITY if any count
 * exceeds its pair_capacity (that view rendered nothing), and
 * TGS_ERR_UNSUPPORTED if a view reached 2^32 - 1 pairs (its count reads
 * 4294967295). */
tgs_status tgs_pair_counts(tgs_context* ctx, int32_t views, tgs_state* states, void* stream);

/* ---- Fused Adam step (the optimiser of the fitting loop that follows
 * stage (d2); Adam as in the 3DGS recipe the paper trains with, Tab. 2).
 *
 * For every element of every group, with t the step after this call:
 *   m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
 *   p <- p - lr / (1 - b1^t) * m / (sqrt(v) / sqrt(1 - b2^t) + eps).
 * The step counter t and the bias corrections live in `state` (device
 * memory of TGS_ADAM_STATE_BYTES bytes, 16-byte aligned, zero before the
 * first step, one per optimiser); each call increments it on the device, so
 * the call can be captured in a graph and replayed. */
#define TGS_ADAM_STATE_BYTES 16
#define TGS_MAX_ADAM_GROUPS 8

typedef struct tgs_adam_group {
    float* param;            /* device [count], updated in place          */
    const float* grad;       /* device [count]                            */
    float* exp_avg;          /* device [count], first moment, in place    */
    float* exp_avg_sq;       /* device [count], second moment, in place   */
    int64_t count;           /* >= 0                                      */
    float lr;                /* learning rate of the group, >= 0          */
} tgs_adam_group;

/* 1 <= n_groups <= TGS_MAX_ADAM_GROUPS; 0 <= beta1, beta2 < 1; eps > 0.
 * Arrays of different groups must not overlap. */
tgs_status tgs_adam_step(tgs_context* ctx, const tgs_adam_group* groups, int32_t n_groups,
                         float beta1, float beta2, float eps, void* state, void* stream);

/* ---- Densification selection (Sec. 4.3) from statistics accumulated over
 * views and iterations (sums of the per-view pos_stat / col_stat and the
 * number of views that saw each Gaussian, e.g. the sums of `visible`).
 *
 * selected[i] = 1 when count[i] > 0 and either pos_sum[i] / count[i] >=
 * tau_pos or, when color_active != 0, col_sum[i] / count[i] >= tau_col
 * (the paper sets tau_col = 0.01 tau_pos and activates the appearance branch
 * in 20% of the densification events; the caller draws that decision).
 * Means and ratios are computed in float32 with IEEE division.  With
 * budget >= 0 (the number of Gaussians the convergence-aware schedule of
 * Sec. 4.2 still allows), only the `budget` candidates with the largest
 * score max(mean_pos / tau_pos, mean_col / tau_col) stay selected, equal
 * scores in ascending index; budget = -1 keeps every candidate.
 * n_selected: device uint32, the number selected.  workspace: device,
 * 256-byte aligned, at least tgs_densify_query bytes; col_sum may be NULL
 * when color_active is 0. */
tgs_status tgs_densify_query(int64_t n, uint64_t* workspace_bytes);
tgs_status tgs_densify_select(tgs_context* ctx, int64_t n, const float* pos_sum,
                              const float* col_sum, const int32_t* count, float tau_pos,
                              float tau_col, int32_t color_active, int64_t budget,
                              uint8_t* selected, uint32_t* n_selected, void* workspace,
                              uint64_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TGS_H */
