/*
 * seele.h -- C ABI of the MI355X (gfx950) Gaussian-splatting hot path of
 * "Seele: A Unified Acceleration Framework for Real-Time Gaussian Splatting
 * on Mobile Devices" (arXiv 2503.05168).
 *
 * The pipeline the paper describes for one frame (Sec. 3.1 Preliminaries):
 *   preprocessing  -> seele_preprocess   (frustum/opacity culling, EWA
 *                                          projection, SH colour, tile extent;
 *                                          the opacity-aware extent of Sec. 3.3
 *                                          Eqs. 4-5; the hybrid-preprocessing
 *                                          active set of Sec. 3.3 "Algorithm")
 *   sorting        -> seele_bin_sort     (Gaussian-tile pairs, per-tile
 *                                          closest-to-furthest order)
 *   rasterization  -> seele_rasterize_fwd (Eqs. 1-2, plain or the
 *                                          contribution-aware Algorithm 1 of
 *                                          Sec. 3.4)
 *   fine-tuning    -> seele_rasterize_bwd (Sec. 3.5: gradients of the unchanged
 *                                          pipeline with the HP/CR decisions
 *                                          held fixed)
 *
 * Conventions shared by every entry point
 *  - Every array argument is a device pointer to caller-owned memory unless
 *    the comment says "host".  The library allocates and frees nothing and
 *    keeps no state between calls; calls on different streams may overlap.
 *  - All work is enqueued on `stream` (a hipStream_t; NULL = default stream)
 *    and nothing synchronises.  Inputs are read-only; outputs are fully
 *    overwritten.
 *  - Arguments are validated on the host before anything is enqueued.  On
 *    any non-zero status nothing has been enqueued unless the status is
 *    SEELE_ERR_HIP (a launch failed; the stream state is then undefined).
 *    seele_last_error() returns a thread-local message for the last failure.
 *  - Several views are handled by one call: per-view outputs are stored view
 *    after view (view v's block starts after views 0..v-1's blocks).
 *  - Cameras use OpenCV axes (+x right, +y down, +z forward), a world-to-
 *    camera transform x_c = R x_w + t, pinhole intrinsics and pixel centres
 *    at integer + 0.5.
 */
#ifndef SEELE_H
#define SEELE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes returned by every entry point. */
enum {
  SEELE_OK = 0,
  SEELE_ERR_INVALID_ARG = 1,  /* null/misaligned pointer, bad size or option */
  SEELE_ERR_UNSUPPORTED = 2,  /* valid but not supported by this library     */
  SEELE_ERR_CAPACITY = 3,     /* a caller buffer is too small                */
  SEELE_ERR_HIP = 4           /* a HIP runtime call or launch failed         */
};

/* Tile extent of a projected Gaussian (Sec. 3.3 "Online Filtering"). */
enum {
  SEELE_EXTENT_3SIGMA = 0,  /* circle of radius 3 sqrt(lambda_max(Sigma')), Eq. 3 */
  SEELE_EXTENT_OPACITY = 1  /* box of the ellipse d^T Sigma'^-1 d <= min(2 ln(o/alpha_theta), 9), Eq. 5 */
};

/* Rasterization form. */
enum {
  SEELE_RASTER_PLAIN = 0,   /* every pixel evaluates every listed Gaussian (Eqs. 1-2) */
  SEELE_RASTER_CONTRIB = 1  /* contribution-aware: a pixel group follows its leader's
                               alpha test (Sec. 3.4, Algorithm 1) */
};

/* 3D Gaussians, structure of arrays (device, float32).  sh_degree in 0..3;
 * the SH coefficient stride is always 16 (unused higher-degree slots are
 * not read). */
typedef struct seele_gaussians {
  int64_t n;                    /* number of Gaussians, 0 <= n < 2^31        */
  int32_t sh_degree;            /* 0..3                                       */
  int32_t reserved;
  const float* means;           /* [3][n] world positions                     */
  const float* log_scales;      /* [3][n] log of the per-axis std deviations  */
  const float* quats;           /* [4][n] rotation (w, x, y, z), any norm > 0 */
  const float* opacity_logits;  /* [n]    o = sigmoid(logit)                  */
  const float* sh;              /* [16][3][n] (coefficient, channel, Gaussian)
                                   coefficient index l*l + l + m             */
} seele_gaussians;

/* Gradients in the layout of seele_gaussians (device, float32, overwritten). */
typedef struct seele_gaussian_grads {
  float* means;           /* [3][n]  */
  float* log_scales;      /* [3][n]  */
  float* quats;           /* [4][n]  */
  float* opacity_logits;  /* [n]     */
  float* sh;              /* [16][3][n] */
} seele_gaussian_grads;

/* A pinhole camera (host struct, 72 bytes). */
typedef struct seele_camera {
  float R[9];             /* world->camera rotation, row-major */
  float t[3];             /* world->camera translation         */
  float fx, fy, cx, cy;   /* focal lengths and principal point, pixels */
  int32_t width, height;  /* image size, pixels, >= 1          */
} seele_camera;

/* One projected Gaussian for one view (64 bytes, one aligned 64-byte
 * sector).  Written by seele_preprocess for visible Gaussians only (records
 * of culled Gaussians are left untouched and never read).
 * chol = (l11, l21, l22) is the lower Cholesky factor of k * conic with
 * k = log2(e) / 2, computed in double precision from the float32 conic:
 * k * [[a, b], [b, c]] = [[l11, 0], [l21, l22]] [[l11, l21], [0, l22]],
 * so that exp(-q/2) = exp2(-((l11 dx + l21 dy)^2 + (l22 dy)^2)).
 * rect_x = x0 | x1 << 16 and rect_y = y0 | y1 << 16 give the half-open tile
 * rectangle [x0, x1) x [y0, y1). */
typedef struct seele_splat {
  float mean_x, mean_y;              /* x' (pixels)                         */
  float chol_l11, chol_l21;          /* Cholesky factor of k * conic        */
  float chol_l22;
  float opacity;                     /* o                                   */
  float r, g, b;                     /* view-dependent colour (clamped >= 0) */
  float conic_a, conic_b, conic_c;   /* Sigma'^-1 = [[a, b], [b, c]]       */
  float depth;                       /* camera-space z                      */
  uint32_t rect_x, rect_y;
  uint32_t reserved;                 /* written as 0                        */
} seele_splat;

/* Preprocessing options. */
typedef struct seele_preprocess_opts {
  int32_t tile;             /* tile edge in pixels: 8 or 16                     */
  int32_t extent;           /* SEELE_EXTENT_*                                    */
  float alpha_min;          /* alpha_theta (1/255)                               */
  float lowpass;            /* added to the diagonal of Sigma' (0.3 px^2)        */
  float z_near;             /* Gaussians with camera z <= z_near are culled (0.2) */
  int32_t n_segs;           /* active segments (hybrid preprocessing); 0 = all   */
  const int64_t* seg_begin; /* host [n_segs], disjoint, inside [0, n)            */
  const int64_t* seg_count; /* host [n_segs]                                     */
} seele_preprocess_opts;

/* Rasterization options. */
typedef struct seele_raster_opts {
  int32_t tile;             /* must equal the tile used by preprocess/bin_sort */
  int32_t mode;             /* SEELE_RASTER_*                                  */
  int32_t group_w, group_h; /* contribution-aware pixel group (2, 2); each of
                               1, 2, 4 with group_w * group_h <= 16            */
  int32_t lds_batch;        /* Gaussians staged in LDS per step: 0 = one per
                               pixel of the tile; 16x16 tiles also take 64 or
                               128 (a tuning knob; results do not change)      */
  float alpha_min;          /* alpha_theta (1/255)                             */
  float alpha_max;          /* clamp of alpha (0.99)                           */
  float T_min;              /* a pixel stops before T would fall below (1e-4)   */
  float bg[3];              /* background colour added as T_final * bg         */
} seele_raster_opts;

/* Number of tiles of view v is ceil(W/tile) * ceil(H/tile); this returns the
 * sum over the views (the length of the tile_ranges array), or -1 on bad
 * arguments.  cams is a host array. */
int64_t seele_total_tiles(const seele_camera* cams, int32_t n_views, int32_t tile);

/* Preprocess n_views views of g (Sec. 3.1 "Preprocessing", Sec. 3.3 "Online
 * Filtering").  For view v and Gaussian i, record v*n + i of `splats` and
 * `n_tiles` is written: n_tiles = number of tiles of its rectangle, or 0 if
 * the Gaussian is culled (inactive segment, non-finite attribute, z <=
 * z_near, degenerate Sigma', o < alpha_min (3-sigma extent) or
 * tau <= 0 (opacity extent), empty rectangle).
 *   cams    host [n_views]
 *   splats  device [n_views * n] seele_splat, 16-byte aligned (64 keeps every
 *           record in one 64-byte sector)
 *   n_tiles device [n_views * n] int32 */
int32_t seele_preprocess(const seele_gaussians* g, const seele_camera* cams, int32_t n_views,
                         const seele_preprocess_opts* opts, seele_splat* splats,
                         int32_t* n_tiles, void* stream);

/* Workspace bytes seele_bin_sort needs for n_records = n_views * n records,
 * a pair capacity and the total tile count. */
size_t seele_bin_sort_workspace_size(int64_t n_records, int64_t capacity, int64_t n_tiles_total);

/* Tile binning and depth sort (Sec. 3.1 "Preprocessing" and "Sorting").
 * Every record with n_tiles > 0 yields one pair per tile of its rectangle.
 * Pairs are ordered by (global tile id, float32 depth, record id), where the
 * global tile id of local tile (tx, ty) in view v is
 * sum_{u<v} tiles(u) + ty * ceil(W_v/tile) + tx.
 *   sorted_ids  device [capacity] uint32: record ids v*n + i in that order
 *   tile_ranges device [n_tiles_total][2] int32: [start, end) into sorted_ids
 *                (start = end = 0 for an empty tile)
 *   num_pairs   device [1] int64: the number of pairs the frame needs.
 * If that number exceeds `capacity`, every tile range is written empty and
 * sorted_ids is not written; the caller reads num_pairs, grows the buffer
 * and calls again (the call itself still returns SEELE_OK because the count
 * is only known on the device).  capacity < 2^31.  n_views <= 256; at most
 * 2^24 super-tiles (blocks of 4 x 4 tiles) over all views. */
int32_t seele_bin_sort(const seele_splat* splats, const int32_t* n_tiles, int64_t n,
                       const seele_camera* cams, int32_t n_views, int32_t tile,
                       void* workspace, size_t workspace_bytes, uint32_t* sorted_ids,
                       int64_t capacity, int32_t* tile_ranges, int64_t* num_pairs,
                       void* stream);

/* Super-tiles are blocks of 4 x 4 tiles, ceil(ceil(W/tile)/4) *
 * ceil(ceil(H/tile)/4) per view, numbered row-major per view after the
 * previous views' ones.  This returns their number over the views (the
 * length of the st_ranges array), or -1 on bad arguments.  cams is a host
 * array. */
int64_t seele_total_super_tiles(const seele_camera* cams, int32_t n_views, int32_t tile);

/* The binning and depth sort of seele_bin_sort (Sec. 3.1 "Sorting"), left at
 * super-tile granularity: every record with n_tiles > 0 yields one entry per
 * super-tile its tile rectangle touches, and the entries are ordered by
 * (global super-tile id, float32 depth, record id).
 *   entry_keys device [capacity] uint32: (clip << 24) | global super-tile id,
 *              clip = the rectangle clipped to the super-tile as local
 *              inclusive tile coordinates x0 | x1 << 2 | y0 << 4 | y1 << 6
 *   entry_ids  device [capacity] uint32: record ids v*n + i, same order
 *   st_ranges  device [n_super_tiles][2] int32: [start, end) into the entries
 *              (start = end = 0 for an empty super-tile)
 *   num_pairs  device [2] int64: the Gaussian-tile pairs of the frame (as
 *              for seele_bin_sort), then the entries it needs (never more
 *              than the pairs).
 * Here `capacity` bounds the entries: a frame overflows when its entries
 * exceed it (every range written empty, entries not written), however many
 * pairs it has; the caller reads num_pairs[1], grows both buffers and calls
 * again.  Tile t's list of seele_bin_sort is exactly the subsequence of its
 * super-tile's entries whose clip covers t.  Workspace and other limits are
 * those of seele_bin_sort; the workspace size is
 * seele_bin_sort_workspace_size's. */
int32_t seele_bin_sort_super(const seele_splat* splats, const int32_t* n_tiles, int64_t n,
                             const seele_camera* cams, int32_t n_views, int32_t tile,
                             void* workspace, size_t workspace_bytes, uint32_t* entry_keys,
                             uint32_t* entry_ids, int64_t capacity, int32_t* st_ranges,
                             int64_t* num_pairs, void* stream);

/* seele_preprocess that also does the first step of the binning (visible
 * records and their float32 depth keys in record order, every record's tile
 * rectangle) and leaves it in a bin-sort workspace, for seele_bin_sort_ex
 * with SEELE_BIN_STAGED.  Outputs (splats, n_tiles) and arguments are those
 * of seele_preprocess; workspace / workspace_bytes / capacity are those the
 * following seele_bin_sort_ex call will take (workspace size from
 * seele_bin_sort_workspace_size for n_views * n records).  n_views <= 256.
 * The staged input is valid until the workspace is used for another call;
 * the caller orders the two calls (same stream, or synchronised). */
int32_t seele_preprocess_staged(const seele_gaussians* g, const seele_camera* cams,
                                int32_t n_views, const seele_preprocess_opts* opts,
                                seele_splat* splats, int32_t* n_tiles, void* workspace,
                                size_t workspace_bytes, int64_t capacity, void* stream);

/* Flags of seele_bin_sort_ex. */
enum {
  SEELE_BIN_SUPER = 1,  /* super-tile lists (seele_bin_sort_super's outputs) */
  SEELE_BIN_STAGED = 2  /* take the visible records staged in the workspace by
                           seele_preprocess_staged (same views, n and
                           capacity); splats and n_tiles are then not read */
};

/* seele_bin_sort (flags 0) or seele_bin_sort_super (SEELE_BIN_SUPER), either
 * one optionally from a staged workspace (SEELE_BIN_STAGED); results are
 * identical in every case.  entry_keys is used with SEELE_BIN_SUPER only;
 * ids is sorted_ids / entry_ids; ranges is tile_ranges / st_ranges;
 * num_pairs has 1 element (per-tile lists) or 2 (SEELE_BIN_SUPER: pairs,
 * entries), and capacity bounds the pairs or the entries respectively. */
int32_t seele_bin_sort_ex(int32_t flags, const seele_splat* splats, const int32_t* n_tiles,
                          int64_t n, const seele_camera* cams, int32_t n_views, int32_t tile,
                          void* workspace, size_t workspace_bytes, uint32_t* entry_keys,
                          uint32_t* ids, int64_t capacity, int32_t* ranges, int64_t* num_pairs,
                          void* stream);

/* Bytes of the per-device scratch array behind seele_bin_sort_noalloc. */
#define SEELE_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* seele_bin_sort_ex for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the binning workspace is a file-scope device array of
 * SEELE_NOALLOC_SCRATCH_BYTES in the library (one per GPU, held until the
 * process ends), so the call takes no workspace and allocates nothing.
 * flags: 0 (per-tile lists) or SEELE_BIN_SUPER; SEELE_BIN_STAGED is refused
 * (its input lives in a caller workspace).  Every other argument, output and
 * overflow rule is seele_bin_sort_ex's.  SEELE_ERR_CAPACITY when
 * seele_bin_sort_workspace_size(n_views * n, capacity, total tiles) exceeds
 * SEELE_NOALLOC_SCRATCH_BYTES (e.g. 980k records with 2.45M pairs fit).
 * The array is shared by every call on a GPU and keeps the last call's
 * contents: calls that overlap on one GPU (different streams or host
 * threads without ordering) race and give undefined results. */
int32_t seele_bin_sort_noalloc(int32_t flags, const seele_splat* splats, const int32_t* n_tiles,
                               int64_t n, const seele_camera* cams, int32_t n_views, int32_t tile,
                               uint32_t* entry_keys, uint32_t* ids, int64_t capacity,
                               int32_t* ranges, int64_t* num_pairs, void* stream);

/* Front-to-back blending of every tile of every view (Eqs. 1-2; Algorithm 1
 * when opts->mode == SEELE_RASTER_CONTRIB).
 *   image     device, per view [3][H][W] float32, views concatenated
 *   final_T   device, per view [H][W] float32: transmittance after the last
 *             blended Gaussian (>= T_min)
 *   n_contrib device, per view [H][W] int32: 1-based position, in the pixel's
 *             tile list, of the last Gaussian it blended (0 if none). */
int32_t seele_rasterize_fwd(const seele_splat* splats, const uint32_t* sorted_ids,
                            const int32_t* tile_ranges, const seele_camera* cams,
                            int32_t n_views, const seele_raster_opts* opts, float* image,
                            float* final_T, int32_t* n_contrib, void* stream);

/* seele_rasterize_fwd reading the super-tile lists of seele_bin_sort_super
 * (each tile keeps the entries whose clip covers it, in list order): the
 * outputs are bit-identical to seele_rasterize_fwd on the per-tile lists,
 * and n_contrib still counts positions in the tile's own list.
 *   last_entry NULL, or device, per view [H][W] int32: 1 + the index, from
 *              the start of the pixel's super-tile list, of the last entry
 *              the pixel blended (0 if none); the input of
 *              seele_rasterize_bwd_super
 *   counters   NULL, or device [6] uint64 as for seele_rasterize_fwd_counted
 *              (then the instrumented kernel runs).
 * Default LDS batch (opts->lds_batch 0 or tile * tile) only;
 * SEELE_ERR_UNSUPPORTED otherwise. */
int32_t seele_rasterize_fwd_super(const seele_splat* splats, const uint32_t* entry_keys,
                                  const uint32_t* entry_ids, const int32_t* st_ranges,
                                  const seele_camera* cams, int32_t n_views,
                                  const seele_raster_opts* opts, float* image, float* final_T,
                                  int32_t* n_contrib, int32_t* last_entry, uint64_t* counters,
                                  void* stream);

/* Offline contribution pass of the view-dependent representation (Sec. 3.3
 * "Offline Clustering"): the plain blend of every pixel (Eqs. 1-2, exactly
 * as seele_rasterize_fwd computes it) over the per-tile lists of
 * seele_bin_sort, ranking each pixel's blended records by their contribution
 * T_i alpha_i (a larger one first, equal ones toward the lower record id).
 *   topk_mark   device [n_views * n] uint8: set to 1 for every record among
 *               some pixel's k first (1 <= k <= 32); other entries are left
 *               unchanged, so marks accumulate over calls (the caller clears)
 *   contrib_sum device [n_views * n] float32: T_i alpha_i of every blend is
 *               added to its record's entry (float atomics; summation order
 *               unspecified)
 * opts->mode must be SEELE_RASTER_PLAIN (SEELE_ERR_UNSUPPORTED otherwise). */
int32_t seele_contrib_topk(const seele_splat* splats, const uint32_t* sorted_ids,
                           const int32_t* tile_ranges, const seele_camera* cams, int32_t n_views,
                           int64_t n, const seele_raster_opts* opts, int32_t k,
                           uint8_t* topk_mark, float* contrib_sum, void* stream);

/* Order of the (view, tile) work queue of seele_rasterize_fwd_queue. */
enum {
  SEELE_QUEUE_LIST = 0,           /* tiles in id order                       */
  SEELE_QUEUE_HEAVIEST_FIRST = 1  /* tiles with the longest lists first       */
};

/* Workspace bytes for seele_rasterize_fwd_queue over n_tiles_total tiles. */
size_t seele_raster_queue_workspace_size(int64_t n_tiles_total);

/* seele_rasterize_fwd for batches of views as one persistent launch per 64
 * views: a fixed grid of workgroups (enough to fill the GPU) pulls
 * (view, tile) items from a device counter in `order` until the queue is
 * empty.  Same outputs as seele_rasterize_fwd (bit-identical).  The
 * workspace (caller-owned device memory, 256-byte aligned) holds the queue
 * counter and the heaviest-first order; no host synchronisation, so the call
 * can be captured in a HIP graph. */
int32_t seele_rasterize_fwd_queue(const seele_splat* splats, const uint32_t* sorted_ids,
                                  const int32_t* tile_ranges, const seele_camera* cams,
                                  int32_t n_views, const seele_raster_opts* opts, int32_t order,
                                  void* workspace, size_t workspace_bytes, float* image,
                                  float* final_T, int32_t* n_contrib, void* stream);

/* seele_rasterize_fwd with work counters (an instrumented, slower kernel
 * that visits every record of every tile list and writes the same outputs).
 * counters: device [6] uint64, overwritten:
 *   [0] per-pixel alpha evaluations by pixels that have not stopped
 *       (contribution-aware form: only in groups whose leader accepted),
 *   [1] blends (Gaussians accumulated into a pixel),
 *   [2] leader tests of groups with a pixel that has not stopped,
 *   [3] of those, tests that accepted the Gaussian.
 * [0]-[3] are the algorithmic work units of Eqs. 1-2 and Algorithm 1.  The
 * production kernels skip, per 8x8 pixel block, the records whose
 * alpha >= alpha_min region cannot reach the block (exactly: those records
 * blend into none of its pixels); the work they are left with is
 *   [4] the evaluations of [0] on records that can reach the pixel's block,
 *   [5] (8x8 block, record) visits of such records while the block has a
 *       pixel that has not stopped. */
int32_t seele_rasterize_fwd_counted(const seele_splat* splats, const uint32_t* sorted_ids,
                                    const int32_t* tile_ranges, const seele_camera* cams,
                                    int32_t n_views, const seele_raster_opts* opts, float* image,
                                    float* final_T, int32_t* n_contrib, uint64_t* counters,
                                    void* stream);

/* Gradients of a scalar loss L for the fine-tuning of Sec. 3.5, given
 * dL/dimage (same layout as image).  The forward's decisions (culling,
 * rectangles, order, alpha skips, leader tests, termination) are constants;
 * the blend is recomputed backwards from final_T and n_contrib, so no
 * per-pixel lists are stored.
 *   grad2d device [n_views * n][9] float32, written by the call: per record
 *          dL/d(mean_x, mean_y, conic_a, conic_b, conic_c, opacity, r, g, b)
 *          (zero for records no pixel blended)
 *   grads  overwritten with dL/d(raw parameters), summed over views.
 * g, cams, popts and n_views must be those of the forward call that wrote
 * splats/n_tiles; ropts those of the seele_rasterize_fwd call. */
int32_t seele_rasterize_bwd(const seele_gaussians* g, const seele_camera* cams, int32_t n_views,
                            const seele_preprocess_opts* popts, const seele_raster_opts* ropts,
                            const seele_splat* splats, const int32_t* n_tiles,
                            const uint32_t* sorted_ids, const int32_t* tile_ranges,
                            const float* final_T, const int32_t* n_contrib,
                            const float* dL_dimage, float* grad2d,
                            const seele_gaussian_grads* grads, void* stream);

/* seele_rasterize_bwd over the super-tile lists of seele_bin_sort_super (the
 * lists seele_rasterize_fwd_super read): same outputs, gradients equal up to
 * the order of float sums (Sec. 3.5).  One workgroup takes a 2 x 2-tile
 * quadrant of a super-tile and walks the super-tile's list backwards, so a
 * record's gradient is flushed to grad2d once per quadrant instead of once
 * per tile.  entry_keys / entry_ids / st_ranges as seele_bin_sort_super
 * writes them; last_entry as seele_rasterize_fwd_super wrote it for the same
 * lists (it takes the place of n_contrib).  16 x 16 tiles only
 * (SEELE_ERR_UNSUPPORTED otherwise). */
int32_t seele_rasterize_bwd_super(const seele_gaussians* g, const seele_camera* cams,
                                  int32_t n_views, const seele_preprocess_opts* popts,
                                  const seele_raster_opts* ropts, const seele_splat* splats,
                                  const int32_t* n_tiles, const uint32_t* entry_keys,
                                  const uint32_t* entry_ids, const int32_t* st_ranges,
                                  const float* final_T, const int32_t* last_entry,
                                  const float* dL_dimage, float* grad2d,
                                  const seele_gaussian_grads* grads, void* stream);

/* Offline view-dependent representation (Sec. 3.3 "Offline Clustering").
 *
 * seele_hp_kmeans clusters n_cams sampled poses (host array) into K groups
 * by the pose feature (camera centre / pos_scale, beta * view direction),
 * the one seele_hp_select uses: farthest-point seeding (pose 0 first, then
 * the pose farthest from every chosen centroid, lowest index on ties), then
 * Lloyd iterations (nearest centroid, lowest index on ties; member means; an
 * empty cluster keeps its centroid) until no label changes or `iters` updates.
 * pos_scale <= 0 takes seele_hp_pos_scale(cams, n_cams) (an error if every
 * centre is at the origin); a non-finite pos_scale or beta is an error.
 * Host only: centroids host [K][6], labels host [n_cams]. */
int32_t seele_hp_kmeans(const seele_camera* cams, int32_t n_cams, float pos_scale, float beta,
                        int32_t K, int32_t iters, float* centroids, int32_t* labels);

/* Default position normaliser of the pose feature (Sec. 3.3 "Offline
 * Clustering" normalises the camera position without saying by what): the
 * largest distance of a camera centre from the world origin over the n_cams
 * sampled poses (host array), as float32.  Returns -1 (and sets the last
 * error) on a null array, n_cams < 1 or a non-finite centre.  Host only. */
float seele_hp_pos_scale(const seele_camera* cams, int32_t n_cams);

/* Folds one cluster's seele_contrib_topk results (records v*n + i of its
 * n_views views) into per-Gaussian state, on the device: shared[i] |= any
 * view's top-k mark; if the cluster's summed contribution exceeds best_sum[i]
 * (strictly), best_sum[i] and best_cluster[i] = cluster.  The caller starts
 * from shared = 0, best_sum = 0, best_cluster = -1 and calls once per
 * cluster in index order (so ties keep the earlier cluster).
 *   topk_mark [n_views * n] uint8, contrib_sum [n_views * n] float32,
 *   shared [n] uint8, best_sum [n] float32, best_cluster [n] int32. */
int32_t seele_hp_accumulate(const uint8_t* topk_mark, const float* contrib_sum, int32_t n_views,
                            int64_t n, int32_t cluster, uint8_t* shared, float* best_sum,
                            int32_t* best_cluster, void* stream);

/* The segment layout (host): Gaussians with shared[i] form the shared
 * segment; the others with best_sum[i] > 0 form cluster best_cluster[i]'s
 * exclusive segment; the rest (never blended in any sampled view) go last
 * and belong to no segment.  Within a segment the original order is kept.
 *   perm          host [n] int64: perm[new position] = original index
 *   layout_begin  host [1 + K] int64: shared segment, then clusters 0..K-1
 *   layout_count  host [1 + K] int64   (the layout seele_hp_segments reads) */
int32_t seele_hp_partition(const uint8_t* shared, const float* best_sum,
                           const int32_t* best_cluster, int64_t n, int32_t K, int64_t* perm,
                           int64_t* layout_begin, int64_t* layout_count);

/* dst[c] = src[perm[c]] for every attribute, c < n_out (perm device int64);
 * dst holds device arrays in the seele_gaussians layout for n_out Gaussians
 * (the writable struct seele_gaussian_grads describes them); the SH rows
 * src->sh_degree uses are copied. */
int32_t seele_gather_gaussians(const seele_gaussians* src, const int64_t* perm, int64_t n_out,
                               const seele_gaussian_grads* dst, void* stream);

/* Hybrid preprocessing, runtime cluster choice (Sec. 3.3 "Algorithm").  The
 * camera feature is (centre / pos_scale, beta * view direction); the nearest
 * of the K centroids (host [K][6]) is chosen, then the M centroids nearest to
 * it; ties go to the lower index.  clusters: host [1 + M] output.  Host only,
 * enqueues nothing. */
int32_t seele_hp_select(const float* centroids, int32_t K, const seele_camera* cam,
                        float pos_scale, float beta, int32_t M, int32_t* clusters);

/* Active segments for the chosen clusters of a layout
 * [shared | excl_0 | ... | excl_{K-1}] given by host arrays
 * layout_begin[1 + K], layout_count[1 + K]: the shared segment plus each
 * chosen cluster's segment, sorted by begin, empty ones dropped.  out_begin
 * and out_count are host arrays of capacity 1 + n_sel; *n_out receives the
 * segment count.  Host only. */
int32_t seele_hp_segments(const int64_t* layout_begin, const int64_t* layout_count, int32_t K,
                          const int32_t* clusters, int32_t n_sel, int64_t* out_begin,
                          int64_t* out_count, int32_t* n_out);

/* Scene prefetching (Sec. 3.3 "Scene Prefetching"): clusters predicted for
 * coming frames are copied to the GPU ahead of time on a dedicated stream,
 * the future pose predicted by linear extrapolation of the camera pose.
 *
 * seele_pose_extrapolate: the pose s frames after `cur`, given the frame
 * before it: camera centre c_cur + s (c_cur - c_prev) and rotation
 * (R_cur R_prev^T)^s R_cur, the power taken on the relative rotation's
 * rotation vector (angle scaled by s about the same axis); intrinsics and
 * image size from `cur`.  s = 0 gives cur, s = -1 prev.  Host only. */
int32_t seele_pose_extrapolate(const seele_camera* prev, const seele_camera* cur, float s,
                               seele_camera* out);

/* Resident-set planning for a device pool that holds the shared segment and
 * n_slots slots of slot_cap Gaussians each.  slot_cluster[n_slots] (cluster
 * held by each slot, -1 empty) and slot_stamp[n_slots] (frame of its last
 * use or load) are host arrays updated in place; cluster_count[K] gives each
 * cluster's exclusive-segment size.
 *   1. Every needed cluster (need[n_need], this frame's selection) that is
 *      resident is held and stamped with `frame`.
 *   2. Each needed cluster that is not resident is loaded (a demand load)
 *      into the lowest empty slot, else into the slot that is not held with
 *      the oldest stamp, slots whose cluster is not in `want` first, the
 *      lowest index on ties.
 *   3. Each predicted cluster (want[n_want], in priority order) that is not
 *      resident is loaded into the lowest empty slot, else into the oldest
 *      slot (lowest index on ties) that is not held, not predicted and
 *      stamped before `frame`; planning stops at the first one with no such
 *      slot.  Loaded slots are stamped with `frame` and held.
 * load_cluster / load_slot (host, capacity n_slots) receive the loads in
 * order, *n_loads their number and *n_demand how many lead (the demand
 * loads).  Errors: a cluster outside 0..K-1 or larger than slot_cap, more
 * distinct needed clusters than slots, an inconsistent slot table.  The
 * caller copies each load (seele_load_segments) after the last reader of the
 * evicted cluster is done.  Host only. */
int32_t seele_resident_plan(int32_t* slot_cluster, int64_t* slot_stamp, int32_t n_slots,
                            const int64_t* cluster_count, int32_t K, int64_t slot_cap,
                            const int32_t* need, int32_t n_need, const int32_t* want,
                            int32_t n_want, int64_t frame, int32_t* load_cluster,
                            int32_t* load_slot, int32_t* n_loads, int32_t* n_demand);

/* Host-to-device segment copies of a row-major attribute table: for each
 * load j, columns [src_begin[j], src_begin[j] + count[j]) of all `rows`
 * rows of host_src (row stride src_stride floats) go to columns starting at
 * dst_begin[j] of dev_pool (row stride dst_stride floats), one 2D copy per
 * load enqueued on `stream`.  host_src must be pinned host memory for the
 * copies to run asynchronously; both tables stay owned by the caller and
 * must live until the copies complete.  Errors: a load out of either
 * table's bounds (nothing is enqueued). */
int32_t seele_load_segments(const float* host_src, int64_t src_stride, float* dev_pool,
                            int64_t dst_stride, int32_t rows, const int64_t* src_begin,
                            const int64_t* dst_begin, const int64_t* count, int32_t n_loads,
                            void* stream);

/* Fine-tuning (Sec. 3.5): the pipeline trains through its unchanged
 * backward; these are the loss and optimizer steps around it.
 *
 * Photometric loss of 3DGS training (the L_3DGS term): per view
 *   L_v = (1 - lambda) mean|x - y| + lambda (1 - SSIM(x, y))
 * over the [3][H][W] render x and target y, SSIM being the mean over pixels
 * and channels of the SSIM map with an 11 x 11 Gaussian window (sigma 1.5,
 * normalised, zero padding), C1 = 0.01^2, C2 = 0.03^2.  loss (device,
 * [n_views]) receives L_v; dL_dimage (device, the image layout) the
 * gradient of the mean of L_v over the views (at x = y the L1 term
 * contributes 0).  image and target: device, views concatenated as the
 * rasterizer writes them.  workspace: device, 256-byte aligned, at least
 * seele_photometric_loss_workspace_size bytes; contents undefined after. */
size_t seele_photometric_loss_workspace_size(const seele_camera* cams, int32_t n_views);
int32_t seele_photometric_loss(const float* image, const float* target, const seele_camera* cams,
                               int32_t n_views, float lambda, void* workspace,
                               size_t workspace_bytes, float* loss, float* dL_dimage,
                               void* stream);

typedef struct seele_adam_opts {
  float lr_means, lr_log_scales, lr_quats, lr_opacity, lr_sh_dc, lr_sh_rest;
  float beta1, beta2, eps;
} seele_adam_opts;

/* One Adam step over every attribute element of n Gaussians (the optimizer
 * of 3DGS training): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * p -= lr * (m / (1 - b1^step)) / (sqrt(v) / sqrt(1 - b2^step) + eps), with
 * the learning rate of the element's attribute (SH degree-0 rows and the
 * higher rows separately).  params (written in place), grads, m and v are
 * device arrays in the seele_gaussians layout (the writable descriptor
 * seele_gaussian_grads describes each); m and v start at zero; step counts
 * from 1.  SH rows beyond 3 (sh_degree + 1)^2 are not touched. */
int32_t seele_adam_step(const seele_gaussian_grads* params, const seele_gaussian_grads* grads,
                        const seele_gaussian_grads* m, const seele_gaussian_grads* v, int64_t n,
                        int32_t sh_degree, const seele_adam_opts* opts, int64_t step,
                        void* stream);

/* View-consistency term of the fine-tuning loss (Sec. 3.5): FLIP (LDR)
 * between each view's render (`image`, sRGB [3][H][W] per view, clamped to
 * [0, 1]) and its `reference`, for a viewer at `ppd` pixels per degree
 * (FLIP's default 67.02: 0.7 m from a 0.7 m wide 3840-pixel screen).  flip
 * (device [n_views]) receives each view's mean FLIP; dL_dimage receives
 * scale * d(mean over views of the per-view means)/d image, written, or
 * added to its contents when accumulate != 0 (so the photometric loss's
 * gradient and gamma * this one sum in place).  workspace: device, 256-byte
 * aligned, at least seele_flip_loss_workspace_size bytes.  Errors: ppd
 * whose filters exceed 24-pixel radii (ppd above about 177). */
size_t seele_flip_loss_workspace_size(const seele_camera* cams, int32_t n_views);
int32_t seele_flip_loss(const float* image, const float* reference, const seele_camera* cams,
                        int32_t n_views, float ppd, float scale, int32_t accumulate,
                        void* workspace, size_t workspace_bytes, float* flip, float* dL_dimage,
                        void* stream);

/* Storage order of a scene (a layout choice, not a step of the method):
 * the permutation that sorts the Gaussians by the 30-bit Morton code of
 * their means, bit 3k + a holding bit k of axis a's quantised coordinate
 * q_a = min(1023, floor((x_a - lo_a) * (1024 / (hi_a - lo_a)))) computed in
 * float32 over the box [lo, hi] of the finite coordinates (q_a = 1023 for a
 * non-finite coordinate, 0 on a flat axis); equal codes keep their original
 * order.  Gathering the scene in this order (seele_gather_gaussians) lets a
 * view's culled and visible Gaussians, and a tile's list, occupy contiguous
 * runs of memory.  perm: device int64 [n], new position -> original index.
 * workspace: device, 256-byte aligned, seele_spatial_order_workspace_size
 * bytes. */
size_t seele_spatial_order_workspace_size(int64_t n);
int32_t seele_spatial_order(const seele_gaussians* g, void* workspace, size_t workspace_bytes,
                            int64_t* perm, void* stream);

/* Thread-local message describing the last non-OK status on this thread. */
const char* seele_last_error(void);
/* Static name of a status code. */
const char* seele_status_string(int32_t status);
/* ABI version (major * 100 + minor). */
int32_t seele_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SEELE_H */
