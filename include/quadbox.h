/*
 * quadbox.h -- C ABI of the MI355X (gfx950) QuadBox rasterizer hot path.
 *
 * Implements the forward rasterization of 3D Gaussian Splatting with the
 * QuadBox tile culling and the QPass traversal of "QuadBox: Accelerating 3D
 * Gaussian Splatting with Geometry-Aware Boxes" (arXiv 2605.04844):
 *   qb_project    Sec. 2 (EWA projection, Eq. 1; Preprocess), Sec. 3.1 (boxes,
 *                 Eqs. 3-12), Sec. 3.2 (tile-space bounds)
 *   qb_intersect  Sec. 2 (DuplicateWithKeys), Sec. 3.2 (QPass)
 *   qb_sort       Sec. 2 (SortPairs) and the per-tile ranges
 *   qb_render     Sec. 2, Eq. (2) (front-to-back alpha compositing)
 *   qb_tile_order the order in which the render takes tiles (scheduling only:
 *                 results do not depend on it)
 *   qb_render_backward, qb_project_backward
 *                 gradients (the rasterizer is trained through, Sec. 4.1)
 *   qb_*_views    the same stages over several views per launch
 *
 * Conventions shared by every entry point
 *   - Array arguments are DEVICE pointers owned by the caller; the library never
 *     allocates, frees or retains caller memory.  Scratch memory comes from a
 *     caller-provided workspace of qb_*_workspace_size() bytes (256-byte aligned).
 *   - Every call but qb_check_capacity is asynchronous on the given HIP
 *     stream (0 = null stream) and returns after enqueueing its kernels.
 *   - Argument errors (null pointers, negative or oversized counts, bad modes,
 *     bad image sizes) are detected on the host before anything is launched and
 *     return QB_ERR_INVALID_ARG; a failed launch returns QB_ERR_HIP.  Nothing
 *     aborts or throws across the ABI.
 *   - Tiles are 16x16 pixels; tile id = ty * tiles_x + tx with
 *     tiles_x = ceil(W/16), tiles_y = ceil(H/16).
 *   - Floating point is IEEE binary32.  Values that decide tile sets, keys and
 *     the render's 1/255 cutoff follow one fixed operation order (no
 *     contraction, correctly rounded divide and sqrt, transcendentals evaluated
 *     in binary64 and rounded once), so they are reproducible bit for bit.
 */
#ifndef QUADBOX_H
#define QUADBOX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* qb_stream_t; /* a hipStream_t */

typedef enum {
    QB_OK = 0,
    QB_ERR_INVALID_ARG = -1,
    QB_ERR_CAPACITY = -2,   /* more pairs than the caller's capacity            */
    QB_ERR_HIP = -3,        /* a HIP runtime call or kernel launch failed        */
    QB_ERR_UNSUPPORTED = -4 /* no gfx950 device / feature not built              */
} qb_status;

/* Box that decides which tiles a Gaussian is listed in. */
typedef enum {
    QB_BOX_3SIGMA = 0,  /* square of side 6 sqrt(lambda_max) (Sec. 2)               */
    QB_BOX_ADR = 1,     /* opacity-aware AABB, half extents sqrt(gamma*Sigma2D_ii)
                           (Sec. 3.1, Eqs. 9, 11)                                   */
    QB_BOX_QUADBOX = 2, /* four quadrant boxes: two full (major axis) and two
                           scaled by f = sqrt(1 - b^2/(ac)) (Sec. 3.1, Eq. 12)      */
    QB_BOX_DUALBOX = 3, /* the two major-axis quadrant boxes only (Sec. 3.1);
                           not conservative, ablation only (Table 3)              */
    QB_BOX_QUADBOX_NAIVE = 4 /* the QuadBox tile set enumerated without QPass: each
                           sub-box's tile rect walked with nested loops, tiles
                           of earlier sub-boxes skipped by rect tests (Sec. 3.2;
                           the dagger row of Table 3).  Same sets, counts, pairs
                           after sorting and image as QB_BOX_QUADBOX.            */
} qb_box_mode;

/* Flag added to an opacity-aware qb_box_mode (ADR, QUADBOX, DUALBOX,
 * QUADBOX_NAIVE) in qb_project, qb_project_views and qb_intersect: each
 * sub-box's tile rect is intersected with the tile rect of the 3-sigma square
 * (QB_BOX_3SIGMA's box).  The tile set is then the mode's set intersected
 * with the 3-sigma set for every Gaussian, so it never exceeds the 3-sigma
 * baseline's (the unclipped set does where gamma > 9, i.e. o > e^4.5/255: the
 * 1/255 ellipse leaves the 3-sigma square), and with ADR or QUADBOX the image
 * equals the 3-sigma image (the render finds the same contributions).  The
 * unclipped modes are the paper's. */
#define QB_CLIP_3SIGMA 16

/* Pinhole camera.  R (row-major) and t map world to camera coordinates:
 * p = R mu + t, x right, y down, z forward; pixel (i, j) samples the image
 * point (i, j); u = fx x/z + cx.  campos is the camera centre in world space
 * (used for the view direction of the SH colour).  Gaussians with p.z <=
 * near_plane are culled.  Every entry point that takes a camera returns
 * QB_ERR_INVALID_ARG unless width, height, fx, fy and near_plane are
 * positive and every field is finite (depth keys are the binary32 bits of
 * p.z, which sort correctly only for positive depths). */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float near_plane;
    float R[9];
    float t[3];
    float campos[3];
} qb_camera;

/* Projected record of one Gaussian, written by qb_project (48 bytes, 16-byte
 * aligned, array of N):
 *   u, v         image-plane mean (pixels)
 *   depth        view-space z (only meaningful when the Gaussian is visible)
 *   opacity      o = sigmoid(logit)
 *   a, b, c      conic Lambda = inverse(Sigma2D) = [a b; b c]
 *   gamma        2 ln(o / (1/255)): the 1/255 level of Eqs. (3), (4)
 *   r, g, bl     view-dependent colour from the SH coefficients
 *   visible      1.0f when the Gaussian survived culling, else 0.0f          */
typedef struct {
    float u, v, depth, opacity;
    float a, b, c, gamma;
    float r, g, bl, visible;
} qb_splat;

/* Per-Gaussian tile rects: four sub-boxes of (tx0, tx1, ty0, ty1), inclusive
 * tile bounds, int16 each (32 bytes).  An empty sub-box has tx0 > tx1.  The
 * Gaussian's tile set is the union of the four.  QB_BOX_3SIGMA and
 * QB_BOX_ADR store their single rect in slot 0. */
typedef struct {
    int16_t r[4][4];
} qb_rects;

/* ------------------------------------------------------------------------- */

/* qb_project -- Preprocess (Sec. 2) with the box of `mode` (Sec. 3.1) and
 * the tile count of the union of its sub-boxes (Sec. 3.2).
 *   n                number of Gaussians, 0 <= n < 2^31 (n = 0 is a no-op)
 *   means            [3][n] float, structure of arrays (x plane, y plane, z)
 *   log_scales       [3][n] float; scale s = exp(log_scale)
 *   quats            [4][n] float (w, x, y, z); need not be unit length
 *   opacity_logits   [n] float; opacity o = sigmoid(logit)
 *   sh               [(sh_degree+1)^2 * 3][n] float; plane k*3+ch holds SH
 *                    coefficient k = l*l + l + m of colour channel ch
 *   sh_degree        0..3
 *   cam              host pointer, read during the call only
 *   out_splats       [n] qb_splat
 *   out_rects        [n] qb_rects
 *   out_counts       [n] int32: number of tiles in the Gaussian's tile set
 *                    (0 when culled or off-screen)
 * Culled: p.z <= near, non-finite values, zero quaternion, det(Sigma2D) <= 0,
 * and (all modes but 3SIGMA) o <= 1/255. */
qb_status qb_project(int64_t n, const float* means, const float* log_scales, const float* quats,
                     const float* opacity_logits, const float* sh, int32_t sh_degree,
                     const qb_camera* cam, int32_t mode, qb_splat* out_splats,
                     qb_rects* out_rects, int32_t* out_counts, qb_stream_t stream);

/* qb_project_ex -- qb_project that also writes the keys of qb_intersect's
 * depth sort, so that qb_intersect_ex need not read the splats back for them:
 *   out_depth_keys   [n] uint32: float_bits(depth) where out_counts[i] > 0,
 *                    else 0xFFFFFFFF (the Gaussian emits no pair); may be
 *                    NULL, which is qb_project
 * Every other output as qb_project's. */
qb_status qb_project_ex(int64_t n, const float* means, const float* log_scales, const float* quats,
                        const float* opacity_logits, const float* sh, int32_t sh_degree,
                        const qb_camera* cam, int32_t mode, qb_splat* out_splats,
                        qb_rects* out_rects, int32_t* out_counts, uint32_t* out_depth_keys,
                        qb_stream_t stream);

/* The three binary32 activations of qb_project (each evaluated in binary64
 * and rounded once; Eq. (3) for gamma), on arbitrary inputs, so that their
 * agreement with another implementation can be checked on every binary32
 * value of a range:
 *   QB_ACT_SCALE     s = exp(log_scale)
 *   QB_ACT_OPACITY   o = sigmoid(logit) = 1 / (1 + exp(-logit))
 *   QB_ACT_GAMMA     gamma = 2 ln(255 o), from an opacity o
 * qb_project evaluates exactly these device functions. */
typedef enum { QB_ACT_SCALE = 0, QB_ACT_OPACITY = 1, QB_ACT_GAMMA = 2 } qb_activation;

/* qb_activations -- out[i] = activation `which` of x[i] for i < n (device
 * arrays of n floats; x and out may alias). */
qb_status qb_activations(int64_t n, const float* x, int32_t which, float* out, qb_stream_t stream);

/* Workspace bytes qb_intersect needs for n Gaussians. */
size_t qb_intersect_workspace_size(int64_t n);

/* qb_intersect -- DuplicateWithKeys with the QPass traversal (Sec. 2, 3.2).
 * Orders the Gaussians by (depth bits, id), takes the exclusive prefix sum of
 * their tile counts in that order, then writes for every tile of every
 * Gaussian's tile set, enumerated by QPass, exactly one pair
 *     (tile, id):  the pair with key (uint64)tile << 32 | float_bits(depth).
 * The pairs of one Gaussian are contiguous and the Gaussians appear in
 * ascending (depth, id) order; qb_sort relies on that order.
 *   splats, rects, counts   outputs of qb_project for the same n and camera
 *   width, height           image size; at most 65536 tiles
 *   mode                    the qb_box_mode given to qb_project; only
 *                           QB_BOX_QUADBOX_NAIVE changes the traversal (one
 *                           lane per Gaussian walks its sub-box rects)
 *   pair_capacity           entries available in pair_tiles / pair_ids
 *   pair_tiles, pair_ids    [pair_capacity] uint16 tile id / uint32 Gaussian id
 *   num_pairs               device int64: receives the total pair count P,
 *                           also when P > pair_capacity; then no pair is
 *                           written, qb_sort writes empty ranges and the
 *                           caller re-runs with a larger capacity
 *   workspace               qb_intersect_workspace_size(n) bytes
 * Returns QB_ERR_UNSUPPORTED for more than 65536 tiles, QB_ERR_INVALID_ARG
 * for an unknown mode. */
qb_status qb_intersect(int64_t n, const qb_splat* splats, const qb_rects* rects,
                       const int32_t* counts, int32_t width, int32_t height, int32_t mode,
                       int64_t pair_capacity,
                       uint16_t* pair_tiles, uint32_t* pair_ids, int64_t* num_pairs, void* workspace,
                       size_t workspace_bytes, qb_stream_t stream);

/* Launch shapes of qb_intersect's stages: the depth sort's radix workgroups
 * (lanes x keys per lane) and the emission's workgroup size (Gaussians per
 * workgroup).  Every combination gives the same pairs in the same order. */
typedef enum {
    QB_DEPTH_512x4 = 0,   /* 2048 keys per workgroup (qb_intersect's shape) */
    QB_DEPTH_256x8 = 1,   /* 2048 keys per workgroup                        */
    QB_DEPTH_512x8 = 2,   /* 4096 keys per workgroup                        */
    QB_DEPTH_1024x4 = 3,  /* 4096 keys per workgroup                        */
    QB_DEPTH_VARIANTS = 4
} qb_depth_variant;

typedef enum {
    QB_EMIT_256 = 0,      /* 256 Gaussians per workgroup (qb_intersect's)   */
    QB_EMIT_128 = 1,
    QB_EMIT_512 = 2,
    QB_EMIT_256_2CHAINS = 3,  /* 256, each wave walking two pair ranges at once */
    QB_EMIT_128_2CHAINS = 4,  /* 128, likewise                                   */
    QB_EMIT_VARIANTS = 5
} qb_emit_variant;

/* qb_pair_id_bits -- the id width of packed pairs for n Gaussians on a
 * width x height image: ceil(log2(n)) (at least 1) when that many id bits and
 * the tile id's bits fit 32 bits together, else 0 (pairs cannot be packed). */
int32_t qb_pair_id_bits(int64_t n, int32_t width, int32_t height);

/* qb_intersect_ex -- qb_intersect with the depth-sort keys written by
 * qb_project_ex for the same projection (depth_keys, [n] uint32, read only;
 * NULL: derived from splats and counts as qb_intersect does), explicit
 * launch shapes (a qb_depth_variant and a qb_emit_variant; the emission shape
 * does not apply to QB_BOX_QUADBOX_NAIVE) and a pair format:
 *   packed_id_bits   0: pairs as qb_intersect writes them; b > 0 (at most
 *                    qb_pair_id_bits): pair i is the one uint32
 *                    pair_ids[i] = tile << b | id and pair_tiles is not used
 *                    (may be NULL); QB_ERR_INVALID_ARG when n > 2^b or the
 *                    tile id and b exceed 32 bits together
 * Same workspace size, pair count and pair order as qb_intersect. */
qb_status qb_intersect_ex(int64_t n, const qb_splat* splats, const qb_rects* rects,
                          const int32_t* counts, int32_t width, int32_t height, int32_t mode,
                          int64_t pair_capacity, uint16_t* pair_tiles, uint32_t* pair_ids, int64_t* num_pairs,
                          void* workspace, size_t workspace_bytes, const uint32_t* depth_keys,
                          int32_t depth_variant, int32_t emit_variant, int32_t packed_id_bits,
                          qb_stream_t stream);

/* Workspace bytes qb_sort needs for a pair capacity. */
size_t qb_sort_workspace_size(int64_t pair_capacity);

/* qb_sort -- SortPairs (Sec. 2): the P = *num_pairs pairs written by
 * qb_intersect, in ascending (key, id) order, and per-tile ranges of the
 * sorted list:
 *   ranges[2t] = first index with tile >= t, ranges[2t+1] = first index with
 *   tile > t (empty tiles get start == end).
 * Only the tile bits are sorted (a stable LSD radix sort), since qb_intersect
 * emits the pairs in (depth, id) order.  When P > pair_capacity nothing is
 * sorted and every range is [0, 0).
 *   num_tiles              tiles_x * tiles_y, 1 .. 65536
 *   pair_tiles, pair_ids   from qb_intersect; not modified
 *   splats                 from qb_project; read only when keys != NULL
 *   keys                   [pair_capacity] uint64 sorted keys, or NULL to skip
 *   ids                    [pair_capacity] uint32 sorted Gaussian ids
 *   ranges                 [num_tiles][2] uint32                              */
qb_status qb_sort(int64_t pair_capacity, const int64_t* num_pairs, int32_t num_tiles,
                  const uint16_t* pair_tiles, const uint32_t* pair_ids, const qb_splat* splats,
                  uint64_t* keys, uint32_t* ids, uint32_t* ranges, void* workspace,
                  size_t workspace_bytes, qb_stream_t stream);

/* Launch shapes of the tile sort: lanes x pairs per lane of one radix
 * workgroup (larger workgroups write longer runs per digit and launch fewer
 * workgroups; smaller ones keep more workgroups per compute unit), and the
 * digit widths of its two passes over more than 8 tile bits (even by default:
 * 6 + 6 bits at 3600 tiles; the NARROW / WIDE variants give the first pass 2
 * bits fewer / more, within 1..8 bits per pass).  Every variant gives the
 * same sorted list and ranges. */
typedef enum {
    QB_SORT_512x8 = 0,    /* 4096 pairs per workgroup (qb_sort's shape) */
    QB_SORT_1024x8 = 1,   /* 8192 pairs per workgroup                   */
    QB_SORT_512x16 = 2,   /* 8192 pairs per workgroup                   */
    QB_SORT_256x16 = 3,   /* 4096 pairs per workgroup                   */
    QB_SORT_512x8_NARROW_FIRST = 4,  /* 512 x 8, first digit 2 bits narrower */
    QB_SORT_512x8_WIDE_FIRST = 5,    /* 512 x 8, first digit 2 bits wider    */
    QB_SORT_VARIANTS = 6
} qb_sort_variant;

/* qb_sort_ex -- qb_sort with an explicit launch shape (a qb_sort_variant,
 * chosen for example by timing each on the workload) and the pair format
 * qb_intersect_ex wrote (packed_id_bits: 0 for tiles and ids apart, b > 0
 * for packed pairs tile << b | id in pair_ids, pair_tiles then not used and
 * may be NULL; the radix passes then move 4 bytes per pair instead of 6).
 * Same results as qb_sort (plain ids, keys and ranges), the same workspace
 * size. */
qb_status qb_sort_ex(int64_t pair_capacity, const int64_t* num_pairs, int32_t num_tiles,
                     const uint16_t* pair_tiles, const uint32_t* pair_ids, const qb_splat* splats,
                     uint64_t* keys, uint32_t* ids, uint32_t* ranges, void* workspace,
                     size_t workspace_bytes, int32_t variant, int32_t packed_id_bits, qb_stream_t stream);

/* qb_render -- Eq. (2) per pixel over its tile's sorted list: front to back,
 * skipping a Gaussian where its quadratic form exceeds gamma (alpha < 1/255,
 * Eq. (4)), alpha = min(0.99, o exp(-q/2)), stopping before the first
 * Gaussian that would take T below 1e-4; output C + T * bg.
 *   ranges, ids      from qb_sort
 *   splats           from qb_project
 *   bg               host pointer to 3 floats
 *   image            [3][H][W] float
 *   final_T          [H][W] float (may be NULL)
 *   n_contrib        [H][W] uint32: 1 + list index of the last contributor,
 *                    0 if none (may be NULL)
 *   n_touched        [H][W] uint32: list entries the pixel examined, i.e. its
 *                    stop index, or the list length when it never stopped
 *                    (may be NULL; the count of Eq. (2) evaluations)        */
qb_status qb_render(int32_t width, int32_t height, const uint32_t* ranges, const uint32_t* ids,
                    const qb_splat* splats, const float* bg, float* image, float* final_T,
                    uint32_t* n_contrib, uint32_t* n_touched, qb_stream_t stream);

/* Launch shapes of the render (the same image, T and counts from each):
 * pixels per lane of a tile row (256 / pixels lanes per 16x16 tile), and
 * whether each wave first drops the batch entries whose cutoff ellipse cannot
 * reach its rows (a per-entry row range; pays off for loose boxes).  The
 * render backward accepts the first three and always drops such entries. */
typedef enum {
    QB_RENDER_2PX = 0,        /* 128 lanes, 2 pixels each (qb_render's shape)  */
    QB_RENDER_1PX = 1,        /* 256 lanes, 1 pixel each                       */
    QB_RENDER_4PX = 2,        /* 64 lanes, 4 pixels each                       */
    QB_RENDER_2PX_ROWS = 3,   /* 2 pixels each, row-range entry skip           */
    QB_RENDER_1PX_ROWS = 4,   /* 1 pixel each, row-range entry skip            */
    QB_RENDER_2PX_XROW = 5,   /* 2 pixels each; the row terms of the quadratic
                                 form computed once per tile row and shared
                                 across the row's lanes                        */
    QB_RENDER_4PX_XROW = 6,   /* 4 pixels each, row terms shared likewise      */
    QB_RENDER_2PX_XROW1 = 7,  /* as 2PX_XROW, one branch per entry instead of
                                 one per pair of entries                       */
    QB_RENDER_VARIANTS = 8
} qb_render_variant;

/* qb_tile_order -- the order in which the render's workgroups (one per
 * tile) take tiles, heaviest first.  Scheduling only: the render and its
 * backward compute every tile exactly as in row-major order; on a frame
 * where all tiles' workgroups are resident at once, this order decides how
 * evenly the work spreads over the compute units.
 *   work[t]   estimated cost of tile t: the number of list entries the tile's
 *             centre pixel (x0 + w/2, y0 + h/2 of the tile's pixel rect)
 *             examines before its transmittance drops below 1e-4 (Eq. (2)),
 *             followed over the first 256 entries with the transmittance
 *             carried as a sum of log2(1 - alpha) in binary32; a pixel still
 *             open there gets 256 * log2(1e-4) / log2(T_256) (its stop at the
 *             same rate of attenuation), capped at the list length, or the
 *             list length when T_256 = 1
 *   order     a permutation of 0 .. tiles-1, tiles in non-increasing
 *             min(work, 4095); equal values in no fixed order
 *   ranges, ids, splats   from qb_sort / qb_project for this frame
 *   work, order           [tiles_x * tiles_y] uint32 each                    */
qb_status qb_tile_order(int32_t width, int32_t height, const uint32_t* ranges, const uint32_t* ids,
                        const qb_splat* splats, uint32_t* work, uint32_t* order, qb_stream_t stream);

/* qb_render_ex -- qb_render with an explicit launch shape (chosen, for
 * example, by timing each on the workload) and tile order.  Same arguments
 * as qb_render plus `variant` (a qb_render_variant) and `tile_order`
 * (qb_tile_order's order, or NULL for row-major; entries >= the tile count
 * are skipped, so an order must be a permutation to render every tile);
 * results identical for every variant and order. */
qb_status qb_render_ex(int32_t width, int32_t height, const uint32_t* ranges, const uint32_t* ids,
                       const qb_splat* splats, const float* bg, float* image, float* final_T,
                       uint32_t* n_contrib, uint32_t* n_touched, int32_t variant, const uint32_t* tile_order,
                       qb_stream_t stream);

/* qb_render_stats -- qb_render_ex that also counts the work of Eq. (2) per
 * pixel, for measurement (the same image, T and contributor counts):
 *   n_touched      [H][W] uint32, required: list entries the pixel examined
 *                  (as in qb_render)
 *   n_composited   [H][W] uint32, required: entries that passed the 1/255
 *                  cutoff and were composited (the pixel's stop excluded)
 * Other arguments as qb_render_ex. */
qb_status qb_render_stats(int32_t width, int32_t height, const uint32_t* ranges, const uint32_t* ids,
                          const qb_splat* splats, const float* bg, float* image, float* final_T,
                          uint32_t* n_contrib, uint32_t* n_touched, uint32_t* n_composited, int32_t variant,
                          const uint32_t* tile_order, qb_stream_t stream);

/* qb_render_backward -- gradient of Eq. (2) (the rasterizer is trained
 * through; Sec. 4.1) with respect to each Gaussian's 2D parameters.  For
 * every pixel, walks its tile's list back to front from its last contributor,
 * re-evaluating the forward's alpha decisions, and accumulates
 *   grad2d[i] = dL/d(u, v, a, b, c, opacity, r, g, b)   (9 floats per Gaussian)
 * where (a, b, c) is the conic.  grad2d is cleared first, then summed with
 * float atomics (order-dependent rounding).
 *   ranges, ids, splats, bg   as given to qb_render for this frame
 *   final_T, n_contrib        qb_render's outputs for this frame
 *   dL_dimage                 [3][H][W] float
 *   n                         number of Gaussians (rows of grad2d)
 *   grad2d                    [n][9] float                                   */
qb_status qb_render_backward(int32_t width, int32_t height, const uint32_t* ranges, const uint32_t* ids,
                             const qb_splat* splats, const float* bg, const float* final_T,
                             const uint32_t* n_contrib, const float* dL_dimage, int64_t n, float* grad2d,
                             qb_stream_t stream);

/* qb_render_backward_ex -- qb_render_backward with an explicit launch shape
 * (a qb_render_variant: pixels per lane) and tile order (as for qb_render_ex;
 * the forward's order fits, the work per tile being alike); the same
 * gradients up to the order
 * of the float atomic additions. */
qb_status qb_render_backward_ex(int32_t width, int32_t height, const uint32_t* ranges, const uint32_t* ids,
                                const qb_splat* splats, const float* bg, const float* final_T,
                                const uint32_t* n_contrib, const float* dL_dimage, int64_t n, float* grad2d,
                                int32_t variant, const uint32_t* tile_order, qb_stream_t stream);

/* qb_project_backward -- chain rule from grad2d (qb_render_backward) to the
 * inputs of qb_project (Sec. 2, Eq. 1; the projection of Sec. 2): through the
 * conic inverse, the EWA covariance with its clamped Jacobian, the mean
 * projection, Sigma3D = R S S^T R^T, the quaternion normalisation, the
 * exp / sigmoid activations and the SH colour (no gradient where the colour
 * was clamped at 0).  The 1/255 cutoff, the 0.99 cap and the tile sets are
 * piecewise constant and contribute nothing.
 *   n .. cam          as given to qb_project; splats its output
 *   grad2d            [n][9] from qb_render_backward
 *   d_means .. d_sh   gradients in the input layouts ([3][n], [3][n], [4][n],
 *                     [n], [(sh_degree+1)^2 * 3][n]); culled Gaussians get 0 */
qb_status qb_project_backward(int64_t n, const float* means, const float* log_scales, const float* quats,
                              const float* opacity_logits, const float* sh, int32_t sh_degree,
                              const qb_camera* cam, const qb_splat* splats, const float* grad2d,
                              float* d_means, float* d_log_scales, float* d_quats, float* d_opacity_logits,
                              float* d_sh, qb_stream_t stream);

/* ---- Several views of one Gaussian set in one launch per stage ------------
 * For multi-view training (many cameras of one scene per step).  Each view
 * keeps its own projected splats, pairs, ranges and image; the preprocessing
 * of a view (qb_intersect, qb_sort) stays per view, while the stages below
 * treat all views at once: projection over (view, Gaussian), the render and
 * its backward over every (view, tile), and the projection backward over
 * Gaussians with the sum over views taken in registers.  At most
 * QB_MAX_VIEWS views per call; the per-view tables travel as kernel
 * arguments, so a call holds no device memory of its own and can be
 * captured in a HIP graph as long as the buffers stay put. */
#define QB_MAX_VIEWS 32

/* Per-view buffers of a batched forward/backward (device pointers). */
typedef struct {
    int32_t width, height;
    const uint32_t* ranges;  /* qb_sort ranges of this view                     */
    const uint32_t* ids;     /* qb_sort sorted Gaussian ids of this view         */
    const qb_splat* splats;  /* qb_project(_views) splats of this view, [n]      */
    float* image;            /* [3][height][width], written by qb_render_views   */
    float* final_T;          /* [height][width], written by qb_render_views      */
    uint32_t* n_contrib;     /* [height][width], written by qb_render_views      */
    const float* dL_dimage;  /* [3][height][width], read by the backward         */
    float* grad2d;           /* [n][9], cleared and written by the backward      */
} qb_view;

/* qb_project_views -- qb_project for num_views cameras in one launch.
 *   cams          host array of num_views cameras
 *   out_splats    [num_views][n] qb_splat;  out_rects [num_views][n];
 *   out_counts    [num_views][n] int32 (view v's block starts at v*n)
 * Same results per view as qb_project with that camera. */
qb_status qb_project_views(int64_t n, const float* means, const float* log_scales, const float* quats,
                           const float* opacity_logits, const float* sh, int32_t sh_degree,
                           const qb_camera* cams, int32_t num_views, int32_t mode, qb_splat* out_splats,
                           qb_rects* out_rects, int32_t* out_counts, qb_stream_t stream);

/* qb_project_views_ex -- qb_project_views that also writes each view's
 * depth-sort keys as qb_project_ex does: out_depth_keys [num_views][n] uint32
 * (NULL: qb_project_views). */
qb_status qb_project_views_ex(int64_t n, const float* means, const float* log_scales, const float* quats,
                              const float* opacity_logits, const float* sh, int32_t sh_degree,
                              const qb_camera* cams, int32_t num_views, int32_t mode, qb_splat* out_splats,
                              qb_rects* out_rects, int32_t* out_counts, uint32_t* out_depth_keys,
                              qb_stream_t stream);

/* qb_render_views -- qb_render of every view in one launch (one workgroup
 * per tile of every view).  views: host array; uses width, height, ranges,
 * ids, splats, image, final_T, n_contrib (final_T and n_contrib required).
 * Same image, T and contributor counts per view as qb_render. */
qb_status qb_render_views(int32_t num_views, const qb_view* views, const float* bg, qb_stream_t stream);

/* qb_tile_order_views -- qb_tile_order over the tiles of every view, in
 * one order: global tile b is tile b - start(v) of view v, where start(v) is
 * the tile count of views 0 .. v-1.  views as for qb_render_views (uses
 * width, height, ranges, ids, splats); work, order [total tiles] uint32. */
qb_status qb_tile_order_views(int32_t num_views, const qb_view* views, uint32_t* work, uint32_t* order,
                              qb_stream_t stream);

/* qb_render_views_ex -- qb_render_views with a launch shape (qb_render_variant)
 * and a tile order over global tiles (qb_tile_order_views, or NULL). */
qb_status qb_render_views_ex(int32_t num_views, const qb_view* views, const float* bg, int32_t variant,
                             const uint32_t* tile_order, qb_stream_t stream);

/* qb_render_backward_views -- qb_render_backward of every view in one
 * launch; each view's grad2d ([n][9]) is cleared first.  Uses every field of
 * each view except image. */
qb_status qb_render_backward_views(int32_t num_views, const qb_view* views, const float* bg, int64_t n,
                                   qb_stream_t stream);

/* qb_render_backward_views_ex -- with a launch shape (qb_render_variant) and a
 * tile order over global tiles (qb_tile_order_views, or NULL). */
qb_status qb_render_backward_views_ex(int32_t num_views, const qb_view* views, const float* bg, int64_t n,
                                      int32_t variant, const uint32_t* tile_order, qb_stream_t stream);

/* qb_project_backward_views -- gradients of the loss summed over views:
 * one lane per Gaussian runs the chain rule of qb_project_backward for each
 * view (camera cams[v], splats[v][n], grad2d[v][n][9]) and writes the sums
 * once (no atomics).  d_* as in qb_project_backward. */
qb_status qb_project_backward_views(int64_t n, const float* means, const float* log_scales, const float* quats,
                                    const float* opacity_logits, const float* sh, int32_t sh_degree,
                                    const qb_camera* cams, int32_t num_views, const qb_splat* splats,
                                    const float* grad2d, float* d_means, float* d_log_scales, float* d_quats,
                                    float* d_opacity_logits, float* d_sh, qb_stream_t stream);

/* A batched training step without the clear of grad2d (32 views of 2M
 * Gaussians hold 2.3 GB of it).  For callers that run the backward step
 * after step on the same grad2d buffers: the projection backward already
 * reads every row, so it can leave the rows at zero behind it, and the next
 * render backward then adds into them without clearing.  The caller keeps
 * the invariant "grad2d is all zero between steps": allocate it zeroed, and
 * after anything else wrote it (qb_render_backward_views_ex without
 * qb_project_backward_views_ex's clear) use the clearing entry points once. */

/* qb_render_backward_views_acc -- qb_render_backward_views_ex that adds to
 * each view's grad2d instead of clearing it first.  With grad2d all zero on
 * entry the result is bit-identical to qb_render_backward_views_ex. */
qb_status qb_render_backward_views_acc(int32_t num_views, const qb_view* views, const float* bg, int64_t n,
                                       int32_t variant, const uint32_t* tile_order, qb_stream_t stream);

/* qb_project_backward_views_ex -- qb_project_backward_views; clear_grad2d 1:
 * also sets every grad2d row to zero once read (grad2d is then written, hence
 * not const), with the same d_* bit for bit; 0: exactly
 * qb_project_backward_views.  INVALID_ARG for other clear_grad2d values and
 * wherever qb_project_backward_views returns it.  A row that is zero apart
 * from the sign of its zeros is left as it is. */
qb_status qb_project_backward_views_ex(int64_t n, const float* means, const float* log_scales, const float* quats,
                                       const float* opacity_logits, const float* sh, int32_t sh_degree,
                                       const qb_camera* cams, int32_t num_views, const qb_splat* splats,
                                       float* grad2d, float* d_means, float* d_log_scales, float* d_quats,
                                       float* d_opacity_logits, float* d_sh, int32_t clear_grad2d,
                                       qb_stream_t stream);

/* ---- Loss gradient of a training step -----------------------------------
 * Training (Sec. 4.1) drives the render backward with dL/dimage.  For the
 * mean absolute (L1) error of an image against a target, that gradient is
 * scale * sign(image - target) elementwise, scale = 1 / element count. */
typedef struct {
    int64_t count;        /* elements (3 * width * height for an image), >= 0  */
    const float* image;   /* [count] rendered image (device)                   */
    const float* target;  /* [count] target (device)                           */
    float* grad;          /* [count] written: scale * sign(image - target)     */
    float scale;          /* the factor of the sign                            */
} qb_l1_item;

/* qb_l1_grad -- grad = scale * sign(image - target) for every item, one
 * launch for all of them.  sign is +1, -1 or 0 (for equal values, either
 * zero, and NaN), so grad holds exactly +scale, -scale or +0.
 *   num_items   0 .. QB_MAX_VIEWS (0 is a no-op)
 *   items       host array of num_items items; pointers may be NULL only
 *               where count is 0; grad must not overlap image or target
 * Returns QB_ERR_INVALID_ARG (before any device work) for a count < 0, a
 * missing pointer or num_items out of range. */
qb_status qb_l1_grad(int32_t num_items, const qb_l1_item* items, qb_stream_t stream);

/* qb_check_capacity -- the pair-capacity check of a frame (Sec. 2: the pair
 * buffers of DuplicateWithKeys are sized before the frame).  qb_intersect
 * writes the true pair count P to its device num_pairs also when P exceeds
 * pair_capacity; it then emits no pair, qb_sort writes empty ranges and the
 * frame renders no Gaussian.  Because the count lives on the device, no
 * asynchronous call can report the overflow; this call does, once per frame
 * (or per multi-view step), outside any HIP graph capture:
 *   count        number of frames (views) to check, >= 1
 *   num_pairs    DEVICE array [count] int64: the num_pairs of each frame's
 *                qb_intersect (for one frame, its single int64)
 *   capacities   HOST array [count] int64: the pair_capacity each was given
 *   out_counts   HOST array [count] int64 receiving the counts, or NULL when
 *                count <= 64
 * Waits for the work queued on `stream` (the counts are read after it) and
 * returns QB_ERR_CAPACITY when any count exceeds its capacity (the caller
 * grows the pair and sort buffers and runs the frame again), QB_ERR_HIP when
 * the copy or the wait fails, QB_OK otherwise.  The only entry point that
 * synchronises. */
qb_status qb_check_capacity(int32_t count, const int64_t* num_pairs, const int64_t* capacities,
                            int64_t* out_counts, qb_stream_t stream);

/* qb_intersect_noalloc -- qb_intersect for callers that cannot allocate
 * device memory: code recorded under HIP graph capture that may not call
 * hipMalloc, tight serving loops, and harnesses that forbid allocation.  It
 * takes no workspace: its scratch (the depth sort's buffers, the pair offsets
 * and the scan partials, qb_intersect_workspace_size(n) bytes) lives in a
 * static device array of the library, 60 MiB, one copy on every GPU the
 * library runs on, held from the library's load until the process ends.
 * The call itself allocates nothing: no hipMalloc, no hipFree, no
 * allocating library routine.  The first call on a device looks up that
 * device's copy (hipGetSymbolAddress, with the device current).
 *   n         0 <= n <= QB_NOALLOC_MAX_GAUSSIANS; a larger n returns
 *             QB_ERR_INVALID_ARG (use qb_intersect with a workspace)
 *   others    as for qb_intersect; the outputs are identical to qb_intersect's
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (each call writes every scratch value it reads, so nothing needs
 * clearing): calls that overlap on one GPU -- on different streams, or from
 * different host threads without ordering -- race and give wrong results.
 * Returns QB_ERR_HIP when the device's copy cannot be looked up. */
#define QB_NOALLOC_MAX_GAUSSIANS 2097152
qb_status qb_intersect_noalloc(int64_t n, const qb_splat* splats, const qb_rects* rects,
                               const int32_t* counts, int32_t width, int32_t height, int32_t mode,
                               int64_t pair_capacity, uint16_t* pair_tiles, uint32_t* pair_ids,
                               int64_t* num_pairs, qb_stream_t stream);

/* Human-readable name of a status code (static string). */
const char* qb_status_string(qb_status s);

/* Library version, major*10000 + minor*100 + patch. */
int32_t qb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QUADBOX_H */
