/*
 * gs.h -- C ABI of the MI355X (gfx950) rendering path of CityGaussian
 * (arXiv 2404.01133): block-wise level-of-detail selection (Sec. 3.3.2) feeding
 * a differentiable tile-based 3D Gaussian splatting rasterizer (Sec. 3.1, Eq. 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Memory: every array argument is DEVICE memory allocated and owned by the
 *    caller, unless its comment says "host".  The library never allocates or
 *    frees; scratch comes from a caller-provided workspace whose size is given
 *    by gs_workspace_bytes().
 *  - Streams: every call is asynchronous and ordered on `stream` (a
 *    hipStream_t passed as void*; NULL = the default stream).  Argument checks
 *    happen on the host before any launch; a failed check returns an error
 *    code and launches nothing.
 *  - Sizes that depend on the data (selected Gaussians, visible Gaussians,
 *    tile pairs) stay on the device, in the caller's `counts` array (int64[8],
 *    see GS_COUNT_*), so a whole frame can be captured in a HIP graph.  Each
 *    stage clamps to the capacity the caller passed and raises a bit in
 *    counts[GS_COUNT_FLAGS] when a capacity was too small; the outputs of that
 *    frame are then invalid and the caller re-runs with larger buffers.
 *  - Gaussians are structure-of-arrays FP32:
 *        means [3][n], scales [3][n] (> 0), quats [4][n] (w, x, y, z, any norm > 0),
 *        opac [n] in (0, 1), sh [16][3][n] (degree-3 real SH, coefficient-major).
 *    Gaussians with non-finite geometry, a zero quaternion or opacity below
 *    1/255 are culled silently; they are not errors.
 *  - Cameras: world->camera rotation R (row-major) and translation t, camera
 *    axes x right, y down, z forward; pixel (i, j) has centre (i + 0.5, j + 0.5);
 *    every view of one call has the same width and height.
 *  - Images: rgb [V][3][H][W] FP32, transmittance T_final [V][H][W], and
 *    n_last [V][H][W] = number of tile-list entries walked by each pixel
 *    (consumed by the backward pass).
 *  - Return value: GS_OK or a negative gs_status.  gs_status_string() names it;
 *    after GS_ERR_HIP it also carries the HIP error text of the calling thread.
 */
#ifndef GS_H_
#define GS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gs_status;
#define GS_OK 0
#define GS_ERR_INVALID_ARG (-1)
#define GS_ERR_UNSUPPORTED (-2)
#define GS_ERR_WORKSPACE (-3)
#define GS_ERR_CAPACITY (-4)
#define GS_ERR_HIP (-5)
#define GS_ERR_SCRATCH (-6) /* capacities need more scratch than GS_STATIC_SCRATCH_BYTES */

/* indices into the device int64 counts[8] array */
#define GS_COUNT_RECORDS 0 /* selected (view, Gaussian) records, written by gs_lod_select */
#define GS_COUNT_VISIBLE 1 /* records that survived culling, written by gs_bin_sort */
#define GS_COUNT_PAIRS 2   /* (tile, record) pairs, written by gs_bin_sort */
#define GS_COUNT_FLAGS 3   /* bit 0: record capacity exceeded; bit 1: pair capacity exceeded;
                              bit 2: a device-side wait gave up (see GS_FLAG_WAIT);
                              bit 3: GS_TUNE_SHARED_SELECTION was set but the views did not
                              select the same records (see GS_FLAG_SELECTION) */
#define GS_COUNT_SLOTS 8
#define GS_FLAG_RECORDS 1
#define GS_FLAG_PAIRS 2
#define GS_FLAG_WAIT 4
#define GS_FLAG_SELECTION 8

/* Camera (device array [V] of these; 152 bytes, 8-byte aligned). */
typedef struct gs_camera {
  double R[9];   /* world -> camera rotation, row-major */
  double t[3];   /* world -> camera translation */
  double fx, fy; /* focal lengths, pixels */
  double cx, cy; /* principal point, pixels */
  double znear;  /* Gaussians and block corners need camera z > znear */
  int32_t width, height;
  int32_t pad[2];
} gs_camera;

/* One detail level of the scene: device SoA arrays (see conventions).
 * Centres are always FP32.  A coarse level may store its other attributes at
 * lower precision and fewer SH bands (Sec. 3.3.1: distant levels need less
 * feature dimension and lower data precision):
 *   attr_half = 1: scales, quats, opac and sh are IEEE binary16 arrays
 *   sh_degree:     bands stored, 0..3; sh holds (sh_degree + 1)^2 coefficient
 *                  planes [K][3][n]; a render uses min(its sh_degree, this)
 * gs_gaussians values of zero for both fields mean FP32 with sh_degree 0, so
 * callers set sh_degree explicitly (3 for full SH). */
typedef struct gs_gaussians {
  const float* means; /* [3][n] FP32 */
  const void* scales; /* [3][n] */
  const void* quats;  /* [4][n] */
  const void* opac;   /* [n] */
  const void* sh;     /* [(sh_degree+1)^2][3][n] */
  int64_t n;
  int32_t sh_degree;
  int32_t attr_half;
} gs_gaussians;

/* Gradient buffers with the shapes of gs_gaussians, always FP32 (device, accumulated +=);
 * sh has the level's stored (sh_degree+1)^2 planes. */
typedef struct gs_gaussian_grads {
  float* means;
  float* scales;
  float* quats;
  float* opac;
  float* sh;
} gs_gaussian_grads;

/* Block table (all pointers device).  Block b of level l occupies
 * [lvl_off[b*L + l], lvl_off[b*L + l] + lvl_cnt[b*L + l]) of level l's arrays.
 * lo/hi are the block's bounding box (Eq. 6), cell its half-open xy cell.
 * contraction: NULL (cells are world xy rectangles), or device double[6] =
 * p_min[3], p_max[3] of the foreground box of a contracted partition
 * (gs_partition): cells are then rectangles of the contracted x, y, and the
 * camera centre is normalised and contracted (Eq. 2) before the cell test. */
typedef struct gs_blocks {
  const double* lo;       /* [B][3] */
  const double* hi;       /* [B][3] */
  const double* cell;     /* [B][4] = x0, x1, y0, y1 */
  const int64_t* lvl_off; /* [B][L] */
  const int64_t* lvl_cnt; /* [B][L] */
  int32_t n_blocks;
  int32_t n_levels;
  const double* contraction; /* NULL or [6] */
} gs_blocks;

/* Launch shape of the tile kernels.  tile_w x tile_h pixels per tile
 * (supported: 16x16, 8x8, 16x8, 32x8, 32x16); batch = Gaussians staged in LDS per
 * round (64, 128 or 256).  The image does not depend on these choices. */
typedef struct gs_tuning {
  int32_t tile_w, tile_h;
  int32_t batch;
  int32_t flags; /* GS_TUNE_* bits */
} gs_tuning;

/* tuning.flags: every view of the call selected the same records (gs_lod_select in
 * GS_LOD_ALL_FINEST mode, e.g. several training views of one block).  preprocess and
 * rasterize_bwd then iterate Gaussian-major: one thread handles a Gaussian for all
 * views, reading its parameters from HBM once and accumulating its gradient without
 * atomics.  Segments and levels of view 0 are used for every view.  gs_preprocess
 * checks this on the device: if the record count is not V times view 0's, or a
 * view's segment offsets or levels differ from view 0's (shifted by its first
 * record), it raises GS_FLAG_SELECTION, marks every record culled (tiles_touched
 * 0) and projects nothing, so the frame is empty; gs_rasterize_bwd then adds
 * nothing.  Block-wise selections only (with a point-wise gather list the flag
 * returns GS_ERR_UNSUPPORTED). */
#define GS_TUNE_SHARED_SELECTION 1
/* tuning.flags: rasterize_fwd / rasterize_bwd run as persistent kernels that take
 * tiles from a device work queue, longest tile lists first. */
#define GS_TUNE_WORK_QUEUE 2
/* tuning.flags: bit-reproducible gradients from gs_rasterize_bwd (Sec. 3.1, the
 * adjoint of Eq. 1 summed over pixels, tiles and views).  Without it partial
 * sums are added with FP32 atomics, whose order varies from run to run.  With
 * it every sum has a fixed order: within a tile, per-quadrant sums are added in
 * quadrant order; each (tile, record) partial goes to its own workspace slot
 * and a record's slots are summed in ascending tile order; a Gaussian's
 * records are summed in view order.  Costs a larger workspace (36 bytes per
 * pair of capacity, see gs_workspace_bytes) and time.  Supported for one view,
 * for GS_TUNE_SHARED_SELECTION, and for several block-wise views (then each
 * level must store its blocks in ascending block order); several point-wise
 * views return GS_ERR_UNSUPPORTED.  Ignored by the other entry points. */
#define GS_TUNE_DETERMINISTIC 4
/* tuning.flags, gs_preprocess and gs_rasterize_bwd: the selection is a packed
 * gather list from gs_lod_refine (entries level << GS_PACKED_INDEX_BITS | index
 * within the level, offsets [V+1] per view, level unused).  gs_rasterize_bwd
 * returns GS_ERR_UNSUPPORTED for it with GS_TUNE_SHARED_SELECTION, or with
 * GS_TUNE_DETERMINISTIC and several views. */
#define GS_TUNE_PACKED_SELECTION 8

/* Size in bytes of one projected record (an opaque device structure). */
size_t gs_record_bytes(void);

/* Workspace needed by gs_bin_sort / gs_rasterize_bwd for the given capacities
 * (for gs_rasterize_bwd with GS_TUNE_DETERMINISTIC in tuning->flags, size it
 * with the pair capacity given to gs_bin_sort: it holds one slot per pair). */
#define GS_WS_BIN_SORT 1
#define GS_WS_RASTERIZE_BWD 2
size_t gs_workspace_bytes(int32_t which, int64_t record_capacity, int64_t pair_capacity, int32_t n_views,
                          int32_t width, int32_t height, const gs_tuning* tuning /* host */);

/* Block-wise level-of-detail selection (Sec. 3.3.2).
 * For every (view v, block b): the level is chosen from the minimum distance
 * between the camera centre and the eight corners of the block's box, against
 * the ascending distance thresholds (half-open intervals; near = finest level
 * L-1); the block is kept if the bounding box of its corners in front of the
 * camera (z > znear), projected, overlaps the screen with positive area, or if
 * the camera's xy lies in the block's cell.  The chosen levels are concatenated
 * in block order (the aggregation step), as offsets into one record space:
 *   level   [V][B] int8: chosen level or -1 (not rendered)
 *   offsets [V*B + 1] int64: record range of (v, b) is [offsets[v*B+b], offsets[v*B+b+1])
 *   counts[GS_COUNT_RECORDS] = offsets[V*B].
 * mode: GS_LOD_BLOCKWISE (the paper's method) or GS_LOD_ALL_FINEST (every
 * non-empty block at level L-1, no culling: the plain comparator).
 * thresholds: host array [L-1], ascending, scene units. */
#define GS_LOD_BLOCKWISE 0
#define GS_LOD_ALL_FINEST 1
gs_status gs_lod_select(const gs_blocks* blocks /* host struct */, const double* thresholds /* host */,
                        int32_t mode, const gs_camera* cams, int32_t n_views, int8_t* level, int64_t* offsets,
                        int64_t* counts, void* stream);

/* Point-wise level-of-detail selection: the baseline Sec. 3.3.2 sets against
 * the block-wise strategy (ablated in Table 5).  Each Gaussian of each level is
 * tested on its own: level l keeps the Gaussians whose centre distance to the
 * camera centre lies in level l's interval (same thresholds and numbering as
 * gs_lod_select: near = finest level L-1) and whose centre is in the frustum:
 * camera z > znear and projection (u, v) with -0.15 W < u < 1.15 W and
 * -0.15 H < v < 1.15 H.  All tests are FP64 in a fixed operation order.
 *   levels: host array [n_levels] of device Gaussian sets (only means are read)
 *   thresholds: host array [n_levels-1], ascending, scene units
 *   gather [record_capacity] u32: the selection, index within the level
 *   offsets [V*L + 1] int64: segment v*L + l (view v, level l) is
 *     gather[offsets[v*L+l] .. offsets[v*L+l+1]), ascending indices
 *   counts[GS_COUNT_RECORDS] = offsets[V*L]; GS_FLAG_RECORDS is raised (and the
 *     gather list truncated) if that exceeds record_capacity
 *   ws / ws_bytes: workspace of at least gs_points_workspace_bytes(...).
 * The selection feeds gs_preprocess / gs_rasterize_bwd through their gather
 * argument. */
size_t gs_points_workspace_bytes(const int64_t* level_sizes /* host [n_levels] */, int32_t n_levels,
                                 int32_t n_views);
gs_status gs_lod_select_points(const gs_gaussians* levels, int32_t n_levels, const double* thresholds,
                               const gs_camera* cams, int32_t n_views, int64_t record_capacity, uint32_t* gather,
                               int64_t* offsets, int64_t* counts, void* ws, size_t ws_bytes, void* stream);

/* Chunk refinement of a block-wise selection (between the selection of Sec.
 * 3.3.2 and the projection of Eq. 1; it changes no rendered value).  Every
 * (block, level) run is cut into chunks of GS_CHUNK Gaussians in storage order.
 * gs_chunk_bounds (once per scene) keeps per chunk the box of its centres and
 * its largest scale component; gs_lod_refine drops, per view, the chunks of the
 * selected runs that the projection would cull whole (the box behind the near
 * plane, or its projection farther outside the image than a bound on the
 * 3-sigma radius of any Gaussian of the chunk) and lists the records left, in
 * the block-wise order, so gs_preprocess (with GS_TUNE_PACKED_SELECTION), the
 * binning and the compositing give the same images as with the unrefined
 * selection.
 *   gs_chunk_capacity: host helper, entries to allocate for chunk tables (-1 on
 *     bad arguments); levels host [n_levels]
 *   gs_chunk_bounds: chunk_off [B*L + 1] int64 (first chunk of run b*L + l, then
 *     the total), bounds [max_chunks][8] f32 (lo xyz, hi xyz, largest |scale|,
 *     the run b*L + l as int32 bits); GS_ERR_CAPACITY if max_chunks <
 *     gs_chunk_capacity, GS_ERR_UNSUPPORTED if a level holds 2^GS_PACKED_INDEX_BITS
 *     Gaussians or more
 *   gs_lod_refine: level from gs_lod_select; gather [record_capacity] u32
 *     (level << GS_PACKED_INDEX_BITS | index); view_offsets [V + 1] int64;
 *     counts[GS_COUNT_RECORDS] = records kept; GS_FLAG_RECORDS is raised (and
 *     the list truncated) past record_capacity or if the chunk table holds more
 *     than max_chunks; ws / ws_bytes: at least gs_refine_workspace_bytes(V,
 *     max_chunks); chunk_off and bounds as gs_chunk_bounds wrote them.
 * All arrays are caller-owned device memory except the host structures noted;
 * calls are ordered on `stream`.  The tables describe the Gaussians as they were
 * when gs_chunk_bounds ran: rebuild them after moving or rescaling Gaussians,
 * or visible Gaussians may be dropped.  Errors: GS_ERR_INVALID_ARG (NULL
 * pointers, sizes out of range, record_capacity >= 2^32, V * max_chunks >=
 * 2^31), GS_ERR_WORKSPACE (ws_bytes too small), before any launch. */
#define GS_CHUNK 2048
#define GS_PACKED_INDEX_BITS 29
int64_t gs_chunk_capacity(const gs_gaussians* levels /* host [n_levels] */, const gs_blocks* blocks /* host */);
gs_status gs_chunk_bounds(const gs_gaussians* levels, const gs_blocks* blocks, int64_t* chunk_off, float* bounds,
                          int64_t max_chunks, void* stream);
size_t gs_refine_workspace_bytes(int32_t n_views, int64_t max_chunks);
gs_status gs_lod_refine(const gs_blocks* blocks, const int8_t* level, const gs_camera* cams, int32_t n_views,
                        int32_t width, int32_t height, const int64_t* chunk_off, const float* bounds,
                        int64_t max_chunks, int64_t record_capacity, uint32_t* gather, int64_t* view_offsets,
                        int64_t* counts, void* ws, size_t ws_bytes, void* stream);

/* Projection of every selected record (Sec. 3.1, "proj" in Eq. 1, following
 * 3DGS): EWA splat of the 3D covariance R S S^T R^T through the pinhole
 * Jacobian (guard band 1.3x the half field of view) with a 0.3 px^2 dilation,
 * 3-sigma screen footprint, view-dependent colour from degree <= sh_degree real
 * SH (clamped at 0), depth = camera z.  Geometry is computed in FP64 in a fixed
 * operation order so footprints and depth keys are reproducible bit for bit.
 *   levels: host array [n_levels] of device Gaussian sets
 *   selection: gather == NULL: block-wise, from gs_lod_select (level, offsets
 *     [V*B+1]); gather != NULL: point-wise, from gs_lod_select_points (offsets
 *     [V*L+1], level unused and may be NULL, blocks only supplies n_levels);
 *     with GS_TUNE_PACKED_SELECTION: refined, from gs_lod_refine (packed
 *     gather, offsets [V+1])
 *   records [record_capacity] of gs_record_bytes(); depth_keys [record_capacity]
 *   u32 (float bits of depth; 0xFFFFFFFF if culled); tiles_touched
 *   [record_capacity] int32 (0 if culled). */
gs_status gs_preprocess(const gs_gaussians* levels, const gs_blocks* blocks, const int8_t* level,
                        const int64_t* offsets, const uint32_t* gather, const gs_camera* cams, int32_t n_views,
                        int32_t width,
                        int32_t height, int32_t sh_degree, const gs_tuning* tuning, int64_t record_capacity,
                        void* records, uint32_t* depth_keys, int32_t* tiles_touched, int64_t* counts,
                        void* stream);

/* Tile binning (Sec. 3.1, Eq. 1): the colour of a pixel blends the Gaussians
 * that cover it in depth order, front to back; this call lists, per screen
 * tile, the visible records whose footprint meets the tile in that order.
 * One (tile, record) pair per tile under each visible record's footprint,
 * sorted by (view*tiles + tile, depth, record index) with a stable LSD radix
 * sort (depth digits on the visible records, tile digits on the pairs), so
 * ties go to the lower record index.
 * Inputs: records, depth_keys and tiles_touched as written by gs_preprocess
 * with the same width, height and tile shape (record_capacity entries;
 * counts[GS_COUNT_RECORDS] of them are read; tiles_touched must equal the
 * tiles under each record's footprint, which the binning also derives from the
 * record itself).
 * Writes counts[GS_COUNT_VISIBLE] and counts[GS_COUNT_PAIRS]; raises
 * GS_FLAG_PAIRS (pairs beyond pair_capacity are dropped, the frame is
 * invalid) and GS_FLAG_WAIT.  Errors: GS_ERR_INVALID_ARG for NULL pointers,
 * non-positive sizes or capacities of 2^30 and more; GS_ERR_UNSUPPORTED for a
 * tile shape outside the supported list; GS_ERR_WORKSPACE when ws_bytes is too
 * small.
 *   pair_tiles / pair_records [pair_capacity] u32: sorted pairs
 *   tile_ranges [V*tiles][2] u32: [start, end) of each tile in the sorted pairs
 *   tile_queue: NULL, or u32[2 + V*tiles]; with GS_TUNE_WORK_QUEUE it receives the
 *     tiles ordered by decreasing list length (power-of-two buckets) and its two
 *     head counters are reset, for the persistent tile kernels
 *   ws / ws_bytes: workspace of at least gs_workspace_bytes(GS_WS_BIN_SORT, ...). */
gs_status gs_bin_sort(const void* records, const uint32_t* depth_keys, const int32_t* tiles_touched,
                      int32_t n_views, int32_t width, int32_t height, const gs_tuning* tuning,
                      int64_t record_capacity, int64_t pair_capacity, uint32_t* pair_tiles,
                      uint32_t* pair_records, uint32_t* tile_ranges, uint32_t* tile_queue, int64_t* counts,
                      void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory at all (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): gs_bin_sort
 * with its workspace taken from a library-owned device array of
 * GS_STATIC_SCRATCH_BYTES (64 MiB), one copy per GPU, held from the library's
 * first call on that GPU until the process ends.  Same arguments, outputs,
 * flags and errors as gs_bin_sort, without ws / ws_bytes, plus:
 *   GS_ERR_SCRATCH when gs_workspace_bytes(GS_WS_BIN_SORT, record_capacity,
 *     pair_capacity, ...) exceeds GS_STATIC_SCRATCH_BYTES (about 25 B per
 *     record of capacity plus 10 B per pair of capacity; e.g. 1M records with
 *     4M pairs fit); nothing is launched.
 *   GS_ERR_HIP if the array's device address cannot be obtained.
 * It calls no allocating routine.  The array is looked up for the device that is
 * current at the call, which must be the device of `stream`.  Every call on one
 * GPU uses the same array and leaves its contents behind (each call clears what
 * it needs first): two calls that overlap in time on one GPU (different
 * streams, or different host threads, without ordering) race and give wrong
 * results. */
#define GS_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
gs_status gs_bin_sort_static(const void* records, const uint32_t* depth_keys, const int32_t* tiles_touched,
                             int32_t n_views, int32_t width, int32_t height, const gs_tuning* tuning,
                             int64_t record_capacity, int64_t pair_capacity, uint32_t* pair_tiles,
                             uint32_t* pair_records, uint32_t* tile_ranges, uint32_t* tile_queue, int64_t* counts,
                             void* stream);

/* Per-tile front-to-back alpha compositing of Eq. 1: for each pixel, walk its
 * tile's list; skip entries whose footprint does not hold the pixel; alpha =
 * min(0.99, opacity * exp(-d^T conic d / 2)); skip alpha < 1/255; stop before an
 * entry that would take the transmittance below 1e-4.
 *   bg: host float[3] background colour.
 *   tile_queue: NULL (one work-group per tile), or the queue gs_bin_sort filled
 *     with GS_TUNE_WORK_QUEUE (persistent work-groups take tiles from it, using
 *     the first head counter; the last work-group to finish puts it back to
 *     zero, so the call can be repeated on the same sorted frame).  Two calls
 *     that share a queue must not overlap in time (same stream, or ordered). */
gs_status gs_rasterize_fwd(const void* records, const uint32_t* pair_records, const uint32_t* tile_ranges,
                           uint32_t* tile_queue, int32_t n_views, int32_t width, int32_t height, const float* bg,
                           const gs_tuning* tuning, float* rgb, float* T_final, int32_t* n_last, void* stream);

/* Adjoint of the forward pass (Sec. 3.1, differentiable rendering): given
 * d_rgb = dL/d rgb [V][3][H][W], accumulates (+=) dL/d(parameters) into
 * grads[n_levels] (host array of device buffers shaped like the levels).  The
 * blend state of each pixel is recomputed front to back from the saved T_final
 * and n_last, so no per-(pixel, Gaussian) state is stored.  Accumulation uses
 * FP32 atomics: results are reproducible to rounding, not bit for bit, unless
 * tuning->flags holds GS_TUNE_DETERMINISTIC (then bit for bit; the workspace
 * then holds one slot per pair: pairs beyond the slots it has are not summed,
 * so it must be sized with the pair capacity the frame was binned with).
 * tile_queue: as for gs_rasterize_fwd (uses the second head counter, reset the same
 *   way, so several backward calls may follow one forward).
 * level / offsets / gather: the selection passed to gs_preprocess (a refined one
 *   with GS_TUNE_PACKED_SELECTION in tuning->flags, as there).
 * ws: at least gs_workspace_bytes(GS_WS_RASTERIZE_BWD, ...). */
gs_status gs_rasterize_bwd(const void* records, const uint32_t* pair_records, const uint32_t* tile_ranges,
                           uint32_t* tile_queue, int32_t n_views, int32_t width, int32_t height, const float* bg,
                           const gs_tuning* tuning, const float* rgb, const float* T_final, const int32_t* n_last,
                           const float* d_rgb, const gs_gaussians* levels, const gs_blocks* blocks,
                           const int8_t* level, const int64_t* offsets, const uint32_t* gather,
                           const gs_camera* cams, int32_t sh_degree, int64_t record_capacity,
                           const int64_t* counts, const gs_gaussian_grads* grads,
                           void* ws, size_t ws_bytes, void* stream);

/* Block bounds of Eq. 6 for every block from its finest-level centres:
 * per axis, med = lower median (rank floor((n-1)/2)), MAD = lower median of
 * |p - med| (FP64), lo = max(min p, med - n_mad * MAD), hi = min(max p,
 * med + n_mad * MAD).  Empty blocks get lo = +inf, hi = -inf.
 *   finest: device Gaussian set of the finest level; lvl_off/lvl_cnt: device
 *   [B][L]; lo, hi: device [B][3] FP64.  ws: gs_mad_workspace_bytes(). */
size_t gs_mad_workspace_bytes(int64_t max_block_count);
gs_status gs_mad_bounds(const gs_gaussians* finest, const int64_t* lvl_off, const int64_t* lvl_cnt,
                        int32_t n_blocks, int32_t n_levels, int64_t max_block_count, double n_mad, double* lo,
                        double* hi, void* ws, size_t ws_bytes, void* stream);

/* Block partition of a Gaussian cloud (Sec. 3.2.2, Eq. 2), the set-up step
 * that builds the block table.  Per centre p (FP64, fixed operation order):
 * p_hat_i = (2 (p_i - min_i)) / (max_i - min_i) - 1 with the foreground box
 * x, y from xy_box and z from the min and max centre z; c = p_hat if
 * max_i |p_hat_i| <= 1, else (2 - 1/n) (p_hat / n) with n = max_i |p_hat_i|;
 * ix = number of boundaries -2 + 4k/nx (k = 1 .. nx-1) <= c_x, iy likewise
 * for c_y; block = iy * nx + ix.
 *   means: device [3][n] FP32 centres (finite)
 *   xy_box: host double[4] = x_a, y_a, x_b, y_b (the ends of each interval in
 *     either order; the extents must be non-zero)
 *   block_id: device u32[n] or NULL; perm: device u32[n], the Gaussians listed
 *     block by block, ascending original index inside a block (stable)
 *   block_off: device int64[nx*ny + 1]: block b is perm[block_off[b] .. block_off[b+1])
 *   cells: device double[nx*ny][4] or NULL: each block's cell in contracted
 *     x, y (the boundaries above, outermost ends infinite), for gs_blocks.cell
 *     together with gs_blocks.contraction
 *   nx * ny <= 65536; ws: gs_partition_workspace_bytes(n). */
size_t gs_partition_workspace_bytes(int64_t n);
gs_status gs_partition(const float* means, int64_t n, const double* xy_box, int32_t nx, int32_t ny,
                       uint32_t* block_id, uint32_t* perm, int64_t* block_off, double* cells, void* ws,
                       size_t ws_bytes, void* stream);

/* dst = src[perm]: every attribute array of a Gaussian set gathered into a new
 * order (dst holds n Gaussians; src->n is the source count; perm entries
 * < src->n).  Used to store a partitioned set block by block.  FP32 sets only
 * (attr_half = 0, else GS_ERR_UNSUPPORTED); sh_degree planes are gathered. */
gs_status gs_gather_gaussians(const gs_gaussians* src, const uint32_t* perm, int64_t n,
                              const gs_gaussian_grads* dst, void* stream);

/* ---- training-data assignment (Sec. 3.2.2, Eqs. 3-5) ------------------------
 * Eq. 3 compares, per pose, the render of every block with the render without
 * block j.  gs_lod_select_exclude selects, for view v, every block at the
 * finest level except block exclude[v] (device int32[V]; -1 = none), no cull;
 * outputs as gs_lod_select. */
gs_status gs_lod_select_exclude(const gs_blocks* blocks /* host struct */, const gs_camera* cams, int32_t n_views,
                                const int32_t* exclude, int8_t* level, int64_t* offsets, int64_t* counts,
                                void* stream);

/* Records of each selection segment that survived the preprocess cull
 * (tiles_touched > 0): visible[p] for segment p of offsets[n_segments + 1]
 * (device arrays).  A block with no visible record in a pose cannot change its
 * render, so its leave-one-out render can be skipped (SSIM = 1 exactly). */
gs_status gs_segment_visible(const int32_t* tiles_touched, const int64_t* offsets, int32_t n_segments,
                             int64_t record_capacity, int32_t* visible, void* stream);

/* SSIM (Wang et al. 2004) of image pairs: 11 x 11 Gaussian window, std 1.5,
 * normalised, zero padding outside the image, C1 = 0.01^2, C2 = 0.03^2, mean
 * over pixels and the three channels.  images: device [n_images][3][H][W]
 * FP32; pairs: device int32 [n_pairs][2] image indices (an index out of range
 * gives NaN); ssim: device float[n_pairs].  FP32 filtering, FP64 sums reduced
 * in a fixed order (deterministic).  ws: gs_ssim_workspace_bytes(). */
size_t gs_ssim_workspace_bytes(int32_t n_pairs, int32_t width, int32_t height);
gs_status gs_ssim(const float* images, int32_t n_images, int32_t width, int32_t height, const int32_t* pairs,
                  int32_t n_pairs, float* ssim, void* ws, size_t ws_bytes, void* stream);

/* Eqs. 3-5 for P poses and the B blocks of `blocks`: B1 = (1 - ssim[p][j]) >
 * eps (SSIM loss between the full render and the render without block j);
 * B2 = the pose's camera centre lies in block j's cell (normalised and
 * contracted first when blocks->contraction is set); B = B1 or B2.
 * ssim: device float[P][B]; b1, b2 (may be NULL), b: device uint8[P][B]. */
gs_status gs_assign(const gs_blocks* blocks /* host struct */, const gs_camera* cams, int32_t n_poses,
                    const float* ssim, double eps, uint8_t* b1, uint8_t* b2, uint8_t* b, void* stream);

/* Name of a status code (static string, or a thread-local buffer after GS_ERR_HIP). */
const char* gs_status_string(gs_status status);

#ifdef __cplusplus
}
#endif

#endif /* GS_H_ */
