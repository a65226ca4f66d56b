/*
 * ccl.h — C ABI of the MI355X (gfx950) connected-components labeller.
 *
 * Method: the block-based coarse-to-fine labelling of Chen et al., "Efficient
 * Parallel Connected Components Labeling with a Coarse-to-fine Strategy"
 * (arXiv 1712.09789), Section 3: (1) local labelling of each image tile
 * (initialisation, row-column connection, label-equivalence unification,
 * refinement, ID conversion; Algorithm "Local labeling with coarse-to-fine
 * strategy" and Section 3.1), (2) block merge that inspects only pixels on
 * tile borders (Algorithm "Boundary analysis", Section 3.2, Eq. 1-2), and
 * (3) the global root-find that writes the final label map (Section 3.3).
 *
 * Output convention (all entry points): labels[y * W + x] is 0 for a
 * background pixel and, for a foreground pixel, 1 + the smallest raster
 * position y' * W + x' of its connected component.  The paper's labels are
 * exactly these root positions (Section 3.1.1: the provisional label of a
 * pixel is its position and the root of a list is the element whose label is
 * its own address; Sections 3.1.3 and 3.2: the larger root always points at
 * the smaller); the "+1" reserves 0 for background.  The result is therefore
 * unique and does not depend on tile shape, batch composition or timing.
 *
 * Input convention: the image is uint8, H rows of W pixels, row y starting
 * at img + y * pitch_bytes.  A pixel is foreground when its byte is nonzero
 * (the paper's binary intensity I(x, y) in {0, 1}, Section 3).  Bytes between
 * W and pitch_bytes are never read.
 *
 * Pointers named img/labels are DEVICE pointers on the current HIP device.
 * `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 * enqueued on `stream` and the call returns without waiting; the labels are
 * valid once the stream has reached that point.  Argument errors are detected
 * on the host before anything is enqueued, and `labels` is then untouched.
 *
 * The library owns a per-(device, stream) workspace cache that grows on
 * demand (hipMalloc); concurrent calls on DIFFERENT streams use different
 * workspaces and may overlap freely.  Calls on the same stream are ordered
 * by the stream.
 */
#ifndef CCL_H
#define CCL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CCL_OK = 0,
    CCL_ERR_INVALID_ARG = -1, /* null pointer, negative size, pitch < W,
                                 connectivity not 4/8, img and labels overlap */
    CCL_ERR_TOO_LARGE = -2,   /* H * W > 2^31 - 1 (labels are int32)         */
    CCL_ERR_OUT_OF_MEMORY = -3, /* the workspace could not grow              */
    CCL_ERR_HIP = -4          /* a HIP call or kernel launch failed           */
} ccl_status;

/*
 * Label one image (Section 3, all three steps).
 *   img          device, uint8, H rows, row stride pitch_bytes (>= W);
 *                caller-owned, only read.
 *   H, W         image size in pixels; H == 0 or W == 0 is a no-op.
 *   connectivity 4 (the paper's setting, Section 4.2) or 8.
 *   labels       device, int32, dense H * W (row stride W); caller-owned,
 *                fully overwritten.  Must not overlap img.
 * Returns a ccl_status; on error ccl_last_error() holds a message.
 */
int ccl_label(const uint8_t* img, int32_t H, int32_t W, int64_t pitch_bytes,
              int32_t connectivity, int32_t* labels, void* stream);

/*
 * ccl_label with an explicit tile height.  The paper's one tuning knob is the
 * block (tile) shape (Section 4.1, effectiveness of coarse labelling); the
 * library is built for tiles 64 pixels wide and 32, 64 or 128 rows high, and
 * ccl_label takes the height from the launch policy (ccl_set_launch_policy).
 *   tile_rows  32, 64 or 128; 0 = the policy's choice (as ccl_label).
 * Labels do not depend on the tile height.  Errors as ccl_label, and
 * CCL_ERR_INVALID_ARG for a height that is not built.
 */
int ccl_label_tiled(const uint8_t* img, int32_t H, int32_t W, int64_t pitch_bytes,
                    int32_t connectivity, int32_t* labels, int32_t tile_rows, void* stream);

/*
 * ccl_label for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same labels, computed with no hipMalloc, hipFree or other allocating call.
 * The workspace is a fixed 32 MiB device array inside the library, one per
 * device, held from the time the library's code is loaded on that device
 * until the process ends; it fits images of up to about 4300 tiles of 64 x
 * 64 pixels (4096 x 4096 fits).  The built-in tile shape and launch grids are
 * used (the launch policy does not apply).  Every call on a device shares
 * that device's array, so calls that overlap on one device (on different
 * streams, or from several threads) race and must be serialised by the
 * caller; consecutive calls on one stream are ordered by the stream.
 * Arguments and errors as ccl_label; CCL_ERR_TOO_LARGE also when the image
 * needs more workspace than the array holds (checked before anything is
 * enqueued).  The first call on a device looks up the array's device
 * address (hipGetSymbolAddress); CCL_ERR_HIP if that fails.
 */
int ccl_label_noalloc(const uint8_t* img, int32_t H, int32_t W, int64_t pitch_bytes,
                      int32_t connectivity, int32_t* labels, void* stream);

/* One image of a batch; same meaning as the ccl_label arguments. */
typedef struct {
    const uint8_t* img;
    int32_t H;
    int32_t W;
    int64_t pitch_bytes;
    int32_t connectivity;
    int32_t* labels;
} ccl_image_desc;

/*
 * Label n independent images (the same three steps per image).
 *   descs   HOST array of n descriptors, read during the call only.
 *   n       number of images; 0 is a no-op.
 * Every descriptor is validated before anything is enqueued; the first bad
 * one fails the whole call (its index is in ccl_last_error()).  Outputs are
 * identical to labelling each image alone with ccl_label.
 */
int ccl_label_batch(const ccl_image_desc* descs, int32_t n, void* stream);

/* ccl_label_batch with an explicit tile height for every connectivity class
 * (32, 64 or 128; 0 = the policy's choice).  Labels do not depend on it. */
int ccl_label_batch_tiled(const ccl_image_desc* descs, int32_t n, int32_t tile_rows,
                          void* stream);

/*
 * Prepared batches, for callers that launch the same batch repeatedly (new
 * pixels written into the same buffers) or capture it into a HIP graph.
 * ccl_plan_create validates the descriptors exactly like ccl_label_batch,
 * allocates the plan's own device memory (hipMalloc), copies the image
 * tables and fills the tile index on `stream`, and waits for that stream.
 * The image and label pointers of every descriptor are bound to the plan.
 * ccl_plan_run enqueues only kernel launches on `stream` — no allocation, no
 * copy, no synchronisation — so it may be captured into a graph; outputs are
 * identical to ccl_label_batch on the same descriptors.  Runs of one plan on
 * different streams must not overlap (they share its workspace).
 * ccl_plan_destroy synchronises the plan's device and frees it (NULL is a
 * no-op).
 */
typedef struct ccl_plan ccl_plan;
int ccl_plan_create(const ccl_image_desc* descs, int32_t n, void* stream, ccl_plan** plan);
int ccl_plan_run(ccl_plan* plan, void* stream);
int ccl_plan_destroy(ccl_plan* plan);

/*
 * Statistics of one connected component.  The paper's introduction names
 * what a labelling is for: the size and the location of each connected set;
 * these are that size, its box and the sums that give its centroid.
 */
typedef struct {
    int32_t label;   /* 1 + raster position of the component's smallest pixel */
    int32_t area;    /* number of pixels                                       */
    int32_t x_min;   /* inclusive bounding box: smallest and largest column    */
    int32_t y_min;   /* and row among the component's pixels                   */
    int32_t x_max;
    int32_t y_max;
    int64_t sum_x;   /* sum of the pixels' columns (centroid x = sum_x / area) */
    int64_t sum_y;   /* sum of the pixels' rows    (centroid y = sum_y / area) */
} ccl_component;     /* 40 bytes */

/*
 * Label one image (as ccl_label) and compute the statistics of every
 * component.
 *   comps     device array of `capacity` entries, caller-owned.  Entry i
 *             describes the component with the i-th smallest label, so the
 *             array is sorted by label.  Entries [0, min(*count, capacity))
 *             are written; the rest are untouched.
 *   capacity  entries comps holds (>= 0; 0 computes the count only).
 *   count     device int64: the number of components, also when it exceeds
 *             capacity (call again with a larger array to get them all).
 *             A negative count (-1) reports an internal consistency failure
 *             found on the device (a label that cannot belong to its pixel);
 *             the labels and records of that call must not be used.
 * Other arguments and errors as ccl_label; additionally CCL_ERR_INVALID_ARG
 * for a null count, capacity < 0, or a null comps with capacity > 0.  An
 * empty image writes *count = 0.  Enqueued on `stream` like ccl_label.
 */
int ccl_label_stats(const uint8_t* img, int32_t H, int32_t W, int64_t pitch_bytes,
                    int32_t connectivity, int32_t* labels, ccl_component* comps,
                    int64_t capacity, int64_t* count, void* stream);

/*
 * Label a volume (the paper's introduction names 2-D and 3-D images): voxel
 * position P = x + y * W + z * W * H; labels[P] = 0 for background, else 1 +
 * the smallest position in the voxel's component.  The paper's method with
 * a third axis: bricks of 64 x 8 x 8 voxels (x, y, z) are labelled in LDS
 * (runs along x united across the brick's rows and slices), components are
 * united across brick faces in the label map (the block merge), and every
 * label is rewritten to its root.  No workspace.
 *   vol           device, uint8, D slices of H rows; row y of slice z starts
 *                 at vol + z * slice_pitch_bytes + y * pitch_bytes;
 *                 caller-owned, only read.
 *   pitch_bytes   >= W; slice_pitch_bytes >= (H - 1) * pitch_bytes + W
 *                 (ignored when D == 1).
 *   connectivity  6 (face neighbours) or 26 (the 3 x 3 x 3 block).
 *   labels        device, int32, dense D * H * W; caller-owned, fully
 *                 overwritten.  Must not overlap vol.
 * Errors as ccl_label (CCL_ERR_TOO_LARGE when D * H * W > 2^31 - 1); an
 * empty volume is a no-op.
 */
int ccl_label_3d(const uint8_t* vol, int32_t D, int32_t H, int32_t W, int64_t pitch_bytes,
                 int64_t slice_pitch_bytes, int32_t connectivity, int32_t* labels, void* stream);

/*
 * The paper's ablation of its local step (Section 4, effectiveness of coarse
 * labelling), for study rather than speed: the local step is rerun with the
 * coarse labelling along rows and columns (CCL_C2FL, the method), along rows
 * only (CCL_RC2FL), along columns only (CCL_CC2FL) or not at all
 * (CCL_NC2FL), followed by the usual block merge and final update.  Row
 * connection makes each row run one union-find node (without it every
 * foreground pixel is a node); column connection starts each node linked to
 * the node above it.  4-connectivity (the paper's setting).
 *   variant   CCL_C2FL .. CCL_NC2FL.
 *   labels    as in ccl_label: identical for every variant.
 *   counters  NULL, or a device uint32 array of 2 * tile count entries
 *             (tiles in row-major order, ccl_tile_cols() x ccl_tile_rows()
 *             pixels each): per tile, the number of find-loop steps (the
 *             paper's iterations) and of atomic merge attempts in the local
 *             step.
 * Other arguments and errors as ccl_label; CCL_ERR_INVALID_ARG for an
 * unknown variant.
 */
enum { CCL_C2FL = 0, CCL_RC2FL = 1, CCL_CC2FL = 2, CCL_NC2FL = 3 };
int ccl_label_ablation(const uint8_t* img, int32_t H, int32_t W, int64_t pitch_bytes,
                       int32_t variant, int32_t* labels, uint32_t* counters, void* stream);

/*
 * Debugging aid for the local step alone (Section 3.1): every tile is
 * labelled as if it were a separate image, and each foreground pixel gets
 * 1 + the raster position (in the whole image) of the smallest pixel of its
 * component INSIDE its tile.  Tiles are ccl_tile_cols() wide and
 * ccl_tile_rows() high (the built-in shape), aligned at (0, 0).  Same
 * arguments and errors as ccl_label.
 */
int ccl_label_local(const uint8_t* img, int32_t H, int32_t W, int64_t pitch_bytes,
                    int32_t connectivity, int32_t* labels, void* stream);

/*
 * Launch policy, for callers that tune it (paper_1712_09789_amd/tune.py
 * does): per launch class, pixel bucket and connectivity, the tile height
 * (the paper's block shape, Section 4.1) and the grid of the two per-tile
 * kernels (the local step and the final relabel).  Each of those runs either
 * as a persistent grid (one workgroup per resident slot, the next tile's
 * loads in flight while the current one is labelled) or with one workgroup
 * per tile (the dispatcher balances tiles of unequal cost).  Labels never
 * depend on any of these choices.
 *   batch         0 = calls with one image (ccl_label, plans of one image),
 *                 1 = calls with several (ccl_label_batch, plans); chosen by
 *                 the number of non-empty images of one connectivity
 *   bucket        0 .. ccl_launch_buckets() - 1: launches whose total pixel
 *                 count (over the images of one connectivity) is at most the
 *                 bucket's bound and above the previous one
 *   connectivity  4 or 8
 *   tile_rows     0 = built-in (64), or 32, 64, 128
 *   local, final_ -1 = the built-in choice (local step per tile beyond four
 *                 times the resident workgroups, final relabel persistent),
 *                 0 = persistent, 1 = one workgroup per tile
 * ccl_label_stats, ccl_label_3d, ccl_label_ablation and ccl_label_local
 * always use the built-in tile height and grids.  Process-wide; applies to
 * launches enqueued (and plans created) afterwards.  CCL_OK, or
 * CCL_ERR_INVALID_ARG for a value out of range.
 */
int ccl_set_launch_policy(int32_t batch, int32_t bucket, int32_t connectivity,
                          int32_t tile_rows, int32_t local, int32_t final_);

/* Number of pixel buckets of ccl_set_launch_policy; writes the first
 * min(n, buckets) upper bounds (pixels; the last is INT64_MAX) into `upper`
 * (host memory, may be NULL). */
int32_t ccl_launch_buckets(int64_t* upper, int32_t n);

/* Tile height the current policy picks for a launch class (0 = one image,
 * 1 = several) of `pixels` pixels and the given connectivity; -1 for
 * arguments out of range. */
int32_t ccl_policy_tile_rows(int32_t batch, int64_t pixels, int32_t connectivity);

/* Number of tile heights built into the library; writes the first min(n,
 * count) of them (ascending) into `rows` (host memory, may be NULL). */
int32_t ccl_tile_shapes(int32_t* rows, int32_t n);

/* Built-in tile shape (pixels): 64 columns, 64 rows. */
int32_t ccl_tile_cols(void);
int32_t ccl_tile_rows(void);

/* Workspace bytes one ccl_label call of this size needs under any tile
   height (the largest of them; 0 for an empty image, -1 for invalid
   sizes). */
int64_t ccl_workspace_bytes(int32_t H, int32_t W);

/* Bytes of the workspace the library currently keeps for `stream` on the
   current device (0 if none): it grows to 1.25 x the largest need seen on
   that stream and is kept until ccl_release_workspace.  For callers that
   account device memory (a serving loop's admission). */
int64_t ccl_workspace_cached(void* stream);

/* Thread-local message describing the last non-OK status ("" if none). */
const char* ccl_last_error(void);

/* Free every cached workspace of `device` (synchronises that device). */
int ccl_release_workspace(int32_t device);

/*
 * Per-kernel timing with HIP events recorded on the launch stream.
 * ccl_timing_enable(mask) clears the counters and starts recording events
 * around every kernel of the kinds whose bit is set in `mask` (bit k = kind
 * k; 0 stops recording).  Kinds: 0 = local step, 1 = merge across tile
 * groups, 2 = final relabel, 3 = copy, 4 = merge inside tile groups,
 * 5 = the statistics kernels of ccl_label_stats (one interval per call),
 * 6 = the merge across brick faces of ccl_label_3d, 7 = its final relabel,
 * 8 = its local step (bricks).
 * ccl_timing_read() waits for the recorded events and fills, for each kind
 * k < n, the summed milliseconds ms[k] and launch count launches[k].
 * Returns the number of kinds (9).
 */
int ccl_timing_enable(int32_t enable);
int ccl_timing_read(double* ms, int64_t* launches, int32_t n);

/*
 * Benchmark hook: enqueue `reps` more launches of one kernel of the most
 * recent plain labelling (ccl_label, ccl_label_tiled, ccl_label_batch,
 * ccl_label_batch_tiled) made by the calling thread on the current device,
 * back to back on `stream`, with that call's arguments, workspace and launch
 * shape, so that a timer around the call measures that kernel alone.
 *   kind  0 = the local step, 2 = the final relabel (the kinds of
 *         ccl_timing_enable).
 * The final relabel rewrites the same labels.  The local step resets the
 * block merge's state in the workspace, so after it the labels of that call
 * are valid only once it is made again.  The workspace must not have been
 * used by a larger call on the same stream since.  CCL_ERR_INVALID_ARG for
 * another kind, reps < 0, or no such call.
 */
int ccl_replay_last(int32_t kind, int32_t reps, void* stream);

/*
 * Plain device-to-device copy of `bytes` bytes (both device pointers,
 * 16-byte aligned, non-overlapping) by a streaming kernel.  Used only to
 * calibrate bandwidth figures and hardware byte counters.
 */
int ccl_copy_bytes(const void* src, void* dst, int64_t bytes, void* stream);

/*
 * Gathering copy for the same calibration, in the request size of the local
 * step's image reads: `bytes` bytes go to dst (contiguous) from segments of
 * `segment_bytes` taken one every `src_stride_bytes` bytes of src (src must
 * hold bytes / segment_bytes such strides).  All sizes, the stride and both
 * pointers 16-byte aligned, bytes a multiple of the segment, stride >=
 * segment.
 */
int ccl_copy_segments(const void* src, void* dst, int64_t bytes, int32_t segment_bytes,
                      int64_t src_stride_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CCL_H */
