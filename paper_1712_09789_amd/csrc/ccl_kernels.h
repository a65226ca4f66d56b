// Internal interface between the host library and the HIP kernels.
//
// The kernels are compiled once per tile height (ccl_kernels.hip built with
// -DCCL_TILE_ROWS=<rows> -DCCL_SHAPE_NS=r<rows>); each build exports its
// launchers through a ShapeOps table, and the host picks a tile shape per
// call.  Everything in this header that depends on the tile height takes it
// as an argument.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccl {

// Tile width: one 64-bit foreground mask per tile row, one wavefront lane per
// row in the local kernels.
constexpr int TW = 64;

// Tile heights built into the library, and the built-in choice.  The
// statistics, ablation and volume paths always use the built-in height.
constexpr int NSHAPES = 3;
constexpr int SHAPE_ROWS[NSHAPES] = {32, 64, 128};
constexpr int DEFAULT_ROWS = 64;

// Border pixels per tile (top row, bottom row, left column, right column).
constexpr int nslots(int rows) { return 2 * TW + 2 * rows; }
// Run-table entries per tile: one per run, at most one run per two columns.
constexpr int runtab_per_tile(int rows) { return rows * TW / 2; }
// Threads of a tile workgroup: one sixteen-pixel chunk of a row each.
constexpr int tile_threads(int rows) { return 4 * rows; }

struct ImageArgs {
    const uint8_t* img;
    int64_t pitch;    // bytes between rows of img
    int32_t* labels;  // dense H x W
    int32_t H, W;
    int32_t ntx, nty;  // tile grid
    uint32_t wmagic;   // floor(2^32 / W) (0xffffffff for W = 1), for division by W
    int32_t lbase;     // added to every label written (a slice's first voxel position)
    int32_t unused;    // keeps the layout at 64 bytes
    int32_t vec_out;   // labels rows are 16-byte aligned (W % 4 == 0)
    int64_t tbase;     // global index of the image's first tile in the workspace
};
// 64 bytes: the kernels read an image's entry with one scalar load.
static_assert(sizeof(ImageArgs) == 64, "ImageArgs is one 64-byte scalar load");

// A volume whose slices were labelled as a batch of images (labels lifted to
// voxel positions by lbase); the labels alone carry what the merge across
// slices needs (nonzero exactly on foreground).
struct VolArgs {
    const uint8_t* vol;     // voxel (z, y, x) at vol[z * spitch + y * pitch + x]
    int64_t pitch, spitch;  // bytes between rows / slices
    int32_t* labels;        // dense D x H x W
    int32_t D, H, W;
    int32_t nbx, nby, nbz;  // bricks along x, y, z
    int32_t vec;            // labels is 16-byte aligned
    uint32_t wmagic, smagic;  // floor(2^32 / W), floor(2^32 / (H * W)); 0xffffffff for 1
};
constexpr int VOL_BRICK_W = 64, VOL_BRICK_H = 8, VOL_BRICK_D = 8;  // voxels per brick (x, y, z)

// Images labelled by one set of launches (all of one connectivity).  With n
// == 1 the image travels in `one` and the tables are unused; otherwise the
// device tables map global tiles, merge groups and k_seam workgroups to
// their image.
struct BatchArgs {
    ImageArgs one;
    const ImageArgs* imgs;  // [n]
    const int64_t* tile_off;   // [n+1] first global tile of each image (= tbase)
    const int64_t* group_off;  // [n+1] first global merge group of each image
    const int64_t* seam_off;   // [n+1] first k_seam workgroup of each image
    int32_t* tile_img;   // [ntiles]  filled by k_index
    int32_t* group_img;  // [ngroups]
    int32_t* seam_img;   // [nseamwg]
    int32_t n;
    int64_t ntiles, ngroups, nseamwg;
};

// Device workspace of one image.
struct Workspace {
    uint64_t* bits;    // [ntiles][rows] foreground masks
    int32_t* slots;    // [ntiles][nslots] forest node of each border pixel, -1 = bg
    uint64_t* forest;  // [ntiles][nslots] (key of parent << 32) | parent node
    uint16_t* runtab;  // [ntiles][runtab_per_tile] local root of each run
    uint32_t* nruns;   // [ntiles] runs of each tile (valid run-table entries)
};

inline int64_t workspace_bytes(int64_t ntiles, int rows)
{
    auto up = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    const int64_t ns = nslots(rows);
    return up(ntiles * rows * 8) + up(ntiles * ns * 4) + up(ntiles * ns * 8) +
           up(ntiles * runtab_per_tile(rows) * 2) + up(ntiles * 4);
}

inline Workspace carve_workspace(void* base, int64_t ntiles, int rows)
{
    auto up = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    const int64_t ns = nslots(rows);
    char* p = static_cast<char*>(base);
    Workspace ws;
    ws.bits = reinterpret_cast<uint64_t*>(p);
    p += up(ntiles * rows * 8);
    ws.slots = reinterpret_cast<int32_t*>(p);
    p += up(ntiles * ns * 4);
    ws.forest = reinterpret_cast<uint64_t*>(p);
    p += up(ntiles * ns * 8);
    ws.runtab = reinterpret_cast<uint16_t*>(p);
    p += up(ntiles * runtab_per_tile(rows) * 2);
    ws.nruns = reinterpret_cast<uint32_t*>(p);
    return ws;
}

// Per-component statistics (same layout as ccl_component in ccl.h).
struct CompStats {
    int32_t label;
    int32_t area;
    int32_t x_min, y_min, x_max, y_max;
    int64_t sum_x, sum_y;
};

// Statistics workspace and outputs of one image (tiles of DEFAULT_ROWS
// rows).  Components are numbered in raster order of their smallest pixel:
// the count of such pixels per (image row, tile column) segment is scanned,
// and a component's number is the scanned count of its segment plus the
// smallest pixels left of it there.
constexpr int SCAN_T = 1024;                // scan workgroup size
constexpr int SCAN_BLK = 4 * SCAN_T;        // segments per first-level scan block
// Partial statistics of one component over part of the image, in global
// coordinates.
struct StatRec {
    int32_t label;  // the component's label
    int32_t area, x_min, x_max, y_min, y_max;
    int64_t sum_x, sum_y;
};
constexpr int MERGE_FAN = 4;     // a merge workgroup takes the records of 4 x 4 tiles
constexpr int MERGE_HT = 2048;   // its hash table of distinct components

// Written to the component count by the statistics kernels when the label
// a run is given is impossible for its pixel (see ccl.h).
constexpr int64_t CCL_STATS_INCONSISTENT = -1;

struct StatsWs {
    uint64_t* rootbits;  // [ntiles][rows] smallest pixels of components, by tile row
    uint32_t* seg;       // [ntiles * rows] per segment: count, then exclusive scan in its block
    uint32_t* bsum;      // [nblk] segments' total per scan block
    uint32_t* boff;      // [nblk] exclusive scan of bsum
    StatRec* rec0;       // [ntiles][nslots] per tile: partials of its border components
    uint32_t* cnt0;      // [ntiles]
    int32_t* fin;        // [ntiles][nslots] final label of the component at each
                         // foreground border slot
    int64_t nseg, nblk;
    int32_t g1x, g1y;    // grid of merge workgroups (4 x 4 tiles each)
    CompStats* comps;    // caller's output [capacity]
    int64_t capacity;
    int64_t* count;      // caller's output: number of components
};

inline int64_t stats_workspace_bytes(int64_t ntiles)
{
    auto up = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    const int64_t nseg = ntiles * DEFAULT_ROWS, nblk = (nseg + SCAN_BLK - 1) / SCAN_BLK;
    return up(nseg * 8) + up(nseg * 4) + 2 * up(nblk * 4) +
           up(ntiles * nslots(DEFAULT_ROWS) * (int64_t)sizeof(StatRec)) + up(ntiles * 4) +
           up(ntiles * nslots(DEFAULT_ROWS) * 4);
}

inline StatsWs carve_stats(void* base, int64_t ntiles, int ntx, int nty)
{
    auto up = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    char* p = static_cast<char*>(base);
    StatsWs s{};
    s.nseg = ntiles * DEFAULT_ROWS;
    s.nblk = (s.nseg + SCAN_BLK - 1) / SCAN_BLK;
    s.g1x = (ntx + MERGE_FAN - 1) / MERGE_FAN;
    s.g1y = (nty + MERGE_FAN - 1) / MERGE_FAN;
    s.rootbits = reinterpret_cast<uint64_t*>(p);
    p += up(s.nseg * 8);
    s.seg = reinterpret_cast<uint32_t*>(p);
    p += up(s.nseg * 4);
    s.bsum = reinterpret_cast<uint32_t*>(p);
    p += up(s.nblk * 4);
    s.boff = reinterpret_cast<uint32_t*>(p);
    p += up(s.nblk * 4);
    s.rec0 = reinterpret_cast<StatRec*>(p);
    p += up(ntiles * nslots(DEFAULT_ROWS) * (int64_t)sizeof(StatRec));
    s.cnt0 = reinterpret_cast<uint32_t*>(p);
    p += up(ntiles * 4);
    s.fin = reinterpret_cast<int32_t*>(p);
    return s;
}

enum {
    KIND_LOCAL = 0, KIND_SEAM = 1, KIND_FINAL = 2, KIND_COPY = 3, KIND_BLOCK = 4,
    KIND_STATS = 5, KIND_VMERGE = 6, KIND_VFINAL = 7, KIND_VLOCAL = 8, NKINDS = 9
};

struct KernelTimer;  // host-side event recorder, null when timing is off
void timer_begin(KernelTimer* t, int kind, hipStream_t st);
void timer_end(KernelTimer* t, int kind, hipStream_t st);

constexpr int SEAM_WG = 256;  // k_seam workgroup size

// Launch grid of k_local and k_final: -1 = built-in rule, 0 = persistent (one
// workgroup per resident slot), 1 = one workgroup per tile.
struct GridChoice {
    int local = -1;
    int final_ = -1;
};

// Launchers and tile-grid quantities of one tile-height build.
struct ShapeOps {
    int rows;
    int64_t (*image_groups)(int ntx, int nty);  // merge groups of an image
    int64_t (*image_seam_items)(int ntx, int nty, int H, int W, int conn);  // k_seam work items
    // k_index: fills the image-of-tile/group/seam-workgroup tables of a
    // batch (n > 1); must precede label on the same stream.
    hipError_t (*index)(const BatchArgs& b, hipStream_t st);
    // With `stats` (a single image, DEFAULT_ROWS build only) k_final also
    // records the smallest pixels of components, and the statistics kernels
    // follow it.
    hipError_t (*label)(const BatchArgs& b, int conn, const Workspace& ws, hipStream_t st,
                        KernelTimer* timer, bool local_only, GridChoice grid,
                        const StatsWs* stats);
    // `reps` back-to-back launches of one kernel of a labelling (KIND_LOCAL
    // or KIND_FINAL) with the arguments and launch shape `label` used.
    hipError_t (*replay)(const BatchArgs& b, int conn, const Workspace& ws, hipStream_t st,
                         GridChoice grid, int kind, int reps);
};

namespace r32 {
extern const ShapeOps ops;
}
namespace r128 {
extern const ShapeOps ops;
}
namespace r64 {
extern const ShapeOps ops;
// The local step's ablation variants (0 = rows and columns, 1 = rows only,
// 2 = columns only, 3 = none), 4-connectivity, a single image, followed by
// the usual merge and final kernels; `counters` (2 per tile) may be null.
hipError_t launch_ablation(const BatchArgs& b, const Workspace& ws, hipStream_t st, int variant,
                           uint32_t* counters);
// Unite components across adjacent slices of a volume (6- or 26-connectivity)
// and write canonical labels; the slices' labels must already be in place.
hipError_t launch_volume(const VolArgs& v, int conn, hipStream_t st, KernelTimer* timer);
// Writes *count = 0 (an empty image has no components).
hipError_t launch_zero_count(int64_t* count, hipStream_t st);
hipError_t launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t st,
                       KernelTimer* timer);
// Segments of seg_bytes (a multiple of 16), one every src_stride bytes of src,
// gathered into dst.
hipError_t launch_copy_segments(const void* src, void* dst, int64_t bytes, int seg_bytes,
                                int64_t src_stride, hipStream_t st, KernelTimer* timer);
}  // namespace r64

}  // namespace ccl
