// Internal interface between the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccl {

// Tile width: one 64-bit foreground mask per tile row, one wavefront lane per
// row in the local kernels.
constexpr int TW = 64;

#ifndef CCL_TILE_ROWS
#define CCL_TILE_ROWS 64
#endif
constexpr int TILE_ROWS = CCL_TILE_ROWS;
constexpr int NSLOTS = 2 * TW + 2 * TILE_ROWS;  // border pixels per tile
constexpr int RUNTAB_PER_TILE = TILE_ROWS * TW / 2;  // run-table entries per tile

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
    int32_t* labels;  // dense D x H x W
    int32_t D, H, W;
    int32_t vec;      // labels is 16-byte aligned
};

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
    uint64_t* bits;    // [ntiles][TILE_ROWS] foreground masks
    int32_t* slots;    // [ntiles][NSLOTS] forest node of each border pixel, -1 = bg
    uint64_t* forest;  // [ntiles][NSLOTS] (key of parent << 32) | parent node
    uint16_t* runtab;  // [ntiles][RUNTAB_PER_TILE] local root of each run
    uint32_t* nruns;   // [ntiles] runs of each tile (valid run-table entries)
};

inline int64_t workspace_bytes(int64_t ntiles)
{
    auto up = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    return up(ntiles * TILE_ROWS * 8) + up(ntiles * NSLOTS * 4) + up(ntiles * NSLOTS * 8) +
           up(ntiles * RUNTAB_PER_TILE * 2) + up(ntiles * 4);
}

inline Workspace carve_workspace(void* base, int64_t ntiles)
{
    auto up = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    char* p = static_cast<char*>(base);
    Workspace ws;
    ws.bits = reinterpret_cast<uint64_t*>(p);
    p += up(ntiles * TILE_ROWS * 8);
    ws.slots = reinterpret_cast<int32_t*>(p);
    p += up(ntiles * NSLOTS * 4);
    ws.forest = reinterpret_cast<uint64_t*>(p);
    p += up(ntiles * NSLOTS * 8);
    ws.runtab = reinterpret_cast<uint16_t*>(p);
    p += up(ntiles * RUNTAB_PER_TILE * 2);
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

// Statistics workspace and outputs of one image.  Components are numbered in
// raster order of their smallest pixel: the count of such pixels per
// (image row, tile column) segment is scanned, and a component's number is
// the scanned count of its segment plus the smallest pixels left of it there.
constexpr int SCAN_T = 1024;                // scan workgroup size
constexpr int SCAN_BLK = 4 * SCAN_T;        // segments per first-level scan block
// Partial statistics of one component over part of the image, in global
// coordinates.
struct StatRec {
    int32_t num;  // component number
    int32_t area, x_min, x_max, y_min, y_max;
    int64_t sum_x, sum_y;
};
constexpr int MERGE_FAN = 4;     // a merge workgroup takes the records of 4 x 4 tiles
constexpr int MERGE_HT = 2048;   // its hash table of distinct components

// Written to the component count by the statistics kernels when a label
// read back from the label map is impossible for its pixel (see ccl.h).
constexpr int64_t CCL_STATS_INCONSISTENT = -1;

struct StatsWs {
    uint64_t* rootbits;  // [ntiles][TILE_ROWS] smallest pixels of components, by tile row
    uint32_t* seg;       // [ntiles * TILE_ROWS] per segment: count, then exclusive scan in its block
    uint32_t* bsum;      // [nblk] segments' total per scan block
    uint32_t* boff;      // [nblk] exclusive scan of bsum
    StatRec* rec0;       // [ntiles][NSLOTS] per tile: partials of its border components
    uint32_t* cnt0;      // [ntiles]
    int64_t nseg, nblk;
    int32_t g1x, g1y;    // grid of merge workgroups (4 x 4 tiles each)
    CompStats* comps;    // caller's output [capacity]
    int64_t capacity;
    int64_t* count;      // caller's output: number of components
};

inline int64_t stats_workspace_bytes(int64_t ntiles)
{
    auto up = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    const int64_t nseg = ntiles * TILE_ROWS, nblk = (nseg + SCAN_BLK - 1) / SCAN_BLK;
    return up(nseg * 8) + up(nseg * 4) + 2 * up(nblk * 4) +
           up(ntiles * NSLOTS * (int64_t)sizeof(StatRec)) + up(ntiles * 4);
}

inline StatsWs carve_stats(void* base, int64_t ntiles, int ntx, int nty)
{
    auto up = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    char* p = static_cast<char*>(base);
    StatsWs s{};
    s.nseg = ntiles * TILE_ROWS;
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
    p += up(ntiles * NSLOTS * (int64_t)sizeof(StatRec));
    s.cnt0 = reinterpret_cast<uint32_t*>(p);
    return s;
}

enum {
    KIND_LOCAL = 0, KIND_SEAM = 1, KIND_FINAL = 2, KIND_COPY = 3, KIND_BLOCK = 4,
    KIND_STATS = 5, NKINDS = 6
};

struct KernelTimer;  // host-side event recorder, null when timing is off
void timer_begin(KernelTimer* t, int kind, hipStream_t st);
void timer_end(KernelTimer* t, int kind, hipStream_t st);

// Tile-grid quantities of one image, shared by the host and the launchers.
int64_t image_groups(int ntx, int nty);      // merge groups
int64_t image_seam_items(int ntx, int nty, int H, int W, int conn);  // k_seam work items
constexpr int SEAM_WG = 256;                 // k_seam workgroup size

// k_index: fills the image-of-tile/group/seam-workgroup tables of a batch
// (n > 1); must precede launch_label on the same stream.
hipError_t launch_index(const BatchArgs& b, hipStream_t st);
// With `stats` (a single image only) k_final also records the smallest
// pixels of components, and the statistics kernels follow it.
hipError_t launch_label(const BatchArgs& b, int conn, const Workspace& ws, hipStream_t st,
                        KernelTimer* timer, bool local_only, const StatsWs* stats = nullptr);
// The local step's ablation variants (0 = rows and columns, 1 = rows only,
// 2 = columns only, 3 = none), 4-connectivity, a single image, followed by
// the usual merge and final kernels; `counters` (2 per tile) may be null.
hipError_t launch_ablation(const BatchArgs& b, const Workspace& ws, hipStream_t st, int variant,
                           uint32_t* counters);
// Unite components across adjacent slices of a volume (6- or 26-connectivity)
// and write canonical labels; the slices' labels must already be in place.
hipError_t launch_volume(const VolArgs& v, int conn, hipStream_t st);
// Launch shape of k_local / k_final per launch class (batch 0 = one image,
// 1 = several) and tile-count bucket: -1 = built-in rule, 0 = persistent
// grid, 1 = one workgroup per tile.  Returns -1 for values out of range.
constexpr int POLICY_BUCKETS = 5;
int set_launch_policy(int batch, int bucket, int local, int final_);
int64_t policy_bucket_bound(int bucket);  // largest tile count of the bucket
// Writes *count = 0 (an empty image has no components).
hipError_t launch_zero_count(int64_t* count, hipStream_t st);
hipError_t launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t st,
                       KernelTimer* timer);

}  // namespace ccl
