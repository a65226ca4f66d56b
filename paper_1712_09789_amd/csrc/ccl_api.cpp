// Host side of the C ABI declared in include/ccl.h: argument validation,
// the per-(device, stream) workspace cache, and the optional event timer.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "ccl.h"
#include "ccl_kernels.h"

namespace ccl {

static thread_local std::string g_err;

static int fail(int status, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int status, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return status;
}

// ---------------------------------------------------------------------------
// workspace cache: one grow-only buffer per (device, stream)
// ---------------------------------------------------------------------------

struct WsEntry {
    void* ptr = nullptr;
    int64_t bytes = 0;
};

static std::mutex g_ws_mu;
static std::map<std::pair<int, hipStream_t>, WsEntry> g_ws;

static int get_workspace(int64_t need, hipStream_t st, void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(CCL_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(g_ws_mu);
    WsEntry& w = g_ws[{dev, st}];
    if (w.bytes < need) {
        if (w.ptr) {
            // earlier work on this stream may still read the old buffer
            e = hipStreamSynchronize(st);
            if (e != hipSuccess)
                return fail(CCL_ERR_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
            (void)hipFree(w.ptr);
            w.ptr = nullptr;
            w.bytes = 0;
        }
        int64_t grow = need + need / 4;
        e = hipMalloc(&w.ptr, (size_t)grow);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            w.ptr = nullptr;
            e = hipMalloc(&w.ptr, (size_t)need);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                w.ptr = nullptr;
                return fail(CCL_ERR_OUT_OF_MEMORY, "workspace of %lld bytes: %s",
                            (long long)need, hipGetErrorString(e));
            }
            grow = need;
        }
        w.bytes = grow;
    }
    *out = w.ptr;
    return CCL_OK;
}

// ---------------------------------------------------------------------------
// pinned staging for the batch tables
// ---------------------------------------------------------------------------
//
// The image tables of a batch go to the device with hipMemcpyAsync.  From
// pageable memory that call waits until the copy has read its source, i.e.
// until the stream's earlier work is done; from pinned memory it returns at
// once.  Each (device, stream) keeps a small ring of pinned buffers; a buffer
// is reused once the event recorded after its last copy has passed (by then
// normally long ago), so a call never overwrites a table still in flight.

struct Stage {
    void* host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool used = false;
};
constexpr int STAGE_RING = 4;
struct StageRing {
    Stage s[STAGE_RING];
    int next = 0;
};

static std::mutex g_stage_mu;
static std::map<std::pair<int, hipStream_t>, StageRing> g_stage;

// Copies `bytes` bytes of `src` to device `dst` on `st` through a pinned
// buffer; the call does not wait for earlier work on the stream.
static hipError_t stage_copy(void* dst, const void* src, size_t bytes, hipStream_t st)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_stage_mu);
    StageRing& ring = g_stage[{dev, st}];
    Stage& b = ring.s[ring.next];
    ring.next = (ring.next + 1) % STAGE_RING;
    if (b.used && (e = hipEventSynchronize(b.done)) != hipSuccess) return e;
    if (b.bytes < bytes) {
        if (b.host) (void)hipHostFree(b.host);
        b.host = nullptr;
        b.bytes = 0;
        const size_t want = bytes < 65536 ? 65536 : bytes + bytes / 4;
        if ((e = hipHostMalloc(&b.host, want, hipHostMallocDefault)) != hipSuccess) return e;
        b.bytes = want;
    }
    if (!b.done && (e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming)) != hipSuccess)
        return e;
    std::memcpy(b.host, src, bytes);
    if ((e = hipMemcpyAsync(dst, b.host, bytes, hipMemcpyHostToDevice, st)) != hipSuccess)
        return e;
    b.used = true;
    return hipEventRecord(b.done, st);
}

// ---------------------------------------------------------------------------
// event timer
// ---------------------------------------------------------------------------

struct KernelTimer {
    struct Rec {
        int kind;
        hipEvent_t a, b;
    };
    std::mutex mu;
    std::vector<hipEvent_t> pool;
    std::vector<Rec> done;
    hipEvent_t open[NKINDS] = {};
    double ms[NKINDS] = {};
    int64_t launches[NKINDS] = {};

    hipEvent_t take()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};

static KernelTimer g_timer;
static std::atomic<uint32_t> g_timing_mask{0};  // bit k: time kernel kind k

void timer_begin(KernelTimer* t, int kind, hipStream_t st)
{
    if (!t || !((g_timing_mask >> kind) & 1u)) return;
    std::lock_guard<std::mutex> lk(t->mu);
    hipEvent_t e = t->take();
    if (e && hipEventRecord(e, st) == hipSuccess) t->open[kind] = e;
}

void timer_end(KernelTimer* t, int kind, hipStream_t st)
{
    if (!t || !((g_timing_mask >> kind) & 1u)) return;
    std::lock_guard<std::mutex> lk(t->mu);
    hipEvent_t a = t->open[kind];
    t->open[kind] = nullptr;
    if (!a) return;
    hipEvent_t b = t->take();
    if (b && hipEventRecord(b, st) == hipSuccess) t->done.push_back({kind, a, b});
}

static KernelTimer* active_timer() { return g_timing_mask ? &g_timer : nullptr; }

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------

static int validate(const uint8_t* img, int32_t H, int32_t W, int64_t pitch, int32_t conn,
                    const int32_t* labels, const char* who)
{
    if (H < 0 || W < 0) return fail(CCL_ERR_INVALID_ARG, "%s: negative size %dx%d", who, H, W);
    if (conn != 4 && conn != 8)
        return fail(CCL_ERR_INVALID_ARG, "%s: connectivity %d is not 4 or 8", who, conn);
    if (H == 0 || W == 0) return CCL_OK;
    if ((int64_t)H * (int64_t)W > (int64_t)INT32_MAX)
        return fail(CCL_ERR_TOO_LARGE, "%s: %dx%d pixels exceed int32 labels", who, H, W);
    if (!img || !labels) return fail(CCL_ERR_INVALID_ARG, "%s: null pointer", who);
    if (pitch < W)
        return fail(CCL_ERR_INVALID_ARG, "%s: pitch %lld < width %d", who, (long long)pitch, W);
    const uintptr_t i0 = (uintptr_t)img, i1 = i0 + (uintptr_t)((int64_t)(H - 1) * pitch + W);
    const uintptr_t l0 = (uintptr_t)labels, l1 = l0 + (uintptr_t)((int64_t)H * W * 4);
    if (i0 < l1 && l0 < i1) return fail(CCL_ERR_INVALID_ARG, "%s: img and labels overlap", who);
    return CCL_OK;
}

// Tiles of an H x W image with tiles of `rows` rows.
static int64_t tiles_of(int32_t H, int32_t W, int rows)
{
    return (((int64_t)W + TW - 1) / TW) * (((int64_t)H + rows - 1) / rows);
}

// Forest node ids (one per border slot of every tile) must fit in int32.
static bool node_ids_fit(int64_t ntiles, int rows)
{
    return ntiles * nslots(rows) <= (int64_t)INT32_MAX;
}

static ImageArgs make_args(const uint8_t* img, int32_t H, int32_t W, int64_t pitch,
                           int32_t* labels, int rows)
{
    ImageArgs a;
    a.img = img;
    a.pitch = pitch;
    a.labels = labels;
    a.H = H;
    a.W = W;
    a.ntx = (int32_t)(((int64_t)W + TW - 1) / TW);
    a.nty = (int32_t)(((int64_t)H + rows - 1) / rows);
    a.unused = 0;
    a.vec_out = ((uintptr_t)labels % 16 == 0) && (W % 4 == 0);
    a.wmagic = W == 1 ? 0xffffffffu : (uint32_t)((1ull << 32) / (uint64_t)W);
    a.lbase = 0;
    a.tbase = 0;
    return a;
}

static int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }

// ---------------------------------------------------------------------------
// tile shape and launch grid per call
// ---------------------------------------------------------------------------
//
// A policy entry per (launch class: one image / several, pixel bucket,
// connectivity) fixes the tile height and the launch grids of k_local and
// k_final; zero / -1 entries keep the built-in choices (64-row tiles, the
// kernels' own grid rule).  A tuner (tune.py) measures and sets them.

static const ShapeOps* const kShapes[NSHAPES] = {&r32::ops, &r64::ops, &r128::ops};
constexpr int POLICY_BUCKETS = 5;
static const int64_t kBucketPx[POLICY_BUCKETS] = {int64_t(1) << 22, int64_t(1) << 24,
                                                  int64_t(1) << 26, int64_t(1) << 28, INT64_MAX};

struct PolicyEntry {
    std::atomic<int> rows{0};  // 0 = built-in (DEFAULT_ROWS)
    std::atomic<int> local{-1}, final_{-1};
};
static PolicyEntry g_policy[2][POLICY_BUCKETS][2];  // [batch][bucket][connectivity == 8]

static int policy_bucket(int64_t px)
{
    int k = 0;
    while (k < POLICY_BUCKETS - 1 && px > kBucketPx[k]) ++k;
    return k;
}

static const ShapeOps* shape_for_rows(int rows)
{
    for (const ShapeOps* o : kShapes)
        if (o->rows == rows) return o;
    return nullptr;
}

struct Choice {
    const ShapeOps* ops;
    GridChoice grid;
};

// Tile shape and grids for a launch class of `px` pixels; `forced_rows` > 0
// overrides the policy's tile height (and then the built-in grids hold).
static Choice choose(bool batch, int64_t px, int conn, int forced_rows)
{
    Choice c;
    if (forced_rows > 0) {
        c.ops = shape_for_rows(forced_rows);
        return c;
    }
    const PolicyEntry& e = g_policy[batch][policy_bucket(px)][conn == 8];
    const int rows = e.rows.load(std::memory_order_relaxed);
    c.ops = shape_for_rows(rows ? rows : DEFAULT_ROWS);
    c.grid.local = e.local.load(std::memory_order_relaxed);
    c.grid.final_ = e.final_.load(std::memory_order_relaxed);
    return c;
}

// Sizes of one connectivity class of a batch.
struct ClassLayout {
    int n = 0;
    int rows = DEFAULT_ROWS;
    std::vector<int64_t> toff, goff, soff;  // prefix offsets (n+1 each)
    int64_t ntiles = 0, ngroups = 0, nseamwg = 0;
    int64_t head = 0;  // bytes of the device tables (0 for a single image)
    int64_t bytes() const { return head + workspace_bytes(ntiles, rows); }
};

static int layout_class(std::vector<ImageArgs>& imgs, int conn, const ShapeOps& ops,
                        ClassLayout& L, const char* who)
{
    const int n = (int)imgs.size();
    L.n = n;
    L.rows = ops.rows;
    L.toff.assign(n + 1, 0);
    L.goff.assign(n + 1, 0);
    L.soff.assign(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        ImageArgs& a = imgs[i];
        a.tbase = L.toff[i];
        L.toff[i + 1] = L.toff[i] + (int64_t)a.ntx * a.nty;
        L.goff[i + 1] = L.goff[i] + ops.image_groups(a.ntx, a.nty);
        const int64_t items = ops.image_seam_items(a.ntx, a.nty, a.H, a.W, conn);
        L.soff[i + 1] = L.soff[i] + (items + SEAM_WG - 1) / SEAM_WG;
    }
    L.ntiles = L.toff[n];
    L.ngroups = L.goff[n];
    L.nseamwg = L.soff[n];
    if (!node_ids_fit(L.ntiles, L.rows))
        return fail(CCL_ERR_TOO_LARGE, "%s: %lld tiles exceed the node id range", who,
                    (long long)L.ntiles);
    L.head = 0;
    if (n > 1)
        L.head = align256(n * (int64_t)sizeof(ImageArgs)) + 3 * align256((n + 1) * 8) +
                 align256(L.ntiles * 4) + align256(L.ngroups * 4) + align256(L.nseamwg * 4);
    return CCL_OK;
}

// Point the batch arguments and the workspace at device memory `base`
// (L.bytes() long) and enqueue the copy of the image tables.
static int bind_class(const std::vector<ImageArgs>& imgs, const ClassLayout& L, void* base,
                      bool local_only, hipStream_t st, BatchArgs& b, Workspace& ws,
                      const char* who)
{
    const int n = L.n;
    b = BatchArgs{};
    b.n = n;
    b.ntiles = L.ntiles;
    b.ngroups = local_only ? 0 : L.ngroups;
    b.nseamwg = local_only ? 0 : L.nseamwg;
    char* d = static_cast<char*>(base);
    if (n == 1) {
        b.one = imgs[0];
    } else {
        const int64_t tables = align256(n * (int64_t)sizeof(ImageArgs)) + 3 * align256((n + 1) * 8);
        std::vector<char> host((size_t)tables, 0);
        char* h = host.data();
        std::memcpy(h, imgs.data(), n * sizeof(ImageArgs));
        b.imgs = reinterpret_cast<const ImageArgs*>(d);
        int64_t o = align256(n * (int64_t)sizeof(ImageArgs));
        const std::vector<int64_t>* tabs[3] = {&L.toff, &L.goff, &L.soff};
        const int64_t* dtabs[3];
        for (int k = 0; k < 3; ++k) {
            std::memcpy(h + o, tabs[k]->data(), (n + 1) * 8);
            dtabs[k] = reinterpret_cast<const int64_t*>(d + o);
            o += align256((n + 1) * 8);
        }
        b.tile_off = dtabs[0];
        b.group_off = dtabs[1];
        b.seam_off = dtabs[2];
        hipError_t e = stage_copy(d, h, host.size(), st);
        if (e != hipSuccess)
            return fail(CCL_ERR_HIP, "%s: table copy: %s", who, hipGetErrorString(e));
        b.tile_img = reinterpret_cast<int32_t*>(d + o);
        o += align256(L.ntiles * 4);
        b.group_img = reinterpret_cast<int32_t*>(d + o);
        o += align256(L.ngroups * 4);
        b.seam_img = reinterpret_cast<int32_t*>(d + o);
    }
    ws = carve_workspace(d + L.head, L.ntiles, L.rows);
    return CCL_OK;
}

// Caller's outputs of the statistics path.
struct StatsOut {
    ccl_component* comps;
    int64_t capacity;
    int64_t* count;
};

// Label images of one connectivity with one set of launches.  A single image
// travels in the kernel arguments; several get a device table (copied into
// the head of the workspace) that maps global tiles, merge groups and seam
// workgroups back to their image.

// The most recent plain labelling launched by this thread (for ccl_replay_last).
struct LastLaunch {
    bool valid = false;
    int device = 0;
    int conn = 0;
    Choice ch{};
    BatchArgs b{};
    Workspace ws{};
};
static thread_local LastLaunch g_last;

static int run_batch(std::vector<ImageArgs>& imgs, int conn, const Choice& ch, hipStream_t st,
                     bool local_only, const char* who, const StatsOut* so = nullptr,
                     int ablation = -1, uint32_t* counters = nullptr)
{
    if (imgs.empty()) return CCL_OK;
    ClassLayout L;
    int rc = layout_class(imgs, conn, *ch.ops, L, who);
    if (rc != CCL_OK) return rc;
    const int64_t label_bytes = align256(L.bytes());
    void* base = nullptr;
    rc = get_workspace(label_bytes + (so ? stats_workspace_bytes(L.ntiles) : 0), st, &base);
    if (rc != CCL_OK) return rc;
    BatchArgs b;
    Workspace ws;
    rc = bind_class(imgs, L, base, local_only, st, b, ws, who);
    if (rc != CCL_OK) return rc;
    StatsWs sw{};
    if (so) {
        sw = carve_stats(static_cast<char*>(base) + label_bytes, L.ntiles, imgs[0].ntx, imgs[0].nty);
        sw.comps = reinterpret_cast<CompStats*>(so->comps);
        sw.capacity = so->capacity;
        sw.count = so->count;
    }
    hipError_t e = ch.ops->index(b, st);
    if (e == hipSuccess && ablation >= 0)
        e = r64::launch_ablation(b, ws, st, ablation, counters);
    else if (e == hipSuccess)
        e = ch.ops->label(b, conn, ws, st, active_timer(), local_only, ch.grid,
                          so ? &sw : nullptr);
    if (e != hipSuccess) return fail(CCL_ERR_HIP, "%s: launch failed: %s", who, hipGetErrorString(e));
    if (!so && ablation < 0 && !local_only) {
        g_last.valid = hipGetDevice(&g_last.device) == hipSuccess;
        g_last.conn = conn;
        g_last.ch = ch;
        g_last.b = b;
        g_last.ws = ws;
    }
    return CCL_OK;
}

// One image with the tile shape of `ch`.
static int label_one(const uint8_t* img, int32_t H, int32_t W, int64_t pitch, int32_t conn,
                     int32_t* labels, hipStream_t st, bool local_only, const Choice& ch,
                     const char* who)
{
    int rc = validate(img, H, W, pitch, conn, labels, who);
    if (rc != CCL_OK || H == 0 || W == 0) return rc;
    if (!node_ids_fit(tiles_of(H, W, ch.ops->rows), ch.ops->rows))
        return fail(CCL_ERR_TOO_LARGE, "%s: %dx%d needs too many tiles", who, H, W);
    std::vector<ImageArgs> one(1, make_args(img, H, W, pitch, labels, ch.ops->rows));
    return run_batch(one, conn, ch, st, local_only, who);
}

// The built-in tile shape and grids (statistics, ablation, volumes, local step).
static Choice builtin_choice() { return Choice{&r64::ops, GridChoice{}}; }

// ---------------------------------------------------------------------------
// fixed device scratch of ccl_label_noalloc
// ---------------------------------------------------------------------------
//
// The workspace of ccl_label_noalloc lives in this file-scope device array,
// which every device holds from the time the library's code is loaded on it
// until the process ends.  In host code `scratch` names a host-side stand-in,
// not device memory: its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is
// ever passed to kernels.  Nothing in the workspace needs to start at zero:
// the local step writes every entry the later kernels read.

constexpr int64_t NOALLOC_SCRATCH_BYTES = int64_t(32) << 20;
static __device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_addr;  // device -> address of its copy of scratch

static int scratch_address(void** out, const char* who)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(CCL_ERR_HIP, "%s: hipGetDevice: %s", who, hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    const auto it = g_scratch_addr.find(dev);
    if (it != g_scratch_addr.end()) {
        *out = it->second;
        return CCL_OK;
    }
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(CCL_ERR_HIP, "%s: hipGetSymbolAddress(scratch) on device %d: %s", who, dev,
                    hipGetErrorString(e));
    g_scratch_addr[dev] = ptr;
    *out = ptr;
    return CCL_OK;
}

// Labels a batch: one set of launches per connectivity class, each with the
// tile shape the policy (or `forced_rows`) picks for it.
static int label_batch(const ccl_image_desc* descs, int32_t n, int forced_rows, hipStream_t st,
                       const char* who)
{
    if (n < 0) return fail(CCL_ERR_INVALID_ARG, "%s: n = %d", who, n);
    if (n == 0) return CCL_OK;
    if (!descs) return fail(CCL_ERR_INVALID_ARG, "%s: null descriptor array", who);
    int64_t class_px[2] = {0, 0}, class_n[2] = {0, 0};
    for (int32_t i = 0; i < n; ++i) {
        const ccl_image_desc& d = descs[i];
        char w[64];
        snprintf(w, sizeof w, "%s[%d]", who, i);
        int rc = validate(d.img, d.H, d.W, d.pitch_bytes, d.connectivity, d.labels, w);
        if (rc != CCL_OK) return rc;
        if (d.H == 0 || d.W == 0) continue;
        class_px[d.connectivity == 8] += (int64_t)d.H * d.W;
        class_n[d.connectivity == 8] += 1;
    }
    Choice ch[2];
    for (int c = 0; c < 2; ++c) ch[c] = choose(class_n[c] > 1, class_px[c], c ? 8 : 4, forced_rows);
    // the node ids of each connectivity class must fit in int32 (checked
    // before anything is enqueued)
    int64_t class_tiles[2] = {0, 0};
    for (int32_t i = 0; i < n; ++i) {
        const ccl_image_desc& d = descs[i];
        if (d.H == 0 || d.W == 0) continue;
        const int c = d.connectivity == 8;
        class_tiles[c] += tiles_of(d.H, d.W, ch[c].ops->rows);
    }
    for (int c = 0; c < 2; ++c)
        if (class_n[c] && !node_ids_fit(class_tiles[c], ch[c].ops->rows))
            return fail(CCL_ERR_TOO_LARGE, "%s: %lld tiles of connectivity %d "
                        "exceed the node id range", who, (long long)class_tiles[c], c ? 8 : 4);
    std::vector<ImageArgs> by_conn[2];
    for (int32_t i = 0; i < n; ++i) {
        const ccl_image_desc& d = descs[i];
        if (d.H == 0 || d.W == 0) continue;
        const int c = d.connectivity == 8;
        by_conn[c].push_back(make_args(d.img, d.H, d.W, d.pitch_bytes, d.labels, ch[c].ops->rows));
    }
    for (int c = 0; c < 2; ++c) {
        int rc = run_batch(by_conn[c], c ? 8 : 4, ch[c], st, false, who);
        if (rc != CCL_OK) return rc;
    }
    return CCL_OK;
}

}  // namespace ccl

using namespace ccl;

static_assert(sizeof(CompStats) == sizeof(ccl_component) &&
                  offsetof(CompStats, sum_x) == offsetof(ccl_component, sum_x),
              "statistics layout");

// A prepared batch: own device memory, tables filled, ready to launch.
struct ccl_plan {
    int device = 0;
    void* mem = nullptr;
    struct Class {
        int conn;
        Choice ch;  // tile shape and grids, fixed when the plan is made
        BatchArgs b;
        Workspace ws;
    };
    std::vector<Class> classes;
};

extern "C" {

int ccl_label(const uint8_t* img, int32_t H, int32_t W, int64_t pitch_bytes,
              int32_t connectivity, int32_t* labels, void* stream)
{
    g_err.clear();
    const Choice ch = choose(false, (int64_t)H * W, connectivity, 0);
    return label_one(img, H, W, pitch_bytes, connectivity, labels,
                     static_cast<hipStream_t>(stream), false, ch, "ccl_label");
}

int ccl_label_noalloc(const uint8_t* img, int32_t H, int32_t W, int64_t pitch_bytes,
                      int32_t connectivity, int32_t* labels, void* stream)
{
    g_err.clear();
    const char* who = "ccl_label_noalloc";
    int rc = validate(img, H, W, pitch_bytes, connectivity, labels, who);
    if (rc != CCL_OK || H == 0 || W == 0) return rc;
    // the built-in tile shape and grids: the scratch is sized for them
    const Choice ch = builtin_choice();
    const int64_t ntiles = tiles_of(H, W, ch.ops->rows);
    const int64_t need = node_ids_fit(ntiles, ch.ops->rows)
                             ? workspace_bytes(ntiles, ch.ops->rows)
                             : INT64_MAX;
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(CCL_ERR_TOO_LARGE, "%s: %dx%d needs %lld workspace bytes; the fixed scratch "
                    "holds %lld (about %lld tiles of %dx%d pixels)", who, H, W,
                    (long long)(need == INT64_MAX ? -1 : need), (long long)NOALLOC_SCRATCH_BYTES,
                    (long long)(NOALLOC_SCRATCH_BYTES /
                                (ch.ops->rows * 8 + nslots(ch.ops->rows) * 12 +
                                 runtab_per_tile(ch.ops->rows) * 2 + 4)),
                    ch.ops->rows, TW);
    void* base = nullptr;
    rc = scratch_address(&base, who);
    if (rc != CCL_OK) return rc;
    std::vector<ImageArgs> one(1, make_args(img, H, W, pitch_bytes, labels, ch.ops->rows));
    ClassLayout L;
    rc = layout_class(one, connectivity, *ch.ops, L, who);
    if (rc != CCL_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    BatchArgs b;
    Workspace ws;
    // a single image: no device tables, so nothing is copied
    rc = bind_class(one, L, base, false, st, b, ws, who);
    if (rc != CCL_OK) return rc;
    hipError_t e = ch.ops->label(b, connectivity, ws, st, nullptr, false, ch.grid, nullptr);
    if (e != hipSuccess) return fail(CCL_ERR_HIP, "%s: launch failed: %s", who, hipGetErrorString(e));
    return CCL_OK;
}

int ccl_label_tiled(const uint8_t* img, int32_t H, int32_t W, int64_t pitch_bytes,
                    int32_t connectivity, int32_t* labels, int32_t tile_rows, void* stream)
{
    g_err.clear();
    if (tile_rows != 0 && !shape_for_rows(tile_rows))
        return fail(CCL_ERR_INVALID_ARG, "ccl_label_tiled: tile height %d is not built "
                    "(32, 64 or 128; 0 = policy)", tile_rows);
    const Choice ch = choose(false, (int64_t)H * W, connectivity, tile_rows);
    return label_one(img, H, W, pitch_bytes, connectivity, labels,
                     static_cast<hipStream_t>(stream), false, ch, "ccl_label_tiled");
}

int ccl_label_stats(const uint8_t* img, int32_t H, int32_t W, int64_t pitch_bytes,
                    int32_t connectivity, int32_t* labels, ccl_component* comps,
                    int64_t capacity, int64_t* count, void* stream)
{
    g_err.clear();
    const char* who = "ccl_label_stats";
    int rc = validate(img, H, W, pitch_bytes, connectivity, labels, who);
    if (rc != CCL_OK) return rc;
    if (!count) return fail(CCL_ERR_INVALID_ARG, "%s: null count pointer", who);
    if (capacity < 0) return fail(CCL_ERR_INVALID_ARG, "%s: capacity %lld < 0", who,
                                  (long long)capacity);
    if (capacity > 0 && !comps)
        return fail(CCL_ERR_INVALID_ARG, "%s: null component array with capacity %lld", who,
                    (long long)capacity);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (H == 0 || W == 0) {
        hipError_t e = r64::launch_zero_count(count, st);
        if (e != hipSuccess) return fail(CCL_ERR_HIP, "%s: launch failed: %s", who, hipGetErrorString(e));
        return CCL_OK;
    }
    if (!node_ids_fit(tiles_of(H, W, DEFAULT_ROWS), DEFAULT_ROWS))
        return fail(CCL_ERR_TOO_LARGE, "%s: %dx%d needs too many tiles", who, H, W);
    std::vector<ImageArgs> one(1, make_args(img, H, W, pitch_bytes, labels, DEFAULT_ROWS));
    StatsOut so{comps, capacity, count};
    return run_batch(one, connectivity, builtin_choice(), st, false, who, &so);
}

int ccl_label_3d(const uint8_t* vol, int32_t D, int32_t H, int32_t W, int64_t pitch_bytes,
                 int64_t slice_pitch_bytes, int32_t connectivity, int32_t* labels, void* stream)
{
    g_err.clear();
    const char* who = "ccl_label_3d";
    if (D < 0 || H < 0 || W < 0)
        return fail(CCL_ERR_INVALID_ARG, "%s: negative size %dx%dx%d", who, D, H, W);
    if (connectivity != 6 && connectivity != 26)
        return fail(CCL_ERR_INVALID_ARG, "%s: connectivity %d is not 6 or 26", who, connectivity);
    if (D == 0 || H == 0 || W == 0) return CCL_OK;
    if ((int64_t)D * H * W > (int64_t)INT32_MAX)
        return fail(CCL_ERR_TOO_LARGE, "%s: %dx%dx%d voxels exceed int32 labels", who, D, H, W);
    if (!vol || !labels) return fail(CCL_ERR_INVALID_ARG, "%s: null pointer", who);
    if (pitch_bytes < W)
        return fail(CCL_ERR_INVALID_ARG, "%s: pitch %lld < width %d", who, (long long)pitch_bytes, W);
    if (D > 1 && slice_pitch_bytes < (int64_t)(H - 1) * pitch_bytes + W)
        return fail(CCL_ERR_INVALID_ARG, "%s: slice pitch %lld is smaller than a slice", who,
                    (long long)slice_pitch_bytes);
    const uintptr_t v0 = (uintptr_t)vol,
                    v1 = v0 + (uintptr_t)((int64_t)(D - 1) * slice_pitch_bytes +
                                          (int64_t)(H - 1) * pitch_bytes + W);
    const uintptr_t l0 = (uintptr_t)labels, l1 = l0 + (uintptr_t)((int64_t)D * H * W * 4);
    if (v0 < l1 && l0 < v1) return fail(CCL_ERR_INVALID_ARG, "%s: vol and labels overlap", who);
    hipStream_t st = static_cast<hipStream_t>(stream);
    VolArgs v;
    v.vol = vol;
    v.pitch = pitch_bytes;
    v.spitch = D > 1 ? slice_pitch_bytes : 0;
    v.labels = labels;
    v.D = D;
    v.H = H;
    v.W = W;
    v.nbx = (W + VOL_BRICK_W - 1) / VOL_BRICK_W;
    v.nby = (H + VOL_BRICK_H - 1) / VOL_BRICK_H;
    v.nbz = (D + VOL_BRICK_D - 1) / VOL_BRICK_D;
    v.vec = ((uintptr_t)labels & 15) == 0;
    auto magic = [](int64_t d) { return d == 1 ? 0xffffffffu : (uint32_t)((1ull << 32) / (uint64_t)d); };
    v.wmagic = magic(W);
    v.smagic = magic((int64_t)H * W);
    hipError_t e = r64::launch_volume(v, connectivity, st, active_timer());
    if (e != hipSuccess) return fail(CCL_ERR_HIP, "%s: launch failed: %s", who, hipGetErrorString(e));
    return CCL_OK;
}

int ccl_label_ablation(const uint8_t* img, int32_t H, int32_t W, int64_t pitch_bytes,
                       int32_t variant, int32_t* labels, uint32_t* counters, void* stream)
{
    g_err.clear();
    const char* who = "ccl_label_ablation";
    if (variant < CCL_C2FL || variant > CCL_NC2FL)
        return fail(CCL_ERR_INVALID_ARG, "%s: variant %d is not one of 0..3", who, variant);
    int rc = validate(img, H, W, pitch_bytes, 4, labels, who);
    if (rc != CCL_OK || H == 0 || W == 0) return rc;
    if (!node_ids_fit(tiles_of(H, W, DEFAULT_ROWS), DEFAULT_ROWS))
        return fail(CCL_ERR_TOO_LARGE, "%s: %dx%d needs too many tiles", who, H, W);
    std::vector<ImageArgs> one(1, make_args(img, H, W, pitch_bytes, labels, DEFAULT_ROWS));
    return run_batch(one, 4, builtin_choice(), static_cast<hipStream_t>(stream), false, who,
                     nullptr, variant, counters);
}

int ccl_label_local(const uint8_t* img, int32_t H, int32_t W, int64_t pitch_bytes,
                    int32_t connectivity, int32_t* labels, void* stream)
{
    g_err.clear();
    return label_one(img, H, W, pitch_bytes, connectivity, labels,
                     static_cast<hipStream_t>(stream), true, builtin_choice(), "ccl_label_local");
}

int ccl_label_batch(const ccl_image_desc* descs, int32_t n, void* stream)
{
    g_err.clear();
    return label_batch(descs, n, 0, static_cast<hipStream_t>(stream), "ccl_label_batch");
}

int ccl_label_batch_tiled(const ccl_image_desc* descs, int32_t n, int32_t tile_rows,
                          void* stream)
{
    g_err.clear();
    if (tile_rows != 0 && !shape_for_rows(tile_rows))
        return fail(CCL_ERR_INVALID_ARG, "ccl_label_batch_tiled: tile height %d is not built "
                    "(32, 64 or 128; 0 = policy)", tile_rows);
    return label_batch(descs, n, tile_rows, static_cast<hipStream_t>(stream),
                       "ccl_label_batch_tiled");
}

int ccl_plan_create(const ccl_image_desc* descs, int32_t n, void* stream, ccl_plan** plan)
{
    g_err.clear();
    if (!plan) return fail(CCL_ERR_INVALID_ARG, "ccl_plan_create: null plan pointer");
    *plan = nullptr;
    if (n < 0 || (n > 0 && !descs)) return fail(CCL_ERR_INVALID_ARG, "ccl_plan_create: bad descriptors");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int64_t class_px[2] = {0, 0}, class_n[2] = {0, 0};
    for (int32_t i = 0; i < n; ++i) {
        const ccl_image_desc& d = descs[i];
        char who[64];
        snprintf(who, sizeof who, "ccl_plan_create[%d]", i);
        int rc = validate(d.img, d.H, d.W, d.pitch_bytes, d.connectivity, d.labels, who);
        if (rc != CCL_OK) return rc;
        if (d.H == 0 || d.W == 0) continue;
        class_px[d.connectivity == 8] += (int64_t)d.H * d.W;
        class_n[d.connectivity == 8] += 1;
    }
    Choice ch[2];
    for (int c = 0; c < 2; ++c) ch[c] = choose(class_n[c] > 1, class_px[c], c ? 8 : 4, 0);
    std::vector<ImageArgs> by_conn[2];
    for (int32_t i = 0; i < n; ++i) {
        const ccl_image_desc& d = descs[i];
        if (d.H == 0 || d.W == 0) continue;
        const int c = d.connectivity == 8;
        by_conn[c].push_back(make_args(d.img, d.H, d.W, d.pitch_bytes, d.labels, ch[c].ops->rows));
    }
    ClassLayout L[2];
    int64_t total = 0;
    for (int c = 0; c < 2; ++c) {
        if (by_conn[c].empty()) continue;
        int rc = layout_class(by_conn[c], c ? 8 : 4, *ch[c].ops, L[c], "ccl_plan_create");
        if (rc != CCL_OK) return rc;
        total += align256(L[c].bytes());
    }
    ccl_plan* p = new ccl_plan;
    (void)hipGetDevice(&p->device);
    if (total > 0) {
        hipError_t e = hipMalloc(&p->mem, (size_t)total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete p;
            return fail(CCL_ERR_OUT_OF_MEMORY, "ccl_plan_create: %lld bytes: %s",
                        (long long)total, hipGetErrorString(e));
        }
    }
    char* base = static_cast<char*>(p->mem);
    for (int c = 0; c < 2; ++c) {
        if (by_conn[c].empty()) continue;
        ccl_plan::Class k;
        k.conn = c ? 8 : 4;
        k.ch = ch[c];
        int rc = bind_class(by_conn[c], L[c], base, false, st, k.b, k.ws, "ccl_plan_create");
        hipError_t e = rc == CCL_OK ? k.ch.ops->index(k.b, st) : hipSuccess;
        if (rc != CCL_OK || e != hipSuccess) {
            (void)hipStreamSynchronize(st);
            (void)hipFree(p->mem);
            delete p;
            return rc != CCL_OK ? rc : fail(CCL_ERR_HIP, "ccl_plan_create: %s", hipGetErrorString(e));
        }
        p->classes.push_back(k);
        base += align256(L[c].bytes());
    }
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFree(p->mem);
        delete p;
        return fail(CCL_ERR_HIP, "ccl_plan_create: %s", hipGetErrorString(e));
    }
    *plan = p;
    return CCL_OK;
}

int ccl_plan_run(ccl_plan* plan, void* stream)
{
    g_err.clear();
    if (!plan) return fail(CCL_ERR_INVALID_ARG, "ccl_plan_run: null plan");
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (auto& k : plan->classes) {
        hipError_t e = k.ch.ops->label(k.b, k.conn, k.ws, st, active_timer(), false, k.ch.grid,
                                       nullptr);
        if (e != hipSuccess) return fail(CCL_ERR_HIP, "ccl_plan_run: %s", hipGetErrorString(e));
    }
    return CCL_OK;
}

int ccl_plan_destroy(ccl_plan* plan)
{
    g_err.clear();
    if (!plan) return CCL_OK;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(plan->device);
    (void)hipDeviceSynchronize();
    if (plan->mem) (void)hipFree(plan->mem);
    (void)hipSetDevice(prev);
    delete plan;
    return CCL_OK;
}

int ccl_set_launch_policy(int32_t batch, int32_t bucket, int32_t connectivity,
                          int32_t tile_rows, int32_t local, int32_t final_)
{
    g_err.clear();
    if (batch < 0 || batch > 1 || bucket < 0 || bucket >= POLICY_BUCKETS ||
        (connectivity != 4 && connectivity != 8) || (tile_rows != 0 && !shape_for_rows(tile_rows)) ||
        local < -1 || local > 1 || final_ < -1 || final_ > 1)
        return fail(CCL_ERR_INVALID_ARG,
                    "ccl_set_launch_policy: batch %d (0|1), bucket %d (0..%d), connectivity %d "
                    "(4|8), tile rows %d (0|32|64|128), local %d, final %d (-1|0|1)",
                    batch, bucket, POLICY_BUCKETS - 1, connectivity, tile_rows, local, final_);
    PolicyEntry& e = g_policy[batch][bucket][connectivity == 8];
    e.rows.store(tile_rows, std::memory_order_relaxed);
    e.local.store(local, std::memory_order_relaxed);
    e.final_.store(final_, std::memory_order_relaxed);
    return CCL_OK;
}

int32_t ccl_launch_buckets(int64_t* upper, int32_t n)
{
    for (int32_t k = 0; upper && k < n && k < POLICY_BUCKETS; ++k) upper[k] = kBucketPx[k];
    return POLICY_BUCKETS;
}

int32_t ccl_policy_tile_rows(int32_t batch, int64_t pixels, int32_t connectivity)
{
    if (batch < 0 || batch > 1 || pixels < 0 || (connectivity != 4 && connectivity != 8))
        return -1;
    return choose(batch == 1, pixels, connectivity, 0).ops->rows;
}

int32_t ccl_tile_shapes(int32_t* rows, int32_t n)
{
    for (int32_t k = 0; rows && k < n && k < NSHAPES; ++k) rows[k] = SHAPE_ROWS[k];
    return NSHAPES;
}

int32_t ccl_tile_cols(void) { return TW; }
int32_t ccl_tile_rows(void) { return DEFAULT_ROWS; }

int64_t ccl_workspace_bytes(int32_t H, int32_t W)
{
    if (H < 0 || W < 0) return -1;
    if (H == 0 || W == 0) return 0;
    int64_t most = 0;
    for (const ShapeOps* o : kShapes) {
        const int64_t b = workspace_bytes(tiles_of(H, W, o->rows), o->rows);
        most = b > most ? b : most;
    }
    return most;
}

int64_t ccl_workspace_cached(void* stream)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    const auto it = g_ws.find({dev, static_cast<hipStream_t>(stream)});
    return it == g_ws.end() ? 0 : it->second.bytes;
}

const char* ccl_last_error(void) { return g_err.c_str(); }

int ccl_release_workspace(int32_t device)
{
    g_err.clear();
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return fail(CCL_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(g_ws_mu);
    bool any = false;
    for (auto it = g_ws.begin(); it != g_ws.end();) {
        if (it->first.first == device) {
            if (!any) {
                if ((e = hipSetDevice(device)) != hipSuccess)
                    return fail(CCL_ERR_HIP, "hipSetDevice: %s", hipGetErrorString(e));
                (void)hipDeviceSynchronize();
                any = true;
            }
            if (it->second.ptr) (void)hipFree(it->second.ptr);
            it = g_ws.erase(it);
        } else {
            ++it;
        }
    }
    {
        // the device is synchronised above if it had a workspace; the staging
        // buffers' copies are then complete as well
        std::lock_guard<std::mutex> sl(g_stage_mu);
        for (auto it = g_stage.begin(); it != g_stage.end();) {
            if (it->first.first != device) {
                ++it;
                continue;
            }
            for (Stage& s : it->second.s) {
                if (s.used) (void)hipEventSynchronize(s.done);
                if (s.done) (void)hipEventDestroy(s.done);
                if (s.host) (void)hipHostFree(s.host);
            }
            it = g_stage.erase(it);
        }
    }
    if (any) (void)hipSetDevice(prev);
    return CCL_OK;
}

int ccl_timing_enable(int32_t enable)
{
    std::lock_guard<std::mutex> lk(g_timer.mu);
    for (auto& r : g_timer.done) {
        g_timer.pool.push_back(r.a);
        g_timer.pool.push_back(r.b);
    }
    g_timer.done.clear();
    for (int k = 0; k < NKINDS; ++k) {
        g_timer.ms[k] = 0.0;
        g_timer.launches[k] = 0;
    }
    g_timing_mask = (uint32_t)enable & ((1u << NKINDS) - 1u);
    return CCL_OK;
}

int ccl_timing_read(double* ms, int64_t* launches, int32_t n)
{
    g_err.clear();
    std::lock_guard<std::mutex> lk(g_timer.mu);
    for (auto& r : g_timer.done) {
        float t = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
        if (e != hipSuccess) return fail(CCL_ERR_HIP, "timing: %s", hipGetErrorString(e));
        g_timer.ms[r.kind] += t;
        g_timer.launches[r.kind] += 1;
        g_timer.pool.push_back(r.a);
        g_timer.pool.push_back(r.b);
    }
    g_timer.done.clear();
    for (int k = 0; k < n && k < NKINDS; ++k) {
        if (ms) ms[k] = g_timer.ms[k];
        if (launches) launches[k] = g_timer.launches[k];
    }
    return NKINDS;
}

int ccl_replay_last(int32_t kind, int32_t reps, void* stream)
{
    g_err.clear();
    const char* who = "ccl_replay_last";
    if (kind != KIND_LOCAL && kind != KIND_FINAL)
        return fail(CCL_ERR_INVALID_ARG, "%s: kind %d is not 0 (local step) or 2 (final relabel)",
                    who, kind);
    if (reps < 0) return fail(CCL_ERR_INVALID_ARG, "%s: reps = %d", who, reps);
    int dev = -1;
    if (!g_last.valid || hipGetDevice(&dev) != hipSuccess || dev != g_last.device)
        return fail(CCL_ERR_INVALID_ARG, "%s: no labelling call on this thread and device", who);
    hipError_t e = g_last.ch.ops->replay(g_last.b, g_last.conn, g_last.ws,
                                         static_cast<hipStream_t>(stream), g_last.ch.grid, kind,
                                         reps);
    if (e != hipSuccess) return fail(CCL_ERR_HIP, "%s: %s", who, hipGetErrorString(e));
    return CCL_OK;
}

int ccl_copy_bytes(const void* src, void* dst, int64_t bytes, void* stream)
{
    g_err.clear();
    if (bytes < 0 || (bytes > 0 && (!src || !dst)))
        return fail(CCL_ERR_INVALID_ARG, "ccl_copy_bytes: bad arguments");
    if (((uintptr_t)src | (uintptr_t)dst | (uintptr_t)bytes) % 16)
        return fail(CCL_ERR_INVALID_ARG, "ccl_copy_bytes: pointers and size must be 16-byte aligned");
    if (bytes == 0) return CCL_OK;
    hipError_t e =
        r64::launch_copy(src, dst, bytes, static_cast<hipStream_t>(stream), active_timer());
    if (e != hipSuccess) return fail(CCL_ERR_HIP, "ccl_copy_bytes: %s", hipGetErrorString(e));
    return CCL_OK;
}

int ccl_copy_segments(const void* src, void* dst, int64_t bytes, int32_t segment_bytes,
                      int64_t src_stride_bytes, void* stream)
{
    g_err.clear();
    if (bytes < 0 || (bytes > 0 && (!src || !dst)) || segment_bytes <= 0 ||
        src_stride_bytes < segment_bytes)
        return fail(CCL_ERR_INVALID_ARG, "ccl_copy_segments: bad arguments");
    if (((uintptr_t)src | (uintptr_t)dst | (uintptr_t)bytes | (uintptr_t)segment_bytes |
         (uintptr_t)src_stride_bytes) % 16 || bytes % segment_bytes)
        return fail(CCL_ERR_INVALID_ARG, "ccl_copy_segments: pointers, sizes and stride must be "
                    "16-byte aligned, and bytes a multiple of the segment");
    if (bytes == 0) return CCL_OK;
    hipError_t e = r64::launch_copy_segments(src, dst, bytes, segment_bytes, src_stride_bytes,
                                             static_cast<hipStream_t>(stream), active_timer());
    if (e != hipSuccess) return fail(CCL_ERR_HIP, "ccl_copy_segments: %s", hipGetErrorString(e));
    return CCL_OK;
}

}  // extern "C"
