// Block-based coarse-to-fine connected-components labelling for gfx950.
//
// The image is cut into tiles of 64 x TILE_ROWS pixels: one 64-bit
// foreground mask per tile row, so the paper's row scan becomes bit
// arithmetic on a word.  A workgroup of 4 * TILE_ROWS threads owns a tile
// (one sixteen-pixel chunk of a row each).  The file is compiled once per
// tile height (32, 64 and 128 rows: the paper's block shape is its tuning
// knob), and the host picks the height per call.
//
// Nodes of the tile-local union-find are runs: maximal horizontal stretches
// of foreground.  Under 8-connectivity two rows are fused into a strip first:
// any run of (row 2k | row 2k+1) is 8-connected (neighbouring columns that
// each hold a foreground pixel in one of the two rows always touch), so a
// strip run is a node.  "Line" below means a row (4-connectivity) or a strip
// (8-connectivity); runs get dense ids in line-major, left-to-right order.
//
// Four kernels per image (the paper's Section 3):
//   k_local  (Section 3.1)  load the tile, label it in LDS, and publish what
//            the merge and the relabel need: the foreground bitmask, a run
//            table (local root of each run), one forest node id per border
//            pixel, and one forest node per component that touches the tile
//            border.
//   k_block  (Section 3.2, inside groups of 256 x 256 pixels)  unite the border
//            nodes across the seams inside the group in LDS and write the
//            group roots to the forest.
//   k_seam   (Section 3.2, between groups)  for every foreground pair
//            straddling a group seam, unite the two group roots in HBM
//            (atomicMin).
//   k_final  (Section 3.3)  look up the global root of each border component
//            and write every label exactly once, from the bitmask and the run
//            table (no union-find work is repeated).
// Batches of images share one launch of each (k_index maps tiles, groups and
// seam workgroups to their image).  Optional extras: per-component statistics
// (k_scan1/2, k_stats, k_stats_merge) and the paper's ablation
// variants of the local step (k_local_ablate).
//
// Labels are canonical: 1 + the smallest raster position of the component.
// Every node carries a key, the tile position of its smallest pixel; parents
// are packed as (key << 16 | id), so "point the larger root at the smaller"
// (the paper's merge) is an atomicMin on the packed word, and the root of a
// tile component is the node with the smallest key.  Both tile order and
// raster order are row-major, so the smallest key is the smallest raster
// position.  Across tiles the HBM forest orders roots by raster position.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <utility>

#include "ccl_kernels.h"

// One build per tile height: CCL_TILE_ROWS rows, launchers in namespace
// ccl::CCL_SHAPE_NS.
#ifndef CCL_TILE_ROWS
#define CCL_TILE_ROWS 64
#endif
#ifndef CCL_SHAPE_NS
#define CCL_SHAPE_NS r64
#endif

namespace ccl {
namespace CCL_SHAPE_NS {

constexpr int TILE_ROWS = CCL_TILE_ROWS;
static_assert(TILE_ROWS == 32 || TILE_ROWS == 64 || TILE_ROWS == 128, "built tile heights");
constexpr int NSLOTS = nslots(TILE_ROWS);             // border pixels per tile
constexpr int RUNTAB_PER_TILE = runtab_per_tile(TILE_ROWS);
constexpr int NT = tile_threads(TILE_ROWS);           // threads per tile workgroup
constexpr int SPT = (NSLOTS + NT - 1) / NT;           // border slots per thread, at most

// Geometry of one connectivity: D = 0 (4-connectivity, lines are rows) or
// D = 1 (8-connectivity, lines are two-row strips).
template <int D>
struct Geo {
    static constexpr int NL = D ? TILE_ROWS / 2 : TILE_ROWS;  // lines per tile
    static constexpr int TPL = NT / NL;                       // threads per line
    static constexpr int WIN = TW / TPL;                      // columns per thread
    static constexpr int MAXR = NL * (TW / 2);                // runs per tile, at most
    // refinement edges per tile, at most: one per column and line boundary
    // (8-connectivity), one per stretch start of T & B (4-connectivity)
    static constexpr int MAXE = NL * (D ? TW : TW / 2);
};
static_assert(Geo<0>::MAXR <= RUNTAB_PER_TILE && Geo<1>::MAXR <= RUNTAB_PER_TILE, "run table");
// packed LDS parents hold a 16-bit tile key and a 16-bit run id
static_assert(TILE_ROWS * TW <= 0x8000 && Geo<0>::MAXR <= 0x10000, "16-bit keys and ids");

// ---------------------------------------------------------------------------
// bit helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int ctz64(uint64_t v) { return __builtin_ctzll(v); }
__device__ __forceinline__ int ctz64_or64(uint64_t v) { return v ? __builtin_ctzll(v) : 64; }
__device__ __forceinline__ uint32_t popc64(uint64_t v) { return (uint32_t)__popcll(v); }
__device__ __forceinline__ int msb64(uint64_t v) { return 63 - __builtin_clzll(v); }

// Bits 0..x inclusive (x in 0..63).
__device__ __forceinline__ uint64_t upto(int x) { return (2ull << x) - 1ull; }
// Bits lo..hi inclusive, 0 <= lo <= hi <= 63.
__device__ __forceinline__ uint64_t span_mask(int lo, int hi)
{
    return (~0ull << lo) & (~0ull >> (63 - hi));
}

// Nonzero bytes of a dword -> 4-bit mask (bit i = byte i != 0).
__device__ __forceinline__ uint32_t nz_nibble(uint32_t d)
{
    uint32_t t = (((d & 0x7f7f7f7fu) + 0x7f7f7f7fu) | d) >> 7;
    return ((t & 0x01010101u) * 0x01020408u) >> 24;
}

// ---------------------------------------------------------------------------
// LDS union-find over run ids, parents packed as (key << 16) | id
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t pk(uint32_t key, uint32_t id) { return (key << 16) | id; }
__device__ __forceinline__ uint32_t pk_id(uint32_t v) { return v & 0xffffu; }
__device__ __forceinline__ uint32_t pk_key(uint32_t v) { return v >> 16; }

__device__ __forceinline__ uint32_t lds_ld(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Packed root of x.  Halves the path on the way: x takes its grandparent,
// whose key is smaller.  The halving write is an atomic min, not a store: a
// stale grandparent read before another thread pointed x straight at the
// root must not overwrite that pointer (the run table and the border slots
// rely on every run holding its root after the unification passes).  Along
// a path keys only decrease, so the root is the smallest value x can hold.
__device__ uint32_t pfind(uint32_t* P, uint32_t x)
{
    uint32_t v = lds_ld(P + x);
    while (pk_id(v) != x) {
        const uint32_t p = pk_id(v);
        const uint32_t w = lds_ld(P + p);
        if (pk_id(w) == p) return w;
        __hip_atomic_fetch_min(P + x, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        x = pk_id(w);
        v = lds_ld(P + x);
    }
    return v;
}

// Counting versions for the ablation study: `it` counts steps of the find
// loops (the paper's iterations), `at` the atomic merge attempts.
__device__ uint32_t pfind_count(uint32_t* P, uint32_t x, uint32_t& it)
{
    uint32_t v = lds_ld(P + x);
    while (pk_id(v) != x) {
        ++it;
        const uint32_t p = pk_id(v);
        const uint32_t w = lds_ld(P + p);
        if (pk_id(w) == p) return w;
        __hip_atomic_fetch_min(P + x, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        x = pk_id(w);
        v = lds_ld(P + x);
    }
    return v;
}

__device__ void punion_count(uint32_t* P, uint32_t a, uint32_t b, uint32_t& it, uint32_t& at)
{
    while (true) {
        uint32_t ra = pfind_count(P, a, it), rb = pfind_count(P, b, it);
        if (ra == rb) return;
        if (ra < rb) { uint32_t t = ra; ra = rb; rb = t; }
        ++at;
        const uint32_t old = __hip_atomic_fetch_min(P + pk_id(ra), rb, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old == ra) return;
        a = pk_id(old);
        b = pk_id(rb);
    }
}

// The paper's merge (Section 3.1.3): compare the two roots and point the one
// with the larger key at the other, atomically; if it stopped being a root
// in the meantime, continue with the parent it had.
__device__ void punion(uint32_t* P, uint32_t a, uint32_t b)
{
    while (true) {
        uint32_t ra = pfind(P, a), rb = pfind(P, b);
        if (ra == rb) return;
        if (ra < rb) { uint32_t t = ra; ra = rb; rb = t; }
        const uint32_t old = __hip_atomic_fetch_min(P + pk_id(ra), rb, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old == ra) return;
        a = pk_id(old);
        b = pk_id(rb);
    }
}

// Caller buffers (image, labels, statistics) are reached through pointers
// read from memory, which the compiler cannot place in an address space, so
// it would use flat instructions; flat accesses also count against the LDS
// wait counter, and every LDS wait would then wait for them too (the
// next-tile prefetch and the label stores included).  These accessors name
// the global address space explicitly.
template <typename V>
__device__ __forceinline__ V ld_global(const V* p)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return *(const __attribute__((address_space(1))) V*)p;
#else
    return *p;  // host pass: never executed
#endif
}
template <typename V>
__device__ __forceinline__ void st_global(V* p, const V& v)
{
#if defined(__HIP_DEVICE_COMPILE__)
    *(__attribute__((address_space(1))) V*)p = v;
#else
    *p = v;  // host pass: never executed
#endif
}
// 16-byte accesses go through plain vector types: the copy of HIP's uint4 /
// int4 classes would turn the global lvalue back into a generic one.
typedef uint32_t v4u32 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ld_global16(const void* p)
{
    const v4u32 v = ld_global(reinterpret_cast<const v4u32*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st_global16(void* p, int32_t a, int32_t b, int32_t c, int32_t d)
{
    v4u32 v;
    v.x = (uint32_t)a;
    v.y = (uint32_t)b;
    v.z = (uint32_t)c;
    v.w = (uint32_t)d;
    st_global(reinterpret_cast<v4u32*>(p), v);
}

// ---------------------------------------------------------------------------
// HBM forest over border components.  Entry = (key of parent << 32) | parent
// node; a root stores its own key and id.  Keys (raster position of a tile
// component's smallest pixel) are distinct across components, so atomicMin
// on the packed word only ever moves a parent to a smaller key.
// ---------------------------------------------------------------------------

struct Root {
    uint32_t node;
    uint32_t key;
};

__device__ __forceinline__ uint64_t g_ld(const uint64_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Reads of the forest during a merge.  A find's first two hops use plain
// (cacheable) loads: most finds end there, at a root many threads share.  A
// stale entry still names an ancestor, and a stale "root" is caught by the
// link's atomic min, which returns the current entry, and the union goes on
// from there; longer chases switch to coherent loads, which keep chains that
// are being rewritten from being walked through old entries.
__device__ __forceinline__ uint64_t g_hop(const uint64_t* p, int step)
{
    return step < 2 ? ld_global(p) : g_ld(p);
}

// Root of n, given v = F[n] already loaded.  Halves the path on the way
// with plain stores: a node is rewritten only after it was read as a
// non-root (roots are never stored to, and a node that has a parent never
// becomes a root again), and only with an ancestor, whose key is smaller.
// Such a store may replace a link another thread made meanwhile with its
// atomic min; that thread found the node no longer a root (the min returned
// another parent) and goes on uniting from that parent, so the link it made
// is not needed.  Atomic mins for the halving made the merge across groups
// slower where one component crosses the seams many times (all chains pass
// the same few nodes); plain stores gained on those images (8192^2
// serpentine 135 -> 111 us) and cost nothing elsewhere.
__device__ Root g_find_from(uint64_t* F, uint32_t n, uint64_t v)
{
    for (int step = 0;; step += 2) {
        uint32_t p = (uint32_t)v;
        if (p == n) return Root{n, (uint32_t)(v >> 32)};
        uint64_t vp = g_hop(F + p, step);
        uint32_t pp = (uint32_t)vp;
        if (pp == p) return Root{p, (uint32_t)(vp >> 32)};
        st_global(F + n, vp);
        n = pp;
        v = g_hop(F + n, step + 1);
    }
}

// The paper's merge on the HBM forest.  The first loads of both finds are
// issued together, so a union whose nodes are still roots costs one round
// trip before the link instead of two.
__device__ void g_union(uint64_t* F, uint32_t a, uint32_t b)
{
    while (true) {
        const uint64_t va = g_hop(F + a, 0), vb = g_hop(F + b, 0);
        Root ra = g_find_from(F, a, va);
        Root rb = g_find_from(F, b, vb);
        if (ra.node == rb.node) return;
        if (ra.key < rb.key) { Root t = ra; ra = rb; rb = t; }
        // ra has the larger key: link it under rb
        const uint64_t self = ((uint64_t)ra.key << 32) | ra.node;
        const uint64_t nv = ((uint64_t)rb.key << 32) | rb.node;
        const uint64_t old = __hip_atomic_fetch_min(F + ra.node, nv, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        if (old == self) return;
        a = (uint32_t)old;
        b = rb.node;
    }
}

// ---------------------------------------------------------------------------
// line structure shared by k_local and k_final
// ---------------------------------------------------------------------------

template <int D>
struct Lines {
    uint64_t M[TILE_ROWS];          // foreground mask of each tile row
    uint64_t LM[Geo<D>::NL];        // foreground columns of each line
    uint64_t LS[Geo<D>::NL];        // run starts of each line
    uint32_t base[Geo<D>::NL + 1];  // id of the first run of each line; base[NL] = runs
};

// Row masks in sh.M -> line masks, run starts and dense run-id bases.  Must be
// called by all threads; ends with a barrier.
template <int D>
__device__ void build_lines(Lines<D>& sh, int tid)
{
    constexpr int NL = Geo<D>::NL;
    constexpr int LPL = (NL + 63) / 64;  // consecutive lines per lane of the first wavefront
    if (tid < 64) {
        uint32_t cnt[LPL], tot = 0;
#pragma unroll
        for (int k = 0; k < LPL; ++k) {
            const int l = tid * LPL + k;
            cnt[k] = 0;
            if (l < NL) {
                const uint64_t lm = D ? (sh.M[2 * l] | sh.M[2 * l + 1]) : sh.M[l];
                const uint64_t ls = lm & ~(lm << 1);
                sh.LM[l] = lm;
                sh.LS[l] = ls;
                cnt[k] = popc64(ls);
            }
            tot += cnt[k];
        }
        // inclusive scan of the run counts across the first wavefront
        uint32_t inc = tot;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off, 64);
            if (tid >= off) inc += o;
        }
        uint32_t run = inc - tot;
#pragma unroll
        for (int k = 0; k < LPL; ++k) {
            const int l = tid * LPL + k;
            if (l < NL) sh.base[l] = run;
            run += cnt[k];
        }
        if (tid == 63) sh.base[NL] = inc;
    }
    __syncthreads();
}

// Dense id of the run of line l that contains foreground column x.
template <int D>
__device__ __forceinline__ uint32_t run_id(const Lines<D>& sh, int l, int x)
{
    return sh.base[l] + popc64(sh.LS[l] & upto(x)) - 1u;
}

// Row of line l that faces the line above / below it.
template <int D>
__device__ __forceinline__ uint64_t top_row(const Lines<D>& sh, int l)
{
    return D ? sh.M[2 * l] : sh.M[l];
}
template <int D>
__device__ __forceinline__ uint64_t bottom_row(const Lines<D>& sh, int l)
{
    return D ? sh.M[2 * l + 1] : sh.M[l];
}

// Tile position (y * 64 + x) of the smallest pixel of run [a, e] of line l.
template <int D>
__device__ __forceinline__ uint32_t run_key(const Lines<D>& sh, int l, int a, int e)
{
    if (!D) return (uint32_t)(l * TW + a);
    const uint64_t top = sh.M[2 * l] & span_mask(a, e);
    return top ? (uint32_t)(2 * l * TW + ctz64(top)) : (uint32_t)((2 * l + 1) * TW + a);
}

// Run list: RL[id] = start column | line << 6, for every run of the tile.
// Thread tid takes one window of Geo<D>::WIN columns of one line.  Needs
// build_lines; the caller synchronises before RL is read.
template <int D>
__device__ __forceinline__ void list_runs(const Lines<D>& sh, uint16_t* RL, int tid)
{
    using G = Geo<D>;
    static_assert(G::WIN <= 16, "column windows fit a 32-bit word");
    const int wl = tid / G::TPL, wlo = (tid % G::TPL) * G::WIN;
    const uint64_t ls = sh.LS[wl];
    uint32_t id = sh.base[wl] + popc64(ls & ~(~0ull << wlo));
    for (uint32_t r = (uint32_t)(ls >> wlo) & ((1u << G::WIN) - 1u); r; r &= r - 1u, ++id)
        RL[id] = (uint16_t)((__builtin_ctz(r) + wlo) | (wl << 6));
}

template <int D>
struct LocalShared : Lines<D> {
    uint32_t P[Geo<D>::MAXR];    // parent of each run, packed (key << 16) | id
    uint32_t nedges;             // refinement edges listed so far
    union {
        uint32_t EL[Geo<D>::MAXE];     // refinement edge: lower run | upper run << 16
        uint16_t h[TILE_ROWS * 4];     // 16-pixel masks as produced by the byte load
        uint64_t w[TILE_ROWS];         // the same bits as one word per row
    } u;
};

// Border slot s -> tile-local (x, y).  Slots: top row, bottom row, left
// column, right column.
__device__ __forceinline__ void slot_xy(int s, int& x, int& y)
{
    if (s < TW) { x = s; y = 0; }
    else if (s < 2 * TW) { x = s - TW; y = TILE_ROWS - 1; }
    else if (s < 2 * TW + TILE_ROWS) { x = 0; y = s - 2 * TW; }
    else { x = TW - 1; y = s - 2 * TW - TILE_ROWS; }
}

// Run-table entry flag: the run's component touches the tile border (low
// bits = its representative border slot; otherwise the entry is the tile
// position of the component's smallest pixel).
constexpr uint16_t RT_BORDER = 0x8000;
constexpr uint32_t REP_TAG = 0x80000000u;

// ---------------------------------------------------------------------------
// images of a batch
// ---------------------------------------------------------------------------

// The batch tables are read-only while the labelling kernels run and are
// indexed by workgroup-uniform values: they are read through the constant
// address space, so the loads go to the scalar unit and do not queue behind
// (or hold up) the vector loads of tile data in flight.
template <typename V>
__device__ __forceinline__ V ld_uniform(const V* p)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return *(const __attribute__((address_space(4))) V*)p;
#else
    return *p;  // host pass: never executed
#endif
}

// The fields are read one by one: a whole-struct copy is lowered to vector
// loads, whose wait would also wait for every store issued before them.
__device__ __forceinline__ ImageArgs batch_image(const BatchArgs& b, int i)
{
    if (b.n == 1) return b.one;
#if defined(__HIP_DEVICE_COMPILE__)
    const __attribute__((address_space(4))) ImageArgs* p =
        (const __attribute__((address_space(4))) ImageArgs*)(b.imgs + i);
#else
    const ImageArgs* p = b.imgs + i;  // host pass: never executed
#endif
    ImageArgs r;
    r.img = p->img;
    r.pitch = p->pitch;
    r.labels = p->labels;
    r.H = p->H;
    r.W = p->W;
    r.ntx = p->ntx;
    r.nty = p->nty;
    r.wmagic = p->wmagic;
    r.lbase = p->lbase;
    r.unused = 0;
    r.vec_out = p->vec_out;
    r.tbase = p->tbase;
    return r;
}
__device__ __forceinline__ int tile_image(const BatchArgs& b, int64_t T)
{
    return b.n == 1 ? 0 : ld_uniform(b.tile_img + T);
}

// Largest i with off[i] <= x, for off[0] = 0 <= x < off[n].
__device__ int upper_index(const int64_t* off, int n, int64_t x)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Image of every global tile, merge group and k_seam workgroup of a batch.
__global__ __launch_bounds__(256) void k_index(BatchArgs b)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < b.ntiles) {
        b.tile_img[x] = upper_index(b.tile_off, b.n, x);
    } else if (x < b.ntiles + b.ngroups) {
        b.group_img[x - b.ntiles] = upper_index(b.group_off, b.n, x - b.ntiles);
    } else if (x < b.ntiles + b.ngroups + b.nseamwg) {
        const int64_t w = x - b.ntiles - b.ngroups;
        b.seam_img[w] = upper_index(b.seam_off, b.n, w);
    }
}

// ---------------------------------------------------------------------------
// k_local
// ---------------------------------------------------------------------------

// Initialisation (Section 3.1.1): sixteen pixels of a tile row, four threads
// per row.  The bytes come from the aligned 16-byte blocks that hold them:
// one block when the row segment is aligned (rows of an image with an
// aligned base and pitch), else two, and the foreground mask is shifted into
// place.  A block is loaded only when it holds a byte of the segment, so it
// lies in the same memory page as image bytes (blocks never cross a page);
// its other bytes are masked off, as are pixels past the image edge.  The
// raw blocks are returned so that the loads of the next tile can be in
// flight while the current one is labelled.
struct Chunk {
    uint4 lo, hi;   // the aligned blocks
    uint32_t off;   // byte of the segment's first pixel in lo
    uint32_t n;     // pixels of the segment inside the image (0 .. 16)
};
// n (1 .. 16) pixels from src, through the aligned blocks that hold them.
__device__ __forceinline__ Chunk fetch_segment(const uint8_t* src, uint32_t n)
{
    Chunk k;
    k.hi = make_uint4(0u, 0u, 0u, 0u);
    k.n = n;
    k.off = (uint32_t)((uintptr_t)src & 15u);
    const uint8_t* blk = src - k.off;
    k.lo = ld_global16(blk);
    if (k.off + k.n > 16u) k.hi = ld_global16(blk + 16);
    return k;
}
__device__ __forceinline__ Chunk fetch_chunk(const ImageArgs& a, int t, int c)
{
    const int gx = (t % a.ntx) * TW + 16 * (c & 3);
    const int gy = (t / a.ntx) * TILE_ROWS + (c >> 2);
    Chunk k;
    k.lo = k.hi = make_uint4(0u, 0u, 0u, 0u);
    k.off = k.n = 0u;
    if (gy < a.H && gx < a.W)
        k = fetch_segment(a.img + (int64_t)gy * a.pitch + gx,
                          (uint32_t)(a.W - gx < 16 ? a.W - gx : 16));
    return k;
}

// Foreground bits of sixteen bytes (bit i = byte i != 0).
__device__ __forceinline__ uint32_t nz16(uint4 v)
{
    return nz_nibble(v.x) | (nz_nibble(v.y) << 4) | (nz_nibble(v.z) << 8) | (nz_nibble(v.w) << 12);
}

// Foreground bits of the chunk's pixels (bit i = pixel i).
__device__ __forceinline__ uint32_t chunk_mask(const Chunk& k)
{
    uint32_t m = nz16(k.lo);
    if (k.off + k.n > 16u) m |= nz16(k.hi) << 16;
    return (m >> k.off) & ((1u << k.n) - 1u);
}

// The local step on tile t; sh.u.h holds its foreground bits on entry.
template <int D>
__device__ void local_tile(const ImageArgs& a, const Workspace& ws, LocalShared<D>& sh, int t,
                           int tid)
{
    using G = Geo<D>;
    const int tx = t % a.ntx, ty = t / a.ntx;
    const int gx0 = tx * TW, gy0 = ty * TILE_ROWS;

    const int64_t T = a.tbase + t;  // global tile index (workspace)
    if (tid < TILE_ROWS) {
        const uint64_t m = sh.u.w[tid];
        sh.M[tid] = m;
        ws.bits[T * TILE_ROWS + tid] = m;
    }
    __syncthreads();
    build_lines<D>(sh, tid);

    // Two passes walk the bits of a column window (the runs that start in it,
    // and its edges to the line above); the union-find passes walk dense run
    // ids (thread tid takes ids tid, tid + NT, ...) so that every lane has
    // work.
    const uint32_t R = sh.base[G::NL];
    if (tid == 0) ws.nruns[T] = R;
    const int wl = tid / G::TPL;              // this thread's line
    const int wlo = (tid % G::TPL) * G::WIN;  // and first column of its window
    constexpr uint32_t WMASK = (1u << G::WIN) - 1u;
    // Row connection (Section 3.1.2): every run is one provisional label,
    // keyed by its smallest pixel (the paper's provisional label =
    // position).  Each thread takes the runs that start in its window.
    {
        const uint64_t ls = sh.LS[wl], lm = sh.LM[wl];
        uint32_t id = sh.base[wl] + popc64(ls & ~(~0ull << wlo));
        for (uint32_t r = (uint32_t)(ls >> wlo) & WMASK; r; r &= r - 1u, ++id) {
            const int s0 = __builtin_ctz(r) + wlo;
            uint32_t key;
            if (!D) {
                key = (uint32_t)(wl * TW + s0);
            } else {
                // first top-row pixel of the strip run, else its bottom-row start
                const int len = ctz64_or64(~(lm >> s0));
                const int tf = ctz64_or64(sh.M[2 * wl] >> s0);
                key = tf < len ? (uint32_t)(2 * wl * TW + s0 + tf)
                               : (uint32_t)((2 * wl + 1) * TW + s0);
            }
            sh.P[id] = pk(key, id);
        }
    }
    if (tid == 0) sh.nedges = 0u;
    __syncthreads();

    // Refinement edges: every adjacency between a line and the one above that
    // the coarse links do not already hold.  They are enumerated bitwise from
    // the two facing rows (lower = this line's top row T, upper = the line
    // above's bottom row B); an edge is dropped when an edge further left
    // joins the same two runs (consecutive foreground pixels of one row lie
    // in one run), which leaves at most one edge per column:
    //   4-connectivity: starts of the stretches of T & B (edge (i, i));
    //   8-connectivity: (i,i)   where neither side continues from i-1,
    //                   (i-1,i) where B does not continue from i-1,
    //                   (i,i-1) where T does not continue from i-1.
    // Each run's first surviving edge, ordered by lower then upper pixel,
    // joins it to the run holding its leftmost upper neighbour: that is its
    // coarse link, so it is masked out.  The first edge position of every
    // run is found for all runs at once: adding the run starts to the
    // columns without an edge carries each start up to its first edge.
    uint32_t cw = 0, c1w = 0, c2w = 0;  // edges in this thread's window (bit j = column wlo + j)
    uint32_t lslw = 0, lsuw = 0;        // run starts of the two lines in the window
    uint32_t prel = 0, preu = 0;        // runs of the two lines starting left of the window
    if (wl > 0) {
        const int l = wl;
        const uint64_t T = top_row<D>(sh, l), B = bottom_row<D>(sh, l - 1);
        const uint64_t lm = sh.LM[l], lsl = sh.LS[l], lsu = sh.LS[l - 1];
        uint64_t c0, c1 = 0, c2 = 0, e0, e2 = 0, first;
        if (!D) {
            const uint64_t o = T & B;
            e0 = o & ~(o << 1);
            const uint64_t q = lm & ~e0;
            first = (lsl & e0) | ((q + (lsl & q)) & e0);
            c0 = e0 & ~first;
        } else {
            e0 = T & B & ~(T << 1) & ~(B << 1);
            const uint64_t e1 = (T << 1) & B & ~(B << 1);  // index = upper pixel
            e2 = T & (B << 1) & ~(T << 1);
            const uint64_t x = e0 | e2 | (e1 >> 1);         // lower pixels with an edge
            const uint64_t q = lm & ~x;
            first = (lsl & x) | ((q + (lsl & q)) & x);
            c0 = e0 & ~(first & e0);
            c2 = e2 & ~(first & e2);
            c1 = e1 & ~((first & ~e0 & ~e2) << 1);
        }
        cw = (uint32_t)((c0 | c1 | c2) >> wlo) & WMASK;
        c1w = (uint32_t)(c1 >> wlo) & WMASK;
        c2w = (uint32_t)(c2 >> wlo) & WMASK;
        lslw = (uint32_t)(lsl >> wlo) & WMASK;
        lsuw = (uint32_t)(lsu >> wlo) & WMASK;
        const uint64_t left = ~(~0ull << wlo);
        prel = sh.base[l] + popc64(lsl & left) - 1u;
        preu = sh.base[l - 1] + popc64(lsu & left) - 1u;
        // Column connection (coarse, Section 3.1.2): a run's first edge
        // joins it to the run holding its leftmost neighbour in the line
        // above; the run takes that run's current entry (its label or, if
        // that run was linked meanwhile, an ancestor with a smaller key).
        // Every run has at most one first edge, so every entry still has
        // one writer.
        for (uint32_t f = (uint32_t)(first >> wlo) & WMASK; f; f &= f - 1u) {
            const int j = __builtin_ctz(f), p = wlo + j;
            int u = p;  // upper pixel: same column, one left (i, i-1) or one right (i-1, i)
            if (D && !((e0 >> p) & 1ull)) u = ((e2 >> p) & 1ull) ? p - 1 : p + 1;
            const uint32_t lo = prel + __builtin_popcount(lslw & ((2u << j) - 1u));
            const uint32_t up = sh.base[l - 1] + popc64(lsu & upto(u)) - 1u;
            lds_st(sh.P + lo, lds_ld(sh.P + up));
        }
    }
    // At most one edge per column, so the edge count of the window is a
    // popcount; edges go to the list in any order.
    if (cw) {
        uint32_t off = atomicAdd(&sh.nedges, (uint32_t)__builtin_popcount(cw));
        for (uint32_t r = cw; r; r &= r - 1u, ++off) {
            const int j = __builtin_ctz(r);
            const uint32_t bit = 1u << j;
            // run holding the lower / upper pixel: runs starting at or left of it
            const int jl = (c1w & bit) ? j : j + 1;  // (i-1, i): lower pixel one left
            const int ju = (c2w & bit) ? j : j + 1;  // (i, i-1): upper pixel one left
            sh.u.EL[off] = (prel + __builtin_popcount(lslw & ((1u << jl) - 1u))) |
                           ((preu + __builtin_popcount(lsuw & ((1u << ju) - 1u))) << 16);
        }
    }
    __syncthreads();
    const uint32_t E = sh.nedges;

    // Label-equivalence unification: every run points at its current root
    // (the coarse links form chains down the lines), so that the
    // refinement's finds start from short paths.  The store is an atomic
    // min: a merge of the refinement may already have linked that run.
    for (uint32_t id = tid; id < R; id += NT)
        __hip_atomic_fetch_min(sh.P + id, pfind(sh.P, id), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);

    // Refinement: the paper's merge on every listed edge.
    for (uint32_t k = tid; k < E; k += NT) {
        const uint32_t ed = sh.u.EL[k];
        punion(sh.P, ed & 0xffffu, ed >> 16);
    }
    __syncthreads();

    // Unification again: every run points straight at its final local root.
    for (uint32_t id = tid; id < R; id += NT) lds_st(sh.P + id, pfind(sh.P, id));
    __syncthreads();

    // Border slots (slots tid, tid + NT, ...): local root of each border pixel.
    bool fg[SPT];
    uint32_t root[SPT], rkey[SPT];
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
        const int s = tid + k * NT;
        fg[k] = false;
        root[k] = rkey[k] = 0;
        if (s < NSLOTS) {
            int sx, sy;
            slot_xy(s, sx, sy);
            fg[k] = (sh.M[sy] >> sx) & 1ull;
            if (fg[k]) {
                const uint32_t v = lds_ld(sh.P + run_id<D>(sh, D ? sy >> 1 : sy, sx));
                root[k] = pk_id(v);
                rkey[k] = pk_key(v);
            }
        }
    }
    __syncthreads();
    // Elect the smallest slot of each border component as its representative
    // (an atomic max on the root entry, which is no longer needed as a parent).
#pragma unroll
    for (int k = 0; k < SPT; ++k)
        if (fg[k])
            __hip_atomic_fetch_max(sh.P + root[k], REP_TAG | (uint32_t)(NSLOTS - 1 - (tid + k * NT)),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __syncthreads();

    // ID conversion (Section 3.1.4): the representative's forest node carries
    // the raster position of the component's smallest pixel.
    const int64_t sbase = T * NSLOTS;
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
        const int s = tid + k * NT;
        if (s >= NSLOTS) continue;
        int32_t node = -1;
        if (fg[k]) {
            const int rep = NSLOTS - 1 - (int)pk_id(lds_ld(sh.P + root[k]));
            node = (int32_t)(sbase + rep);
            if (rep == s) {
                const uint32_t gkey = (uint32_t)((int64_t)(gy0 + (int)(rkey[k] / TW)) * a.W +
                                                 gx0 + (int)(rkey[k] % TW));
                ws.forest[node] = ((uint64_t)gkey << 32) | (uint32_t)node;
            }
        }
        ws.slots[sbase + s] = node;
    }

    // Run table: interior components store their root's tile key; border
    // components store their representative slot.
    uint16_t* rt = ws.runtab + T * RUNTAB_PER_TILE;
    for (uint32_t id = tid; id < R; id += NT) {
        const uint32_t v = lds_ld(sh.P + id);
        uint16_t ent;
        if (v & REP_TAG) {
            ent = (uint16_t)(RT_BORDER | (NSLOTS - 1 - pk_id(v)));
        } else {
            const uint32_t w = pk_id(v) == id ? v : lds_ld(sh.P + pk_id(v));
            ent = (w & REP_TAG) ? (uint16_t)(RT_BORDER | (NSLOTS - 1 - pk_id(w)))
                                : (uint16_t)pk_key(v);
        }
        rt[id] = ent;
    }
}

// Each workgroup labels tiles blockIdx.x, +gridDim.x, ... and loads the next
// tile's bytes while labelling the current one, so that with a grid smaller
// than the tile count (tile_grid) the load latency overlaps the LDS work.
static_assert(TILE_ROWS * 4 == NT, "one sixteen-byte chunk per thread");
template <int D>
__global__ __launch_bounds__(NT) void k_local(BatchArgs b, Workspace ws)
{
    __shared__ LocalShared<D> sh;
    const int tid = threadIdx.x;
    int64_t T = blockIdx.x;
    if (T >= b.ntiles) return;
    ImageArgs a = batch_image(b, tile_image(b, T));
    int t = (int)(T - a.tbase);
    Chunk raw = fetch_chunk(a, t, tid);
    for (; T < b.ntiles; T += gridDim.x) {
        sh.u.h[tid] = (uint16_t)chunk_mask(raw);
        const int64_t TN = T + gridDim.x;
        ImageArgs an = a;
        int tn = 0;
        if (TN < b.ntiles) {
            an = batch_image(b, tile_image(b, TN));
            tn = (int)(TN - an.tbase);
            raw = fetch_chunk(an, tn, tid);
        }
        __syncthreads();
        local_tile<D>(a, ws, sh, t, tid);
        __syncthreads();
        a = an;
        t = tn;
    }
}

// ---------------------------------------------------------------------------
// block merge (Section 3.2), in two levels
// ---------------------------------------------------------------------------
//
// The paper merges blocks by inspecting only the pixels on block borders
// (Eq. 1-2: the candidates shrink by the block width along each axis).  The
// same boundary analysis runs here at two scales:
//   k_block  one workgroup per group of BX x BY tiles unites, in LDS, the
//            border components of its tiles across the seams inside the
//            group, then writes every component's group root into the HBM
//            forest (plain stores: no other workgroup touches those nodes);
//   k_seam   the seams between groups, united in the HBM forest with atomics.
//
// Along a seam, A[k] / B[k] are the node ids of the pixels at seam index k on
// the first / second side (-1 = background).  Work item i owns the edges
// whose larger index is i: (i, i) and, with diagonals, (i-1, i) and (i, i-1).
// An edge is skipped when an edge of smaller index sum joins the same two
// nodes; by induction on the index sum every node pair that is adjacent
// somewhere along the seam is still united, and a foreground stretch along a
// seam costs one union instead of one per pixel.  For 8-connectivity:
//   (i, i)   is covered by (i-1, i) when A[i-1] == A[i], by (i, i-1) when
//            B[i-1] == B[i];
//   (i-1, i) is covered by (i-1, i-1) when B[i-1] == B[i];
//   (i, i-1) is covered by (i-1, i-1) when A[i-1] == A[i].
// For 4-connectivity only (i, i) exists, covered by (i-1, i-1) when both
// sides repeat.  Node ids are unique across tiles, so a covering edge always
// joins the same two tiles as the edge it covers.

// tiles per merge group: a group is 256 x 256 pixels for every tile height
constexpr int BX = 4, BY = 256 / TILE_ROWS;
constexpr int BPX = BX * TW, BPY = BY * TILE_ROWS;  // group size in pixels
constexpr int BN = BX * BY * NSLOTS;             // border slots per group
static_assert(BPX * BPY <= 65536 && BN <= 65536, "16-bit group keys and ids");

// q = v / d, r = v % d for a runtime divisor, from magic = floor(2^32 / d)
// (0xffffffff for d = 1): the estimate is low by at most two.
__device__ __forceinline__ void divmod_w(uint32_t v, uint32_t d, uint32_t magic, uint32_t& q,
                                         uint32_t& r)
{
    q = __umulhi(v, magic);
    r = v - q * d;
    while (r >= d) { ++q; r -= d; }
}

enum { E_II = 1, E_PI = 2, E_IP = 4 };  // edges (i,i), (i-1,i), (i,i-1)
constexpr int SEAM_HASH = 512;           // pair table per k_seam workgroup (power of two)

// Which of the three edges at seam index i survive the deduplication above.
template <int D>
__device__ __forceinline__ int seam_edges(int32_t ap, int32_t ac, int32_t bp, int32_t bc)
{
    const bool ra = ap == ac, rb = bp == bc;
    int m = 0;
    if (D == 0) {
        if (ac >= 0 && bc >= 0 && !(ra && rb)) m |= E_II;
    } else {
        if (ac >= 0 && bc >= 0 && !ra && !rb) m |= E_II;
        if (ap >= 0 && bc >= 0 && !rb) m |= E_PI;
        if (ac >= 0 && bp >= 0 && !ra) m |= E_IP;
    }
    return m;
}

// Node ids at seam index i-1 and i of a horizontal seam (tile rows k-1 | k)
// at image column x, or of a vertical seam (tile columns j-1 | j) at image
// row y (index i = row within the tile row; i-1 < 0 gives -1).
struct SeamNodes {
    int32_t ap, ac, bp, bc;
};

__device__ __forceinline__ SeamNodes hseam_nodes(const ImageArgs& a, const int32_t* slots, int k,
                                                 int x)
{
    const int64_t top = a.tbase + (int64_t)(k - 1) * a.ntx, bot = a.tbase + (int64_t)k * a.ntx;
    SeamNodes n;
    n.ac = slots[(top + x / TW) * NSLOTS + TW + x % TW];
    n.bc = slots[(bot + x / TW) * NSLOTS + x % TW];
    n.ap = n.bp = -1;
    if (x > 0) {
        const int xp = x - 1;
        n.ap = slots[(top + xp / TW) * NSLOTS + TW + xp % TW];
        n.bp = slots[(bot + xp / TW) * NSLOTS + xp % TW];
    }
    return n;
}

__device__ __forceinline__ SeamNodes vseam_nodes(const ImageArgs& a, const int32_t* slots, int j,
                                                 int y)
{
    const int k = y / TILE_ROWS, yl = y - k * TILE_ROWS;
    const int32_t* left =
        slots + (a.tbase + (int64_t)k * a.ntx + j - 1) * NSLOTS + 2 * TW + TILE_ROWS;
    const int32_t* right = slots + (a.tbase + (int64_t)k * a.ntx + j) * NSLOTS + 2 * TW;
    SeamNodes n;
    n.ac = left[yl];
    n.bc = right[yl];
    n.ap = yl > 0 ? left[yl - 1] : -1;
    n.bp = yl > 0 ? right[yl - 1] : -1;
    return n;
}

constexpr int NTB = 1024;  // threads per merge-group workgroup

template <int D>
__global__ __launch_bounds__(NTB) void k_block(BatchArgs b, Workspace ws)
{
    __shared__ uint32_t P[BN];           // (group key << 16) | group index
    __shared__ int32_t S[BN];            // the group's slot tables (node ids, -1 = bg)
    __shared__ uint32_t isrep[BN / 32];  // group indices that are forest nodes
    const int tid = threadIdx.x;
    const int img = b.n == 1 ? 0 : ld_uniform(b.group_img + blockIdx.x);
    const ImageArgs a = batch_image(b, img);
    const int g = (int)(blockIdx.x - (b.n == 1 ? 0 : ld_uniform(b.group_off + img)));
    const int nbx = (a.ntx + BX - 1) / BX;
    const int tx0 = (g % nbx) * BX, ty0 = (g / nbx) * BY;
    const int px0 = tx0 * TW, py0 = ty0 * TILE_ROWS;

    // The group's slot tables and forest entries: all loads are issued before
    // any is used (one round trip instead of one per pass).  Tiles past the
    // image edge read the group's first tile and count as background.  Nodes
    // are keyed by the position of their smallest pixel relative to the group
    // origin (same order as raster position).
    constexpr int PER = BN / NTB;
    static_assert(BN % NTB == 0 && NTB % 64 == 0, "whole wavefronts per pass");
    int32_t nd[PER];
    uint32_t fk[PER];
    int64_t ix[PER];
    bool in[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int li = tid + k * NTB;
        const int ti = li / NSLOTS, sl = li % NSLOTS;
        const int tx = tx0 + ti % BX, ty = ty0 + ti / BX;
        in[k] = tx < a.ntx && ty < a.nty;
        ix[k] = (a.tbase + (int64_t)(in[k] ? ty : ty0) * a.ntx + (in[k] ? tx : tx0)) * NSLOTS + sl;
        nd[k] = ws.slots[ix[k]];
        fk[k] = (uint32_t)(ws.forest[ix[k]] >> 32);
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int li = tid + k * NTB;
        const int32_t node = in[k] ? nd[k] : -1;
        const bool rep = node == (int32_t)ix[k];
        // every entry gets a value; only those of representatives are read
        uint32_t gy, gx;
        divmod_w(fk[k], (uint32_t)a.W, a.wmagic, gy, gx);
        P[li] = pk((gy - py0) * BPX + (gx - px0), li);
        const uint64_t bal = __ballot(rep);
        if ((tid & 63) == 0) {
            isrep[li >> 5] = (uint32_t)bal;
            isrep[(li >> 5) + 1] = (uint32_t)(bal >> 32);
        }
        S[li] = node;
    }
    __syncthreads();

    // Node id -> group index, for a node of the group tile (txl, tyl).
    auto gidx = [&](int32_t node, int txl, int tyl) {
        const int ti = tyl * BX + txl;
        const int64_t base = (a.tbase + (int64_t)(ty0 + tyl) * a.ntx + tx0 + txl) * NSLOTS;
        return (uint32_t)(ti * NSLOTS + (int)(node - base));
    };
    // seams between tile columns inside the group
    for (int it = tid; it < (BX - 1) * BPY; it += NTB) {
        const int j = it / BPY + 1, yy = it % BPY;
        if (tx0 + j >= a.ntx || py0 + yy >= a.H) continue;
        const int tyl = yy / TILE_ROWS, yl = yy % TILE_ROWS;
        const int32_t* L = S + (tyl * BX + j - 1) * NSLOTS + 2 * TW + TILE_ROWS;
        const int32_t* Rr = S + (tyl * BX + j) * NSLOTS + 2 * TW;
        const int32_t ac = L[yl], bc = Rr[yl];
        const int32_t ap = yl > 0 ? L[yl - 1] : -1, bp = yl > 0 ? Rr[yl - 1] : -1;
        const int m = seam_edges<D>(ap, ac, bp, bc);
        if (m & E_II) punion(P, gidx(ac, j - 1, tyl), gidx(bc, j, tyl));
        if (m & E_PI) punion(P, gidx(ap, j - 1, tyl), gidx(bc, j, tyl));
        if (m & E_IP) punion(P, gidx(ac, j - 1, tyl), gidx(bp, j, tyl));
    }
    // seams between tile rows inside the group; diagonal edges that reach the
    // group to the left belong to k_seam
    for (int it = tid; it < (BY - 1) * BPX; it += NTB) {
        const int k = it / BPX + 1, xx = it % BPX;
        if (ty0 + k >= a.nty || px0 + xx >= a.W) continue;
        const int txl = xx / TW, xl = xx % TW;
        const int32_t* A = S + ((k - 1) * BX + txl) * NSLOTS + TW;  // bottom row of the upper tile
        const int32_t* B = S + (k * BX + txl) * NSLOTS;             // top row of the lower tile
        const int32_t ac = A[xl], bc = B[xl];
        int32_t ap = -1, bp = -1;
        int txp = txl;
        if (xx > 0) {
            txp = (xx - 1) / TW;
            const int xp = (xx - 1) % TW;
            ap = S[((k - 1) * BX + txp) * NSLOTS + TW + xp];
            bp = S[(k * BX + txp) * NSLOTS + xp];
        }
        const int m = seam_edges<D>(ap, ac, bp, bc);
        if (m & E_II) punion(P, gidx(ac, txl, k - 1), gidx(bc, txl, k));
        if (m & E_PI) punion(P, gidx(ap, txp, k - 1), gidx(bc, txl, k));
        if (m & E_IP) punion(P, gidx(ac, txl, k - 1), gidx(bp, txp, k));
    }
    __syncthreads();

    // Every node of the group now points at its group root in the forest, and
    // the border slots that k_seam reads (the group's outer rows and columns,
    // and the end pixels of tile rows at the group's left and right columns)
    // name that group root directly.
    for (int li = tid; li < BN; li += NTB) {
        const int ti = li / NSLOTS, sl = li % NSLOTS;
        const int txl = ti % BX, tyl = ti / BX;
        const int tx = tx0 + txl, ty = ty0 + tyl;
        if (tx >= a.ntx || ty >= a.nty) continue;
        const int64_t base = (a.tbase + (int64_t)ty * a.ntx + tx) * NSLOTS;
        auto node_of = [&](uint32_t l) {
            const int tj = (int)(l / NSLOTS);
            return (uint32_t)((a.tbase + (int64_t)(ty0 + tj / BX) * a.ntx + tx0 + tj % BX) *
                                  NSLOTS +
                              (int)(l % NSLOTS));
        };
        if ((isrep[li >> 5] >> (li & 31)) & 1u) {
            const uint32_t r = pfind(P, (uint32_t)li);
            const uint32_t rk = pk_key(r);
            const uint32_t gkey =
                (uint32_t)((int64_t)(py0 + (int)(rk / BPX)) * a.W + px0 + (int)(rk % BPX));
            ws.forest[base + sl] = ((uint64_t)gkey << 32) | node_of(pk_id(r));
        }
        const int32_t node = S[li];
        if (node < 0) continue;
        const bool top = sl < TW, bot = sl >= TW && sl < 2 * TW;
        const int xs = sl % TW;
        const bool outer = (top && tyl == 0) || (bot && tyl == BY - 1) ||
                           (sl >= 2 * TW && sl < 2 * TW + TILE_ROWS && txl == 0) ||
                           (sl >= 2 * TW + TILE_ROWS && txl == BX - 1) ||
                           ((top || bot) && ((xs == 0 && txl == 0) || (xs == TW - 1 && txl == BX - 1)));
        if (outer) {
            const uint32_t r = pfind(P, gidx(node, txl, tyl));
            ws.slots[base + sl] = (int32_t)node_of(pk_id(r));
        }
    }
}

// Seams between merge groups, united in the HBM forest.  Work items: every
// position of the horizontal seams on group rows, of the vertical seams on
// group columns, and (8-connectivity) the two diagonal edges that cross a
// group column at each seam between tile rows inside a group.
template <int D>
__global__ __launch_bounds__(SEAM_WG) void k_seam(BatchArgs b, Workspace ws)
{
    const int img = b.n == 1 ? 0 : ld_uniform(b.seam_img + blockIdx.x);
    const ImageArgs a = batch_image(b, img);
    const int64_t wg = blockIdx.x - (b.n == 1 ? 0 : ld_uniform(b.seam_off + img));
    const int64_t gid = wg * SEAM_WG + threadIdx.x;
    const int nkh = (a.nty - 1) / BY, nkv = (a.ntx - 1) / BX;
    const int nbx = (a.ntx + BX - 1) / BX;
    const int64_t nh = (int64_t)nkh * a.W, nv = (int64_t)nkv * a.H;
    const int64_t nc = D ? (int64_t)(a.nty - 1 - nkh) * (nbx - 1) : 0;
    SeamNodes n;
    int m;
    if (gid < nh) {
        n = hseam_nodes(a, ws.slots, (int)(gid / a.W + 1) * BY, (int)(gid % a.W));
        m = seam_edges<D>(n.ap, n.ac, n.bp, n.bc);
    } else if (gid < nh + nv) {
        const int64_t g = gid - nh;
        n = vseam_nodes(a, ws.slots, (int)(g / a.H + 1) * BX, (int)(g % a.H));
        m = seam_edges<D>(n.ap, n.ac, n.bp, n.bc);
    } else if (gid < nh + nv + nc) {
        const int64_t g = gid - nh - nv;
        const int kk = (int)(g / (nbx - 1));
        const int k = kk + kk / (BY - 1) + 1;  // skip tile rows that start a group
        const int x = (int)(g % (nbx - 1) + 1) * BPX;
        n = hseam_nodes(a, ws.slots, k, x);
        m = seam_edges<D>(n.ap, n.ac, n.bp, n.bc) & (E_PI | E_IP);
    } else {
        m = 0;
        n.ap = n.ac = n.bp = n.bc = -1;
    }
    // The slots read here name group roots (k_block rewrote them); drop pairs
    // another item of this workgroup already holds: along a seam most
    // foreground stretches join the same two group roots, and one union per
    // distinct pair is enough.  A full table only costs duplicates.
    __shared__ unsigned long long seen[SEAM_HASH];
    for (int i = threadIdx.x; i < SEAM_HASH; i += blockDim.x) seen[i] = ~0ull;
    __syncthreads();
    uint64_t* F = ws.forest;
    auto unite = [&](uint32_t x, uint32_t y) {
        if (x == y) return;
        if (x > y) { uint32_t t = x; x = y; y = t; }
        const unsigned long long key = ((unsigned long long)x << 32) | y;
        uint32_t h = (x * 0x9e3779b1u) ^ (y * 0x85ebca77u);
        for (int probe = 0; probe < 8; ++probe, ++h) {
            const unsigned long long prev = atomicCAS(seen + (h & (SEAM_HASH - 1)), ~0ull, key);
            if (prev == key) return;         // already united by this workgroup
            if (prev == ~0ull) break;        // claimed a fresh entry
        }
        g_union(F, x, y);
    };
    if (m & E_II) unite((uint32_t)n.ac, (uint32_t)n.bc);
    if (m & E_PI) unite((uint32_t)n.ap, (uint32_t)n.bc);
    if (m & E_IP) unite((uint32_t)n.ac, (uint32_t)n.bp);
}

// ---------------------------------------------------------------------------
// k_final
// ---------------------------------------------------------------------------

template <int D>
struct FinalShared : Lines<D> {
    uint64_t rb[TILE_ROWS];                // with statistics: smallest pixels of components
    int32_t lab[Geo<D>::MAXR];             // final label of each run
    int32_t fin[NSLOTS];                   // final label of the component at each border slot
    alignas(16) uint16_t ent[RUNTAB_PER_TILE];  // the tile's run table
};
static_assert(RUNTAB_PER_TILE == 8 * NT, "one 16-byte run-table load per thread");

struct FinalFetch {
    int32_t node[SPT];
    uint32_t nruns;
    uint64_t m;
};

// Loads of one tile for k_final that depend on no other: the border slots of
// this thread (tid, tid + NT, ...), the row masks and the run count (which
// sizes the run-table load issued when the tile's turn comes).
__device__ __forceinline__ FinalFetch final_fetch(const Workspace& ws, int64_t T, int tid)
{
    FinalFetch f;
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
        const int s = tid + k * NT;
        f.node[k] = s < NSLOTS ? ws.slots[T * NSLOTS + s] : -1;
    }
    f.nruns = ws.nruns[T];
    f.m = tid < TILE_ROWS ? ws.bits[T * TILE_ROWS + tid] : 0ull;
    return f;
}

// Update of the global label map (Section 3.3) for global tile T.  Each
// border component takes 1 + the key of its global root, every other
// component 1 + the raster position of its local root; each label is
// written once.  With LOCAL_ONLY the forest is read before any merge (every
// tile labelled as an image).
template <int D, bool LOCAL_ONLY, bool STATS>
__device__ void final_tile(const BatchArgs& b, const Workspace& ws, const StatsWs& st,
                           FinalShared<D>& sh, int64_t T, const FinalFetch& f, int tid)
{
    const ImageArgs a = batch_image(b, tile_image(b, T));
    const int t = (int)(T - a.tbase);
    const int tx = t % a.ntx, ty = t / a.ntx;
    const int gx0 = tx * TW, gy0 = ty * TILE_ROWS;

    // The run table (only the chunks holding the tile's runs, eight entries
    // per thread) and the first forest hop are issued before the line set-up,
    // so their latency overlaps it.
    uint4 ent = make_uint4(0u, 0u, 0u, 0u);
    if (8u * tid < f.nruns)
        ent = reinterpret_cast<const uint4*>(ws.runtab + T * RUNTAB_PER_TILE)[tid];
    uint64_t v[SPT];
#pragma unroll
    for (int k = 0; k < SPT; ++k) v[k] = f.node[k] >= 0 ? ws.forest[f.node[k]] : 0;
    if (tid < TILE_ROWS) {
        sh.M[tid] = f.m;
        if (STATS) sh.rb[tid] = 0ull;
    }
    __syncthreads();
    build_lines<D>(sh, tid);
    const uint32_t R = sh.base[Geo<D>::NL];
    reinterpret_cast<uint4*>(sh.ent)[tid] = ent;
    // Global root of the component at each of this thread's border slots.
    // The slot names a forest node of that component (its tile
    // representative, or the group root after the block merge); before any
    // merge the node is the root.
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
        if (f.node[k] < 0) continue;
        uint64_t vk = v[k];
        if (!LOCAL_ONLY) {
            // The merge is over, so every node's root is fixed and any
            // ancestor is a valid parent: beyond the first hop (whose node
            // the whole group's tiles share) the path is halved with plain
            // stores, which keeps later chases short on images whose merge
            // left long chains (one component snaking through many groups).
            uint32_t n = (uint32_t)f.node[k];
            bool first = true;
            while ((uint32_t)vk != n) {
                const uint32_t p = (uint32_t)vk;
                const uint64_t vp = ld_global(ws.forest + p);
                if (!first && (uint32_t)vp != p) st_global(ws.forest + n, vp);
                first = false;
                n = p;
                vk = vp;
            }
        }
        sh.fin[tid + k * NT] = (int32_t)((uint32_t)(vk >> 32) + 1u) + a.lbase;
        // with statistics, every foreground border slot publishes its
        // component's label; the statistics pass reads it at the component's
        // representative slot (the slot itself may name another node: the
        // block merge rewrites outer slots to group roots)
        if (STATS) st.fin[T * NSLOTS + tid + k * NT] = sh.fin[tid + k * NT];
    }
    __syncthreads();
    for (uint32_t id = tid; id < R; id += NT) {
        const uint32_t e = sh.ent[id];
        // border component: its global root; otherwise ID conversion of the
        // interior component's local root
        sh.lab[id] = (e & RT_BORDER)
                         ? sh.fin[e & 0x7fff]
                         : (int32_t)((int64_t)(gy0 + (int)(e / TW)) * a.W + gx0 + (int)(e % TW) + 1 +
                                     a.lbase);
    }
    __syncthreads();

    // With statistics: mark the smallest pixel of every component that has
    // it in this tile (label - 1 is its raster position), and count them per
    // tile row for the numbering scan.
    if (STATS) {
        for (uint32_t id = tid; id < R; id += NT) {
            uint32_t ry, rx;
            divmod_w((uint32_t)sh.lab[id] - 1u, (uint32_t)a.W, a.wmagic, ry, rx);
            ry -= (uint32_t)gy0;
            rx -= (uint32_t)gx0;
            if (ry < (uint32_t)TILE_ROWS && rx < (uint32_t)TW)
                atomicOr(reinterpret_cast<unsigned long long*>(sh.rb + ry), 1ull << rx);
        }
        __syncthreads();
        if (tid < TILE_ROWS) {
            const uint64_t rb = sh.rb[tid];
            st.rootbits[T * TILE_ROWS + tid] = rb;
            st.seg[(int64_t)(ty * TILE_ROWS + tid) * a.ntx + tx] = popc64(rb);
        }
    }

    // write the labels: 16 threads per tile row, 4 pixels per thread
    const int xmax = a.W - gx0;  // pixels of this tile inside the image
    if (a.vec_out && xmax >= TW) {
        // whole aligned rows: four consecutive pixels per thread, one
        // 16-byte store
        for (int c = tid; c < TILE_ROWS * 16; c += NT) {
            const int r = c >> 4, x0 = (c & 15) * 4;
            const int gy = gy0 + r;
            if (gy >= a.H) continue;
            const int l = D ? r >> 1 : r;
            const uint64_t ls = sh.LS[l];
            const uint32_t m4 = (uint32_t)(sh.M[r] >> x0) & 15u;
            const uint32_t s4 = (uint32_t)(ls >> x0) & 15u;
            uint32_t cnt = sh.base[l] + popc64(ls & ~(~0ull << x0));  // runs starting left of x0
            int32_t o[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                cnt += (s4 >> k) & 1u;
                // a foreground pixel has its run start at or left of it, so cnt >= 1
                o[k] = ((m4 >> k) & 1u) ? sh.lab[cnt ? cnt - 1 : 0] : 0;
            }
            st_global16(a.labels + (int64_t)gy * a.W + gx0 + x0, o[0], o[1], o[2], o[3]);
        }
    } else {
        // rows not 16-byte aligned, or cut by the image edge: pixels
        // x, x + 16, x + 32, x + 48 per thread, so that each store
        // instruction writes sixteen consecutive labels of a row
        for (int c = tid; c < TILE_ROWS * 16; c += NT) {
            const int r = c >> 4, x = c & 15;
            const int gy = gy0 + r;
            if (gy >= a.H) continue;
            const int l = D ? r >> 1 : r;
            const uint64_t m = sh.M[r];
            int32_t* row = a.labels + (int64_t)gy * a.W + gx0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int xk = x + 16 * k;
                if (xk < xmax)
                    st_global(row + xk, ((m >> xk) & 1ull) ? sh.lab[run_id<D>(sh, l, xk)] : 0);
            }
        }
    }
}

// Persistent over tiles like k_local: each workgroup takes tiles blockIdx.x,
// + gridDim.x, ... and issues the next tile's loads before labelling the
// current one.
template <int D, bool LOCAL_ONLY, bool STATS>
__global__ __launch_bounds__(NT) void k_final(BatchArgs b, Workspace ws, StatsWs st)
{
    __shared__ FinalShared<D> sh;
    const int tid = threadIdx.x;
    int64_t T = blockIdx.x;
    if (T >= b.ntiles) return;
    FinalFetch next = final_fetch(ws, T, tid);
    for (; T < b.ntiles; T += gridDim.x) {
        const FinalFetch cur = next;
        if (T + gridDim.x < b.ntiles) next = final_fetch(ws, T + gridDim.x, tid);
        final_tile<D, LOCAL_ONLY, STATS>(b, ws, st, sh, T, cur, tid);
        __syncthreads();
    }
}

// The statistics, ablation, volume and copy kernels are built only with the
// built-in tile height (their host entry points always use it).
#if CCL_TILE_ROWS == 64
static_assert(NSLOTS == NT, "one border slot per thread in the statistics and ablation kernels");

// ---------------------------------------------------------------------------
// per-component statistics
// ---------------------------------------------------------------------------

// Inclusive scan of v over the workgroup (SCAN_T threads); also returns the
// workgroup total.  `wsum` holds SCAN_T / 64 words of LDS.
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t* wsum, uint32_t& total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(inc, off, 64);
        if (lane >= off) inc += o;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        uint32_t w = lane < SCAN_T / 64 ? wsum[lane] : 0u;
#pragma unroll
        for (int off = 1; off < SCAN_T / 64; off <<= 1) {
            const uint32_t o = __shfl_up(w, off, 64);
            if (lane >= off) w += o;
        }
        if (lane < SCAN_T / 64) wsum[lane] = w;
    }
    __syncthreads();
    total = wsum[SCAN_T / 64 - 1];
    const uint32_t r = inc + (wave > 0 ? wsum[wave - 1] : 0u);
    __syncthreads();  // wsum may be reused by the caller
    return r;
}

// First scan level: each block of SCAN_BLK segment counts becomes its
// exclusive scan within the block; the block totals go to bsum.
__global__ __launch_bounds__(SCAN_T) void k_scan1(StatsWs st)
{
    __shared__ uint32_t wsum[SCAN_T / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_BLK + 4 * (int64_t)threadIdx.x;
    uint32_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = base + k < st.nseg ? st.seg[base + k] : 0u;
    const uint32_t mine = v[0] + v[1] + v[2] + v[3];
    uint32_t total;
    uint32_t run = block_scan(mine, wsum, total) - mine;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (base + k < st.nseg) st.seg[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) st.bsum[blockIdx.x] = total;
}

// Second level (one workgroup): exclusive scan of the block totals, and the
// number of components.
__global__ __launch_bounds__(SCAN_T) void k_scan2(StatsWs st)
{
    __shared__ uint32_t wsum[SCAN_T / 64];
    uint64_t carry = 0;
    for (int64_t c0 = 0; c0 < st.nblk; c0 += SCAN_T) {
        const int64_t i = c0 + threadIdx.x;
        const uint32_t v = i < st.nblk ? st.bsum[i] : 0u;
        uint32_t total;
        const uint32_t inc = block_scan(v, wsum, total);
        if (i < st.nblk) st.boff[i] = (uint32_t)(carry + inc - v);
        carry += total;
    }
    if (threadIdx.x == 0) st_global(st.count, (int64_t)carry);
}

// Sum of the positions of the set bits of m.
__device__ __forceinline__ uint32_t bit_position_sum(uint64_t m)
{
    return popc64(m & 0xAAAAAAAAAAAAAAAAull) + 2u * popc64(m & 0xCCCCCCCCCCCCCCCCull) +
           4u * popc64(m & 0xF0F0F0F0F0F0F0F0ull) + 8u * popc64(m & 0xFF00FF00FF00FF00ull) +
           16u * popc64(m & 0xFFFF0000FFFF0000ull) + 32u * popc64(m & 0xFFFFFFFF00000000ull);
}

template <int D>
struct StatsShared : Lines<D> {
    uint16_t RL[Geo<D>::MAXR];
    alignas(16) uint16_t ent[RUNTAB_PER_TILE];  // the tile's run table
    // Per component part, in tile-local coordinates, three words that take
    // one atomic each per run: the packed sums (area | sum x << 13 | sum y
    // << 31; a tile's totals fit 13, 18 and 18 bits, so no field carries into
    // the next), and the masks of the columns and of the rows it touches (the
    // box is their lowest and highest set bits).
    // border components of the tile, by representative slot
    uint64_t sums[NSLOTS], cols[NSLOTS], rows[NSLOTS];
    int32_t lab[NSLOTS];
    // interior components, at the run holding their smallest pixel
    uint64_t isums[Geo<D>::MAXR], icols[Geo<D>::MAXR], irows[Geo<D>::MAXR];
    uint8_t iroot[Geo<D>::MAXR];
    // this tile's rows: number of the first component whose smallest pixel
    // lies in the row segment, and those smallest pixels
    uint32_t segnum[TILE_ROWS];
    uint64_t rootb[TILE_ROWS];
    uint32_t nrec;
};

// Adds a partial record (global coordinates) to a component's entry.
__device__ __forceinline__ void add_stats(CompStats* c, int area, int xmin, int xmax, int ymax,
                                          uint64_t sx, uint64_t sy)
{
    atomicAdd(&c->area, area);
    atomicMin(&c->x_min, xmin);
    atomicMax(&c->x_max, xmax);
    atomicMax(&c->y_max, ymax);
    atomicAdd(reinterpret_cast<unsigned long long*>(&c->sum_x), (unsigned long long)sx);
    atomicAdd(reinterpret_cast<unsigned long long*>(&c->sum_y), (unsigned long long)sy);
}

// Number of the component with label L: scanned count of its smallest
// pixel's segment plus the smallest pixels left of it in that segment.
__device__ __forceinline__ int64_t component_number(const ImageArgs& a, const StatsWs& st,
                                                    int32_t L)
{
    uint32_t ry, rx;
    divmod_w((uint32_t)L - 1u, (uint32_t)a.W, a.wmagic, ry, rx);
    const int64_t sg = (int64_t)ry * a.ntx + rx / TW;
    const int64_t rt = ((int64_t)(ry / TILE_ROWS) * a.ntx + rx / TW) * TILE_ROWS + ry % TILE_ROWS;
    return (int64_t)st.seg[sg] + st.boff[sg / SCAN_BLK] +
           popc64(st.rootbits[rt] & ((1ull << (rx % TW)) - 1ull));
}

// Number of a component whose smallest pixel is at tile position (ky, kx)
// of the tile in sh (its rows' scanned counts and smallest pixels staged).
template <typename SH>
__device__ __forceinline__ int64_t tile_number(const SH& sh, int ky, int kx)
{
    return (int64_t)sh.segnum[ky] + popc64(sh.rootb[ky] & ((1ull << kx) - 1ull));
}

// Statistics of every run of a tile.  A run's label is its border
// component's final label (published by the relabel at the component's
// representative slot) or its interior component's root position, so no
// label is read back from the label map.  Runs of interior components
// (wholly in this tile) are summed in LDS at the run holding the component's
// smallest pixel, which then writes the whole entry; runs of border
// components are summed per component in LDS and leave the tile as one
// partial record each, which k_stats_merge combines over 4 x 4 tiles before
// they reach the entries, so that a component spanning the image is not
// updated once per tile.  The run holding a border component's smallest
// pixel writes the entry's starting values (label, top row, empty sums and
// box).  Components whose smallest pixel lies in this tile are numbered
// from the tile's staged row counts; the partial records carry the label.
constexpr int ST = 1024;  // k_stats threads per tile (its LDS allows two workgroups per
                          // compute unit, so a wide workgroup keeps the unit busy)
template <int D>
__global__ __launch_bounds__(ST) void k_stats(BatchArgs b, Workspace ws, StatsWs st)
{
    __shared__ StatsShared<D> sh;
    const int tid = threadIdx.x;
    const int64_t T = blockIdx.x;
    const ImageArgs a = b.one;  // statistics are computed for a single image
    const int t = (int)T;
    const int tx = t % a.ntx, ty = t / a.ntx;
    const int gx0 = tx * TW, gy0 = ty * TILE_ROWS;

    if (tid < TILE_ROWS) {
        sh.M[tid] = ws.bits[T * TILE_ROWS + tid];
        sh.rootb[tid] = st.rootbits[T * TILE_ROWS + tid];
        const int64_t sg = (int64_t)(gy0 + tid) * a.ntx + tx;
        sh.segnum[tid] = gy0 + tid < a.H ? st.seg[sg] + st.boff[sg / SCAN_BLK] : 0u;
    }
    if (tid < NSLOTS) {
        sh.sums[tid] = sh.cols[tid] = sh.rows[tid] = 0ull;
        sh.lab[tid] = st.fin[T * NSLOTS + tid];  // used at representative slots only
    }
    // the whole run table, in the same round trip as the loads above (its
    // entries past the tile's run count are never read)
    static_assert(RUNTAB_PER_TILE % 8 == 0 && RUNTAB_PER_TILE / 8 <= ST, "one chunk per thread");
    if (tid < RUNTAB_PER_TILE / 8)
        reinterpret_cast<uint4*>(sh.ent)[tid] = ld_global16(ws.runtab + T * RUNTAB_PER_TILE + 8 * tid);
    if (tid == 0) sh.nrec = 0u;
    __syncthreads();
    build_lines<D>(sh, tid);
    if (tid < NT) list_runs<D>(sh, sh.RL, tid);
    const uint32_t R = sh.base[Geo<D>::NL];
    for (uint32_t id = tid; id < R; id += ST) {
        sh.isums[id] = sh.icols[id] = sh.irows[id] = 0ull;
        sh.iroot[id] = 0;
    }
    __syncthreads();
    for (uint32_t id = tid; id < R; id += ST) {
        const uint32_t rec = sh.RL[id];
        const int s0 = rec & 63, l = rec >> 6;
        const int e = s0 + ctz64_or64(~(sh.LM[l] >> s0)) - 1;
        uint32_t area, key, sx, sy;
        uint64_t rowm;  // rows of the tile the run's pixels lie in
        if (!D) {
            area = (uint32_t)(e - s0 + 1);
            rowm = 1ull << l;
            sx = (uint32_t)(s0 + e) * area / 2u;
            sy = (uint32_t)l * area;
            key = (uint32_t)(l * TW + s0);
        } else {
            const uint64_t span = span_mask(s0, e);
            const uint64_t top = sh.M[2 * l] & span, bot = sh.M[2 * l + 1] & span;
            const uint32_t at = popc64(top), ab = popc64(bot);
            area = at + ab;
            rowm = (top ? 1ull << (2 * l) : 0ull) | (bot ? 1ull << (2 * l + 1) : 0ull);
            sx = bit_position_sum(top) + bit_position_sum(bot);
            sy = (uint32_t)(2 * l) * at + (uint32_t)(2 * l + 1) * ab;
            key = top ? (uint32_t)(2 * l * TW + ctz64(top)) : (uint32_t)((2 * l + 1) * TW + s0);
        }
        // its first and last columns are foreground (in one of its rows)
        const uint64_t colm = span_mask(s0, e);
        const uint64_t packed = (uint64_t)area | ((uint64_t)sx << 13) | ((uint64_t)sy << 31);
        const int64_t kpos = (int64_t)(gy0 + (int)(key / TW)) * a.W + gx0 + (int)(key % TW);
        // the run's label: a border component's from the relabel (at its
        // representative slot), an interior one's from its root's tile key
        const uint32_t en = sh.ent[id];
        const bool border = (en & RT_BORDER) != 0;
        const int32_t L = border ? sh.lab[en & 0x7fff]
                                 : (int32_t)((int64_t)(gy0 + (int)(en / TW)) * a.W + gx0 +
                                             (int)(en % TW) + 1);
        if (L <= 0 || (int64_t)L > kpos + 1) {
            // a foreground pixel's label is 1 + a position at or before it;
            // anything else means the labels are wrong: poison the count so
            // the caller sees the failure instead of missing statistics
            st_global(st.count, (int64_t)CCL_STATS_INCONSISTENT);
            continue;
        }
        const bool is_root = kpos == (int64_t)L - 1;
        if (!border) {
            // the run holding the smallest pixel (tile position = the entry)
            const int ky = (int)(en / TW), kx = (int)(en % TW);
            const int rl = D ? ky >> 1 : ky;
            const uint32_t rr = sh.base[rl] + popc64(sh.LS[rl] & upto(kx)) - 1u;
            atomicAdd(&sh.isums[rr], packed);
            atomicOr(&sh.icols[rr], colm);
            atomicOr(&sh.irows[rr], rowm);
            if (is_root) sh.iroot[id] = 1;
            continue;
        }
        {
            const int rep = en & 0x7fff;
            atomicAdd(&sh.sums[rep], packed);
            atomicOr(&sh.cols[rep], colm);
            atomicOr(&sh.rows[rep], rowm);
            if (!is_root) continue;
        }
        // the component's entry starts from its label and top row; the
        // merge adds every tile's part to it
        const int64_t num = tile_number(sh, (int)(key / TW), (int)(key % TW));
        if (num >= st.capacity) continue;
        CompStats c;
        c.label = L;
        c.area = 0;
        c.x_min = INT32_MAX;
        c.y_min = (int32_t)(kpos / a.W);
        c.x_max = c.y_max = -1;
        c.sum_x = c.sum_y = 0;
        st_global(st.comps + num, c);
    }
    __syncthreads();
    // interior components: the whole entry from the run holding the smallest pixel
    for (uint32_t id = tid; id < R; id += ST) {
        if (!sh.iroot[id]) continue;
        const uint32_t rec = sh.RL[id];
        const int s0 = rec & 63, l = rec >> 6;
        // smallest pixel: the run's first foreground pixel in raster order
        int ky = l, kx = s0;
        if (D) {
            const int e = s0 + ctz64_or64(~(sh.LM[l] >> s0)) - 1;
            const uint64_t top = sh.M[2 * l] & span_mask(s0, e);
            ky = top ? 2 * l : 2 * l + 1;
            kx = top ? ctz64(top) : s0;
        }
        const int64_t kpos = (int64_t)(gy0 + ky) * a.W + gx0 + kx;
        const int32_t L = (int32_t)(kpos + 1);
        const int64_t num = tile_number(sh, ky, kx);
        if (num >= st.capacity) continue;
        const uint64_t v = sh.isums[id], cm = sh.icols[id], rm = sh.irows[id];
        const int area = (int)(v & 0x1fffu);
        CompStats c;
        c.label = L;
        c.area = area;
        c.x_min = gx0 + ctz64(cm);
        c.y_min = gy0 + ky;
        c.x_max = gx0 + msb64(cm);
        c.y_max = gy0 + msb64(rm);
        c.sum_x = (int64_t)(((v >> 13) & 0x3ffffu) + (uint64_t)area * gx0);
        c.sum_y = (int64_t)(((v >> 31) & 0x3ffffu) + (uint64_t)area * gy0);
        st_global(st.comps + num, c);
    }
    // one partial record per border component of the tile
    const uint64_t v = tid < NSLOTS ? sh.sums[tid] : 0ull;
    const int area = (int)(v & 0x1fffu);
    if (area > 0) {
        {
            StatRec r;
            r.label = sh.lab[tid];
            r.area = area;
            const uint64_t cm = sh.cols[tid], rm = sh.rows[tid];
            r.x_min = gx0 + ctz64(cm);
            r.x_max = gx0 + msb64(cm);
            r.y_min = gy0 + ctz64(rm);
            r.y_max = gy0 + msb64(rm);
            r.sum_x = (int64_t)(((v >> 13) & 0x3ffffu) + (uint64_t)area * gx0);
            r.sum_y = (int64_t)(((v >> 31) & 0x3ffffu) + (uint64_t)area * gy0);
            st.rec0[T * NSLOTS + atomicAdd(&sh.nrec, 1u)] = r;
        }
    }
    __syncthreads();
    if (tid == 0) st.cnt0[T] = sh.nrec;
}

// Merge of the tiles' partial records: workgroup (I, J) combines the
// records of tiles (4I .. 4I+3, 4J .. 4J+3) in an LDS hash table keyed by
// label, and numbers each combined record once (the tiles leave their
// records unnumbered, which spares them a round trip to the scanned counts
// per tile).  A combined record whose box stays off the region's
// inner edges (image edges do not count) is the whole component: it cannot
// reach outside without crossing them, so its fields are stored into the
// component's entry (started by the tile holding its smallest pixel, which
// wrote the label and top row).  The others are added to the entry with
// atomics, where a component's parts from several regions meet.  Records
// that find the table full go straight to the entries with atomics; then
// the workgroup stores nothing plainly, since a store could hide them.
constexpr int MERGE_T = 1024;
__global__ __launch_bounds__(MERGE_T) void k_stats_merge(StatsWs st, const StatRec* in,
                                                          const uint32_t* in_cnt, int in_cap,
                                                          int inx, int iny, int outx,
                                                          ImageArgs a)
{
    const int W = a.W, H = a.H;
    __shared__ int32_t hkey[MERGE_HT], harea[MERGE_HT], hxmin[MERGE_HT], hxmax[MERGE_HT],
        hymin[MERGE_HT], hymax[MERGE_HT];
    __shared__ unsigned long long hsx[MERGE_HT], hsy[MERGE_HT];
    __shared__ int overflow;
    const int tid = threadIdx.x;
    for (int h = tid; h < MERGE_HT; h += MERGE_T) {
        hkey[h] = -1;
        harea[h] = 0;
        hxmin[h] = hymin[h] = INT32_MAX;
        hxmax[h] = hymax[h] = -1;
        hsx[h] = hsy[h] = 0ull;
    }
    if (tid == 0) overflow = 0;
    __syncthreads();
    const int I = (int)(blockIdx.x % (unsigned)outx), J = (int)(blockIdx.x / (unsigned)outx);
    // one wavefront per tile of the region: every tile's count and records
    // are loaded at once (one round trip each, not one per tile in turn)
    constexpr int PARTS = MERGE_FAN * MERGE_FAN, TPP = MERGE_T / PARTS;  // threads per tile
    static_assert(MERGE_T % PARTS == 0 && TPP == 64, "a wavefront per tile");
    const int part = tid / TPP, pl = tid % TPP;
    const int i = I * MERGE_FAN + part % MERGE_FAN, j = J * MERGE_FAN + part / MERGE_FAN;
    const int64_t sg = (int64_t)j * inx + i;
    const uint32_t n = (i < inx && j < iny) ? ld_global(in_cnt + sg) : 0u;
    constexpr int RPT = 4;  // records loaded together per thread
    for (uint32_t k0 = 0; k0 < n; k0 += RPT * TPP) {
        StatRec rec[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const uint32_t k = k0 + pl + q * TPP;
            if (k < n) rec[q] = ld_global(in + sg * in_cap + k);
        }
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            if (k0 + pl + q * TPP >= n) continue;
            const StatRec& r = rec[q];
            uint32_t h = ((uint32_t)r.label * 0x9E3779B1u) >> (32 - 11);
            static_assert(MERGE_HT == 1 << 11, "hash width");
            bool placed = false;
            for (int probe = 0; probe < 64 && !placed; ++probe, h = (h + 1u) & (MERGE_HT - 1)) {
                const int32_t old = atomicCAS(&hkey[h], -1, r.label);
                if (old == -1 || old == r.label) {
                    atomicAdd(&harea[h], r.area);
                    atomicMin(&hxmin[h], r.x_min);
                    atomicMax(&hxmax[h], r.x_max);
                    atomicMin(&hymin[h], r.y_min);
                    atomicMax(&hymax[h], r.y_max);
                    atomicAdd(&hsx[h], (unsigned long long)r.sum_x);
                    atomicAdd(&hsy[h], (unsigned long long)r.sum_y);
                    placed = true;
                }
            }
            if (!placed) {
                overflow = 1;
                const int64_t num = component_number(a, st, r.label);
                if (num < st.capacity)
                    add_stats(st.comps + num, r.area, r.x_min, r.x_max, r.y_max,
                              (uint64_t)r.sum_x, (uint64_t)r.sum_y);
            }
        }
    }
    __syncthreads();
    // the region's inner edges
    const int span = TW * MERGE_FAN;
    const int x0 = I * span, y0 = J * span;
    const int x1 = min(x0 + span, W) - 1, y1 = min(y0 + span, H) - 1;
    const bool plain_ok = overflow == 0;
    for (int h = tid; h < MERGE_HT; h += MERGE_T) {
        const int32_t label = hkey[h];
        if (label < 0) continue;
        const int64_t num = component_number(a, st, label);
        if (num >= st.capacity) continue;
        const bool crosses = (hxmin[h] == x0 && x0 > 0) || (hxmax[h] == x1 && x1 < W - 1) ||
                             (hymin[h] == y0 && y0 > 0) || (hymax[h] == y1 && y1 < H - 1);
        CompStats* c = st.comps + num;
        if (crosses || !plain_ok) {
            add_stats(c, harea[h], hxmin[h], hxmax[h], hymax[h], hsx[h], hsy[h]);
        } else {
            st_global(&c->area, harea[h]);
            st_global(&c->x_min, hxmin[h]);
            st_global(&c->x_max, hxmax[h]);
            st_global(&c->y_max, hymax[h]);
            st_global(&c->sum_x, (int64_t)hsx[h]);
            st_global(&c->sum_y, (int64_t)hsy[h]);
        }
    }
}

__global__ void k_zero_count(int64_t* count) { st_global(count, (int64_t)0); }

// ---------------------------------------------------------------------------
// ablations of the local step (4-connectivity, the paper's setting)
// ---------------------------------------------------------------------------

// The paper's revisions of its local step (Section 4): coarse labelling along
// rows and columns (C2FL, the method), along rows only (RC2FL), along
// columns only (CC2FL), or none (NC2FL).  Row connection = a row's run of
// foreground pixels is one node; without it every foreground pixel is its
// own node.  Column connection = each node starts linked to the node holding
// the leftmost foreground pixel above it; without it every node starts as
// its own root.  Refinement then merges every adjacency the coarse structure
// does not already hold.  The products are those of k_local (the run table
// indexed by row runs), so the merge and final kernels run unchanged; with a
// counter array each tile also reports its find-loop steps and atomic merge
// attempts.  One 256-thread workgroup per tile.
enum { ABL_ROW = 1, ABL_COL = 2 };
constexpr int ABL_MAXN = TILE_ROWS * TW;          // nodes per tile, at most (pixels)
constexpr int ABL_MAXE = 2 * TILE_ROWS * TW;      // refinement edges, at most

struct AblationShared : Lines<0> {
    uint64_t NS[TILE_ROWS];       // node starts of each row
    uint32_t nbase[TILE_ROWS + 1];  // id of the first node of each row
    uint32_t P[ABL_MAXN];
    uint16_t NL[ABL_MAXN];        // node record: start column | row << 6
    uint32_t EL[ABL_MAXE];
    uint32_t nedges, cit, cat;
};

// Node of row l holding foreground column x.
__device__ __forceinline__ uint32_t abl_node(const AblationShared& sh, int l, int x)
{
    return sh.nbase[l] + popc64(sh.NS[l] & upto(x)) - 1u;
}

template <int MODE>
__global__ __launch_bounds__(NT) void k_local_ablate(BatchArgs b, Workspace ws, uint32_t* counters)
{
    constexpr bool ROW = MODE & ABL_ROW, COL = MODE & ABL_COL;
    __shared__ AblationShared sh;
    const int tid = threadIdx.x;
    const int64_t T = blockIdx.x;
    const ImageArgs a = b.one;
    const int t = (int)T;
    const int tx = t % a.ntx, ty = t / a.ntx;
    const int gx0 = tx * TW, gy0 = ty * TILE_ROWS;

    // initialisation: the tile's foreground bits
    const uint32_t m16 = chunk_mask(fetch_chunk(a, t, tid));
    uint16_t* h = reinterpret_cast<uint16_t*>(sh.M);
    h[tid] = (uint16_t)m16;
    if (tid == 0) sh.nedges = sh.cit = sh.cat = 0u;
    __syncthreads();
    if (tid < TILE_ROWS) ws.bits[T * TILE_ROWS + tid] = sh.M[tid];
    build_lines<0>(sh, tid);  // row runs (for the run table)
    if (tid == 0) ws.nruns[T] = sh.base[TILE_ROWS];
    // nodes: runs (row connection) or single pixels
    if (tid < TILE_ROWS) {
        const uint64_t m = sh.M[tid];
        const uint64_t ns = ROW ? (m & ~(m << 1)) : m;
        sh.NS[tid] = ns;
        const uint32_t c = popc64(ns);
        uint32_t inc = c;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off, 64);
            if (tid >= off) inc += o;
        }
        sh.nbase[tid] = inc - c;
        if (tid == TILE_ROWS - 1) sh.nbase[TILE_ROWS] = inc;
    }
    __syncthreads();
    const uint32_t N = sh.nbase[TILE_ROWS];
    {
        // node list, one 16-column window of a row per thread
        const int l = tid >> 2, lo = (tid & 3) * 16;
        uint32_t id = sh.nbase[l] + popc64(sh.NS[l] & ~(~0ull << lo));
        for (uint32_t r = (uint32_t)(sh.NS[l] >> lo) & 0xffffu; r; r &= r - 1u, ++id)
            sh.NL[id] = (uint16_t)((__builtin_ctz(r) + lo) | (l << 6));
    }
    __syncthreads();
    uint32_t it = 0, at = 0;
    // provisional labels; coarse column links
    for (uint32_t id = tid; id < N; id += NT) {
        const uint32_t rec = sh.NL[id];
        const int s0 = rec & 63, l = rec >> 6;
        const int e = ROW ? s0 + ctz64_or64(~(sh.M[l] >> s0)) - 1 : s0;
        uint32_t v = pk((uint32_t)(l * TW + s0), id);
        if (COL && l > 0) {
            const uint64_t contact = sh.M[l - 1] & span_mask(s0, e);
            if (contact) {
                const uint64_t below = sh.NS[l - 1] & upto(ctz64(contact));
                v = pk((uint32_t)((l - 1) * TW + msb64(below)), sh.nbase[l - 1] + popc64(below) - 1u);
            }
        }
        sh.P[id] = v;
    }
    __syncthreads();
    // label-equivalence unification
    for (uint32_t id = tid; id < N; id += NT) lds_st(sh.P + id, pfind_count(sh.P, id, it));
    // refinement edges: adjacencies the coarse structure does not hold
    {
        const int l = tid >> 2, lo = (tid & 3) * 16;
        const uint64_t m = sh.M[l], ns = sh.NS[l];
        uint64_t vert = 0, horz = 0;
        if (l > 0) {
            const uint64_t o = m & sh.M[l - 1];
            // a column continues the previous column's edge when both nodes do
            const uint64_t same = (o << 1) & o & ~ns & ~sh.NS[l - 1];
            vert = o & ~same;
            if (COL) {
                // each node's first edge (leftmost contact above) is its coarse link
                const uint64_t q = m & ~vert;
                const uint64_t first = (ns & vert) | ((q + (ns & q)) & vert);
                vert &= ~first;
            }
        }
        if (!ROW) horz = m & (m << 1);  // pixel x joins pixel x - 1
        const uint32_t wv = (uint32_t)(vert >> lo) & 0xffffu, wh = (uint32_t)(horz >> lo) & 0xffffu;
        const uint32_t n = (uint32_t)__builtin_popcount(wv) + (uint32_t)__builtin_popcount(wh);
        if (n) {
            uint32_t off = atomicAdd(&sh.nedges, n);
            for (uint32_t r = wv; r; r &= r - 1u, ++off) {
                const int x = __builtin_ctz(r) + lo;
                sh.EL[off] = abl_node(sh, l, x) | (abl_node(sh, l - 1, x) << 16);
            }
            for (uint32_t r = wh; r; r &= r - 1u, ++off) {
                const int x = __builtin_ctz(r) + lo;
                sh.EL[off] = abl_node(sh, l, x) | (abl_node(sh, l, x - 1) << 16);
            }
        }
    }
    __syncthreads();
    const uint32_t E = sh.nedges;
    for (uint32_t k = tid; k < E; k += NT) {
        const uint32_t ed = sh.EL[k];
        punion_count(sh.P, ed & 0xffffu, ed >> 16, it, at);
    }
    __syncthreads();
    for (uint32_t id = tid; id < N; id += NT) lds_st(sh.P + id, pfind_count(sh.P, id, it));
    __syncthreads();

    // border slots, representatives, forest nodes (as in k_local)
    const int s = tid;
    int sx, sy;
    slot_xy(s, sx, sy);
    const bool fg = (sh.M[sy] >> sx) & 1ull;
    uint32_t root = 0, rkey = 0;
    if (fg) {
        const uint32_t v = lds_ld(sh.P + abl_node(sh, sy, sx));
        root = pk_id(v);
        rkey = pk_key(v);
    }
    __syncthreads();
    if (fg)
        __hip_atomic_fetch_max(sh.P + root, REP_TAG | (uint32_t)(NSLOTS - 1 - s),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __syncthreads();
    const int64_t sbase = T * NSLOTS;
    {
        int32_t node = -1;
        if (fg) {
            const int rep = NSLOTS - 1 - (int)pk_id(lds_ld(sh.P + root));
            node = (int32_t)(sbase + rep);
            if (rep == s) {
                const uint32_t gkey = (uint32_t)((int64_t)(gy0 + (int)(rkey / TW)) * a.W +
                                                 gx0 + (int)(rkey % TW));
                ws.forest[node] = ((uint64_t)gkey << 32) | (uint32_t)node;
            }
        }
        ws.slots[sbase + s] = node;
    }
    // run table over row runs: the entry of the node holding each run's first pixel
    uint16_t* rtab = ws.runtab + T * RUNTAB_PER_TILE;
    const uint32_t R = sh.base[TILE_ROWS];
    for (uint32_t rid = tid; rid < R; rid += NT) {
        // row of run rid: last row whose first run id is <= rid
        int lo = 0, hi = TILE_ROWS - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sh.base[mid] <= rid) lo = mid;
            else hi = mid - 1;
        }
        uint64_t ls = sh.LS[lo];
        for (uint32_t k = rid - sh.base[lo]; k; --k) ls &= ls - 1ull;
        const uint32_t id = abl_node(sh, lo, ctz64(ls));
        const uint32_t v = lds_ld(sh.P + id);
        uint16_t ent;
        if (v & REP_TAG) {
            ent = (uint16_t)(RT_BORDER | (NSLOTS - 1 - pk_id(v)));
        } else {
            const uint32_t w = pk_id(v) == id ? v : lds_ld(sh.P + pk_id(v));
            ent = (w & REP_TAG) ? (uint16_t)(RT_BORDER | (NSLOTS - 1 - pk_id(w)))
                                : (uint16_t)pk_key(v);
        }
        rtab[rid] = ent;
    }
    if (counters) {
        atomicAdd(&sh.cit, it);
        atomicAdd(&sh.cat, at);
        __syncthreads();
        if (tid == 0) {
            counters[2 * T] = sh.cit;
            counters[2 * T + 1] = sh.cat;
        }
    }
}

// ---------------------------------------------------------------------------
// volumes
// ---------------------------------------------------------------------------

// The paper's method with a third axis (Section 3 lifted to 3-D): the
// volume is cut into bricks of 64 x VB_H x VB_D voxels (x, y, z), each
// labelled on its own in LDS (runs along x, united across the rows and
// slices of the brick), then the bricks are merged across their faces, and
// a final pass gives every voxel its component's label.
//
// k_vlocal writes every voxel's provisional label: 1 + the position of the
// smallest voxel of its component within the brick.  The label map is then
// itself the forest of the merge: every entry is 1 + an ancestor's position,
// the smallest voxel of each brick component is a root, and k_vmerge unites
// components that touch across a brick face by pointing the larger root at
// the smaller with an atomic min, so entries only decrease.  k_vfinal
// replaces each label by its root's.
constexpr int VB_W = VOL_BRICK_W, VB_H = VOL_BRICK_H, VB_D = VOL_BRICK_D;  // 64 rows of 64
constexpr int VB_ROWS = VB_H * VB_D;          // brick row r = z * VB_H + y
constexpr int VNT = 256;                      // threads per brick: 16 voxels each
constexpr int VMAXR = VB_ROWS * (VB_W / 2);   // runs per brick, at most
static_assert(VB_ROWS * 4 == VNT && VB_ROWS == 64, "one 16-voxel segment per thread");
static_assert(VB_ROWS * VB_W <= 0x8000 && VMAXR <= 0x10000, "16-bit keys and run ids");

// Entry of a node during the merge: the first two hops of a find use plain
// loads, later ones coherent loads (as g_hop for the 2-D forest).
__device__ __forceinline__ uint32_t vl_hop(const int32_t* p, int step)
{
    return (uint32_t)(step < 2 ? ld_global(p)
                               : __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) -
           1u;
}

// Root of r, given its parent p and grandparent pp (p not a root, pp != p):
// halves the path on the way, with plain stores of ancestors into entries
// read as non-roots (safe for the reasons given at g_find_from).  Entries
// always name smaller positions, so a chase ends at a root; the bound check
// only keeps a corrupted entry from reading outside the map.
__device__ uint32_t v_find_on(int32_t* lab, uint32_t r, uint32_t p, uint32_t pp, uint32_t n)
{
    for (int step = 2;; step += 2) {
        st_global(lab + r, (int32_t)(pp + 1u));
        r = pp;
        p = vl_hop(lab + r, step);
        if (p == r || p >= n) return r;
        pp = vl_hop(lab + p, step + 1);
        if (pp == p || pp >= n) return p;
    }
}

__device__ void v_union(int32_t* lab, uint32_t a, uint32_t b, uint32_t n)
{
    while (true) {
        // the first two hops of both finds, each hop's two loads issued
        // together (most finds end within them)
        uint32_t pa = vl_hop(lab + a, 0), pb = vl_hop(lab + b, 0);
        if (pa >= n) pa = a;
        if (pb >= n) pb = b;
        uint32_t qa = pa, qb = pb;
        if (pa != a) qa = vl_hop(lab + pa, 1);
        if (pb != b) qb = vl_hop(lab + pb, 1);
        if (pa != a) a = (qa == pa || qa >= n) ? pa : v_find_on(lab, a, pa, qa, n);
        if (pb != b) b = (qb == pb || qb >= n) ? pb : v_find_on(lab, b, pb, qb, n);
        if (a == b) return;
        if (a < b) { const uint32_t t = a; a = b; b = t; }
        const int32_t old = __hip_atomic_fetch_min(lab + a, (int32_t)(b + 1u), __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
        if (old == (int32_t)(a + 1u)) return;
        a = (uint32_t)old - 1u;  // a was no root (linked meanwhile, or read stale): go on from its parent
    }
}

// Brick (bx, by, bz) of workgroup / work item `i` (bricks in raster order).
struct Brick {
    int x0, y0, z0;
};
__device__ __forceinline__ Brick brick_of(const VolArgs& v, int64_t i)
{
    Brick k;
    const int64_t per_slab = (int64_t)v.nbx * v.nby;
    const int bz = (int)(i / per_slab), r = (int)(i - bz * per_slab);
    k.x0 = (r % v.nbx) * VB_W;
    k.y0 = (r / v.nbx) * VB_H;
    k.z0 = bz * VB_D;
    return k;
}

struct VolLocalShared {
    uint64_t M[VB_ROWS];          // foreground of each brick row
    uint64_t S[VB_ROWS];          // run starts of each row
    uint32_t base[VB_ROWS + 1];   // id of the first run of each row; base[64] = runs
    uint32_t P[VMAXR];            // parent of each run, packed (brick key << 16) | id
    int32_t lab[VMAXR];           // label of each run (1 + its root's volume position)
    uint16_t h[VNT];              // 16-voxel masks as loaded
};

// Dense id of the run of brick row r that contains foreground column x.
__device__ __forceinline__ uint32_t vrun(const VolLocalShared& sh, int r, int x)
{
    return sh.base[r] + popc64(sh.S[r] & upto(x)) - 1u;
}

// Unites the runs of brick row r with those of an earlier row nr that they
// touch, for the edges whose index lies in columns c0 .. c0+15.  Face
// neighbours (6-connectivity: nr is the row above or the same row of the
// slice below) touch where the rows overlap: one edge per overlapping
// stretch.  With diagonals (26-connectivity) the edges are those of two
// 8-connected rows: (i, i) where neither row continues from i-1, (i-1, i)
// where nr does not continue from i-1, (i, i-1) where r does not (at most
// one per column; for two touching runs, the edge at the larger of their
// first columns is listed).
// With `last`, an edge is dropped when the two runs' current parents are
// the pair this thread united last (after the unification most runs point at
// their root, and the runs one run touches mostly share one), and for face
// neighbours also when the two runs have the same parent (already one set;
// 512^3 volumes 1-3 % faster under 6-connectivity, while under 26 the
// early exit only split the wavefronts: Bernoulli 0.5 656 -> 694 us).
template <bool DIAG>
__device__ __forceinline__ void vlink_rows(VolLocalShared& sh, int r, int nr, int c0,
                                           uint32_t* last = nullptr)
{
    const uint64_t T = sh.M[r], B = sh.M[nr];
    auto join = [&](uint32_t a, uint32_t b) {
        if (last) {
            const uint32_t pa = pk_id(lds_ld(sh.P + a)), pb = pk_id(lds_ld(sh.P + b));
            if (!DIAG && pa == pb) return;
            const uint32_t pair = (pa << 16) | pb;
            if (pair == *last) return;
            *last = pair;
        }
        punion(sh.P, a, b);
    };
    if (!DIAG) {
        const uint64_t o = T & B;
        for (uint32_t e = (uint32_t)((o & ~(o << 1)) >> c0) & 0xffffu; e; e &= e - 1u) {
            const int x = __builtin_ctz(e) + c0;
            join(vrun(sh, r, x), vrun(sh, nr, x));
        }
        return;
    }
    const uint64_t e0 = T & B & ~(T << 1) & ~(B << 1);
    const uint64_t e1 = (T << 1) & B & ~(B << 1);  // r at i-1, nr at i
    const uint64_t e2 = T & (B << 1) & ~(T << 1);  // r at i, nr at i-1
    for (uint32_t e = (uint32_t)((e0 | e1 | e2) >> c0) & 0xffffu; e; e &= e - 1u) {
        const int i = __builtin_ctz(e) + c0;
        const int xr = ((e1 >> i) & 1ull) ? i - 1 : i, xn = ((e2 >> i) & 1ull) ? i - 1 : i;
        join(vrun(sh, r, xr), vrun(sh, nr, xn));
    }
}

// k_vlocal: one workgroup per brick.  Thread tid loads sixteen voxels of
// brick row tid / 4; every run is a provisional label keyed by its first
// voxel (Section 3.1.2), runs are united with the runs they touch in the
// row above and in the rows of the slice below (Section 3.1.3, the
// neighbourhood restricted to the brick), every run then takes its root
// (Section 3.1.4), and each voxel is written as 1 + the position of its
// root run's first voxel, the smallest voxel of its brick component.
template <int C>
__global__ __launch_bounds__(VNT) void k_vlocal(VolArgs v)
{
    __shared__ VolLocalShared sh;
    const int tid = threadIdx.x;
    const Brick bk = brick_of(v, blockIdx.x);
    const int r = tid >> 2, c0 = (tid & 3) * 16;
    const int ky = r % VB_H, kz = r / VB_H;
    const int x = bk.x0 + c0, y = bk.y0 + ky, z = bk.z0 + kz;
    const bool live = z < v.D && y < v.H && x < v.W;
    uint32_t m16 = 0u;
    if (live) {
        const Chunk k = fetch_segment(v.vol + (int64_t)z * v.spitch + (int64_t)y * v.pitch + x,
                                      (uint32_t)(v.W - x < 16 ? v.W - x : 16));
        m16 = chunk_mask(k);
    }
    sh.h[tid] = (uint16_t)m16;
    __syncthreads();
    if (tid < 64) {  // rows, run starts and run-id bases (first wavefront)
        const uint64_t m = (uint64_t)sh.h[4 * tid] | ((uint64_t)sh.h[4 * tid + 1] << 16) |
                           ((uint64_t)sh.h[4 * tid + 2] << 32) | ((uint64_t)sh.h[4 * tid + 3] << 48);
        const uint64_t st = m & ~(m << 1);
        sh.M[tid] = m;
        sh.S[tid] = st;
        const uint32_t cnt = popc64(st);
        uint32_t inc = cnt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off, 64);
            if (tid >= off) inc += o;
        }
        sh.base[tid] = inc - cnt;
        if (tid == 63) sh.base[VB_ROWS] = inc;
    }
    __syncthreads();
    {  // runs starting in this thread's sixteen columns
        const uint64_t st = sh.S[r];
        uint32_t id = sh.base[r] + popc64(st & ~(~0ull << c0));
        for (uint32_t w = (uint32_t)(st >> c0) & 0xffffu; w; w &= w - 1u, ++id)
            sh.P[id] = pk((uint32_t)(r * VB_W + __builtin_ctz(w) + c0), id);
    }
    __syncthreads();
    // Coarse links (Section 3.1.2, column connection lifted to 3-D): every
    // run takes the entry of a run it touches in the first of its earlier
    // neighbour rows that has one (the row above, then the rows of the slice
    // below), a plain store since each run has one writer.  The entry read is
    // that run's label or an ancestor with a smaller key.
    {
        const uint64_t st = sh.S[r], m = sh.M[r];
        uint32_t id = sh.base[r] + popc64(st & ~(~0ull << c0));
        for (uint32_t w = (uint32_t)(st >> c0) & 0xffffu; w; w &= w - 1u, ++id) {
            const int s0 = __builtin_ctz(w) + c0;
            const int e = s0 + ctz64_or64(~(m >> s0)) - 1;
            const uint64_t span = C == 26 ? span_mask(s0 > 0 ? s0 - 1 : 0, e < 63 ? e + 1 : 63)
                                          : span_mask(s0, e);
            int nr = -1;
            uint64_t t = 0;
            if (ky > 0 && (t = sh.M[r - 1] & span)) nr = r - 1;
            else if (kz > 0) {
                if (C == 26 && ky > 0 && (t = sh.M[r - VB_H - 1] & span)) nr = r - VB_H - 1;
                else if ((t = sh.M[r - VB_H] & span)) nr = r - VB_H;
                else if (C == 26 && ky < VB_H - 1 && (t = sh.M[r - VB_H + 1] & span))
                    nr = r - VB_H + 1;
            }
            if (nr >= 0) lds_st(sh.P + id, lds_ld(sh.P + vrun(sh, nr, ctz64(t))));
        }
    }
    __syncthreads();
    // Unification: every run points at its coarse root, then the edges to
    // the earlier rows are merged (Section 3.1.3); an edge whose two runs'
    // current parents are the pair this thread merged last is dropped.
    const uint32_t R = sh.base[VB_ROWS];
    for (uint32_t id = tid; id < R; id += VNT)
        __hip_atomic_fetch_min(sh.P + id, pfind(sh.P, id), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    __syncthreads();
    {
        uint32_t last = ~0u;
        if (ky > 0) vlink_rows<C == 26>(sh, r, r - 1, c0, &last);
        if (kz > 0) {
            if (C == 6) {
                vlink_rows<false>(sh, r, r - VB_H, c0, &last);
            } else {
                if (ky > 0) vlink_rows<true>(sh, r, r - VB_H - 1, c0, &last);
                vlink_rows<true>(sh, r, r - VB_H, c0, &last);
                if (ky < VB_H - 1) vlink_rows<true>(sh, r, r - VB_H + 1, c0, &last);
            }
        }
    }
    __syncthreads();
    // every run's label: 1 + the volume position of its root's first voxel
    const int64_t S = (int64_t)v.H * v.W;
    const int64_t org = (int64_t)bk.z0 * S + (int64_t)bk.y0 * v.W + bk.x0 + 1;
    for (uint32_t id = tid; id < R; id += VNT) {
        const uint32_t key = pk_key(pfind(sh.P, id));
        const int kr = (int)(key / VB_W);
        sh.lab[id] = (int32_t)(org + (int64_t)(kr / VB_H) * S + (int64_t)(kr % VB_H) * v.W +
                               (int)(key % VB_W));
    }
    __syncthreads();
    // Labels out: each wavefront store covers four whole brick rows (row
    // w * 16 + 4q + lane / 16, columns 4 * (lane % 16) .. +3).
    const int lane = tid & 63, wave = tid >> 6;
    const int xw = 4 * (lane % 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int rr = wave * 16 + 4 * q + lane / 16;
        const int yy = bk.y0 + rr % VB_H, zz = bk.z0 + rr / VB_H, xx = bk.x0 + xw;
        if (zz >= v.D || yy >= v.H || xx >= v.W) continue;
        const uint64_t m = sh.M[rr];
        int32_t o[4];
        uint32_t id = vrun(sh, rr, xw);  // the last run starting at or left of xw
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int xj = xw + j;
            if (j > 0 && ((m >> xj) & 1ull) && !((m >> (xj - 1)) & 1ull)) ++id;  // a run starts
            o[j] = ((m >> xj) & 1ull) ? sh.lab[id] : 0;
        }
        int32_t* dst = v.labels + (int64_t)zz * S + (int64_t)yy * v.W + xx;
        if (v.W - xx >= 4 && v.vec && (((uintptr_t)dst & 15u) == 0)) {
            st_global16(dst, o[0], o[1], o[2], o[3]);
        } else {
            for (int j = 0; j < 4; ++j)
                if (xx + j < v.W) st_global(dst + j, o[j]);
        }
    }
}

// k_vmerge: the merge across brick faces (Section 3.2, boundary analysis in
// 3-D), in the label map.  One workgroup per brick takes the voxel pairs
// that cross its three lower faces, each pair exactly once over the volume:
//   z face (z = z0 against z0-1): every neighbour in the slice below,
//       whatever brick it is in (26: the nine voxels around);
//   y face (y = y0 against y0-1): neighbours in the row above within the
//       brick's own slab of slices (26: z-1 .. z+1, x-1 .. x+1);
//   x face (x = x0 against x0-1): neighbours in the column to the left
//       within the brick's own slab and row band (26: z and y +-1).
// A pair crossing several faces belongs to the first of them in that order.
// The z and y faces are rows of 64 voxels against rows of the neighbouring
// plane, staged in LDS: within the brick's 64 columns a stretch of
// foreground of one row lies in one brick component, so, as in the local
// step, one union per pair of touching stretches suffices (face neighbours:
// one per overlapping stretch; with diagonals the 8-connected row edges,
// plus the two voxels at the ends of the row against the neighbouring
// bricks' columns x0-1 and x0+64).  The x face is taken voxel by voxel.
// A thread drops a pair equal to the one it united last, and the workgroup
// drops pairs another of its threads already holds (LDS hash); labels read
// may be stale (roots are lowered meanwhile): any ancestor serves.
constexpr int VM_HASH = 1024;
constexpr int VM_ROWS = 2 * VB_H + 2 + 2 * VB_D;  // staged rows: zA, zB, yA, yB
struct VMergeShared {
    int32_t zA[VB_H][VB_W];          // plane z0, rows y0 .. y0+VB_H-1
    int32_t zB[VB_H + 2][VB_W + 2];  // plane z0-1, rows y0-1 .. y0+VB_H, columns x0-1 .. x0+64
    int32_t yA[VB_D][VB_W];          // row y0 of slices z0 .. z0+VB_D-1
    int32_t yB[VB_D][VB_W + 2];      // row y0-1 of those slices, columns x0-1 .. x0+64
    uint64_t zAm[VB_H], zBm[VB_H + 2], yAm[VB_D], yBm[VB_D];  // foreground of x0 .. x0+63
    unsigned long long seen[VM_HASH];
};

template <int C>
__global__ __launch_bounds__(VNT) void k_vmerge(VolArgs v)
{
    __shared__ VMergeShared sh;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int k = tid; k < VM_HASH; k += VNT) sh.seen[k] = ~0ull;
    const Brick bk = brick_of(v, blockIdx.x);
    const int64_t S = (int64_t)v.H * v.W;
    const uint32_t n = (uint32_t)((int64_t)v.D * S);
    const int zend = min(bk.z0 + VB_D, v.D), yend = min(bk.y0 + VB_H, v.H);
    // staged row q: 0 .. 7 zA, 8 .. 17 zB, 18 .. 25 yA, 26 .. 33 yB
    auto row_of = [&](int q, int& z, int& y) {
        if (q < VB_H) { z = bk.z0; y = bk.y0 + q; return bk.z0 > 0 && y < v.H; }
        q -= VB_H;
        if (q < VB_H + 2) {
            z = bk.z0 - 1;
            y = bk.y0 - 1 + q;
            return bk.z0 > 0 && y >= 0 && y < v.H && (C == 26 || (q > 0 && q <= VB_H));
        }
        q -= VB_H + 2;
        if (q < VB_D) { z = bk.z0 + q; y = bk.y0; return bk.y0 > 0 && z < v.D; }
        q -= VB_D;
        z = bk.z0 + q;
        y = bk.y0 - 1;
        return bk.y0 > 0 && z < v.D;
    };
    constexpr int RPW = (VM_ROWS + 3) / 4;  // staged rows per wavefront
    int32_t val[RPW];
    const int xl = bk.x0 + lane;
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        int z, y;
        const int q = wave + 4 * i;
        val[i] = 0;
        if (q < VM_ROWS && row_of(q, z, y) && xl < v.W)
            val[i] = ld_global(v.labels + (int64_t)z * S + (int64_t)y * v.W + xl);
    }
    // rim columns x0-1 and x0+64 of the zB and yB rows (26 only)
    int32_t rim = 0;
    if (C == 26 && tid < 2 * (VB_H + 2 + VB_D)) {
        int z, y;
        const int q = tid >> 1, side = tid & 1;
        const int qq = q < VB_H + 2 ? VB_H + q : VB_H + (VB_H + 2) + VB_D + (q - (VB_H + 2));
        const int xr = side ? bk.x0 + VB_W : bk.x0 - 1;
        if (row_of(qq, z, y) && xr >= 0 && xr < v.W)
            rim = ld_global(v.labels + (int64_t)z * S + (int64_t)y * v.W + xr);
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        const int q = wave + 4 * i;
        if (q >= VM_ROWS) continue;  // wave-uniform
        const uint64_t m = __ballot(val[i] != 0);
        if (q < VB_H) {
            sh.zA[q][lane] = val[i];
            if (lane == 0) sh.zAm[q] = m;
        } else if (q < 2 * VB_H + 2) {
            sh.zB[q - VB_H][lane + 1] = val[i];
            if (lane == 0) sh.zBm[q - VB_H] = m;
        } else if (q < 2 * VB_H + 2 + VB_D) {
            sh.yA[q - (2 * VB_H + 2)][lane] = val[i];
            if (lane == 0) sh.yAm[q - (2 * VB_H + 2)] = m;
        } else {
            sh.yB[q - (2 * VB_H + 2 + VB_D)][lane + 1] = val[i];
            if (lane == 0) sh.yBm[q - (2 * VB_H + 2 + VB_D)] = m;
        }
    }
    if (C == 26 && tid < 2 * (VB_H + 2 + VB_D)) {
        const int q = tid >> 1, col = (tid & 1) ? VB_W + 1 : 0;
        if (q < VB_H + 2) sh.zB[q][col] = rim;
        else sh.yB[q - (VB_H + 2)][col] = rim;
    }
    if (C == 6) {  // columns x0-1 and x0+64 are never read, but keep them defined
        if (tid < VB_H + 2) sh.zB[tid][0] = sh.zB[tid][VB_W + 1] = 0;
        if (tid < VB_D) sh.yB[tid][0] = sh.yB[tid][VB_W + 1] = 0;
    }
    __syncthreads();

    uint32_t la = ~0u, lb = ~0u;  // the pair this thread united last
    auto unite = [&](int32_t A, int32_t B) {
        const uint32_t a = (uint32_t)A - 1u, b = (uint32_t)B - 1u;
        if (a >= n || b >= n || a == b || (a == la && b == lb)) return;
        la = a;
        lb = b;
        const unsigned long long key = ((unsigned long long)a << 32) | b;
        uint32_t h = (a * 0x9e3779b1u) ^ (b * 0x85ebca77u);
        for (int probe = 0; probe < 8; ++probe, ++h) {
            const unsigned long long old = atomicCAS(sh.seen + (h & (VM_HASH - 1)), ~0ull, key);
            if (old == key) return;   // another thread of the workgroup unites this pair
            if (old == ~0ull) break;  // claimed a fresh entry
        }
        v_union(v.labels, a, b, n);
    };
    // row A (columns x0 .. x0+63) against row B (B[0] = column x0-1), the
    // edges whose index lies in the window of WW columns from c0
    constexpr int NB = C == 26 ? 3 : 1;        // neighbouring rows per face row
    constexpr int WW = C == 26 ? 16 : 8;       // so that the row pairs fill 192 threads
    constexpr int TPR = VB_W / WW;             // threads per row pair
    constexpr uint32_t WMASK = (1u << WW) - 1u;
    static_assert((VB_H + VB_D) * NB * TPR <= VNT - VB_H * VB_D, "row pairs, then the x face");
    auto rows = [&](const int32_t* A, uint64_t TA, const int32_t* B, uint64_t TB, int c0) {
        if (C == 6) {
            const uint64_t o = TA & TB;
            for (uint32_t e = (uint32_t)((o & ~(o << 1)) >> c0) & WMASK; e; e &= e - 1u) {
                const int i = __builtin_ctz(e) + c0;
                unite(A[i], B[i + 1]);
            }
            return;
        }
        const uint64_t e0 = TA & TB & ~(TA << 1) & ~(TB << 1);
        const uint64_t e1 = (TA << 1) & TB & ~(TB << 1);  // A at i-1, B at i
        const uint64_t e2 = TA & (TB << 1) & ~(TA << 1);  // A at i, B at i-1
        for (uint32_t e = (uint32_t)((e0 | e1 | e2) >> c0) & WMASK; e; e &= e - 1u) {
            const int i = __builtin_ctz(e) + c0;
            const int xa = ((e1 >> i) & 1ull) ? i - 1 : i, xb = ((e2 >> i) & 1ull) ? i - 1 : i;
            unite(A[xa], B[xb + 1]);
        }
        if (c0 == 0 && (TA & 1ull) && B[0] != 0) unite(A[0], B[0]);
        if (c0 == VB_W - WW && (TA >> 63) && B[VB_W + 1] != 0) unite(A[VB_W - 1], B[VB_W + 1]);
    };
    const int task = tid / TPR, c0 = (tid % TPR) * WW;
    if (task < VB_H * NB) {  // z face
        if (bk.z0 > 0) {
            const int k = task / NB, j = k + 1 + (C == 26 ? task % NB - 1 : 0);
            rows(sh.zA[k], sh.zAm[k], sh.zB[j], sh.zBm[j], c0);
        }
    } else if (task < (VB_H + VB_D) * NB) {  // y face
        const int t2 = task - VB_H * NB, k = t2 / NB, k2 = k + (C == 26 ? t2 % NB - 1 : 0);
        if (bk.y0 > 0 && k2 >= 0 && k2 < VB_D && bk.z0 + k2 < zend)
            rows(sh.yA[k], sh.yAm[k], sh.yB[k2], sh.yBm[k2], c0);
    }
    // x face: VB_H x VB_D voxels, one per thread of the last quarter
    constexpr int R1 = C == 26 ? 1 : 0;
    const int xt = tid - (VNT - VB_H * VB_D);
    if (bk.x0 > 0 && xt >= 0) {
        const int yy = bk.y0 + xt % VB_H, zz = bk.z0 + xt / VB_H;
        if (yy < yend && zz < zend) {
            const int32_t A = ld_global(v.labels + (int64_t)zz * S + (int64_t)yy * v.W + bk.x0);
            if (A != 0) {
                for (int dz = -R1; dz <= R1; ++dz)
                    for (int dy = -R1; dy <= R1; ++dy) {
                        const int z2 = zz + dz, y2 = yy + dy;
                        if (z2 < bk.z0 || z2 >= zend || y2 < bk.y0 || y2 >= yend) continue;
                        const int32_t B =
                            ld_global(v.labels + (int64_t)z2 * S + (int64_t)y2 * v.W + bk.x0 - 1);
                        if (B != 0) unite(A, B);
                    }
            }
        }
    }
}

// k_vfinal: one workgroup per brick; every foreground voxel takes 1 + its
// root's position.  The brick's labels are staged in LDS (each wavefront
// load and store covers four whole brick rows: row w * 16 + 4q + lane / 16,
// columns 4 * (lane % 16) .. +3).  A voxel's label names the first voxel
// of its brick component, which lies in the brick unless the voxel is that
// first voxel and the merge linked it, so the first hop is mostly an LDS
// read; only components the merge linked (their first voxel's entry no
// longer names itself) are chased in the label map.  A label equal to the
// thread's previous one reuses its root.  The merge is over, so every entry
// read is an ancestor whatever this kernel has already rewritten, and roots
// are never rewritten.
__global__ __launch_bounds__(VNT) void k_vfinal(VolArgs v)
{
    __shared__ int32_t Lb[VB_ROWS][VB_W];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const Brick bk = brick_of(v, blockIdx.x);
    const int64_t S = (int64_t)v.H * v.W;
    const uint32_t n = (uint32_t)((int64_t)v.D * S);
    const int xw = 4 * (lane % 16);
    int32_t in[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int rr = wave * 16 + 4 * q + lane / 16;
        const int yy = bk.y0 + rr % VB_H, zz = bk.z0 + rr / VB_H, xx = bk.x0 + xw;
        in[q][0] = in[q][1] = in[q][2] = in[q][3] = 0;
        if (zz >= v.D || yy >= v.H || xx >= v.W) continue;
        const int32_t* src = v.labels + (int64_t)zz * S + (int64_t)yy * v.W + xx;
        if (v.W - xx >= 4 && v.vec && (((uintptr_t)src & 15u) == 0)) {
            const uint4 w = ld_global16(src);
            in[q][0] = (int32_t)w.x; in[q][1] = (int32_t)w.y;
            in[q][2] = (int32_t)w.z; in[q][3] = (int32_t)w.w;
        } else {
            for (int j = 0; j < 4; ++j)
                if (xx + j < v.W) in[q][j] = ld_global(src + j);
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int rr = wave * 16 + 4 * q + lane / 16;
#pragma unroll
        for (int j = 0; j < 4; ++j) Lb[rr][xw + j] = in[q][j];
    }
    __syncthreads();
    int32_t lastL = 0, lastR = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int rr = wave * 16 + 4 * q + lane / 16;
        const int yy = bk.y0 + rr % VB_H, zz = bk.z0 + rr / VB_H, xx = bk.x0 + xw;
        if (zz >= v.D || yy >= v.H || xx >= v.W) continue;
        int32_t o[4];
        bool changed = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int32_t L = in[q][j];
            o[j] = L;
            if (L == 0 || (uint32_t)L - 1u >= n) continue;
            if (L != lastL) {
                uint32_t p = (uint32_t)L - 1u, zp, rem, yp, xp;
                divmod_w(p, (uint32_t)S, v.smagic, zp, rem);
                divmod_w(rem, (uint32_t)v.W, v.wmagic, yp, xp);
                const int kz = (int)zp - bk.z0, ky = (int)yp - bk.y0, kx = (int)xp - bk.x0;
                const bool here = kz >= 0 && kz < VB_D && ky >= 0 && ky < VB_H && kx >= 0 &&
                                  kx < VB_W;
                uint32_t e = (uint32_t)(here ? Lb[kz * VB_H + ky][kx] : ld_global(v.labels + p)) - 1u;
                while (e != p && e < n) {
                    p = e;
                    e = (uint32_t)ld_global(v.labels + p) - 1u;
                }
                lastL = L;
                lastR = (int32_t)(p + 1u);
            }
            o[j] = lastR;
            changed |= o[j] != L;
        }
        if (!changed) continue;
        int32_t* dst = v.labels + (int64_t)zz * S + (int64_t)yy * v.W + xx;
        if (v.W - xx >= 4 && v.vec && (((uintptr_t)dst & 15u) == 0)) {
            st_global16(dst, o[0], o[1], o[2], o[3]);
        } else {
            for (int j = 0; j < 4; ++j)
                if (xx + j < v.W && o[j] != in[q][j]) st_global(dst + j, o[j]);
        }
    }
}

// ---------------------------------------------------------------------------
// copy kernel (bandwidth / counter calibration)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_copy(const uint4* __restrict__ src,
                                              uint4* __restrict__ dst, int64_t n16)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

// Gathers segments of seg16 16-byte units, one every sstride16 units of src,
// into dst (contiguous): reads in requests of one segment each, as k_local
// reads a tile's rows.
__global__ __launch_bounds__(256) void k_copy_seg(const uint4* __restrict__ src,
                                                  uint4* __restrict__ dst, int64_t n16,
                                                  int seg16, int64_t sstride16)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[(i / seg16) * sstride16 + i % seg16];
}

#endif  // CCL_TILE_ROWS == 64

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

// Workgroups of `kernel` that the current device holds at once (occupancy x
// compute units), cached per device and kernel: the grid of a persistent
// kernel.
template <typename K>
static unsigned resident_blocks(K kernel, int threads)
{
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, unsigned> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    const auto key = std::make_pair(dev, reinterpret_cast<const void*>(kernel));
    const auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess)
        per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 1;
    const unsigned n = (unsigned)(per_cu > 0 ? per_cu : 1) * (unsigned)(cus > 0 ? cus : 1);
    cache[key] = n;
    return n;
}

// Launch shape of k_local and k_final: persistent (one workgroup per
// resident slot, the next tile's loads in flight while the current one is
// labelled) or one workgroup per tile (the dispatcher balances tiles of
// unequal cost, which a fixed round-robin over many tiles does not).  The
// caller may fix the choice (a tuned policy); otherwise the built-in rule
// holds: k_local goes per tile beyond four times the resident workgroups
// (8192^2 with 64-row tiles: 142 -> 126 us on Bernoulli 0.5, 111 -> 79 us on
// the spiral), k_final stays persistent.
// kernel 0 = k_local, 1 = k_final
static unsigned tile_grid(int kernel, const BatchArgs& b, unsigned resident, GridChoice g)
{
    const int v = kernel == 0 ? g.local : g.final_;
    const bool per_tile = v >= 0 ? v == 1 : (kernel == 0 && b.ntiles > 4 * (int64_t)resident);
    return per_tile ? (unsigned)b.ntiles : (unsigned)std::min<int64_t>(b.ntiles, resident);
}

int64_t image_groups(int ntx, int nty)
{
    if (ntx == 1 && nty == 1) return 0;  // nothing to merge
    return (int64_t)((ntx + BX - 1) / BX) * ((nty + BY - 1) / BY);
}

int64_t image_seam_items(int ntx, int nty, int H, int W, int conn)
{
    const int nbx = (ntx + BX - 1) / BX;
    const int nkh = (nty - 1) / BY, nkv = (ntx - 1) / BX;
    return (int64_t)nkh * W + (int64_t)nkv * H +
           (conn == 8 ? (int64_t)(nty - 1 - nkh) * (nbx - 1) : 0);
}

template <int D>
static hipError_t launch_all(const BatchArgs& b, const Workspace& ws, hipStream_t st,
                             KernelTimer* timer, bool local_only, GridChoice grid,
                             const StatsWs* stats)
{
    const StatsWs none{};
    if (b.ntiles <= 0) return hipSuccess;
#if CCL_TILE_ROWS != 64
    if (stats) return hipErrorInvalidValue;  // statistics use the built-in tile height
#endif
    const unsigned lgrid = tile_grid(0, b, resident_blocks(k_local<D>, NT), grid);
    timer_begin(timer, KIND_LOCAL, st);
    k_local<D><<<lgrid, NT, 0, st>>>(b, ws);
    timer_end(timer, KIND_LOCAL, st);
    if (local_only) {
        const unsigned fgrid = tile_grid(1, b, resident_blocks(k_final<D, true, false>, NT), grid);
        timer_begin(timer, KIND_FINAL, st);
        k_final<D, true, false><<<fgrid, NT, 0, st>>>(b, ws, none);
        timer_end(timer, KIND_FINAL, st);
        return hipGetLastError();
    }
    // single-tile images have no merge group (and no seams)
    if (b.ngroups > 0) {
        timer_begin(timer, KIND_BLOCK, st);
        k_block<D><<<(unsigned)b.ngroups, NTB, 0, st>>>(b, ws);
        timer_end(timer, KIND_BLOCK, st);
    }
    if (b.nseamwg > 0) {
        timer_begin(timer, KIND_SEAM, st);
        k_seam<D><<<(unsigned)b.nseamwg, SEAM_WG, 0, st>>>(b, ws);
        timer_end(timer, KIND_SEAM, st);
    }
    if (!stats) {
        const unsigned fgrid =
            tile_grid(1, b, resident_blocks(k_final<D, false, false>, NT), grid);
        timer_begin(timer, KIND_FINAL, st);
        k_final<D, false, false><<<fgrid, NT, 0, st>>>(b, ws, none);
        timer_end(timer, KIND_FINAL, st);
        return hipGetLastError();
    }
#if CCL_TILE_ROWS == 64
    const unsigned fgrid = tile_grid(1, b, resident_blocks(k_final<D, false, true>, NT), grid);
    timer_begin(timer, KIND_FINAL, st);
    k_final<D, false, true><<<fgrid, NT, 0, st>>>(b, ws, *stats);
    timer_end(timer, KIND_FINAL, st);
    timer_begin(timer, KIND_STATS, st);
    k_scan1<<<(unsigned)stats->nblk, SCAN_T, 0, st>>>(*stats);
    k_scan2<<<1, SCAN_T, 0, st>>>(*stats);
    if (stats->capacity > 0) {
        k_stats<D><<<(unsigned)b.ntiles, ST, 0, st>>>(b, ws, *stats);
        const ImageArgs& a = b.one;
        static_assert(TW == TILE_ROWS, "square tiles: merge regions are squares of tiles");
        k_stats_merge<<<(unsigned)(stats->g1x * stats->g1y), MERGE_T, 0, st>>>(
            *stats, stats->rec0, stats->cnt0, NSLOTS, a.ntx, a.nty, stats->g1x, a);
    }
    timer_end(timer, KIND_STATS, st);
#endif
    return hipGetLastError();
}

hipError_t launch_index(const BatchArgs& b, hipStream_t st)
{
    if (b.n <= 1) return hipSuccess;
    const int64_t idx = b.ntiles + b.ngroups + b.nseamwg;
    if (idx > 0) k_index<<<(unsigned)((idx + 255) / 256), 256, 0, st>>>(b);
    return hipGetLastError();
}

hipError_t launch_label(const BatchArgs& b, int conn, const Workspace& ws, hipStream_t st,
                        KernelTimer* timer, bool local_only, GridChoice grid,
                        const StatsWs* stats)
{
    if (conn == 8) return launch_all<1>(b, ws, st, timer, local_only, grid, stats);
    return launch_all<0>(b, ws, st, timer, local_only, grid, stats);
}

template <int D>
static hipError_t replay_all(const BatchArgs& b, const Workspace& ws, hipStream_t st,
                             GridChoice grid, int kind, int reps)
{
    if (b.ntiles <= 0) return hipSuccess;
    if (kind == KIND_LOCAL) {
        const unsigned g = tile_grid(0, b, resident_blocks(k_local<D>, NT), grid);
        for (int r = 0; r < reps; ++r) k_local<D><<<g, NT, 0, st>>>(b, ws);
    } else if (kind == KIND_FINAL) {
        const unsigned g = tile_grid(1, b, resident_blocks(k_final<D, false, false>, NT), grid);
        for (int r = 0; r < reps; ++r) k_final<D, false, false><<<g, NT, 0, st>>>(b, ws, StatsWs{});
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_replay(const BatchArgs& b, int conn, const Workspace& ws, hipStream_t st,
                         GridChoice grid, int kind, int reps)
{
    if (conn == 8) return replay_all<1>(b, ws, st, grid, kind, reps);
    return replay_all<0>(b, ws, st, grid, kind, reps);
}

// The launcher table is host data (the device pass does not see it).
#if !defined(__HIP_DEVICE_COMPILE__)
const ShapeOps ops = {TILE_ROWS, image_groups, image_seam_items, launch_index, launch_label,
                      launch_replay};
#endif

#if CCL_TILE_ROWS == 64
hipError_t launch_ablation(const BatchArgs& b, const Workspace& ws, hipStream_t st, int variant,
                           uint32_t* counters)
{
    if (b.ntiles <= 0) return hipSuccess;
    const unsigned g = (unsigned)b.ntiles;
    switch (variant) {
        case 0: k_local_ablate<ABL_ROW | ABL_COL><<<g, NT, 0, st>>>(b, ws, counters); break;
        case 1: k_local_ablate<ABL_ROW><<<g, NT, 0, st>>>(b, ws, counters); break;
        case 2: k_local_ablate<ABL_COL><<<g, NT, 0, st>>>(b, ws, counters); break;
        default: k_local_ablate<0><<<g, NT, 0, st>>>(b, ws, counters); break;
    }
    if (b.ngroups > 0) k_block<0><<<(unsigned)b.ngroups, NTB, 0, st>>>(b, ws);
    if (b.nseamwg > 0) k_seam<0><<<(unsigned)b.nseamwg, SEAM_WG, 0, st>>>(b, ws);
    const unsigned fgrid =
        tile_grid(1, b, resident_blocks(k_final<0, false, false>, NT), GridChoice{});
    k_final<0, false, false><<<fgrid, NT, 0, st>>>(b, ws, StatsWs{});
    return hipGetLastError();
}

hipError_t launch_volume(const VolArgs& v, int conn, hipStream_t st, KernelTimer* timer)
{
    const int64_t n = (int64_t)v.D * v.H * v.W;
    if (n == 0) return hipSuccess;
    const unsigned g = (unsigned)((int64_t)v.nbx * v.nby * v.nbz);
    timer_begin(timer, KIND_VLOCAL, st);
    if (conn == 26) k_vlocal<26><<<g, VNT, 0, st>>>(v);
    else k_vlocal<6><<<g, VNT, 0, st>>>(v);
    timer_end(timer, KIND_VLOCAL, st);
    if (g > 1) {  // one brick: its components are the volume's, labels final
        timer_begin(timer, KIND_VMERGE, st);
        if (conn == 26) k_vmerge<26><<<g, VNT, 0, st>>>(v);
        else k_vmerge<6><<<g, VNT, 0, st>>>(v);
        timer_end(timer, KIND_VMERGE, st);
        timer_begin(timer, KIND_VFINAL, st);
        k_vfinal<<<g, VNT, 0, st>>>(v);
        timer_end(timer, KIND_VFINAL, st);
    }
    return hipGetLastError();
}

hipError_t launch_zero_count(int64_t* count, hipStream_t st)
{
    k_zero_count<<<1, 1, 0, st>>>(count);
    return hipGetLastError();
}

hipError_t launch_copy_segments(const void* src, void* dst, int64_t bytes, int seg_bytes,
                                int64_t src_stride, hipStream_t st, KernelTimer* timer)
{
    const int64_t n16 = bytes / 16;
    int64_t blocks = (n16 + 255) / 256;
    if (blocks > 256 * 64) blocks = 256 * 64;
    if (blocks < 1) blocks = 1;
    timer_begin(timer, KIND_COPY, st);
    k_copy_seg<<<(unsigned)blocks, 256, 0, st>>>(static_cast<const uint4*>(src),
                                                 static_cast<uint4*>(dst), n16, seg_bytes / 16,
                                                 src_stride / 16);
    timer_end(timer, KIND_COPY, st);
    return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t st,
                       KernelTimer* timer)
{
    const int64_t n16 = bytes / 16;
    int64_t blocks = (n16 + 255) / 256;
    if (blocks > 256 * 64) blocks = 256 * 64;
    if (blocks < 1) blocks = 1;
    timer_begin(timer, KIND_COPY, st);
    k_copy<<<(unsigned)blocks, 256, 0, st>>>(static_cast<const uint4*>(src),
                                             static_cast<uint4*>(dst), n16);
    timer_end(timer, KIND_COPY, st);
    return hipGetLastError();
}
#endif  // CCL_TILE_ROWS == 64

}  // namespace CCL_SHAPE_NS
}  // namespace ccl
