// Block-based coarse-to-fine connected-components labelling for gfx950.
//
// The image is cut into tiles of 64 x TILE_ROWS pixels: one 64-bit
// foreground mask per tile row, so the paper's row scan becomes bit
// arithmetic on a word.  A workgroup of 256 threads owns a tile.
//
// Nodes of the tile-local union-find are runs: maximal horizontal stretches
// of foreground.  Under 8-connectivity two rows are fused into a strip first:
// any run of (row 2k | row 2k+1) is 8-connected (neighbouring columns that
// each hold a foreground pixel in one of the two rows always touch), so a
// strip run is a node.  "Line" below means a row (4-connectivity) or a strip
// (8-connectivity); runs get dense ids in line-major, left-to-right order.
//
// Three kernels per image (the paper's Section 3):
//   k_local  (Section 3.1)  load the tile, label it in LDS, and publish what
//            the merge and the relabel need: the foreground bitmask, a run
//            table (local root of each run), one forest node id per border
//            pixel, and one forest node per component that touches the tile
//            border.
//   k_seam   (Section 3.2)  for every foreground pair straddling a tile seam,
//            unite the two components' forest nodes in HBM (atomicMin).
//   k_final  (Section 3.3)  look up the global root of each border component
//            and write every label exactly once, from the bitmask and the run
//            table (no union-find work is repeated).
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

#include "ccl_kernels.h"

namespace ccl {

constexpr int NT = 256;  // threads per tile workgroup

// Geometry of one connectivity: D = 0 (4-connectivity, lines are rows) or
// D = 1 (8-connectivity, lines are two-row strips).
template <int D>
struct Geo {
    static constexpr int NL = D ? TILE_ROWS / 2 : TILE_ROWS;  // lines per tile
    static constexpr int TPL = NT / NL;                       // threads per line
    static constexpr int WIN = TW / TPL;                      // columns per thread
    static constexpr int MAXR = NL * (TW / 2);                // runs per tile, at most
};
static_assert(Geo<0>::MAXR <= RUNTAB_PER_TILE && Geo<1>::MAXR <= RUNTAB_PER_TILE, "run table");
static_assert(NSLOTS == NT, "one border slot per thread");

// ---------------------------------------------------------------------------
// bit helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int ctz64(uint64_t v) { return __builtin_ctzll(v); }
__device__ __forceinline__ int ctz64_or64(uint64_t v) { return v ? __builtin_ctzll(v) : 64; }
__device__ __forceinline__ uint32_t popc64(uint64_t v) { return (uint32_t)__popcll(v); }

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

// Packed root of x.  Halves the path on the way: every store writes the
// grandparent, whose key is smaller, so entries only ever decrease.
__device__ uint32_t pfind(uint32_t* P, uint32_t x)
{
    uint32_t v = lds_ld(P + x);
    while (pk_id(v) != x) {
        const uint32_t p = pk_id(v);
        const uint32_t w = lds_ld(P + p);
        if (pk_id(w) == p) return w;
        lds_st(P + x, w);
        x = pk_id(w);
        v = lds_ld(P + x);
    }
    return v;
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

__device__ Root g_find(uint64_t* F, uint32_t n)
{
    while (true) {
        uint64_t v = g_ld(F + n);
        uint32_t p = (uint32_t)v;
        if (p == n) return Root{n, (uint32_t)(v >> 32)};
        uint64_t vp = g_ld(F + p);
        uint32_t pp = (uint32_t)vp;
        if (pp == p) return Root{p, (uint32_t)(vp >> 32)};
        __hip_atomic_fetch_min(F + n, vp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        n = pp;
    }
}

__device__ Root g_find_ro(const uint64_t* F, uint32_t n)
{
    while (true) {
        uint64_t v = g_ld(F + n);
        uint32_t p = (uint32_t)v;
        if (p == n) return Root{n, (uint32_t)(v >> 32)};
        n = p;
    }
}

__device__ void g_union(uint64_t* F, uint32_t a, uint32_t b)
{
    while (true) {
        Root ra = g_find(F, a);
        Root rb = g_find(F, b);
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
    if (tid < 64) {
        uint32_t cnt = 0;
        if (tid < NL) {
            const uint64_t lm = D ? (sh.M[2 * tid] | sh.M[2 * tid + 1]) : sh.M[tid];
            const uint64_t ls = lm & ~(lm << 1);
            sh.LM[tid] = lm;
            sh.LS[tid] = ls;
            cnt = popc64(ls);
        }
        // inclusive scan of the run counts across the first wavefront
        uint32_t inc = cnt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off, 64);
            if (tid >= off) inc += o;
        }
        if (tid < NL) sh.base[tid] = inc - cnt;
        if (tid == NL - 1) sh.base[NL] = inc;
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

template <int D>
struct LocalShared : Lines<D> {
    uint32_t P[Geo<D>::MAXR];
    union {
        uint16_t h[TILE_ROWS * 4];  // 16-pixel masks as produced by the byte load
        uint64_t w[TILE_ROWS];      // the same bits as one word per row
    } m16;
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

// Run-table entry flags: the run's component touches the tile border (low
// bits = representative border slot) / this run is that component's root.
constexpr uint16_t RT_BORDER = 0x8000;
constexpr uint16_t RT_ROOT = 0x4000;
constexpr uint32_t REP_TAG = 0x80000000u;

// ---------------------------------------------------------------------------
// k_local
// ---------------------------------------------------------------------------

template <int D>
__global__ __launch_bounds__(NT) void k_local(ImageArgs a, Workspace ws)
{
    using G = Geo<D>;
    __shared__ LocalShared<D> sh;
    const int tid = threadIdx.x;
    const int t = blockIdx.x;
    const int tx = t % a.ntx, ty = t / a.ntx;
    const int gx0 = tx * TW, gy0 = ty * TILE_ROWS;

    // Initialisation: load the tile's bytes, four threads per row, sixteen
    // pixels per thread, and turn them into foreground bits.
    for (int c = tid; c < TILE_ROWS * 4; c += NT) {
        const int r = c >> 2, q = c & 3;
        const int gy = gy0 + r, gx = gx0 + 16 * q;
        uint32_t bits = 0;
        if (gy < a.H && gx < a.W) {
            const uint8_t* src = a.img + (int64_t)gy * a.pitch + gx;
            if (a.vec_in && gx + 16 <= a.W) {
                const uint4 v = *reinterpret_cast<const uint4*>(src);
                bits = nz_nibble(v.x) | (nz_nibble(v.y) << 4) | (nz_nibble(v.z) << 8) |
                       (nz_nibble(v.w) << 12);
            } else {
                const int n = a.W - gx < 16 ? a.W - gx : 16;
                for (int i = 0; i < n; ++i) bits |= (uint32_t)(src[i] != 0) << i;
            }
        }
        sh.m16.h[c] = (uint16_t)bits;
    }
    __syncthreads();
    if (tid < TILE_ROWS) {
        const uint64_t m = sh.m16.w[tid];
        sh.M[tid] = m;
        ws.bits[(int64_t)t * TILE_ROWS + tid] = m;
    }
    __syncthreads();
    build_lines<D>(sh, tid);

    // This thread's line and column window; its runs are those starting in
    // the window, with consecutive ids from id0.
    const int l = tid / G::TPL;
    const int wlo = (tid % G::TPL) * G::WIN;
    const uint64_t wmask = (G::WIN == 64 ? ~0ull : ((1ull << G::WIN) - 1ull)) << wlo;
    const uint64_t lm = sh.LM[l];
    const uint64_t mine = sh.LS[l] & wmask;
    const uint32_t id0 = sh.base[l] + popc64(sh.LS[l] & ~(~0ull << wlo));

    // Row connection: a run is its own provisional root, keyed by its
    // smallest pixel (the paper's provisional label = position).
    {
        uint32_t id = id0;
        for (uint64_t r = mine; r; r &= r - 1, ++id) {
            const int s0 = ctz64(r);
            const int e = s0 + ctz64_or64(~(lm >> s0)) - 1;
            sh.P[id] = pk(run_key<D>(sh, l, s0, e), id);
        }
    }
    __syncthreads();

    // Column connection (coarse): each run records the lowest label among
    // its neighbours in the line above, i.e. the run holding the leftmost
    // pixel there that touches it.  One plain store per run.
    if (l > 0) {
        const uint64_t up = bottom_row<D>(sh, l - 1);
        const uint64_t top = top_row<D>(sh, l);
        uint32_t id = id0;
        for (uint64_t r = mine; r; r &= r - 1, ++id) {
            const int s0 = ctz64(r);
            const int e = s0 + ctz64_or64(~(lm >> s0)) - 1;
            const uint64_t mt = top & span_mask(s0, e);
            const uint64_t reach = D ? (mt | (mt << 1) | (mt >> 1)) : mt;
            const uint64_t contact = up & reach;
            if (contact) sh.P[id] = lds_ld(sh.P + run_id<D>(sh, l - 1, ctz64(contact)));
        }
    }
    __syncthreads();

    // Label-equivalence unification: every run points at its current root.
    {
        uint32_t id = id0;
        for (uint64_t r = mine; r; r &= r - 1, ++id) lds_st(sh.P + id, pfind(sh.P, id));
    }
    __syncthreads();

    // Refinement: unite the runs of every remaining adjacency between this
    // line and the one above.  The adjacencies are enumerated bitwise from
    // the two facing rows (lower = this line's top row T, upper = the line
    // above's bottom row B); an edge is dropped when an edge further left
    // joins the same two runs (consecutive foreground pixels of one row lie
    // in one run), which leaves one edge per touching pair of runs:
    //   4-connectivity: starts of the stretches of T & B;
    //   8-connectivity: (i,i)   where neither side continues from i-1,
    //                   (i-1,i) where B does not continue from i-1,
    //                   (i,i-1) where T does not continue from i-1.
    if (l > 0) {
        const uint64_t T = top_row<D>(sh, l), B = bottom_row<D>(sh, l - 1);
        if (!D) {
            const uint64_t o = T & B;
            for (uint64_t r = o & ~(o << 1) & wmask; r; r &= r - 1) {
                const int i = ctz64(r);
                punion(sh.P, run_id<D>(sh, l, i), run_id<D>(sh, l - 1, i));
            }
        } else {
            const uint64_t e0 = T & B & ~(T << 1) & ~(B << 1);
            const uint64_t e1 = (T << 1) & B & ~(B << 1);
            const uint64_t e2 = T & (B << 1) & ~(T << 1);
            for (uint64_t r = e0 & wmask; r; r &= r - 1) {
                const int i = ctz64(r);
                punion(sh.P, run_id<D>(sh, l, i), run_id<D>(sh, l - 1, i));
            }
            for (uint64_t r = e1 & wmask; r; r &= r - 1) {
                const int i = ctz64(r);
                punion(sh.P, run_id<D>(sh, l, i - 1), run_id<D>(sh, l - 1, i));
            }
            for (uint64_t r = e2 & wmask; r; r &= r - 1) {
                const int i = ctz64(r);
                punion(sh.P, run_id<D>(sh, l, i), run_id<D>(sh, l - 1, i - 1));
            }
        }
    }
    __syncthreads();

    // Unification again: every run points straight at its final local root.
    {
        uint32_t id = id0;
        for (uint64_t r = mine; r; r &= r - 1, ++id) lds_st(sh.P + id, pfind(sh.P, id));
    }
    __syncthreads();

    // Border slots (one per thread): local root of each border pixel.
    const int s = tid;
    int sx, sy;
    slot_xy(s, sx, sy);
    const bool fg = (sh.M[sy] >> sx) & 1ull;
    uint32_t root = 0, rkey = 0;
    if (fg) {
        const uint32_t v = lds_ld(sh.P + run_id<D>(sh, D ? sy >> 1 : sy, sx));
        root = pk_id(v);
        rkey = pk_key(v);
    }
    __syncthreads();
    // Elect the smallest slot of each border component as its representative
    // (an atomic max on the root entry, which is no longer needed as a parent).
    if (fg)
        __hip_atomic_fetch_max(sh.P + root, REP_TAG | (uint32_t)(NSLOTS - 1 - s),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __syncthreads();

    // ID conversion (Section 3.1.4): the representative's forest node carries
    // the raster position of the component's smallest pixel.
    const int64_t sbase = (int64_t)t * NSLOTS;
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

    // Run table: interior components store their root's tile key; border
    // components store their representative slot (and mark the root run).
    {
        uint16_t* rt = ws.runtab + (int64_t)t * RUNTAB_PER_TILE;
        uint32_t id = id0;
        for (uint64_t r = mine; r; r &= r - 1, ++id) {
            const uint32_t v = lds_ld(sh.P + id);
            uint16_t ent;
            if (v & REP_TAG) {
                ent = (uint16_t)(RT_BORDER | RT_ROOT | (NSLOTS - 1 - pk_id(v)));
            } else {
                const uint32_t w = pk_id(v) == id ? v : lds_ld(sh.P + pk_id(v));
                ent = (w & REP_TAG) ? (uint16_t)(RT_BORDER | (NSLOTS - 1 - pk_id(w)))
                                    : (uint16_t)pk_key(v);
            }
            rt[id] = ent;
        }
    }
}

// ---------------------------------------------------------------------------
// k_seam
// ---------------------------------------------------------------------------

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
// sides repeat.
template <int D>
__device__ __forceinline__ void seam_item(uint64_t* F, int32_t a_prev, int32_t a,
                                          int32_t b_prev, int32_t b)
{
    const bool ra = a_prev == a, rb = b_prev == b;
    if (D == 0) {
        if (a >= 0 && b >= 0 && !(ra && rb)) g_union(F, (uint32_t)a, (uint32_t)b);
    } else {
        if (a >= 0 && b >= 0 && !ra && !rb) g_union(F, (uint32_t)a, (uint32_t)b);
        if (a_prev >= 0 && b >= 0 && !rb) g_union(F, (uint32_t)a_prev, (uint32_t)b);
        if (a >= 0 && b_prev >= 0 && !ra) g_union(F, (uint32_t)a, (uint32_t)b_prev);
    }
}

// Block merge with boundary analysis (Section 3.2): only border pixels are
// visited — (ntx-1)*H + (nty-1)*W work items, the paper's P_x + P_y of Eq. 1-2.
// Horizontal seams (between tile rows) run over the full image width, so
// diagonal pairs through a four-tile corner are seen there; vertical seams
// (between tile columns) stay inside one tile row.
template <int D>
__global__ __launch_bounds__(256) void k_seam(ImageArgs a, Workspace ws)
{
    constexpr int NS = NSLOTS;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nh = (int64_t)(a.nty - 1) * a.W;
    const int64_t nv = (int64_t)(a.ntx - 1) * a.H;
    const int32_t* slots = ws.slots;

    int32_t a_prev = -1, a_cur, b_prev = -1, b_cur;
    if (gid < nh) {
        const int k = (int)(gid / a.W) + 1;
        const int x = (int)(gid - (int64_t)(k - 1) * a.W);
        const int64_t top = (int64_t)(k - 1) * a.ntx, bot = (int64_t)k * a.ntx;
        a_cur = slots[(top + x / TW) * NS + TW + x % TW];
        b_cur = slots[(bot + x / TW) * NS + x % TW];
        if (x > 0) {
            const int xp = x - 1;
            a_prev = slots[(top + xp / TW) * NS + TW + xp % TW];
            b_prev = slots[(bot + xp / TW) * NS + xp % TW];
        }
    } else if (gid < nh + nv) {
        const int64_t g = gid - nh;
        const int j = (int)(g / a.H) + 1;
        const int y = (int)(g - (int64_t)(j - 1) * a.H);
        const int k = y / TILE_ROWS, yl = y - k * TILE_ROWS;
        const int64_t left = ((int64_t)k * a.ntx + j - 1) * NS + 2 * TW + TILE_ROWS;
        const int64_t right = ((int64_t)k * a.ntx + j) * NS + 2 * TW;
        a_cur = slots[left + yl];
        b_cur = slots[right + yl];
        if (yl > 0) {
            a_prev = slots[left + yl - 1];
            b_prev = slots[right + yl - 1];
        }
    } else {
        return;
    }
    seam_item<D>(ws.forest, a_prev, a_cur, b_prev, b_cur);
}

// ---------------------------------------------------------------------------
// k_final
// ---------------------------------------------------------------------------

template <int D>
struct FinalShared : Lines<D> {
    int32_t lab[Geo<D>::MAXR];  // final label of each run
    int32_t fin[NSLOTS];        // final label of each border component, by slot
};

// Update of the global label map (Section 3.3).  Each border component takes
// 1 + the key of its global root, every other component 1 + the raster
// position of its local root; each label is written once.  With LOCAL_ONLY
// the forest is read before any merge (every tile labelled as an image).
template <int D, bool LOCAL_ONLY>
__global__ __launch_bounds__(NT) void k_final(ImageArgs a, Workspace ws)
{
    __shared__ FinalShared<D> sh;
    const int tid = threadIdx.x;
    const int t = blockIdx.x;
    const int tx = t % a.ntx, ty = t / a.ntx;
    const int gx0 = tx * TW, gy0 = ty * TILE_ROWS;

    if (tid < TILE_ROWS) sh.M[tid] = ws.bits[(int64_t)t * TILE_ROWS + tid];
    __syncthreads();
    build_lines<D>(sh, tid);
    const uint32_t R = sh.base[Geo<D>::NL];
    const uint16_t* rt = ws.runtab + (int64_t)t * RUNTAB_PER_TILE;
    const int64_t sbase = (int64_t)t * NSLOTS;

    // global root of each border component, looked up once (by its root run)
    for (uint32_t id = tid; id < R; id += NT) {
        const uint16_t e = rt[id];
        if ((e & (RT_BORDER | RT_ROOT)) == (RT_BORDER | RT_ROOT)) {
            const int rep = e & 0x3fff;
            const uint32_t key = LOCAL_ONLY
                                     ? (uint32_t)(g_ld(ws.forest + sbase + rep) >> 32)
                                     : g_find_ro(ws.forest, (uint32_t)(sbase + rep)).key;
            sh.fin[rep] = (int32_t)(key + 1u);
        }
    }
    __syncthreads();
    for (uint32_t id = tid; id < R; id += NT) {
        const uint16_t e = rt[id];
        int32_t v;
        if (e & RT_BORDER) {
            v = sh.fin[e & 0x3fff];
        } else {
            // ID conversion of an interior component's local root
            v = (int32_t)((int64_t)(gy0 + e / TW) * a.W + gx0 + e % TW + 1);
        }
        sh.lab[id] = v;
    }
    __syncthreads();

    // write the labels: 16 threads per tile row, 4 pixels per thread
    const int xmax = a.W - gx0;  // pixels of this tile inside the image
    for (int c = tid; c < TILE_ROWS * 16; c += NT) {
        const int r = c >> 4, x0 = (c & 15) * 4;
        const int gy = gy0 + r;
        if (gy >= a.H || x0 >= xmax) continue;
        const int l = D ? r >> 1 : r;
        const uint64_t mr = sh.M[r], ls = sh.LS[l];
        uint32_t cnt = sh.base[l] + popc64(ls & ~(~0ull << x0));  // runs starting left of x0
        int32_t v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int x = x0 + k;
            cnt += (uint32_t)((ls >> x) & 1ull);
            // a foreground pixel has its run start at or left of it, so cnt >= 1
            v[k] = ((mr >> x) & 1ull) ? sh.lab[cnt ? cnt - 1 : 0] : 0;
        }
        int32_t* dst = a.labels + (int64_t)gy * a.W + gx0 + x0;
        if (a.vec_out && x0 + 4 <= xmax) {
            *reinterpret_cast<int4*>(dst) = make_int4(v[0], v[1], v[2], v[3]);
        } else {
            const int n = xmax - x0 < 4 ? xmax - x0 : 4;
            for (int k = 0; k < n; ++k) dst[k] = v[k];
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

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <int D>
static hipError_t launch_all(const ImageArgs& a, const Workspace& ws, hipStream_t st,
                             KernelTimer* timer, bool local_only)
{
    const unsigned ntiles = (unsigned)a.ntx * (unsigned)a.nty;
    timer_begin(timer, KIND_LOCAL, st);
    k_local<D><<<ntiles, NT, 0, st>>>(a, ws);
    timer_end(timer, KIND_LOCAL, st);
    if (local_only) {
        timer_begin(timer, KIND_FINAL, st);
        k_final<D, true><<<ntiles, NT, 0, st>>>(a, ws);
        timer_end(timer, KIND_FINAL, st);
        return hipGetLastError();
    }
    const int64_t items = (int64_t)(a.nty - 1) * a.W + (int64_t)(a.ntx - 1) * a.H;
    if (items > 0) {
        timer_begin(timer, KIND_SEAM, st);
        k_seam<D><<<(unsigned)((items + 255) / 256), 256, 0, st>>>(a, ws);
        timer_end(timer, KIND_SEAM, st);
    }
    timer_begin(timer, KIND_FINAL, st);
    k_final<D, false><<<ntiles, NT, 0, st>>>(a, ws);
    timer_end(timer, KIND_FINAL, st);
    return hipGetLastError();
}

hipError_t launch_label(const ImageArgs& a, const Workspace& ws, hipStream_t st,
                        KernelTimer* timer, bool local_only)
{
    if (a.conn == 8) return launch_all<1>(a, ws, st, timer, local_only);
    return launch_all<0>(a, ws, st, timer, local_only);
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

}  // namespace ccl
