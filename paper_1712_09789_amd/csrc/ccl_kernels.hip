// Block-based coarse-to-fine connected-components labelling for gfx950.
//
// The image is cut into tiles of TW x TH pixels (TW = 64: one 64-bit mask
// word per tile row).  One workgroup of TH threads owns a tile, one lane per
// tile row, so the row-scan work of the paper's local step becomes bit
// arithmetic on that lane's word.
//
// Three kernels per image (Section 3 of the paper):
//   k_local  (Section 3.1)  load the tile, label it in LDS, and publish what
//            the merge needs: the foreground bitmask, one node id per border
//            pixel, and one forest node per tile-local component that touches
//            the tile border.
//   k_seam   (Section 3.2)  for every foreground pair straddling a tile seam,
//            unite the two components' forest nodes in HBM (atomicMin).
//   k_final  (Section 3.3)  relabel the tile from its bitmask (the local
//            labelling is recomputed instead of stored), look up the global
//            root of each border-touching component, and write every label
//            exactly once.
//
// Labels are canonical: 1 + the smallest raster position of the component.
// Inside a tile the root of a component is its smallest local position
// (links always point the larger root at the smaller), which is also its
// smallest raster position because both orders are row-major.  Across tiles
// the forest orders roots by that raster position (the key).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ccl_kernels.h"

namespace ccl {

// ---------------------------------------------------------------------------
// bit helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int ctz64(uint64_t v) { return __builtin_ctzll(v); }
__device__ __forceinline__ int ctz64_or64(uint64_t v) { return v ? __builtin_ctzll(v) : 64; }
__device__ __forceinline__ int msb64(uint64_t v) { return 63 - __builtin_clzll(v); }

// Bits lo..hi (inclusive), 0 <= lo <= hi <= 63.
__device__ __forceinline__ uint64_t span_mask(int lo, int hi)
{
    return (~0ull << lo) & (~0ull >> (63 - hi));
}

// Start of the run that contains foreground bit x of a row, given the row's
// run-start mask: the highest start bit at or below x.
__device__ __forceinline__ int run_start(uint64_t starts, int x)
{
    return msb64(starts & ((2ull << x) - 1ull));
}

// Nonzero bytes of a dword -> 4-bit mask (bit i = byte i != 0).
__device__ __forceinline__ uint32_t nz_nibble(uint32_t d)
{
    uint32_t t = (((d & 0x7f7f7f7fu) + 0x7f7f7f7fu) | d) >> 7;
    return ((t & 0x01010101u) * 0x01020408u) >> 24;
}

// ---------------------------------------------------------------------------
// LDS union-find over tile positions (32-bit parents, parent <= self)
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t lds_ld(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Root of x, halving the path on the way (every write stores an ancestor,
// which is smaller than the node, so no cycle can form).
__device__ uint32_t lds_find(uint32_t* P, uint32_t x)
{
    while (true) {
        uint32_t p = lds_ld(P + x);
        if (p == x) return x;
        uint32_t gp = lds_ld(P + p);
        if (gp == p) return p;
        lds_st(P + x, gp);
        x = gp;
    }
}

// The paper's merge (Section 3.1.3): compare the two roots and point the
// larger at the smaller, atomically; if the larger stopped being a root in
// the meantime, continue with the parent it had.
__device__ void lds_union(uint32_t* P, uint32_t a, uint32_t b)
{
    while (true) {
        a = lds_find(P, a);
        b = lds_find(P, b);
        if (a == b) return;
        if (a < b) { uint32_t t = a; a = b; b = t; }
        uint32_t old = __hip_atomic_fetch_min(P + a, b, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old == a) return;
        a = old;
    }
}

// ---------------------------------------------------------------------------
// HBM forest over border components.  Entry = (key of parent << 32) | parent
// node; a root stores its own key and id.  Keys (raster position of a tile's
// local root) are distinct across components, so ordering by the packed
// value orders by key: atomicMin on it only ever moves a parent to a smaller
// key, the global analogue of "larger root points at the smaller".
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
        uint64_t self = ((uint64_t)ra.key << 32) | ra.node;
        uint64_t nv = ((uint64_t)rb.key << 32) | rb.node;
        uint64_t old = __hip_atomic_fetch_min(F + ra.node, nv, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
        if (old == self) return;
        a = (uint32_t)old;
        b = rb.node;
    }
}

// ---------------------------------------------------------------------------
// tile-local labelling (shared by k_local and k_final)
// ---------------------------------------------------------------------------

template <int TH>
struct TileShared {
    uint32_t P[TW * TH];  // parent of each run start (position y*TW + x)
    uint64_t M[TH];       // foreground mask per tile row
    uint64_t S[TH];       // run-start mask per tile row
    int32_t slot_lr[2 * TW + 2 * TH];  // local root of each border slot, -1 = bg
    union {
        uint16_t h[TH * 4];  // 16-pixel masks as produced by the byte load
        uint64_t w[TH];      // the same bits as one word per row
    } m16;
};

// Column connection, unification, refinement and the final flatten of the
// local step (Section 3.1.2-3.1.3), at run granularity.  On entry M and S
// hold the tile's masks; on exit P[y*TW + a] is the local root for every run
// start a of every row y.  D is the neighbourhood reach across rows:
// 0 for 4-connectivity, 1 for 8-connectivity (diagonals).
template <int TH, int D>
__device__ void label_tile(TileShared<TH>& sh, int y)
{
    const uint64_t m = sh.M[y];
    const uint64_t s = sh.S[y];
    const uint64_t mu = y > 0 ? sh.M[y - 1] : 0ull;
    const uint64_t su = y > 0 ? sh.S[y - 1] : 0ull;
    const uint32_t row = (uint32_t)y * TW;

    // Coarse column connection: each run records the lowest label among its
    // neighbours in the row above, i.e. the run holding the leftmost
    // neighbouring pixel there; a run with no such neighbour is a root.
    for (uint64_t r = s; r; r &= r - 1) {
        int a = ctz64(r);
        int b = a + ctz64_or64(~(m >> a)) - 1;
        uint64_t u = mu & span_mask(a > D ? a - D : 0, b + D < 63 ? b + D : 63);
        uint32_t p = row + a;
        if (u) p = row - TW + run_start(su, ctz64(u));
        sh.P[row + a] = p;
    }
    __syncthreads();

    // Label-equivalence unification: flatten every run to its current root.
    for (uint64_t r = s; r; r &= r - 1) {
        uint32_t i = row + ctz64(r);
        lds_st(sh.P + i, lds_find(sh.P, i));
    }
    __syncthreads();

    // Refinement: every run of the row above is united with the run holding
    // the leftmost neighbouring pixel in this row.  Together with the coarse
    // links (leftmost neighbour above each run) this covers every adjacency
    // between the two rows: if runs A (this row) and B (above) touch but
    // neither is the other's leftmost neighbour, then A's leftmost neighbour
    // B' and B's leftmost neighbour A' lie further left and touch each other,
    // so A - B' - A' - B is already connected by induction.
    for (uint64_t r = su; r; r &= r - 1) {
        int c = ctz64(r);
        int e = c + ctz64_or64(~(mu >> c)) - 1;
        uint64_t u = m & span_mask(c > D ? c - D : 0, e + D < 63 ? e + D : 63);
        if (u) lds_union(sh.P, row - TW + c, row + run_start(s, ctz64(u)));
    }
    __syncthreads();

    for (uint64_t r = s; r; r &= r - 1) {
        uint32_t i = row + ctz64(r);
        lds_st(sh.P + i, lds_find(sh.P, i));
    }
    __syncthreads();
}

// Border slot s -> tile-local (x, y).  Slots: top row, bottom row, left
// column, right column.
template <int TH>
__device__ __forceinline__ void slot_xy(int s, int& x, int& y)
{
    if (s < TW) { x = s; y = 0; }
    else if (s < 2 * TW) { x = s - TW; y = TH - 1; }
    else if (s < 2 * TW + TH) { x = 0; y = s - 2 * TW; }
    else { x = TW - 1; y = s - 2 * TW - TH; }
}

// Local root of every border slot into sh.slot_lr (-1 for background).
template <int TH>
__device__ void border_roots(TileShared<TH>& sh, int lane)
{
    constexpr int NS = 2 * TW + 2 * TH;
    for (int s = lane; s < NS; s += TH) {
        int x, y;
        slot_xy<TH>(s, x, y);
        int32_t lr = -1;
        if ((sh.M[y] >> x) & 1ull)
            lr = (int32_t)lds_ld(sh.P + y * TW + run_start(sh.S[y], x));
        sh.slot_lr[s] = lr;
    }
}

// ---------------------------------------------------------------------------
// k_local
// ---------------------------------------------------------------------------

template <int TH, int D>
__global__ __launch_bounds__(TH) void k_local(ImageArgs a, Workspace ws)
{
    constexpr int NS = 2 * TW + 2 * TH;
    __shared__ TileShared<TH> sh;
    const int lane = threadIdx.x;
    const int t = blockIdx.x;
    const int tx = t % a.ntx, ty = t / a.ntx;
    const int gx0 = tx * TW, gy0 = ty * TH;

    // Initialisation: load the tile's bytes, four lanes per row, sixteen
    // pixels per lane, and turn them into foreground bits.
    for (int c = lane; c < TH * 4; c += TH) {
        int r = c >> 2, q = c & 3;
        int gy = gy0 + r, gx = gx0 + 16 * q;
        uint32_t bits = 0;
        if (gy < a.H && gx < a.W) {
            const uint8_t* src = a.img + (int64_t)gy * a.pitch + gx;
            if (a.vec_in && gx + 16 <= a.W) {
                uint4 v = *reinterpret_cast<const uint4*>(src);
                bits = nz_nibble(v.x) | (nz_nibble(v.y) << 4) |
                       (nz_nibble(v.z) << 8) | (nz_nibble(v.w) << 12);
            } else {
                int n = a.W - gx < 16 ? a.W - gx : 16;
                for (int i = 0; i < n; ++i) bits |= (uint32_t)(src[i] != 0) << i;
            }
        }
        sh.m16.h[c] = (uint16_t)bits;
    }
    __syncthreads();
    {
        const uint64_t m = sh.m16.w[lane];
        sh.M[lane] = m;
        sh.S[lane] = m & ~(m << 1);
        ws.bits[(int64_t)t * TH + lane] = m;
    }
    __syncthreads();

    label_tile<TH, D>(sh, lane);

    border_roots<TH>(sh, lane);
    __syncthreads();

    // Elect one representative border slot per component (the smallest slot
    // index) by an atomic max on the root's entry; root entries are no
    // longer needed as parents.
    constexpr uint32_t REP = 0x40000000u;
    for (int s = lane; s < NS; s += TH) {
        int32_t lr = sh.slot_lr[s];
        if (lr >= 0)
            __hip_atomic_fetch_max(sh.P + lr, REP | (uint32_t)(NS - 1 - s),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();

    // ID conversion (Section 3.1.4) for border components: the node of the
    // representative slot carries the raster position of the local root.
    const int64_t base = (int64_t)t * NS;
    for (int s = lane; s < NS; s += TH) {
        int32_t lr = sh.slot_lr[s];
        int32_t node = -1;
        if (lr >= 0) {
            int rep = NS - 1 - (int)(lds_ld(sh.P + lr) & ~REP);
            node = (int32_t)(base + rep);
            if (rep == s) {
                uint32_t key = (uint32_t)((gy0 + lr / TW) * (int64_t)a.W + gx0 + lr % TW);
                ws.forest[node] = ((uint64_t)key << 32) | (uint32_t)node;
            }
        }
        ws.slots[base + s] = node;
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
template <int TH, int D>
__global__ __launch_bounds__(256) void k_seam(ImageArgs a, Workspace ws)
{
    constexpr int NS = 2 * TW + 2 * TH;
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
        const int k = y / TH, yl = y - k * TH;
        const int64_t left = ((int64_t)k * a.ntx + j - 1) * NS + 2 * TW + TH;
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

// Update of the global label map (Section 3.3).  The tile's local labelling
// is rebuilt from the bitmask k_local stored; each border component takes the
// key of its global root, every other component keeps its own local root; a
// label is written once per pixel.  With LOCAL_ONLY the global lookup is
// skipped (every tile labelled as a separate image).
template <int TH, int D, bool LOCAL_ONLY>
__global__ __launch_bounds__(TH) void k_final(ImageArgs a, Workspace ws)
{
    constexpr int NS = 2 * TW + 2 * TH;
    constexpr uint32_t FIN = 0x80000000u;  // entry holds a final label
    __shared__ TileShared<TH> sh;
    const int lane = threadIdx.x;
    const int t = blockIdx.x;
    const int tx = t % a.ntx, ty = t / a.ntx;
    const int gx0 = tx * TW, gy0 = ty * TH;

    {
        const uint64_t m = ws.bits[(int64_t)t * TH + lane];
        sh.M[lane] = m;
        sh.S[lane] = m & ~(m << 1);
    }
    __syncthreads();

    label_tile<TH, D>(sh, lane);

    if (!LOCAL_ONLY) {
        border_roots<TH>(sh, lane);
        __syncthreads();
        // the representative slot of each border component looks up its root
        const int64_t base = (int64_t)t * NS;
        for (int s = lane; s < NS; s += TH) {
            int32_t lr = sh.slot_lr[s];
            if (lr >= 0 && ws.slots[base + s] == (int32_t)(base + s)) {
                Root r = g_find_ro(ws.forest, (uint32_t)(base + s));
                lds_st(sh.P + lr, FIN | (r.key + 1u));
            }
        }
        __syncthreads();
    }

    // roots of components that stay inside the tile: ID conversion of the
    // local root (Section 3.1.4)
    const uint64_t m = sh.M[lane], s = sh.S[lane];
    const uint32_t row = (uint32_t)lane * TW;
    for (uint64_t r = s; r; r &= r - 1) {
        const uint32_t i = row + ctz64(r);
        if (lds_ld(sh.P + i) == i)
            lds_st(sh.P + i, FIN | (uint32_t)((gy0 + lane) * (int64_t)a.W + gx0 + (int)(i - row) + 1));
    }
    __syncthreads();
    // every other run start copies its root's final label
    for (uint64_t r = s; r; r &= r - 1) {
        const uint32_t i = row + ctz64(r);
        const uint32_t v = lds_ld(sh.P + i);
        if (!(v & FIN)) lds_st(sh.P + i, lds_ld(sh.P + v));
    }
    __syncthreads();
    (void)m;

    // write the labels: 16 lanes per tile row, 4 pixels per lane
    const int xmax = a.W - gx0;  // pixels of this tile inside the image
    for (int c = lane; c < TH * 16; c += TH) {
        const int r = c >> 4, q = c & 15;
        const int gy = gy0 + r;
        const int x0 = q * 4;
        if (gy >= a.H || x0 >= xmax) continue;
        const uint64_t mr = sh.M[r], sr = sh.S[r];
        int32_t v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int x = x0 + k;
            v[k] = ((mr >> x) & 1ull)
                       ? (int32_t)(lds_ld(sh.P + r * TW + run_start(sr, x)) & ~FIN)
                       : 0;
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

template <int TH, int D>
static hipError_t launch_all(const ImageArgs& a, const Workspace& ws, hipStream_t st,
                             KernelTimer* timer, bool local_only)
{
    const unsigned ntiles = (unsigned)a.ntx * (unsigned)a.nty;
    timer_begin(timer, KIND_LOCAL, st);
    k_local<TH, D><<<ntiles, TH, 0, st>>>(a, ws);
    timer_end(timer, KIND_LOCAL, st);
    if (local_only) {
        timer_begin(timer, KIND_FINAL, st);
        k_final<TH, D, true><<<ntiles, TH, 0, st>>>(a, ws);
        timer_end(timer, KIND_FINAL, st);
        return hipGetLastError();
    }
    const int64_t items = (int64_t)(a.nty - 1) * a.W + (int64_t)(a.ntx - 1) * a.H;
    if (items > 0) {
        timer_begin(timer, KIND_SEAM, st);
        k_seam<TH, D><<<(unsigned)((items + 255) / 256), 256, 0, st>>>(a, ws);
        timer_end(timer, KIND_SEAM, st);
    }
    timer_begin(timer, KIND_FINAL, st);
    k_final<TH, D, false><<<ntiles, TH, 0, st>>>(a, ws);
    timer_end(timer, KIND_FINAL, st);
    return hipGetLastError();
}

hipError_t launch_label(const ImageArgs& a, const Workspace& ws, hipStream_t st,
                        KernelTimer* timer, bool local_only)
{
    if (a.conn == 8) return launch_all<TILE_ROWS, 1>(a, ws, st, timer, local_only);
    return launch_all<TILE_ROWS, 0>(a, ws, st, timer, local_only);
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
