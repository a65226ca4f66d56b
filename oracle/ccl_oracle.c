/*
 * Connected-components labelling oracle — TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain, slow, obviously correct CPU definition that the
 * GPU path is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product library never
 * links, includes or calls it, and it shares no code with the GPU path.
 *
 * What it computes (the problem statement of the paper, Section 3 "Algorithm
 * and implementation", first paragraph, with the pixel position defined as
 * P(x, y) = x + y * W):
 *
 *   fg(x, y)   = img[y * pitch + x] != 0        (the paper's I(x, y) = 1)
 *   G          = graph on fg pixels; edges join 4-neighbours (|dx|+|dy| = 1)
 *                or 8-neighbours (max(|dx|, |dy|) = 1)
 *   L(x, y)    = 0 for background, otherwise
 *                1 + min { P(x', y') : (x', y') in the component of (x, y) }
 *
 * The paper's own labels are the position of the root of each equivalence
 * list; provisional labels are positions (Section 3.1.1), every link points
 * the larger root at the smaller one (Section 3.1.3 and Section 3.2), so the
 * root is the minimum position of the component.  The "+1" keeps 0 free for
 * background.
 *
 * Algorithm: the classical two-pass union-find.
 *   pass 1, raster order: every fg pixel starts as its own set; it is united
 *           with each already-visited fg neighbour (left, up; for
 *           8-connectivity also up-left and up-right);
 *   union:  find both roots; the larger root is pointed at the smaller one,
 *           so every root is the minimum position of its set;
 *   find:   follows parents to the self-pointing root, then compresses the
 *           path it walked;
 *   pass 2: L = 1 + find(p) for fg, 0 for bg.
 *
 * Parity pins: exhaustive brute-force flood fill on every image up to 4x4,
 * scipy.ndimage.label on random images, closed forms (checkerboard, stripes,
 * spirals, serpentines, empty, full) and label-form invariants — see the
 * oracle tests.
 */
#include <stdint.h>
#include <stdlib.h>

#define ORACLE_OK 0
#define ORACLE_ERR_ARG -1
#define ORACLE_ERR_MEM -3

static int64_t find_root(int64_t* parent, int64_t p)
{
    int64_t r = p;
    while (parent[r] != r) r = parent[r];
    /* path compression: point every node on the walked path at the root */
    while (parent[p] != r) {
        int64_t next = parent[p];
        parent[p] = r;
        p = next;
    }
    return r;
}

static void unite(int64_t* parent, int64_t a, int64_t b)
{
    int64_t ra = find_root(parent, a);
    int64_t rb = find_root(parent, b);
    if (ra == rb) return;
    if (ra < rb) parent[rb] = ra;
    else parent[ra] = rb;
}

/*
 * Label one H x W image whose row y starts at img + y * pitch (bytes).
 * out is a dense H x W int32 array (row stride W).  Returns 0 on success.
 */
int oracle_label(const uint8_t* img, int64_t H, int64_t W, int64_t pitch,
                 int32_t connectivity, int32_t* out)
{
    if (H < 0 || W < 0) return ORACLE_ERR_ARG;
    if (connectivity != 4 && connectivity != 8) return ORACLE_ERR_ARG;
    if (H == 0 || W == 0) return ORACLE_OK;
    if (img == NULL || out == NULL || pitch < W) return ORACLE_ERR_ARG;
    if (H * W > (int64_t)INT32_MAX) return ORACLE_ERR_ARG;

    int64_t n = H * W;
    int64_t* parent = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    if (parent == NULL) return ORACLE_ERR_MEM;

    /* pass 1 */
    for (int64_t y = 0; y < H; ++y) {
        for (int64_t x = 0; x < W; ++x) {
            int64_t p = y * W + x;
            parent[p] = p;
            if (img[y * pitch + x] == 0) continue;
            if (x > 0 && img[y * pitch + x - 1] != 0) unite(parent, p, p - 1);
            if (y > 0) {
                if (img[(y - 1) * pitch + x] != 0) unite(parent, p, p - W);
                if (connectivity == 8) {
                    if (x > 0 && img[(y - 1) * pitch + x - 1] != 0)
                        unite(parent, p, p - W - 1);
                    if (x + 1 < W && img[(y - 1) * pitch + x + 1] != 0)
                        unite(parent, p, p - W + 1);
                }
            }
        }
    }

    /* pass 2 */
    for (int64_t y = 0; y < H; ++y) {
        for (int64_t x = 0; x < W; ++x) {
            int64_t p = y * W + x;
            out[p] = img[y * pitch + x] != 0 ? (int32_t)(find_root(parent, p) + 1) : 0;
        }
    }
    free(parent);
    return ORACLE_OK;
}

/*
 * Volumes.  The paper's introduction names 2-D and 3-D images as the inputs
 * of connected-components labelling; the definition carries over with the
 * voxel position P(x, y, z) = x + y * W + z * W * H:
 *
 *   fg(x, y, z) = vol[z * slice_pitch + y * pitch + x] != 0
 *   6-connectivity:  face neighbours        (|dx| + |dy| + |dz| = 1)
 *   26-connectivity: the 3 x 3 x 3 block    (max(|dx|, |dy|, |dz|) = 1)
 *   L = 0 for background, otherwise 1 + the smallest position in the
 *       component.
 *
 * Same two passes as above: in raster order (z, then y, then x) each fg voxel
 * is united with its already-visited fg neighbours (6: left, up, previous
 * slice; 26: left, the three voxels of the row above, and the nine voxels of
 * the previous slice), the larger root pointing at the smaller.
 */
int oracle_label3d(const uint8_t* vol, int64_t D, int64_t H, int64_t W, int64_t pitch,
                   int64_t slice_pitch, int32_t connectivity, int32_t* out)
{
    if (D < 0 || H < 0 || W < 0) return ORACLE_ERR_ARG;
    if (connectivity != 6 && connectivity != 26) return ORACLE_ERR_ARG;
    if (D == 0 || H == 0 || W == 0) return ORACLE_OK;
    if (vol == NULL || out == NULL || pitch < W || slice_pitch < (H - 1) * pitch + W)
        return ORACLE_ERR_ARG;
    if (D * H * W > (int64_t)INT32_MAX) return ORACLE_ERR_ARG;

    const int64_t n = D * H * W, S = H * W;
    int64_t* parent = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    if (parent == NULL) return ORACLE_ERR_MEM;
#define FG(x, y, z) (vol[(z) * slice_pitch + (y) * pitch + (x)] != 0)

    /* pass 1 */
    for (int64_t z = 0; z < D; ++z) {
        for (int64_t y = 0; y < H; ++y) {
            for (int64_t x = 0; x < W; ++x) {
                const int64_t p = z * S + y * W + x;
                parent[p] = p;
                if (!FG(x, y, z)) continue;
                if (connectivity == 6) {
                    if (x > 0 && FG(x - 1, y, z)) unite(parent, p, p - 1);
                    if (y > 0 && FG(x, y - 1, z)) unite(parent, p, p - W);
                    if (z > 0 && FG(x, y, z - 1)) unite(parent, p, p - S);
                    continue;
                }
                if (x > 0 && FG(x - 1, y, z)) unite(parent, p, p - 1);
                if (y > 0) {
                    for (int64_t dx = -1; dx <= 1; ++dx) {
                        const int64_t xx = x + dx;
                        if (xx >= 0 && xx < W && FG(xx, y - 1, z)) unite(parent, p, p - W + dx);
                    }
                }
                if (z > 0) {
                    for (int64_t dy = -1; dy <= 1; ++dy) {
                        const int64_t yy = y + dy;
                        if (yy < 0 || yy >= H) continue;
                        for (int64_t dx = -1; dx <= 1; ++dx) {
                            const int64_t xx = x + dx;
                            if (xx >= 0 && xx < W && FG(xx, yy, z - 1))
                                unite(parent, p, p - S + dy * W + dx);
                        }
                    }
                }
            }
        }
    }

    /* pass 2 */
    for (int64_t z = 0; z < D; ++z)
        for (int64_t y = 0; y < H; ++y)
            for (int64_t x = 0; x < W; ++x) {
                const int64_t p = z * S + y * W + x;
                out[p] = FG(x, y, z) ? (int32_t)(find_root(parent, p) + 1) : 0;
            }
#undef FG
    free(parent);
    return ORACLE_OK;
}
