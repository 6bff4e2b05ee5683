/*
 * hfr.h -- C ABI of the MI355X heightfield renderer library (libhfr.so).
 *
 * The library implements the per-frame path of the two-step adaptive
 * heightfield renderer of Cornel, Horvath and Waser (2022): a truncated
 * Gaussian approximation of an adaptive (quadtree) heightfield is
 * discretized into view-dependent cascade textures, a maximum mipmap is
 * built over each cascade, and every pixel is ray cast against the
 * bilinear patches of the textures.  Gradients of the hit depth with
 * respect to the leaf heights and Gaussian widths are provided as well.
 *
 * Conventions for every entry point:
 *  - Arguments are validated on the host before anything is launched; an
 *    invalid argument returns HFR_EINVAL and launches nothing.
 *  - A non-zero status leaves a message for hfr_last_error() (per thread,
 *    valid until the next call on that thread).  No C++ exception and no
 *    abort crosses the ABI.
 *  - "device" pointers are gfx950 device memory owned by the caller,
 *    contiguous, naturally aligned.  "host" pointers are ordinary host
 *    memory owned by the caller.  The library keeps no pointer after a
 *    call returns; hfr_quadtree and hfr_neighbours objects own copies.
 *  - Device work is enqueued on the given stream (a hipStream_t; NULL is
 *    the null stream) and the call returns without synchronising; it
 *    allocates no device memory, so it may be captured into a HIP graph.
 *    Launch failures return HFR_EDEVICE.
 *  - Coordinates: world x east, y north, z up, metres.  Textures are
 *    row-major [k][j][i] with j the row (y) and i the column (x); texel
 *    (i, j) of cascade k sits at (x0 + i hx, y0 + j hy).  Images are
 *    row-major [row][col] with row 0 at the top.
 */
#ifndef HFR_H
#define HFR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HFR_ABI_VERSION 13
#define HFR_MAX_POLY 32
#define HFR_MAX_CASCADES 8
#define HFR_MAX_TEX_N 8192
#define HFR_MAX_SURFACES 4
#define HFR_HIT_LIMIT (-2) /* hit word of a ray stopped by the walk's iteration cap */

typedef int32_t hfr_status;
enum {
    HFR_OK = 0,
    HFR_EINVAL = -1,       /* invalid argument, nothing launched */
    HFR_ENOMEM = -2,       /* host allocation failed */
    HFR_EDEVICE = -3,      /* HIP runtime or launch error */
    HFR_ECAPACITY = -4,    /* an output does not fit the space given */
    HFR_EUNSUPPORTED = -5  /* valid but not supported by this build */
};

typedef void* hfr_stream; /* hipStream_t */

/* Pinhole camera (the paper casts one ray per pixel, Section 5; the model
 * itself is not stated there).  Forward is
 * (sin yaw cos pitch, cos yaw cos pitch, sin pitch); yaw 0 looks along +y,
 * pitch < 0 looks down; right = (cos yaw, -sin yaw, 0); up = right x forward.
 * Pixel (col, row) is sampled at its centre, the image spans tan(vfov/2)
 * vertically and tan(vfov/2) * width / height horizontally.  Rays have unit
 * length, so depth is Euclidean distance.  znear bounds the frustum used
 * for cascade fitting. */
typedef struct {
    double pos[3];
    double yaw, pitch, vfov;
    int32_t width, height;
    double znear;
} hfr_camera;

/* Heightfield bounding box: the domain rectangle and the z-range of the
 * leaf values (Eq. 2 is a convex combination, so the surface stays inside). */
typedef struct {
    double x0, y0, x1, y1, zmin, zmax;
} hfr_domain;

/* One cascade (Section 3).  The offset of a point p is
 * d(p) = (p - origin) . vhat.  The cascade covers near_d <= d <= far_d;
 * split_d is the split distance s_k, and the overlap with the next cascade
 * is split_d <= d <= far_d (for the last cascade split_d == far_d).  The
 * N x N texture maps texel (i, j) to (x0 + i hx, y0 + j hy); poly is the
 * convex cascade polygon (counter-clockwise, n_poly vertices, possibly 0). */
typedef struct {
    double near_d, far_d, split_d;
    double origin[2], vhat[2];
    double x0, y0, hx, hy;
    int32_t n, n_poly;
    double poly[HFR_MAX_POLY][2];
} hfr_cascade;

/* Leaves of the adaptive grid on the device (all pointers device memory,
 * caller-owned).  The leaves lie on the quadtree lattice of the square
 * [x0, x0 + side] x [y0, y0 + side], levels 0 .. max_depth.
 *  x, y, c, v, sigma : float[n]   centre, cell size, value, Gaussian width
 *                                 (in units of the cell size)
 *  packed            : float[4n]  (x, y, v, s) per leaf in level-index order
 *                                 (packed[p] is leaf order[p]), written by
 *                                 hfr_pack_leaves; s = sqrt(log2(e) / 2) / (sigma c),
 *                                 so that Eq. 1's Gaussian is exp2(-(s r)^2)
 *                                 (HFR_BASIS_WENDLAND: s = 1 / (cutoff sigma c))
 *  level_radius      : float[max_depth + 1], written by hfr_pack_leaves: the
 *                      largest truncation radius cutoff * sigma_j * c_j of the
 *                      leaves of each level (0 where a level has none)
 *  rank, order       : the level index written by hfr_build_level_index (host
 *                      arrays copied to the device); packed is stored in the
 *                      order it defines
 *  cutoff            : truncation radius in units of sigma (the paper's 3.5)
 *  basis             : the weight function in Eq. 2 (HFR_BASIS_*); the packed
 *                      records hold the scale of the basis they were packed for
 *  status            : device int32 or NULL, written by hfr_pack_leaves: HFR_OK,
 *                      or HFR_EINVAL when some leaf has cutoff sigma <= sqrt(2)/2
 *                      (Eq. 2's sum may then be empty where that leaf's cell is
 *                      the only one near: its own reach no longer covers its
 *                      square) or a non-finite value or width
 */
#define HFR_BASIS_GAUSSIAN 0 /* Eq. 1: truncated Gaussian minus its value at the cutoff */
/* Wendland's compactly supported C2 function (1 - u)^4 (4u + 1), u = r / (cutoff
 * sigma c), 0 for u >= 1: the same support as the truncated Gaussian, so the same
 * leaves influence the same texels.  The two-step design of Section 1 admits any
 * reconstruction in the discretization; this one needs no truncation constant. */
#define HFR_BASIS_WENDLAND 1
typedef struct {
    int64_t n;
    const float* x;
    const float* y;
    const float* c;
    const float* v;
    const float* sigma;
    float* packed;
    float* level_radius;
    const int32_t* rank;
    const int32_t* order;
    int32_t max_depth;
    float cutoff;
    double x0, y0, side;
    int32_t basis;
    int32_t* status;
} hfr_leaves;

/* ------------------------------------------------------------------ misc */

int hfr_abi_version(void);
const char* hfr_last_error(void);
/* HIP runtime version the library runs on (hipRuntimeGetVersion). */
hfr_status hfr_runtime_version(int* version);

/* ------------------------------------------------------------ start-up (host) */

typedef struct hfr_quadtree hfr_quadtree;

/* Adaptive quadtree over a square raster (the adaptive grid of Section 2;
 * the paper takes it from a simulation and does not state a refinement
 * rule).  dem: host float[n * n], row-major (row = y), n a power of two,
 * samples at cell centres of a raster spanning [x0, x0 + side] x [y0, y0 + side].
 * Level-l means are 2x2 averages ((a + b) + (c + d)) * 0.25 in FP64; a node
 * at level l < max_depth splits when the largest |second difference| (x or
 * y, edges replicated) of the level l + 1 means under it exceeds tau.  Leaves
 * are listed depth-first with children (0,0), (1,0), (0,1), (1,1).
 * Output: a library-owned object freed with hfr_quadtree_destroy.
 * EINVAL: n not a power of two, max_depth outside [0, log2 n], side <= 0,
 * non-finite samples.  Host only, synchronous. */
hfr_status hfr_build_quadtree(const float* dem, int64_t n, double side, double x0, double y0,
                              int32_t max_depth, double tau, hfr_quadtree** out);
hfr_status hfr_quadtree_size(const hfr_quadtree* q, int64_t* n_leaves);
/* Writes n_leaves entries to each non-NULL host array: centre (x, y), size c,
 * mean value v (FP32), and the integer node (level, i, j). */
hfr_status hfr_quadtree_export(const hfr_quadtree* q, float* x, float* y, float* c, float* v,
                               int32_t* level, int32_t* i, int32_t* j);
void hfr_quadtree_destroy(hfr_quadtree* q);

/* Per-leaf lists of potentially influencing leaves (Section 4: the set I
 * depends only on the grid and is precomputed at start-up).  Leaf j is in
 * the list of leaf i iff dist(p_j, square_i)^2 < ((cutoff sigma_j) c_j (1 + slack))^2
 * (FP64 on the FP32 inputs), so every j with w_j(p) > 0 for some p in
 * square i is listed (Eq. 1).  Leaves must lie on the quadtree lattice of
 * the square [x0, x0 + side] x [y0, y0 + side] with at most max_depth
 * levels.  Host arrays x, y, c, sigma of n leaves.  Lists are sorted by
 * leaf index.  Output: a library-owned object freed with
 * hfr_neighbours_destroy.  EINVAL: off-lattice leaves, cutoff <= 0,
 * slack < 0.  ECAPACITY: more than INT32_MAX entries, which the 32-bit
 * offsets of hfr_neighbours_export cannot address (the device builder's
 * offsets are 64-bit).  Host only, multi-threaded. */
typedef struct hfr_neighbours hfr_neighbours;
hfr_status hfr_build_neighbours(int64_t n, const float* x, const float* y, const float* c,
                                const float* sigma, double x0, double y0, double side,
                                int32_t max_depth, float cutoff, float slack, hfr_neighbours** out);
hfr_status hfr_neighbours_size(const hfr_neighbours* nb, int64_t* nnz);
/* Writes host off[n + 1] (CSR offsets) and idx[nnz] (leaf indices). */
hfr_status hfr_neighbours_export(const hfr_neighbours* nb, int32_t* off, int32_t* idx);
void hfr_neighbours_destroy(hfr_neighbours* nb);

/* The same quadtree built on the device (Section 2's adaptive grid, which the
 * paper builds at start-up; on the device it can follow a raster that changes,
 * such as simulation output).  Decisions are hfr_build_quadtree's, in the same
 * FP64 arithmetic, so the leaves are the same set; they come out sorted by
 * (level, row, column), i.e. already in level-index order (order = 0 .. n-1).
 * Two calls: hfr_build_quadtree_device classifies every lattice node, writes
 * the level index (rank, as hfr_build_level_index) and returns the leaf count
 * (it synchronizes the stream to read it); hfr_quadtree_device_leaves then
 * writes the leaves.  dem: device float[n][n], n a power of two <= 32768.
 * work: device scratch of hfr_quadtree_device_workspace bytes (the FP64 mean
 * pyramid and flags; read again by the second call).  rank: device
 * int32[(4^(max_depth+1) - 1) / 3 + max_depth + 1].  x, y, c, v: device
 * float[n_leaves]; level, i, j: device int32[n_leaves] or NULL.  EINVAL: as
 * hfr_build_quadtree's argument checks, max_depth > 15, NULL pointers; the
 * samples themselves are not checked on the device (a non-finite sample makes
 * the means above it NaN, and a NaN criterion never splits).  The caller
 * owns every buffer. */
hfr_status hfr_quadtree_device_workspace(int64_t n, int32_t max_depth, int64_t* bytes);
hfr_status hfr_build_quadtree_device(const float* dem, int64_t n, double side, double x0, double y0,
                                     int32_t max_depth, double tau, void* work, int32_t* rank,
                                     int64_t* n_leaves, hfr_stream stream);
hfr_status hfr_quadtree_device_leaves(int64_t n, double side, double x0, double y0, int32_t max_depth,
                                      const void* work, const int32_t* rank, int64_t n_leaves, float* x,
                                      float* y, float* c, float* v, int32_t* level, int32_t* i, int32_t* j,
                                      hfr_stream stream);

/* The per-leaf lists of hfr_build_neighbours built on the device, for leaves
 * already on the device with their level index and level radii (L->x, y, c,
 * sigma, rank, order, level_radius after hfr_pack_leaves; L->v and
 * L->packed are not read).  Lists are indexed by sorted position: list p
 * belongs to leaf order[p] and holds the sorted positions q (ascending) of
 * the leaves order[q] in it, under the same FP64 test as
 * hfr_build_neighbours.  For leaves from hfr_quadtree_device_leaves (order =
 * 0 .. n-1) positions are leaf indices and the lists equal
 * hfr_build_neighbours' lists of the same leaves.  Two calls:
 * hfr_build_neighbours_device writes off (device int64[n + 1], CSR offsets)
 * and returns the entry count (it synchronizes the stream to read it), using
 * work (device scratch of hfr_neighbours_device_workspace bytes);
 * hfr_neighbours_device_fill then writes idx (device int32[nnz]).  The
 * caller owns every buffer.  EINVAL: NULL pointers, n outside
 * [1, INT32_MAX], max_depth outside [0, 15], cutoff <= 0, slack < 0. */
hfr_status hfr_neighbours_device_workspace(int64_t n, int64_t* bytes);
hfr_status hfr_build_neighbours_device(const hfr_leaves* L, float slack, void* work, int64_t* off, int64_t* nnz,
                                       hfr_stream stream);
hfr_status hfr_neighbours_device_fill(const hfr_leaves* L, float slack, const int64_t* off, int32_t* idx,
                                      hfr_stream stream);

/* Level index of the leaves (host arrays).  Leaves are ordered by level,
 * then lattice row j (y), then column i (x): order[p] is the leaf at sorted
 * position p (int32[n]).  rank holds, for every level l, 4^l + 1 exclusive
 * prefix counts at offset (4^l - 1) / 3 + l (int32[(4^(max_depth+1) - 1) / 3
 * + max_depth + 1] in all): rank[off_l + j 2^l + i] is the sorted position of
 * the first level-l leaf at or after node (i, j) in row-major order (the
 * leaves of all coarser levels come first).  The level-l leaves of lattice
 * row j with columns ia..ib are therefore the sorted positions
 * [rank[off_l + j 2^l + ia], rank[off_l + j 2^l + ib + 1]), so the influencers
 * of a region are found per level and row without visiting empty nodes.
 * Same lattice requirements as hfr_build_neighbours; EINVAL if the leaves do
 * not tile the square exactly once, max_depth > 15 or n > INT32_MAX. */
hfr_status hfr_build_level_index(int64_t n, const float* x, const float* y, const float* c, double x0,
                                 double y0, double side, int32_t max_depth, int32_t* rank, int32_t* order);

/* --------------------------------------------------------- per frame (host) */

/* Cascade fitting (Section 3): frustum (near plane znear, no far plane)
 * intersected with the domain box, projected to the ground plane, convex
 * hull; n and f are the smallest and largest hull offsets along the
 * horizontal view direction; splits
 * s_k = lambda n' (f/n')^(k/K) + (1 - lambda) (n + (f - n) k / K) with
 * n' = max(n, znear, c_min) (lambda = 1, K = 3 gives the paper's
 * logarithmic splits); near_1 = n, near_{k+1} = s_k, far_k = s_k +
 * overlap (s_k - near_k), far_K = f; each polygon is the hull clipped to
 * [near_k, far_k]; its bounding box is widened to the c_min lattice and
 * to an even multiple of c_min and mapped so its corners are the corner
 * texel centres.  out: host hfr_cascade[K].
 * EINVAL: K outside [1, HFR_MAX_CASCADES], N not a power of two in
 * [2, HFR_MAX_TEX_N], horizontal view direction of zero length, non-finite
 * input, c_min <= 0, lambda outside [0, 1], overlap < 0.  A frustum that
 * misses the box yields cascades with n_poly == 0 (nothing visible). */
hfr_status hfr_fit_cascades(const hfr_camera* cam, const hfr_domain* dom, int32_t K, int32_t N,
                            double lambda, double overlap, double c_min, hfr_cascade* out);

/* The same cascades with texel lattices fixed in the world, so that texels
 * can be reused between frames (hfr_discretize_reuse; not in the paper,
 * whose stable fit of Section 3 keeps the box corners on the c_min lattice
 * but lets the texel spacing follow the box).  Polygons, near, far and
 * split are hfr_fit_cascades'; each axis's spacing h is the smallest
 * c_min 2^(e/4), e an integer, for which the lattice origin (the largest
 * whole multiple of h from the domain origin at or below the box) puts the
 * last texel centre at or beyond the box.  The spacing exceeds the stable
 * fit's by at most a factor 2^(1/4) (N - 1) / (N - 2).  Same arguments and
 * errors as hfr_fit_cascades. */
hfr_status hfr_fit_cascades_aligned(const hfr_camera* cam, const hfr_domain* dom, int32_t K, int32_t N,
                                    double lambda, double overlap, double c_min, hfr_cascade* out);

/* ------------------------------------------------------- per frame (device) */

/* Writes L->packed (each record placed at its leaf's sorted position, found
 * through L->rank) and L->level_radius from x, y, v, c, sigma and cutoff
 * (call again whenever v, sigma or basis change), and L->status when given:
 * the leaves are refused there (HFR_EINVAL) when a width is too small for
 * Eq. 2's sum to be non-empty everywhere (cutoff sigma <= sqrt(2)/2) or a
 * value or width is not finite; the widths live on the device, so the
 * verdict is a device word the caller reads once the stream has reached it.
 * EINVAL (returned) on NULL pointers, n < 1, cutoff <= 0, max_depth outside
 * [0, 15], an unknown basis. */
hfr_status hfr_pack_leaves(const hfr_leaves* L, hfr_stream stream);

/* Discretization (Section 4, Eq. 1 and Eq. 2, and the visibility texture of
 * Section 3).  For every texel of every cascade: the texel is visible when
 * one of its (up to four) incident texture cells meets the closed cascade
 * polygon; a visible texel holds
 *   v_s = sum_j w_j v_j / sum_j w_j,
 *   w_j = max(0, exp(-(|p_j - p_s| / (sigma_j c_j))^2 / 2) - exp(-cutoff^2 / 2)),
 * (HFR_BASIS_WENDLAND: w_j = (1 - u)^4 (4u + 1) for u = |p_j - p_s| /
 * (cutoff sigma_j c_j) < 1, else 0), evaluated at the texel centre clamped into the domain, summed over every
 * leaf with w_j > 0 (found per block of texels from L->rank and
 * L->level_radius); an invisible texel holds -inf.  tex: device float[K][N][N].  mask: device uint32
 * [K][N][(N + 31) / 32] visibility bits (bit i % 32 of word i / 32), or NULL.
 * A texel no leaf influences (impossible when cutoff sigma_j > sqrt(2)/2 for
 * every leaf) holds NaN.  EINVAL: cascades with different N, N outside
 * [2, HFR_MAX_TEX_N], missing leaf arrays. */
hfr_status hfr_discretize(const hfr_leaves* L, const hfr_domain* dom, const hfr_cascade* cas,
                          int32_t K, float* tex, uint32_t* mask, hfr_stream stream);

/* hfr_discretize for the next frame of a camera path, reusing the previous
 * frame's texels (not in the paper; its approximation pass is the cost it
 * names).  prev_cas: the previous frame's host cascades [K]; prev_tex: its
 * device textures [K][N][N], which must not overlap tex.  Where a cascade
 * has the same N, hx and hy as then and its origin moved by whole texels
 * (hfr_fit_cascades_aligned gives such lattices), each 16 x 16 texel block
 * whose visible texels were all visible then copies them from prev_tex
 * instead of evaluating Eq. 2; other blocks and cascades are computed as
 * hfr_discretize does.  A copied texel equals the one computed at the same
 * world position last frame, so the leaves, the basis and the domain must
 * be unchanged since prev_tex was written (the caller's responsibility).
 * reused: device int32 that each copied block increments (caller-zeroed),
 * or NULL (counting costs one atomic per copied block on that one address).  EINVAL as hfr_discretize, NULL prev_cas or prev_tex,
 * overlapping buffers. */
hfr_status hfr_discretize_reuse(const hfr_leaves* L, const hfr_domain* dom, const hfr_cascade* cas,
                                int32_t K, const hfr_cascade* prev_cas, const float* prev_tex, float* tex,
                                uint32_t* mask, int32_t* reused, hfr_stream stream);

/* Maximum mipmap (Tevs et al. 2008, used in Section 5).  Level 0 is N x N
 * by texture cell: the largest of the cell's four corner texels, -inf when
 * one is invisible, -inf on the last row and column; level l + 1 is the
 * 2x2 maximum of level l, down to 1 x 1.  mip: device float[K][(4N^2-1)/3],
 * levels finest first, each row-major.  Level 0 is not stored: its N^2 slot
 * at the start of each cascade's pyramid is left as the caller had it (the
 * ray casts form those maxima from the four texels they load for the patch
 * test); levels 1 .. log2 N are written.  tex: 16-byte aligned.  EINVAL: N
 * not a power of two in [2, HFR_MAX_TEX_N], K outside [1, HFR_MAX_CASCADES],
 * a misaligned tex. */
hfr_status hfr_build_maxmip(const float* tex, int32_t K, int32_t N, float* mip, hfr_stream stream);

/* Ray casting (Section 5).  One ray per pixel, clipped to the domain's xy
 * box and z <= zmax; the cascades are visited in the order the ray sweeps
 * their offsets; inside a cascade the ray walks the maximum mipmap and
 * stops at the first point at or below a bilinear patch of four visible
 * texels.  When that first hit A lies in the overlap with the next cascade
 * visited, that cascade is searched over the overlap only, and a hit B
 * there gives depth (1 - a) t_nearer + a t_farther with
 * a = clamp((d(t_A) - split) / (far - split), 0, 1) of the nearer cascade.
 * depth: device float[H][W], +inf on a miss.  hit: device int32[H][W],
 * (s << 29) | (k << 26) | (j << 13) | i of hit A's cell (s: the surface
 * index, 0 here; see hfr_raycast_nearer), -1 on a miss.  Geometry is FP64
 * throughout.  A walk that reaches its iteration cap (8 N (log2 N + 2) + 64
 * steps per cascade, more than a walk can need: each step descends a level
 * or moves to a later cell) is reported, not taken for a miss: depth NaN and
 * hit HFR_HIT_LIMIT.
 * work: device int32[W H + 2] scratch (its contents on entry do not matter;
 * the call overwrites them), or NULL.  After the call work[0] holds the
 * number of queued long rays and work[1] the number of rays stopped by the
 * iteration cap (a status word the caller may read once the stream has
 * reached it; 0 on a correct walk).  With it, a ray still walking after a
 * fixed number of cell steps is queued there and finished by a second
 * kernel in which 16 lanes share it: each step tests the next 16 nodes of
 * the current pyramid level along the ray at once, with the single-lane
 * walk's arithmetic, so depth and hit agree with the NULL path's (equal on
 * the benchmark frames); the few long rays that graze the surface near the
 * horizon stop setting the frame time.
 * Concurrent calls must not share work.
 * EINVAL: image size outside [1, 16384], K/N as above. */
hfr_status hfr_raycast(const hfr_camera* cam, const hfr_domain* dom, const hfr_cascade* cas,
                       int32_t K, const float* tex, const float* mip, float* depth, int32_t* hit,
                       int32_t* work, hfr_stream stream);

/* Adjoint of hfr_raycast: recomputes every ray (nothing is stored by the
 * forward pass) and ACCUMULATES into the caller-zeroed grad_tex
 * (device float[K][N][N]) the derivative of sum(grad_depth * depth) with
 * respect to the texel heights: dt/dh_c = phi_c(u, v) / f'(t) at a patch
 * root (implicit function theorem on z(t) - B(u(t), v(t)) = 0), chained
 * through the overlap blend; zero for hits at the start of a cascade
 * segment.  grad_depth: device float[H][W] (ignored where the ray misses).
 * work: as for hfr_raycast. */
hfr_status hfr_raycast_backward(const hfr_camera* cam, const hfr_domain* dom,
                                const hfr_cascade* cas, int32_t K, const float* tex,
                                const float* mip, const float* grad_depth, float* grad_tex,
                                int32_t* work, hfr_stream stream);

/* hfr_raycast and hfr_raycast_backward with the frame split at a row (not in
 * the paper; a scheduling choice with the same outputs).  Rows 0 ..
 * band_rows - 1, rounded up to a multiple of 16, are walked first with the
 * long-ray queue in work (required); a second launch then walks the queued
 * rays beside rows band_rows .. H - 1, whose rays each finish on their own
 * lane.  Long rays graze the surface just below the horizon, so a band that
 * ends a few degrees below it takes them all, and their lane-group walks run
 * while the rest of the image is cast instead of after it.  band_rows >= H
 * is hfr_raycast with a workspace; 0 walks every ray on its own lane.
 * Depth and hit are hfr_raycast's (the adjoint's sums differ only in the
 * order of the atomic adds).  EINVAL: band_rows < 0, work NULL, as for
 * hfr_raycast otherwise. */
hfr_status hfr_raycast_split(const hfr_camera* cam, const hfr_domain* dom, const hfr_cascade* cas,
                             int32_t K, const float* tex, const float* mip, float* depth, int32_t* hit,
                             int32_t* work, int32_t band_rows, hfr_stream stream);
hfr_status hfr_raycast_backward_split(const hfr_camera* cam, const hfr_domain* dom,
                                      const hfr_cascade* cas, int32_t K, const float* tex,
                                      const float* mip, const float* grad_depth, float* grad_tex,
                                      int32_t* work, int32_t band_rows, hfr_stream stream);

/* Several heightfields per frame (Section 2: the input is a terrain model and
 * relative water depths on the same adaptive grid; Table 1 times one
 * approximation pass per heightfield and the ray casting of all of them).
 * The visible point of a pixel is the nearest first hit over the surfaces.
 * Draw surface 0 with hfr_raycast, then every further surface s (1 ..
 * HFR_MAX_SURFACES - 1, its own textures and pyramids over the same
 * cascades) with hfr_raycast_nearer: the search for each ray's first hit is
 * clipped at the depth already in depth[p] (the partner hit of an overlap
 * blend is searched unclipped: surface s's depth is its own, whatever lies
 * behind), and a depth of surface s that lies in front replaces depth[p]
 * and hit[p] (tagged with s in bits 29-30); ties keep the earlier surface.
 * depth, hit: device in/out as written by the previous surfaces.  work: as
 * for hfr_raycast.  EINVAL: surface outside [1, HFR_MAX_SURFACES - 1], as
 * for hfr_raycast otherwise. */
hfr_status hfr_raycast_nearer(const hfr_camera* cam, const hfr_domain* dom, const hfr_cascade* cas,
                              int32_t K, const float* tex, const float* mip, int32_t surface,
                              float* depth, int32_t* hit, int32_t* work, hfr_stream stream);

/* Adjoint of the composite depth with respect to surface s's texels: as
 * hfr_raycast_backward on surface s's textures, restricted to the pixels
 * whose final hit (hit, device int32[H][W] as left by the drawing calls)
 * carries tag s.  A pixel's depth is surface s's first hit there, whatever
 * other surfaces lie behind, so the walk is recomputed without a clip.
 * EINVAL: surface outside [0, HFR_MAX_SURFACES - 1], NULL hit. */
hfr_status hfr_raycast_backward_surface(const hfr_camera* cam, const hfr_domain* dom,
                                        const hfr_cascade* cas, int32_t K, const float* tex,
                                        const float* mip, int32_t surface, const int32_t* hit,
                                        const float* grad_depth, float* grad_tex, int32_t* work,
                                        hfr_stream stream);

/* hfr_raycast for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * long-ray queue lives in a library-owned static device array instead of a
 * caller workspace, and the call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine).  Outputs are hfr_raycast's with a workspace.
 * The array holds the queue of at most hfr_raycast_static_max_pixels() pixels
 * (4,194,304: 16 MiB per device, held from the first call on that device until
 * the process ends); a larger image returns HFR_EINVAL.  Every call on one
 * device shares that device's array and clears its count first, so calls on
 * one device that overlap in time (different streams, or threads without
 * ordering) race and give wrong results: order them on one stream.  The
 * stream must belong to the current device (else HFR_EINVAL); the first call
 * on a device looks up the array's address (HFR_EDEVICE if that fails). */
hfr_status hfr_raycast_static(const hfr_camera* cam, const hfr_domain* dom, const hfr_cascade* cas, int32_t K,
                              const float* tex, const float* mip, float* depth, int32_t* hit, hfr_stream stream);
hfr_status hfr_raycast_static_max_pixels(int64_t* pixels);

/* Adjoint of hfr_discretize (Eq. 2 and Eq. 1): ACCUMULATES into the
 * caller-zeroed grad_v and grad_sigma (device float[n])
 *   grad_v[j]     += g_s w_j / S0
 *   grad_sigma[j] += g_s (v_j - v_s) / S0 * exp(-q^2/2) q^2 / sigma_j,
 *   q = |p_j - p_s| / (sigma_j c_j),
 * (HFR_BASIS_WENDLAND: the last factor is 20 u^2 (1 - u)^3 / sigma_j for u < 1)
 * for every visible texel s with g_s = grad_tex[s] != 0, where S0 = sum_j w_j
 * and v_s = tex[s] (the forward output).  Visibility and the cascade fit
 * are treated as constants. */
hfr_status hfr_discretize_backward(const hfr_leaves* L, const hfr_domain* dom,
                                   const hfr_cascade* cas, int32_t K, const float* tex,
                                   const float* grad_tex, float* grad_v, float* grad_sigma,
                                   hfr_stream stream);

/* ------------------------------------------------------------- batching
 *
 * Many views (camera + cascade set) of many heightfields rendered by one
 * set of launches: discretize (one persistent launch for every cascade of
 * every view), max-mipmap (one launch per five-level pass), ray casting
 * (one persistent launch for every pixel of every view), and for the
 * backward pass the two adjoints (one persistent launch each).  Persistent
 * workgroups (ray-cast waves) take runs of work from 64 chunk queues, eight
 * per XCD, starting with one of their own XCD's and moving on to the others
 * when it is empty, so views of uneven size share the GPU without a launch
 * per view.  The per-view work is the same as hfr_discretize,
 * hfr_build_maxmip and hfr_raycast (bit-identical outputs, with or without
 * the long-ray queue) and their adjoints; the batch is not in the paper,
 * which renders one view per frame.
 *
 * The plan is a library-owned host object holding device copies of the
 * field and view descriptors and the long-ray queue (4 B per pixel per 4
 * pixels, allocated by hfr_batch_plan_create, the only call that
 * allocates); every buffer it names stays caller-owned and must
 * outlive the plan.  hfr_batch_launch and hfr_batch_launch_backward
 * allocate nothing, issue no memset and no host synchronisation, and read
 * every per-camera value from device memory, so both may be captured into
 * one HIP graph and replayed after hfr_batch_set_cameras has changed the
 * cameras.  A plan is not thread-safe, and launches of one plan on
 * different streams race on its queues. */

typedef struct hfr_batch_plan hfr_batch_plan;

/* One heightfield.  leaves: as for hfr_discretize (packed records, level
 * radii and level index already built; sigma is needed for the backward
 * pass).  dom: its domain.  grad_v, grad_sigma: device float[leaves.n]
 * written by hfr_batch_launch_backward (summed over every view of this
 * field), or NULL when the plan has no backward pass. */
typedef struct {
    hfr_leaves leaves;
    hfr_domain dom;
    float* grad_v;
    float* grad_sigma;
} hfr_batch_field;

/* One view of field `field`: K cascades of N x N texels (N a power of two in
 * [2, HFR_MAX_TEX_N]) and a width x height image.  split_lambda, overlap,
 * c_min: as for hfr_fit_cascades.  Device buffers: tex float[K][N][N]; mask uint32
 * [K][N][(N+31)/32] or NULL; mip float[K][(4N^2-1)/3]; depth float[H][W];
 * hit int32[H][W]; for the backward pass grad_depth float[H][W] (read) and
 * grad_tex float[K][N][N] (scratch of the plan's backward pass, overwritten),
 * or both NULL. */
typedef struct {
    int32_t field;
    int32_t K, N;
    int32_t width, height;
    double split_lambda, overlap, c_min;
    float* tex;
    uint32_t* mask;
    float* mip;
    float* depth;
    int32_t* hit;
    const float* grad_depth;
    float* grad_tex;
} hfr_batch_view;

/* Launch shape.  disc_blocks_per_cu, ray_blocks_per_cu: persistent
 * workgroups (256 threads) per compute unit for the discretize kernels and
 * the ray-cast kernels, in [1, 16].  ray_tile_w: width of the 64-pixel tile
 * a wave takes at a time (8, 16, 32 or 64; height 64 / ray_tile_w).
 * disc_grain: the most 16 x 16 texel blocks a discretize workgroup takes
 * per queue access, in [1, 64] (a share of what is left in its chunk of the
 * work, at most this many: small runs keep the blocks running at once close
 * together and the finish even, large runs need fewer atomics).
 * ray_queue: 1 = hfr_raycast's long-ray queue for the batch (a ray still
 * walking after 64 steps is queued
 * and finished by a second launch with 16 lanes per ray; the plan holds room
 * for a quarter of each view's pixels and a ray past that finishes in the
 * first launch), 0 = every ray finishes in the first launch; outputs are the
 * same either way.  ray_grain: the most 64-pixel tiles a ray-cast wave takes
 * per queue access, in [1, 32] (a wave takes a share of what is left in its
 * chunk of the work, at most this many: a small cap keeps one wave from
 * being left with a long run of expensive tiles, such as a view's horizon
 * rows, after the others are done; a large one needs fewer atomics).
 * Defaults: 4, 4, 32, 8, 0, 8. */
typedef struct {
    int32_t disc_blocks_per_cu;
    int32_t ray_blocks_per_cu;
    int32_t ray_tile_w;
    int32_t disc_grain;
    int32_t ray_queue;
    int32_t ray_grain;
} hfr_batch_tuning;

/* Validates the fields and views, copies their descriptors to device memory
 * and returns a plan (*out).  Cameras must be set (hfr_batch_set_cameras)
 * before the first launch.  EINVAL: n_fields or n_views outside [1, 4096],
 * a view naming a missing field, K, N or image size out of range, NULL
 * buffers, a total work count above 2^31, or an unknown basis.  Fields may
 * use either basis (each block of a field evaluates that field's).  ENOMEM /
 * EDEVICE: allocation failures.  Synchronous. */
hfr_status hfr_batch_plan_create(const hfr_batch_field* fields, int32_t n_fields, const hfr_batch_view* views,
                                 int32_t n_views, hfr_batch_plan** out);
void hfr_batch_plan_destroy(hfr_batch_plan* plan);

/* Sets the launch shape (synchronous: not to be captured; a graph captured
 * before it must be captured again).  EINVAL on values outside the ranges
 * above. */
hfr_status hfr_batch_set_tuning(hfr_batch_plan* plan, const hfr_batch_tuning* tuning);

/* Fits the cascades of every view to its camera (hfr_fit_cascades, host)
 * and enqueues the upload of the per-view descriptors on `stream` (from a
 * plan-owned pinned buffer; the call first waits for its previous upload
 * to finish).  cams: host hfr_camera[n_views], each with the view's width
 * and height.  EINVAL as hfr_fit_cascades, or a camera whose image size
 * differs from its view's. */
hfr_status hfr_batch_set_cameras(hfr_batch_plan* plan, const hfr_camera* cams, hfr_stream stream);

/* Copies view `view`'s cascades from the last hfr_batch_set_cameras into the
 * host array out[K]. */
hfr_status hfr_batch_cascades(const hfr_batch_plan* plan, int32_t view, hfr_cascade* out);

/* Rays of each view that the last ray-cast launch of the plan (forward or
 * backward) with ray_queue = 1 sent to the long-ray queue, into the host
 * array out[n_views] (may exceed the view's room of a quarter of its
 * pixels: the rest finished in place).  Synchronises the device; not to be
 * captured. */
hfr_status hfr_batch_long_rays(const hfr_batch_plan* plan, int32_t* out);

/* Forward pass of every view: textures, masks, max-mipmaps, depth and hit
 * images, as hfr_discretize + hfr_build_maxmip + hfr_raycast would write
 * them view by view. */
hfr_status hfr_batch_launch(const hfr_batch_plan* plan, hfr_stream stream);

/* Backward pass of every view, after hfr_batch_launch: zeroes every view's
 * grad_tex and every field's grad_v / grad_sigma, then writes the gradient
 * of sum over views of sum(grad_depth * depth) with respect to the leaf
 * values and Gaussian widths (hfr_raycast_backward and
 * hfr_discretize_backward per view, summed per field).  EINVAL when a view
 * or field lacks its gradient buffers. */
hfr_status hfr_batch_launch_backward(const hfr_batch_plan* plan, hfr_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* HFR_H */
