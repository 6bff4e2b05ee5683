// Device-side helpers shared by the HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "hfr_internal.h"

#define HFR_LAUNCH_CHECK(what)                                                              \
    do {                                                                                    \
        hipError_t e_ = hipGetLastError();                                                  \
        if (e_ != hipSuccess) return hfr_fail(HFR_EDEVICE, "%s: %s", what, hipGetErrorString(e_)); \
    } while (0)

// Unfused double-precision helpers: texel and cell-edge positions must be
// formed as separate rounded products and sums so that every caller agrees
// on them bit for bit.
__device__ __forceinline__ double mul_rn(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ double add_rn(double a, double b) { return __dadd_rn(a, b); }

__device__ __forceinline__ double lattice_pos(double base, int m, double h) { return add_rn(base, mul_rn((double)m, h)); }

// Fields of hfr_cascade needed by the texture kernels, passed by value.
struct TexCascade {
    double x0, y0, hx, hy;
    int n, n_poly;
    double poly[HFR_MAX_POLY][2];
};

inline TexCascade tex_cascade(const hfr_cascade& c)
{
    TexCascade t;
    t.x0 = c.x0;
    t.y0 = c.y0;
    t.hx = c.hx;
    t.hy = c.hy;
    t.n = c.n;
    t.n_poly = c.n_poly;
    for (int a = 0; a < HFR_MAX_POLY; ++a) {
        t.poly[a][0] = c.poly[a][0];
        t.poly[a][1] = c.poly[a][1];
    }
    return t;
}

// x-extent [xl, xr] of (convex polygon) intersected with the strip ya <= y <= yb;
// xl > xr when they do not meet.
__device__ inline void strip_extent(const TexCascade& c, double ya, double yb, double* xl, double* xr)
{
    double lo = INFINITY, hi = -INFINITY;
    const int m = c.n_poly;
    for (int a = 0; a < m; ++a) {
        const double px = c.poly[a][0], py = c.poly[a][1];
        if (py >= ya && py <= yb) {
            lo = fmin(lo, px);
            hi = fmax(hi, px);
        }
        const int b = a + 1 == m ? 0 : a + 1;
        const double qx = c.poly[b][0], qy = c.poly[b][1];
        for (int s = 0; s < 2; ++s) {
            const double yc = s ? yb : ya;
            if ((py - yc) * (qy - yc) < 0.0) {
                const double x = px + (yc - py) * (qx - px) / (qy - py);
                lo = fmin(lo, x);
                hi = fmax(hi, x);
            }
        }
    }
    *xl = lo;
    *xr = hi;
}

// Tile (bx, by) of workgroup b of a 1-D grid over gx x gy tiles.  The hardware
// deals consecutive workgroups round-robin to the 8 XCDs; remapping gives each
// XCD one contiguous run of tiles (row-major), so neighbouring tiles, which
// read neighbouring data, share an L2.
__device__ inline void xcd_tile(int b, int gx, int gy, int* bx, int* by)
{
    const int nb = gx * gy;
    const int per = (nb + 7) / 8;
    const int xcd = b & 7, slot = b >> 3;
    const int full = nb - 8 * (per - 1);  // XCDs that receive `per` tiles (the rest get per - 1)
    const int lin = xcd < full ? xcd * per + slot : full * per + (xcd - full) * (per - 1) + slot;
    *bx = lin % gx;
    *by = lin / gx;
}

// Validates the common texture arguments of a set of cascades.
inline hfr_status check_cascades(const hfr_cascade* cas, int32_t K)
{
    HFR_REQUIRE(cas != nullptr, "cascades are NULL");
    HFR_REQUIRE(K >= 1 && K <= HFR_MAX_CASCADES, "K = %d outside [1, %d]", K, HFR_MAX_CASCADES);
    const int N = cas[0].n;
    HFR_REQUIRE(hfr_is_pow2(N) && N >= 2 && N <= HFR_MAX_TEX_N, "N = %d is not a power of two in [2, %d]", N,
                HFR_MAX_TEX_N);
    for (int k = 0; k < K; ++k) {
        const hfr_cascade& c = cas[k];
        HFR_REQUIRE(c.n == N, "cascade %d has N = %d, cascade 0 has %d", k, c.n, N);
        HFR_REQUIRE(c.n_poly >= 0 && c.n_poly <= HFR_MAX_POLY, "cascade %d has %d polygon vertices", k, c.n_poly);
        HFR_REQUIRE(std::isfinite(c.x0) && std::isfinite(c.y0) && c.hx > 0 && c.hy > 0 && std::isfinite(c.hx) &&
                        std::isfinite(c.hy),
                    "cascade %d has an invalid texture mapping", k);
        HFR_REQUIRE(std::isfinite(c.near_d) && std::isfinite(c.far_d) && std::isfinite(c.split_d) &&
                        c.near_d <= c.split_d && c.split_d <= c.far_d,
                    "cascade %d has invalid offsets", k);
        HFR_REQUIRE(std::isfinite(c.vhat[0]) && std::isfinite(c.vhat[1]) && std::isfinite(c.origin[0]) &&
                        std::isfinite(c.origin[1]),
                    "cascade %d has an invalid origin or direction", k);
    }
    return HFR_OK;
}

inline hfr_status check_domain(const hfr_domain* dom)
{
    HFR_REQUIRE(dom != nullptr, "domain is NULL");
    HFR_REQUIRE(std::isfinite(dom->x0) && std::isfinite(dom->x1) && std::isfinite(dom->y0) && std::isfinite(dom->y1) &&
                    std::isfinite(dom->zmin) && std::isfinite(dom->zmax),
                "domain must be finite");
    HFR_REQUIRE(dom->x1 > dom->x0 && dom->y1 > dom->y0 && dom->zmax >= dom->zmin, "empty domain");
    return HFR_OK;
}

// Texture-domain rectangle used by the texture kernels.
struct Dom2 {
    double x0, y0, x1, y1;
};

// Leaf data and constants of one heightfield, as the texture kernels read them.
struct Tables {
    const float4* packed;   // level-index order
    const float* radius;
    const int32_t* rank;    // level index: exclusive prefix counts per level
    const int32_t* order;   // leaf index of each sorted position
    const float* sigma;
    int n, max_depth;
    double x0, y0, side, inv_side;
    float E;   // exp(-cutoff^2 / 2) (Gaussian basis; 0 otherwise)
    float T2;  // (s r)^2 at the truncation radius: cutoff^2 log2(e) / 2 (Wendland basis: 1)
};

// Per-cascade ray-cast constants.
struct RayCas {
    double near_d, far_d, split_d, ox, oy, vx, vy, x0, y0, hx, hy, inv_hx, inv_hy;
    int n, levels;
};

// Everything a ray-cast kernel needs about one view.
struct RayArgs {
    double o[3], fwd[3], right[3], up[3];
    double tx, ty;
    int W, H, K, N;
    double X0, Y0, X1, Y1, zmax;
    RayCas c[HFR_MAX_CASCADES];
};

hfr_status leaf_tables(const hfr_leaves* L, bool backward, Tables* out);
hfr_status ray_args(const hfr_camera* cam, const hfr_domain* dom, const hfr_cascade* cas, int32_t K, RayArgs* A);

// ---------------------------------------------------------------- batching
// Device-resident descriptors of a batch plan.

struct BatchField {
    Tables T;
    Dom2 D;
    float* gv;
    float* gs;
    int basis;  // HFR_BASIS_GAUSSIAN or HFR_BASIS_WENDLAND
};

// One cascade of one view.
struct BatchTex {
    TexCascade C;
    int field, gx;  // gx x gx blocks of 16 x 16 texels
    float* tex;     // this cascade's texture, mask, pyramid and texel gradients
    uint16_t* mask;
    float* mip;
    float* gtex;
};

struct BatchView {
    RayArgs A;
    const float* tex;  // the view's [K][N][N] textures and [K][(4N^2-1)/3] pyramids
    const float* mip;
    float* depth;
    int32_t* hit;
    const float* gdepth;
    float* gtex;
    int tiles_x;       // 64-pixel tiles per image row
    int q_off, q_cap;  // the view's slice of the plan's long-ray queue (pixel indices)
};

// Work queues of the persistent batch launches: each splits its index range
// into HFR_CHUNKS chunks (eight per XCD) with one counter per chunk, each
// counter on its own 128-byte line.
constexpr int HFR_CHUNKS = 64;
constexpr int HFR_CHUNK_STRIDE = 32;  // ints between two chunk counters
constexpr int HFR_QUEUE_SPAN = HFR_CHUNKS * HFR_CHUNK_STRIDE;
constexpr int HFR_QUEUE_DISC = 0, HFR_QUEUE_DISC_BWD = HFR_QUEUE_SPAN, HFR_QUEUE_RAY = 2 * HFR_QUEUE_SPAN,
              HFR_QUEUE_RAY_BWD = 3 * HFR_QUEUE_SPAN;
constexpr int HFR_QUEUE_WORDS = 4 * HFR_QUEUE_SPAN;
constexpr int HFR_MIP_PASSES = 2;  // 64 x 64-cell tiles to level 6, then one workgroup per cascade to the top

struct BatchDev {
    const BatchField* fields;
    const BatchTex* tex;
    const int* tex_start;  // [n_tex + 1] prefix sums of 16 x 16 texel blocks
    const int* mip_start;  // [HFR_MIP_PASSES][n_tex + 1] prefix sums of max-mipmap blocks per pass
    const BatchView* views;
    const int* ray_start;  // [n_views + 1] prefix sums of 64-pixel tiles
    int* queues;           // HFR_QUEUE_WORDS counters, zeroed before each persistent launch
    int* rayq;             // long-ray queue: each view's slice [q_off, q_off + q_cap) holds pixel indices
    int* rayq_count;       // [n_views] rays queued per view, zeroed before each ray-cast launch
    int n_tex, n_views, tile_w;
    int disc_grain;        // texel blocks per discretize queue access
    int ray_queue;         // 1: rays past the step budget go to the queue, then a lane-group launch
    int ray_grain;         // most pixel tiles per ray-cast queue access
    int any_wendland;      // some field uses HFR_BASIS_WENDLAND
};

// Read-only view of descriptor memory through the constant address space: the
// descriptors do not change during a launch, and loads through this address
// space with a wave-uniform index become scalar loads into scalar registers.
template <class T>
__device__ inline const T& as_constant(const T* p, int i)
{
    typedef __attribute__((address_space(4))) const T ConstT;
    return *(const T*)((ConstT*)p + i);
}

hfr_status launch_discretize_batch(const BatchDev& P, int blocks, bool backward, hipStream_t s);
hfr_status launch_maxmip_batch(const BatchDev& P, const int* pass_blocks, hipStream_t s);
hfr_status launch_raycast_batch(const BatchDev& P, int blocks, int tail_blocks, bool backward, hipStream_t s);

// Next range of work indices from nq <= 64 queues that split [0, total) into
// nq contiguous chunks, their counters HFR_CHUNK_STRIDE ints apart; called by
// a whole wave (every lane active), the result wave-uniform.  Guided
// self-scheduling: a grab takes a share of what is left in the chunk,
// remaining / (2 consumers), clamped to [min_grain, max_grain], so early
// grabs are large (few atomics) and the last ones small (an even finish);
// `consumers` is the number of callers per chunk.  A caller starts with its
// home chunk (the hardware deals workgroups to the XCDs round-robin, so
// blockIdx.x & 7 names the workgroup's XCD and the callers pick a home among
// that XCD's chunks: neighbouring work shares an L2; a wrong guess only costs
// locality).  Once the home chunk is exhausted (*scan, false at the first
// call, records it), lane l looks at chunk (home + l) % nq and the wave takes
// from the first one after its home chunk (in that order) with work left.
// Many counters, each on its own cache line, spread the atomics, so the runs
// can stay short without the atomics serialising.  [*w0, *w1) is the range
// taken; false when every chunk is exhausted.  Each counter only grows and a
// failed grab leaves its chunk exhausted, so the loop ends after at most
// nq + 1 failed grabs.
__device__ inline bool queue_grab_wave(int* q, int nq, int total, int home, int min_grain, int max_grain,
                                       int consumers, bool* scan, int* w0, int* w1)
{
    const int lane = __lane_id();
    for (;;) {
        const int c = (home + (*scan ? lane : 0)) % nq;
        const int lo = (int)((int64_t)total * c / nq), hi = (int)((int64_t)total * (c + 1) / nq);
        int left = 0;
        if (*scan ? lane < nq : lane == 0)
            left = hi - lo - __hip_atomic_load(&q[c * HFR_CHUNK_STRIDE], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t m = __ballot(left > 0);
        if (m == 0) {
            if (*scan) return false;
            *scan = true;
            continue;
        }
        const int pick = __ffsll((unsigned long long)m) - 1;
        int idx = 0, end = 0;
        if (lane == pick) {
            const int grain = min(max(left / (2 * consumers), min_grain), max_grain);
            idx = lo + atomicAdd(&q[c * HFR_CHUNK_STRIDE], grain);
            end = min(idx + grain, hi);
        }
        idx = __shfl(idx, pick);
        end = __shfl(end, pick);
        if (idx < end) {
            *w0 = idx;
            *w1 = end;
            return true;
        }
    }
}

// Item holding work index w: the i with start[i] <= w < start[i + 1]
// (start[0] = 0, start[n] > w; empty items are skipped).
__device__ inline int find_item(const int* start, int n, int w)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= w) lo = mid;
        else hi = mid;
    }
    return lo;
}
