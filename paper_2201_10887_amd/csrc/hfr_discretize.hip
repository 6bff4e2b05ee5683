// Discretization of the truncated-Gaussian approximation into cascade
// textures (Eq. 1 and Eq. 2), with the visibility texture fused in, and its
// adjoint.  gfx950, wave64.
//
// Work decomposition.  A workgroup (4 waves) covers a 16 x 16 texel block of
// one cascade; each wave owns one 8 x 8 tile of the block (4 x 16 or 16 x 4
// where the cascade's texels are stretched along one axis).
//  1. Visibility: the 17 cell rows touching the block get their polygon
//     x-extent in LDS; every texel tests its incident cells; the block's
//     16-bit halves of the visibility words are assembled with LDS atomics.
//  2. Candidate search (all 256 lanes): per quadtree level, the lattice rows
//     and columns within that level's largest truncation radius of the block
//     rectangle.  The level index turns each window row into one range of
//     sorted leaf positions (two reads of the rank table per row), so only
//     leaves are visited, never empty lattice nodes.  A block-wide prefix of
//     the row lengths flattens the rows into one element range.
//  3. Element ranges of BCAP are gathered in order: every leaf whose own
//     truncation radius reaches the block rectangle goes to LDS as
//     (s x, s y, s, v), positions relative to the block origin (FP64
//     difference, then FP32), with s = sqrt(log2(e) / 2) / (sigma c) so that
//     Eq. 1's Gaussian is exp2(-(s r)^2) (Wendland basis: s = 1 / (k sigma c),
//     so that (s r)^2 is the squared distance in units of the support).
//  4. Each wave keeps the records whose own truncation radius reaches its
//     tile (a compact copy in LDS), and every lane (texel) runs Eq. 1 / Eq. 2
//     over them with broadcast LDS reads and immediate offsets, subtracting
//     the truncation constant per pair.
// Candidates beyond one element range are handled in rounds (the next range);
// windows of more than RCAP rows in chunks.  The order in which leaves reach
// a texel's sums is (level, row, column) whatever the rounds, so results do
// not depend on them.
#include <cmath>
#include <type_traits>

#include "hfr_device.h"

namespace {

constexpr int BS = 16;        // block side in texels
constexpr int WAVES = 4;      // 2 x 2 tiles per block
constexpr int BCAP = 512;     // candidate elements gathered per round (two per lane)
constexpr int TCAP = 128;     // tile-list records per chunk
constexpr int RCAP = 256;     // window rows per chunk (one per lane)
constexpr float LOG2E = 1.4426950408889634f;


constexpr float HALF_LOG2E = 0.72134752044448170f;


struct Rect {
    double x0, y0, x1, y1;
};

// Packs leaf records in level-index order and finds, per quadtree level, the
// largest support radius.  Thread a reads leaf a (coalesced), finds its
// lattice node (level, i, j) from its size and centre and its sorted position
// p from the rank table, and writes record p: one scattered read and one
// scattered 16-byte write per leaf instead of five scattered reads.  The
// per-level maxima are reduced in LDS first so that each block issues at most
// max_depth + 1 global atomics (one per level it saw).
__global__ __launch_bounds__(256) void pack_leaves_kernel(const float* __restrict__ x, const float* __restrict__ y,
                                                          const float* __restrict__ v, const float* __restrict__ c,
                                                          const float* __restrict__ sigma,
                                                          const int32_t* __restrict__ rank, double x0, double y0,
                                                          float cutoff, float scale, float side, int max_depth,
                                                          float4* __restrict__ out, float* __restrict__ radius,
                                                          int* __restrict__ status, int64_t n)
{
    __shared__ int level_max[16];  // max_depth <= 15; positive floats order as ints, 0 = no leaf seen
    if (threadIdx.x < 16) level_max[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < n; a += (int64_t)gridDim.x * blockDim.x) {
        const float ca = c[a], xa = x[a], ya = y[a];
        const float sc = sigma[a] * ca;
        int l = (int)rintf(log2f(side / ca));
        l = min(max(l, 0), max_depth);
        const int S = 1 << l;
        const int i = min(max((int)floor(((double)xa - x0) / ca), 0), S - 1);
        const int j = min(max((int)floor(((double)ya - y0) / ca), 0), S - 1);
        const int64_t p = rank[((int64_t(1) << (2 * l)) - 1) / 3 + l + (int64_t)j * S + i];
        if (p >= 0 && p < n) out[p] = make_float4(xa, ya, v[a], scale / sc);
        const float R = cutoff * sc * 1.00001f;
        atomicMax(&level_max[l], __float_as_int(R));
        // Eq. 2 needs each leaf's own reach to cover its square (half-diagonal sqrt(2)/2 c)
        if (status != nullptr && !(cutoff * sigma[a] > 0.70710678118654752f && isfinite(v[a]) && isfinite(sigma[a])))
            *status = HFR_EINVAL;
    }
    __syncthreads();
    if (threadIdx.x <= (unsigned)max_depth && level_max[threadIdx.x] != 0)
        atomicMax(reinterpret_cast<int*>(radius) + threadIdx.x, level_max[threadIdx.x]);
}

__global__ void zero_floats_kernel(float* __restrict__ p, int n, int* __restrict__ status)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < n) p[a] = 0.0f;
    if (a == 0 && status != nullptr) *status = HFR_OK;
}

__device__ inline double clampd(double v, double lo, double hi) { return fmin(fmax(v, lo), hi); }

// Clamped centres of texels [i0, i0 + w) x [j0, j0 + h) (cut at N - 1).
__device__ inline Rect texel_rect(const TexCascade& C, const Dom2& D, int i0, int j0, int w, int h)
{
    const int N = C.n;
    const int i1 = min(i0 + w - 1, N - 1), j1 = min(j0 + h - 1, N - 1);
    Rect r;
    r.x0 = clampd(lattice_pos(C.x0, min(i0, N - 1), C.hx), D.x0, D.x1);
    r.x1 = clampd(lattice_pos(C.x0, i1, C.hx), D.x0, D.x1);
    r.y0 = clampd(lattice_pos(C.y0, min(j0, N - 1), C.hy), D.y0, D.y1);
    r.y1 = clampd(lattice_pos(C.y0, j1, C.hy), D.y0, D.y1);
    return r;
}

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Visibility of the block's texels; returns this lane's texel visibility and
// writes the block's 16-bit visibility half-words.  Block-uniform helpers
// live in LDS: rxl / rxr (17 cell-row extents), mbits (16 rows).
__device__ inline bool block_visibility(const TexCascade& C, int bi0, int bj0, int i, int j, double* rxl, double* rxr,
                                        uint32_t* mbits, uint16_t* mask)
{
    const int N = C.n;
    const int t = threadIdx.x;
    if (t <= BS) {
        const int jc = bj0 - 1 + t;
        double lo = INFINITY, hi = -INFINITY;
        if (jc >= 0 && jc <= N - 2) strip_extent(C, lattice_pos(C.y0, jc, C.hy), lattice_pos(C.y0, jc + 1, C.hy), &lo, &hi);
        rxl[t] = lo;
        rxr[t] = hi;
    }
    if (t < BS) mbits[t] = 0u;
    __syncthreads();
    bool vis = false;
    if (i < N && j < N) {
        for (int dj = -1; dj <= 0; ++dj) {
            const int jc = j + dj;
            if (jc < 0 || jc > N - 2) continue;
            const double xl = rxl[jc - (bj0 - 1)], xr = rxr[jc - (bj0 - 1)];
            for (int di = -1; di <= 0; ++di) {
                const int ic = i + di;
                if (ic < 0 || ic > N - 2) continue;
                vis |= (lattice_pos(C.x0, ic, C.hx) <= xr) && (lattice_pos(C.x0, ic + 1, C.hx) >= xl);
            }
        }
    }
    if (vis) atomicOr(&mbits[j - bj0], 1u << (i - bi0));
    __syncthreads();
    if (mask && t < BS && bj0 + t < N) {
        const int halves = 2 * ((N + 31) / 32);
        mask[(int64_t)(bj0 + t) * halves + bi0 / BS] = (uint16_t)mbits[t];
    }
    return vis;
}

// Window of one quadtree level around a block rectangle: columns [ia, ib]
// of lattice rows ja, ja + 1, ... of the level.
struct LevelWin {
    int64_t off;  // offset of the level in the rank table
    int ia, ib, ja, S;
};
constexpr int MAX_LEVELS = 16;

struct ScanShared {
    LevelWin lw[MAX_LEVELS];
    int rstart[MAX_LEVELS + 1];  // first flattened window row of each level
    int seg_pos[RCAP];           // sorted position of the first leaf of each row of the chunk
    int seg_off[RCAP + 1];       // first element of each row of the chunk
    int wcnt[2][WAVES];          // per-wave counts (two buffers: consecutive prefixes need no barrier between)
};

// Largest truncation radius of level threadIdx.x (0 for other threads); loaded
// when a block starts so that its latency hides behind the visibility test.
__device__ inline float level_radius(const Tables& T)
{
    return (int)threadIdx.x <= T.max_depth ? T.radius[threadIdx.x] : 0.0f;
}

// Windows of every level around the block rectangle (lane l of wave 0 fills
// level l from its radius Rf): the lattice nodes within the level's largest
// truncation radius of the rectangle, widened by one node on each side.
// Returns the number of window rows over all levels (block-uniform).
__device__ int block_rows(const Tables& T, const Rect& r, float Rf, ScanShared& sc)
{
    const int t = threadIdx.x;
    if (t < 64) {
        const int l = t;
        int rows = 0;
        if (l <= T.max_depth) {
            LevelWin w{};
            if (Rf > 0.0f) {
                const double R = Rf;
                const double inv_c = ldexp(T.inv_side, l);
                const int S = 1 << l;
                const int ia = max(0, (int)floor((r.x0 - R - T.x0) * inv_c - 0.5) - 1);
                const int ib = min(S - 1, (int)ceil((r.x1 + R - T.x0) * inv_c - 0.5) + 1);
                const int ja = max(0, (int)floor((r.y0 - R - T.y0) * inv_c - 0.5) - 1);
                const int jb = min(S - 1, (int)ceil((r.y1 + R - T.y0) * inv_c - 0.5) + 1);
                if (ib >= ia && jb >= ja) {
                    rows = jb - ja + 1;
                    w = LevelWin{((int64_t(1) << (2 * l)) - 1) / 3 + l, ia, ib, ja, S};
                }
            }
            sc.lw[l] = w;
        }
        // rstart[l + 1] = rows of levels 0 .. l (levels past max_depth add none)
        int incl = rows;
#pragma unroll
        for (int o = 1; o < MAX_LEVELS; o <<= 1) {
            const int y = __shfl_up(incl, o);
            if (l >= o) incl += y;
        }
        if (l < MAX_LEVELS) sc.rstart[l + 1] = incl;
        if (l == 0) sc.rstart[0] = 0;
    }
    __syncthreads();
    return sc.rstart[MAX_LEVELS];
}

// Window rows [r0, r0 + RCAP): lane t reads the sorted-position range of row
// r0 + t from the rank table; seg_off becomes the exclusive prefix of the
// row lengths.  Returns the chunk's element count (block-uniform).
// The previous chunk's rows were last read inside gather_round or before this
// function's own closing barrier, so they may be overwritten without one.
__device__ int chunk_rows(const Tables& T, ScanShared& sc, int r0, int n_rows, int wave, int lane)
{
    const int r = r0 + (int)threadIdx.x;
    int pos = 0, len = 0;
    if (r < n_rows) {
        // the level owning row r: the largest l with rstart[l] <= r (an empty
        // level shares its successor's start, so the largest such l owns rows)
        int l = 0;
#pragma unroll
        for (int step = MAX_LEVELS / 2; step > 0; step >>= 1)
            if (sc.rstart[l + step] <= r) l += step;
        const LevelWin& w = sc.lw[l];
        const int64_t row = w.off + (int64_t)(w.ja + r - sc.rstart[l]) * w.S;
        pos = T.rank[row + w.ia];
        len = T.rank[row + w.ib + 1] - pos;
    }
    int incl = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) sc.wcnt[0][wave] = incl;
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        const int k = sc.wcnt[0][w];
        before += w < wave ? k : 0;
        all += k;
    }
    sc.seg_pos[threadIdx.x] = pos;
    sc.seg_off[threadIdx.x] = before + incl - len;
    if (threadIdx.x == 0) sc.seg_off[RCAP] = all;
    __syncthreads();
    return all;
}

// Elements [e0, e0 + BCAP) of the chunk, 256 at a time (lane t takes one
// element of each): every leaf whose own truncation radius reaches the block
// rectangle goes to brec as (s x, s y, s, v) relative to the block origin,
// in element order; its leaf index to ids and its sigma to bsig when those
// are given.  Returns the number of records (block-uniform).
__device__ int gather_round(const Tables& T, const Rect& r, ScanShared& sc, int e0, int n_e, float4* brec, int* ids,
                            float* bsig, int wave, int lane)
{
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const float lim = T.T2 * 1.001f;  // looser than any tile's test
    int total = 0;
#pragma unroll
    for (int u = 0; u < BCAP / 256; ++u) {
        const int eb = e0 + u * 256;
        if (eb >= n_e) break;  // block-uniform
        const int e = eb + (int)threadIdx.x;
        bool keep = false;
        float4 rec = make_float4(0.f, 0.f, 0.f, 0.f);
        int p = 0;
        if (e < n_e) {
            int sg = 0;
#pragma unroll
            for (int step = RCAP / 2; step > 0; step >>= 1)
                if (sc.seg_off[sg + step] <= e) sg += step;
            p = sc.seg_pos[sg] + (e - sc.seg_off[sg]);
            const float4 q = T.packed[p];
            const double xr = (double)q.x - r.x0, yr = (double)q.y - r.y0;
            const float dx = (float)fmax(fmax(-xr, xr - (r.x1 - r.x0)), 0.0) * q.w;
            const float dy = (float)fmax(fmax(-yr, yr - (r.y1 - r.y0)), 0.0) * q.w;
            keep = fmaf(dx, dx, dy * dy) < lim;
            rec = make_float4((float)xr * q.w, (float)yr * q.w, q.w, q.z);
        }
        const uint64_t m = __ballot(keep);
        if (lane == 0) sc.wcnt[u][wave] = __popcll(m);
        __syncthreads();
        int before = 0, all = 0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            const int k = sc.wcnt[u][w];
            before += w < wave ? k : 0;
            all += k;
        }
        if (keep) {
            const int slot = total + before + __popcll(m & lt);
            brec[slot] = rec;
            if (ids) {
                const int id = T.order[p];
                ids[slot] = id;
                if (bsig) bsig[slot] = T.sigma[id];
            }
        }
        total += all;
    }
    __syncthreads();
    return total;
}

// True when record q (scaled) can reach the rectangle [x0, x1] x [y0, y1]
// (coordinates relative to the block origin): its own truncation radius.
__device__ inline bool reaches(const float4& q, float x0, float x1, float y0, float y1, float lim)
{
    const float dx = fmaxf(fmaxf(fmaf(x0, q.z, -q.x), fmaf(-x1, q.z, q.x)), 0.0f);
    const float dy = fmaxf(fmaxf(fmaf(y0, q.z, -q.y), fmaf(-y1, q.z, q.y)), 0.0f);
    return fmaf(dx, dx, dy * dy) < lim;
}

// Eq. 1 for one (texel, leaf) pair from the scaled offset: exp2(-r2) minus the
// truncation constant, clipped at 0 (one subtract with the output clamp).
// Subtracting per pair keeps long tile lists, where most pairs lie beyond the
// cutoff, from cancelling a large sum of constants at the end.
__device__ __forceinline__ float rbf_weight(float dx, float dy, float E)
{
    return __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(-fmaf(dx, dx, dy * dy)) - E, 0.0f, 1.0f);
}

// Wendland's C2 function (1 - u)^4 (4u + 1) of u = (s r), 0 from u = 1 on.
__device__ __forceinline__ float wendland_weight(float dx, float dy)
{
    const float u = __builtin_amdgcn_sqrtf(fmaf(dx, dx, dy * dy));
    const float t = __builtin_amdgcn_fmed3f(1.0f - u, 0.0f, 1.0f);
    const float t2 = t * t;
    return t2 * t2 * fmaf(4.0f, u, 1.0f);
}

template <int BASIS>
__device__ __forceinline__ float pair_weight(float dx, float dy, float E)
{
    if constexpr (BASIS == HFR_BASIS_WENDLAND) return wendland_weight(dx, dy);
    else return rbf_weight(dx, dy, E);
}

// Weight w and sigma dw/dsigma of one pair from r2 = (s r)^2.
template <int BASIS>
__device__ __forceinline__ void pair_weight_dsigma(float r2, float E, float* w, float* sdw)
{
    if constexpr (BASIS == HFR_BASIS_WENDLAND) {
        const float u = __builtin_amdgcn_sqrtf(r2);
        const float t = fmaxf(1.0f - u, 0.0f);
        const float t3 = t * t * t;
        *w = t3 * t * fmaf(4.0f, u, 1.0f);
        *sdw = 20.0f * r2 * t3;  // (1 - u)^4 (4u + 1) has d/du = -20 u (1 - u)^3, and u scales as 1 / sigma
    } else {
        const float ex = __builtin_amdgcn_exp2f(-r2);
        *w = ex - E;
        *sdw = ex * r2 * (2.0f / LOG2E);  // r2 = q^2 log2(e) / 2
    }
}

// Value of x on lane t (t wave-uniform): a scalar read of one lane, no LDS
// round trip.
__device__ __forceinline__ float lane_value(float x, int t)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), t));
}

struct TileFrame {
    float x0, x1, y0, y1;  // tile rectangle relative to the block origin
    float npx, npy;        // minus the lane's texel centre relative to the block origin
};

__device__ inline TileFrame tile_frame(const TexCascade& C, const Dom2& D, const Rect& br, int ti0, int tj0, int i, int j,
                                       int tw, int th)
{
    const Rect tr = texel_rect(C, D, ti0, tj0, tw, th);
    TileFrame f;
    f.x0 = (float)(tr.x0 - br.x0);
    f.x1 = (float)(tr.x1 - br.x0);
    f.y0 = (float)(tr.y0 - br.y0);
    f.y1 = (float)(tr.y1 - br.y0);
    const int N = C.n;
    f.npx = -(float)(clampd(lattice_pos(C.x0, min(i, N - 1), C.hx), D.x0, D.x1) - br.x0);
    f.npy = -(float)(clampd(lattice_pos(C.y0, min(j, N - 1), C.hy), D.y0, D.y1) - br.y0);
    return f;
}

// The previous frame's texture of a cascade on the same lattice: texel (i, j)
// now is texel (i + di, j + dj) then.  prev == nullptr: nothing to reuse.
struct Reuse {
    const float* prev;
    int di, dj;
};

struct DiscShared {
    float4 brec[BCAP];
    float4 trec_all[WAVES][TCAP];
    double rxl[BS + 1], rxr[BS + 1];
    uint32_t mbits[BS];
    ScanShared scan;
    int any_vis;
};

// Texels of block (bx, by) of one cascade; every thread of the workgroup
// takes part.
template <int BASIS>
__device__ __forceinline__ void discretize_block(const Tables& T, const TexCascade& C, const Dom2& D, int bx, int by,
                                                 float* __restrict__ tex, uint16_t* __restrict__ mask, DiscShared& sh,
                                                 const Reuse* ru = nullptr, int* reused = nullptr)
{
    float4* brec = sh.brec;
    int& any_vis = sh.any_vis;
    const int N = C.n;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int bi0 = bx * BS, bj0 = by * BS;
    // A wave's tile: 8 x 8 texels, or 4 x 16 (16 x 4) when the cascade's texels are more than twice
    // as wide as high (high as wide), so that the tile spans similar lengths on both axes and fewer
    // records reach it (the far cascades' texels are stretched along the view).
    const int lw = C.hx > 2.0 * C.hy ? 2 : (C.hy > 2.0 * C.hx ? 4 : 3);
    const int tw = 1 << lw, th = 64 >> lw, per_row = BS >> lw;
    const int ti0 = bi0 + (wave % per_row) * tw, tj0 = bj0 + (wave / per_row) * th;
    const int i = ti0 + (lane & (tw - 1)), j = tj0 + (lane >> lw);
    const bool inside = i < N && j < N;
    const float Rf = level_radius(T);
    if (threadIdx.x == 0) any_vis = 0;
    const bool vis = block_visibility(C, bi0, bj0, i, j, sh.rxl, sh.rxr, sh.mbits, mask);
    if (vis) any_vis = 1;
    __syncthreads();
    if (!any_vis) {
        if (inside) tex[(int64_t)j * N + i] = -INFINITY;
        return;
    }
    if (ru != nullptr && ru->prev != nullptr) {
        // copy the block when every texel visible now was computed last frame
        const int pi = i + ru->di, pj = j + ru->dj;
        float old = -INFINITY;
        if (vis && pi >= 0 && pi < N && pj >= 0 && pj < N) old = ru->prev[(int64_t)pj * N + pi];
        if (__syncthreads_and(!vis || isfinite(old))) {
            if (inside) tex[(int64_t)j * N + i] = vis ? old : -INFINITY;
            if (reused != nullptr && threadIdx.x == 0) atomicAdd(reused, 1);
            return;
        }
    }
    const Rect br = texel_rect(C, D, bi0, bj0, BS, BS);
    const TileFrame f = tile_frame(C, D, br, ti0, tj0, i, j, tw, th);
    const bool tile_vis = __ballot(vis) != 0;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const float lim = T.T2 * 1.0001f, E = T.E;
    float4* trec = sh.trec_all[wave];
    float s0 = 0.0f, s1 = 0.0f;
    const int n_rows = block_rows(T, br, Rf, sh.scan);
    for (int r0 = 0; r0 < n_rows; r0 += RCAP) {
      const int n_e = chunk_rows(T, sh.scan, r0, n_rows, wave, lane);
      for (int e0 = 0; e0 < n_e; e0 += BCAP) {
        const int nb = gather_round(T, br, sh.scan, e0, n_e, brec, nullptr, nullptr, wave, lane);
        if (tile_vis) {
            int nt = 0;
            for (int c0 = 0; c0 < nb; c0 += 64) {
                const int c = c0 + lane;
                const float4 q = c < nb ? brec[c] : make_float4(0.f, 0.f, 0.f, 0.f);
                const bool keep = c < nb && reaches(q, f.x0, f.x1, f.y0, f.y1, lim);
                const uint64_t m = __ballot(keep);
                const int k = __popcll(m);
                if (nt + k > TCAP) {  // evaluate the full chunk first
                    wave_sync();
                    for (int a = 0; a < nt; ++a) {
                        const float4 r = trec[a];
                        const float g = pair_weight<BASIS>(fmaf(f.npx, r.z, r.x), fmaf(f.npy, r.z, r.y), E);
                        s0 += g;
                        s1 = fmaf(g, r.w, s1);
                    }
                    nt = 0;
                    wave_sync();
                }
                if (keep) trec[nt + __popcll(m & lt)] = q;
                nt += k;
            }
            wave_sync();
            int a = 0;
            for (; a + 4 <= nt; a += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const float4 r = trec[a + u];
                    const float g = pair_weight<BASIS>(fmaf(f.npx, r.z, r.x), fmaf(f.npy, r.z, r.y), E);
                    s0 += g;
                    s1 = fmaf(g, r.w, s1);
                }
            }
            for (; a < nt; ++a) {
                const float4 r = trec[a];
                const float g = pair_weight<BASIS>(fmaf(f.npx, r.z, r.x), fmaf(f.npy, r.z, r.y), E);
                s0 += g;
                s1 = fmaf(g, r.w, s1);
            }
            wave_sync();
        }
        __syncthreads();  // before the next round overwrites brec
      }
    }
    if (!inside) return;
    float out = -INFINITY;
    if (vis) out = s0 > 0.0f ? s1 / s0 : NAN;
    tex[(int64_t)j * N + i] = out;
}

// Up to FUSE cascades of one view in one launch.  Their block rows are
// interleaved (row v holds row v / K of cascade v % K) before the XCD-aware
// mapping, so every XCD's contiguous share mixes the cascades (the far ones
// cost the most) while neighbouring rows of a cascade stay on one XCD; the
// latency-bound blocks of the near cascades overlap the ALU-bound far ones.
constexpr int FUSE = 4;
struct CascadeSet {
    TexCascade c[FUSE];
    Reuse r[FUSE];
    int* reused;  // blocks copied from the previous frame (may be nullptr)
    int K;
};

__device__ inline int fused_block(const CascadeSet& S, int gx, int gy, int* bx, int* by)
{
    int row;
    xcd_tile(blockIdx.x, gx, gy * S.K, bx, &row);
    *by = row / S.K;
    return row - *by * S.K;
}

// 8 waves per SIMD (at most 64 VGPRs, no spills; 8 blocks of LDS fit a CU): the near
// cascades wait on rank-table and record loads, and more resident waves hide that.
template <int BASIS>
__global__ __launch_bounds__(256, 8) void discretize_kernel(Tables T, CascadeSet S, Dom2 D, int gx, int gy,
                                                         float* __restrict__ tex, uint16_t* __restrict__ mask)
{
    __shared__ DiscShared sh;
    int bx, by;
    const int k = __builtin_amdgcn_readfirstlane(fused_block(S, gx, gy, &bx, &by));
    const TexCascade& C = S.c[k];
    const int64_t N = C.n;
    discretize_block<BASIS>(T, C, D, bx, by, tex + k * N * N, mask ? mask + k * N * 2 * ((N + 31) / 32) : nullptr,
                            sh, &S.r[k], S.reused);
}

// Adjoint of Eq. 2 / Eq. 1.  Lanes first own texels (S0 of each texel), then
// own tile-list leaves: for every texel of the tile with a non-zero gradient
// (a wave-uniform loop) each lane adds its leaf's share
//   g w_j / S0   and   g (v_j - v_s) / S0 * exp(-q^2/2) q^2 / sigma_j,
// and finally adds its two sums to the leaf's gradient with one atomic each.
struct DiscBwdShared {
    float4 brec[BCAP];
    int bids[BCAP];
    float bsig[BCAP];
    unsigned short tidx_all[WAVES][BCAP];
    ScanShared scan;
    int any_act;
};

template <int BASIS>
__device__ __forceinline__ void discretize_backward_block(const Tables& T, const TexCascade& C, const Dom2& D, int bx,
                                                          int by, const float* __restrict__ tex,
                                                          const float* __restrict__ gtex, float* __restrict__ gv,
                                                          float* __restrict__ gs, DiscBwdShared& sh)
{
    float4* brec = sh.brec;
    int* bids = sh.bids;
    float* bsig = sh.bsig;
    int& any_act = sh.any_act;
    const int N = C.n;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int bi0 = bx * BS, bj0 = by * BS;
    // A wave's tile: 8 x 8 texels, or 4 x 16 (16 x 4) when the cascade's texels are more than twice
    // as wide as high (high as wide), so that the tile spans similar lengths on both axes and fewer
    // records reach it (the far cascades' texels are stretched along the view).
    const int lw = C.hx > 2.0 * C.hy ? 2 : (C.hy > 2.0 * C.hx ? 4 : 3);
    const int tw = 1 << lw, th = 64 >> lw, per_row = BS >> lw;
    const int ti0 = bi0 + (wave % per_row) * tw, tj0 = bj0 + (wave / per_row) * th;
    const int i = ti0 + (lane & (tw - 1)), j = tj0 + (lane >> lw);
    const bool inside = i < N && j < N;
    const float Rf = level_radius(T);
    float g = 0.0f, vs = 0.0f;
    if (inside) {
        g = gtex[(int64_t)j * N + i];
        vs = tex[(int64_t)j * N + i];
    }
    const bool act = inside && g != 0.0f && isfinite(vs) && isfinite(g);
    if (threadIdx.x == 0) any_act = 0;
    __syncthreads();
    if (act) any_act = 1;
    __syncthreads();
    if (!any_act) return;
    const uint64_t active = __ballot(act);
    const Rect br = texel_rect(C, D, bi0, bj0, BS, BS);
    const TileFrame f = tile_frame(C, D, br, ti0, tj0, i, j, tw, th);
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const float lim = T.T2 * 1.0001f, E = T.E;
    unsigned short* tidx = sh.tidx_all[wave];
    // pass 1: S0 per texel (lanes own texels)
    float s0 = 0.0f;
    const int n_rows = block_rows(T, br, Rf, sh.scan);
    int n_e = 0, nb = 0;
    for (int r0 = 0; r0 < n_rows; r0 += RCAP) {
        n_e = chunk_rows(T, sh.scan, r0, n_rows, wave, lane);
        for (int e0 = 0; e0 < n_e; e0 += BCAP) {
            nb = gather_round(T, br, sh.scan, e0, n_e, brec, bids, bsig, wave, lane);
            if (active) {
                for (int c0 = 0; c0 < nb; c0 += 64) {
                    const int c = c0 + lane;
                    const float4 q0 = c < nb ? brec[c] : make_float4(0.f, 0.f, 0.f, 0.f);
                    const bool keep = c < nb && reaches(q0, f.x0, f.x1, f.y0, f.y1, lim);
                    uint64_t m = __ballot(keep);
                    // two records per step (both reads in flight at once); a missing second
                    // record is one that weighs exactly 0, so s0 sums the same terms in order
                    while (m) {
                        const int t = __ffsll((unsigned long long)m) - 1;
                        m &= m - 1;
                        const float4 qa = brec[c0 + t];
                        float4 qb = make_float4(1e18f, 1e18f, 0.f, 0.f);
                        if (m) {
                            const int t2 = __ffsll((unsigned long long)m) - 1;
                            m &= m - 1;
                            qb = brec[c0 + t2];
                        }
                        s0 += pair_weight<BASIS>(fmaf(f.npx, qa.z, qa.x), fmaf(f.npy, qa.z, qa.y), E);
                        s0 += pair_weight<BASIS>(fmaf(f.npx, qb.z, qb.x), fmaf(f.npy, qb.z, qb.y), E);
                    }
                }
            }
            __syncthreads();  // before the next round overwrites brec
        }
    }
    const float gn = act && s0 > 0.0f ? g / s0 : 0.0f;
    // pass 2: lanes own tile-list leaves; with a single round the block records are still staged
    const bool single = n_rows <= RCAP && n_e <= BCAP;
    for (int r0 = 0; r0 < n_rows; r0 += RCAP) {
        if (!single) n_e = chunk_rows(T, sh.scan, r0, n_rows, wave, lane);
        for (int e0 = 0; e0 < n_e; e0 += BCAP) {
            if (!single) nb = gather_round(T, br, sh.scan, e0, n_e, brec, bids, bsig, wave, lane);
            if (active) {
                int nt = 0;
                for (int c0 = 0; c0 < nb; c0 += 64) {
                    const int c = c0 + lane;
                    const float4 q = c < nb ? brec[c] : make_float4(0.f, 0.f, 0.f, 0.f);
                    const bool keep = c < nb && reaches(q, f.x0, f.x1, f.y0, f.y1, lim);
                    const uint64_t m = __ballot(keep);
                    if (keep) tidx[nt + __popcll(m & lt)] = (unsigned short)c;
                    nt += __popcll(m);
                }
                wave_sync();
                for (int c0 = 0; c0 < nt; c0 += 64) {
                    const int a = c0 + lane;
                    const bool own = a < nt;
                    const int c = own ? tidx[a] : 0;
                    const float4 q = own ? brec[c] : make_float4(1e18f, 1e18f, 0.f, 0.f);
                    const float sj = own ? bsig[c] : 1.0f;
                    float acc_v = 0.0f, acc_s = 0.0f;
                    uint64_t m = active;
                    while (m) {
                        const int t = __ffsll((unsigned long long)m) - 1;  // wave-uniform
                        m &= m - 1;
                        // the texel offsets are read un-negated and negated in the multiply-add
                        // (a lane read cannot take a negation modifier; the values are equal)
                        const float tpx = lane_value(-f.npx, t), tpy = lane_value(-f.npy, t), tg = lane_value(gn, t),
                                    tv = lane_value(vs, t);
                        const float dx = fmaf(-tpx, q.z, q.x), dy = fmaf(-tpy, q.z, q.y);
                        const float r2 = fmaf(dx, dx, dy * dy);
                        float w, sdw;
                        pair_weight_dsigma<BASIS>(r2, E, &w, &sdw);
                        if (w > 0.0f) {
                            acc_v = fmaf(tg, w, acc_v);
                            acc_s = fmaf(tg * (q.w - tv), sdw, acc_s);
                        }
                    }
                    acc_s /= sj;  // d w / d sigma = (sigma d w / d sigma) / sigma: one division per leaf
                    if (own && (acc_v != 0.0f || acc_s != 0.0f)) {
                        atomicAdd(&gv[bids[c]], acc_v);
                        atomicAdd(&gs[bids[c]], acc_s);
                    }
                }
                wave_sync();
            }
            if (!single) __syncthreads();  // before the next round overwrites brec
        }
    }
}

template <int BASIS>
__global__ __launch_bounds__(256, 8) void discretize_backward_kernel(Tables T, CascadeSet S, Dom2 D, int gx, int gy,
                                                                  const float* __restrict__ tex,
                                                                  const float* __restrict__ gtex,
                                                                  float* __restrict__ gv, float* __restrict__ gs)
{
    __shared__ DiscBwdShared sh;
    int bx, by;
    const int k = __builtin_amdgcn_readfirstlane(fused_block(S, gx, gy, &bx, &by));
    const TexCascade& C = S.c[k];
    const int64_t N = C.n;
    discretize_backward_block<BASIS>(T, C, D, bx, by, tex + k * N * N, gtex + k * N * N, gv, gs, sh);
}

// Persistent form over every cascade of every view of a batch: each
// workgroup takes runs of 16 x 16 texel blocks (guided, at most P.disc_grain)
// from HFR_CHUNKS queues, eight per XCD, until all are done; wave 0 grabs for
// the workgroup.  The cascade a block belongs to is found by one search per
// run and followed forward inside it.  The runs stay short: the blocks of an
// XCD then work on neighbouring tiles at once and share node-table rows and
// leaf records in its L2.

// WENDLAND: some field of the batch uses Wendland's basis, so each block
// takes its field's basis; without such a field only the Gaussian body is
// compiled in (both bodies in one kernel need more registers than 7
// workgroups per CU leave, and spill a few).
template <bool BACKWARD, bool WENDLAND>
__global__ __launch_bounds__(256, 7) void discretize_batch_kernel(BatchDev P)
{
    __shared__ typename std::conditional<BACKWARD, DiscBwdShared, DiscShared>::type sh;
    __shared__ int work[3];
    int* q = P.queues + (BACKWARD ? HFR_QUEUE_DISC_BWD : HFR_QUEUE_DISC);
    const int total = P.tex_start[P.n_tex];
    // home chunk: the workgroup's XCD (blockIdx.x & 7), then one of its eight
    // chunks by the workgroup's slot on that XCD
    const int home = (int)(blockIdx.x & 7) * 8 + (int)((blockIdx.x >> 3) & 7);
    const int consumers = max(1, (int)gridDim.x / HFR_CHUNKS);
    bool scan = false;
    for (;;) {
        __syncthreads();  // the previous run's LDS reads are done
        if (threadIdx.x < 64) {  // wave 0, every lane active
            int w0 = -1, w1 = -1;
            const bool got = queue_grab_wave(q, HFR_CHUNKS, total, home, 1, P.disc_grain, consumers, &scan, &w0, &w1);
            if (threadIdx.x == 0) {
                work[0] = got ? w0 : -1;
                work[1] = w1;
                work[2] = got ? find_item(P.tex_start, P.n_tex, w0) : 0;
            }
        }
        __syncthreads();
        const int w0 = __builtin_amdgcn_readfirstlane(work[0]);
        if (w0 < 0) break;
        const int w1 = __builtin_amdgcn_readfirstlane(work[1]);
        int item = __builtin_amdgcn_readfirstlane(work[2]);
        int item_lo = P.tex_start[item], item_hi = P.tex_start[item + 1];
        for (int w = w0; w < w1; ++w) {
            while (w >= item_hi) {  // w < total, so this stops at an item that holds w
                ++item;
                item_lo = item_hi;
                item_hi = P.tex_start[item + 1];
            }
            const BatchTex& it = as_constant(P.tex, item);
            const BatchField& F = as_constant(P.fields, it.field);
            const int local = w - item_lo;
            const int bx = local % it.gx, by = local / it.gx;
            // the field's basis (wave-uniform: one field per block)
            if constexpr (BACKWARD) {
                if (WENDLAND && F.basis == HFR_BASIS_WENDLAND)
                    discretize_backward_block<HFR_BASIS_WENDLAND>(F.T, it.C, F.D, bx, by, it.tex, it.gtex, F.gv, F.gs,
                                                                  sh);
                else
                    discretize_backward_block<HFR_BASIS_GAUSSIAN>(F.T, it.C, F.D, bx, by, it.tex, it.gtex, F.gv, F.gs,
                                                                  sh);
            } else {
                if (WENDLAND && F.basis == HFR_BASIS_WENDLAND)
                    discretize_block<HFR_BASIS_WENDLAND>(F.T, it.C, F.D, bx, by, it.tex, it.mask, sh);
                else discretize_block<HFR_BASIS_GAUSSIAN>(F.T, it.C, F.D, bx, by, it.tex, it.mask, sh);
            }
            __syncthreads();  // LDS is reused by the next block of the run
        }
    }
}

}  // namespace

hfr_status leaf_tables(const hfr_leaves* L, bool backward, Tables* out)
{
    HFR_REQUIRE(L != nullptr, "leaves are NULL");
    HFR_REQUIRE(L->n >= 1 && L->n <= INT32_MAX, "leaf count %lld outside [1, INT32_MAX]", (long long)L->n);
    HFR_REQUIRE(L->packed && L->level_radius && L->rank && L->order,
                "packed records, level radii and the level index are required");
    HFR_REQUIRE(!backward || L->sigma, "sigma is required");
    HFR_REQUIRE(L->max_depth >= 0 && L->max_depth <= 15, "max_depth %d outside [0, 15]", L->max_depth);
    HFR_REQUIRE(std::isfinite(L->cutoff) && L->cutoff > 0, "cutoff must be positive");
    HFR_REQUIRE(std::isfinite(L->side) && L->side > 0 && std::isfinite(L->x0) && std::isfinite(L->y0),
                "invalid lattice square");
    HFR_REQUIRE(L->basis == HFR_BASIS_GAUSSIAN || L->basis == HFR_BASIS_WENDLAND, "unknown basis %d", L->basis);
    const bool gauss = L->basis == HFR_BASIS_GAUSSIAN;
    *out = Tables{reinterpret_cast<const float4*>(L->packed), L->level_radius, L->rank, L->order, L->sigma, (int)L->n,
                  L->max_depth, L->x0, L->y0, L->side, 1.0 / L->side,
                  gauss ? std::exp(-0.5f * L->cutoff * L->cutoff) : 0.0f,
                  gauss ? 0.5f * LOG2E * L->cutoff * L->cutoff : 1.0f};
    return HFR_OK;
}


extern "C" hfr_status hfr_pack_leaves(const hfr_leaves* L, hfr_stream stream)
{
    HFR_REQUIRE(L != nullptr, "leaves are NULL");
    HFR_REQUIRE(L->n >= 1 && L->n <= INT32_MAX, "leaf count %lld outside [1, INT32_MAX]", (long long)L->n);
    HFR_REQUIRE(L->x && L->y && L->v && L->c && L->sigma && L->packed && L->level_radius && L->rank,
                "leaf arrays and the level index must not be NULL");
    HFR_REQUIRE(L->max_depth >= 0 && L->max_depth <= 15, "max_depth %d outside [0, 15]", L->max_depth);
    HFR_REQUIRE(std::isfinite(L->cutoff) && L->cutoff > 0, "cutoff must be positive");
    HFR_REQUIRE(std::isfinite(L->side) && L->side > 0, "side must be positive");
    HFR_REQUIRE(L->basis == HFR_BASIS_GAUSSIAN || L->basis == HFR_BASIS_WENDLAND, "unknown basis %d", L->basis);
    // record scale: exp2(-(s r)^2) is Eq. 1's Gaussian; for Wendland s r is r over the support radius
    const float scale = L->basis == HFR_BASIS_GAUSSIAN ? std::sqrt(HALF_LOG2E) : 1.0f / L->cutoff;
    hipStream_t s = (hipStream_t)stream;
    zero_floats_kernel<<<1, 64, 0, s>>>(L->level_radius, L->max_depth + 1, L->status);
    HFR_LAUNCH_CHECK("pack_leaves (radius reset)");
    const int64_t blocks = std::min<int64_t>((L->n + 255) / 256, 2048);
    pack_leaves_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(
        L->x, L->y, L->v, L->c, L->sigma, L->rank, L->x0, L->y0, L->cutoff, scale, (float)L->side, L->max_depth,
        reinterpret_cast<float4*>(L->packed), L->level_radius, L->status, L->n);
    HFR_LAUNCH_CHECK("pack_leaves");
    return hfr_ok();
}

namespace {

// Whole-texel shift from the previous frame's lattice of a cascade to this one's, when both
// frames use the same spacing and the lattices coincide; false otherwise.
bool lattice_shift(const hfr_cascade& now, const hfr_cascade& then, int* di, int* dj)
{
    if (then.n != now.n || then.hx != now.hx || then.hy != now.hy || then.n_poly == 0 || now.n_poly == 0) return false;
    const double sx = (now.x0 - then.x0) / now.hx, sy = (now.y0 - then.y0) / now.hy;
    if (!(std::fabs(sx) < now.n && std::fabs(sy) < now.n)) return false;
    const double rx = std::nearbyint(sx), ry = std::nearbyint(sy);
    if (std::fabs(sx - rx) > 1e-6 || std::fabs(sy - ry) > 1e-6) return false;
    *di = (int)rx;
    *dj = (int)ry;
    return true;
}

hfr_status discretize_frame(const hfr_leaves* L, const hfr_domain* dom, const hfr_cascade* cas, int32_t K,
                            const hfr_cascade* prev_cas, const float* prev_tex, float* tex, uint32_t* mask,
                            int32_t* reused, hfr_stream stream)
{
    Tables T;
    hfr_status st = leaf_tables(L, false, &T);
    if (st == HFR_OK) st = check_cascades(cas, K);
    if (st == HFR_OK) st = check_domain(dom);
    if (st != HFR_OK) return st;
    HFR_REQUIRE(tex != nullptr, "tex is NULL");
    const int N = cas[0].n;
    const int64_t texels = (int64_t)K * N * N;
    if (prev_cas != nullptr) {
        HFR_REQUIRE(prev_tex != nullptr, "prev_tex is NULL");
        const uintptr_t a0 = reinterpret_cast<uintptr_t>(prev_tex), b0 = reinterpret_cast<uintptr_t>(tex);
        const uintptr_t bytes = (uintptr_t)texels * sizeof(float);
        HFR_REQUIRE(a0 + bytes <= b0 || b0 + bytes <= a0, "prev_tex overlaps tex");
    }
    const Dom2 D{dom->x0, dom->y0, dom->x1, dom->y1};
    const int gx = (N + BS - 1) / BS, gy = (N + BS - 1) / BS;
    const int words = (N + 31) / 32;
    for (int k0 = 0; k0 < K; k0 += FUSE) {
        CascadeSet S;
        S.K = std::min(FUSE, K - k0);
        S.reused = reused;
        for (int k = 0; k < S.K; ++k) {
            S.c[k] = tex_cascade(cas[k0 + k]);
            S.r[k] = Reuse{nullptr, 0, 0};
            int di = 0, dj = 0;
            if (prev_cas != nullptr && lattice_shift(cas[k0 + k], prev_cas[k0 + k], &di, &dj))
                S.r[k] = Reuse{prev_tex + (int64_t)(k0 + k) * N * N, di, dj};
        }
        float* t = tex + (int64_t)k0 * N * N;
        uint16_t* m = mask ? reinterpret_cast<uint16_t*>(mask + (int64_t)k0 * N * words) : nullptr;
        const dim3 grid(gx * gy * S.K), block(64 * WAVES);
        if (L->basis == HFR_BASIS_WENDLAND)
            discretize_kernel<HFR_BASIS_WENDLAND><<<grid, block, 0, (hipStream_t)stream>>>(T, S, D, gx, gy, t, m);
        else
            discretize_kernel<HFR_BASIS_GAUSSIAN><<<grid, block, 0, (hipStream_t)stream>>>(T, S, D, gx, gy, t, m);
        HFR_LAUNCH_CHECK("discretize");
    }
    return hfr_ok();
}

}  // namespace

extern "C" hfr_status hfr_discretize(const hfr_leaves* L, const hfr_domain* dom, const hfr_cascade* cas, int32_t K,
                                     float* tex, uint32_t* mask, hfr_stream stream)
{
    return discretize_frame(L, dom, cas, K, nullptr, nullptr, tex, mask, nullptr, stream);
}

extern "C" hfr_status hfr_discretize_reuse(const hfr_leaves* L, const hfr_domain* dom, const hfr_cascade* cas,
                                           int32_t K, const hfr_cascade* prev_cas, const float* prev_tex, float* tex,
                                           uint32_t* mask, int32_t* reused, hfr_stream stream)
{
    HFR_REQUIRE(prev_cas != nullptr, "prev_cas is NULL (use hfr_discretize for a first frame)");
    return discretize_frame(L, dom, cas, K, prev_cas, prev_tex, tex, mask, reused, stream);
}

extern "C" hfr_status hfr_discretize_backward(const hfr_leaves* L, const hfr_domain* dom, const hfr_cascade* cas,
                                              int32_t K, const float* tex, const float* grad_tex, float* grad_v,
                                              float* grad_sigma, hfr_stream stream)
{
    Tables T;
    hfr_status st = leaf_tables(L, true, &T);
    if (st == HFR_OK) st = check_cascades(cas, K);
    if (st == HFR_OK) st = check_domain(dom);
    if (st != HFR_OK) return st;
    HFR_REQUIRE(tex && grad_tex && grad_v && grad_sigma, "NULL texture or gradient buffer");
    const int N = cas[0].n;
    const Dom2 D{dom->x0, dom->y0, dom->x1, dom->y1};
    const int gx = (N + BS - 1) / BS, gy = (N + BS - 1) / BS;
    for (int k0 = 0; k0 < K; k0 += FUSE) {
        CascadeSet S;
        S.K = std::min(FUSE, K - k0);
        for (int k = 0; k < S.K; ++k) S.c[k] = tex_cascade(cas[k0 + k]);
        const float* t = tex + (int64_t)k0 * N * N;
        const float* g = grad_tex + (int64_t)k0 * N * N;
        const dim3 grid(gx * gy * S.K), block(64 * WAVES);
        if (L->basis == HFR_BASIS_WENDLAND)
            discretize_backward_kernel<HFR_BASIS_WENDLAND><<<grid, block, 0, (hipStream_t)stream>>>(
                T, S, D, gx, gy, t, g, grad_v, grad_sigma);
        else
            discretize_backward_kernel<HFR_BASIS_GAUSSIAN><<<grid, block, 0, (hipStream_t)stream>>>(
                T, S, D, gx, gy, t, g, grad_v, grad_sigma);
        HFR_LAUNCH_CHECK("discretize_backward");
    }
    return hfr_ok();
}

hfr_status launch_discretize_batch(const BatchDev& P, int blocks, bool backward, hipStream_t s)
{
    const dim3 grid(blocks), block(64 * WAVES);
    if (P.any_wendland) {
        if (backward) discretize_batch_kernel<true, true><<<grid, block, 0, s>>>(P);
        else discretize_batch_kernel<false, true><<<grid, block, 0, s>>>(P);
    } else {
        if (backward) discretize_batch_kernel<true, false><<<grid, block, 0, s>>>(P);
        else discretize_batch_kernel<false, false><<<grid, block, 0, s>>>(P);
    }
    HFR_LAUNCH_CHECK(backward ? "discretize_backward (batch)" : "discretize (batch)");
    return HFR_OK;
}
