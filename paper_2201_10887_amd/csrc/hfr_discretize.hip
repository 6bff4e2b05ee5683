// Discretization of the truncated-Gaussian approximation into cascade
// textures (Eq. 1 and Eq. 2), with the visibility texture fused in, and its
// adjoint.  gfx950, wave64.
//
// Work decomposition.  A workgroup covers a 32 x 8 texel block of one
// cascade (one launch per cascade, so the cascade polygon travels as a
// kernel argument); each of its four waves owns an 8 x 8 texel tile.
//  1. The 9 cell rows touching the block get their polygon x-extent in LDS;
//     every texel tests its incident cells; the visibility bits of the
//     block's 8 rows (one 32-bit word each) are assembled with LDS atomics.
//  2. A wave with a visible texel finds every leaf that can influence a
//     point of its tile: per quadtree level, it scans the lattice window
//     within that level's largest truncation radius of the tile rectangle
//     in the dense node table (coalesced rows), keeps the leaves whose
//     centre is closer than the radius to the rectangle (wave ballot +
//     prefix count, no atomics), and stages their records in LDS in
//     tile-local coordinates (FP64 subtraction, then FP32).
//  3. Each lane (texel) runs Eq. 1 / Eq. 2 over the staged records with
//     broadcast LDS reads: no divergent global load in the hot loop.
// More candidates than fit in LDS are handled in rounds (rescan, next slice).
#include <cmath>

#include "hfr_device.h"

namespace {

constexpr int TS = 8;        // tile side in texels (one wave)
constexpr int WAVES = 4;     // tiles per workgroup, side by side along x
constexpr int CAP = 512;     // candidate records staged per round
constexpr float LOG2E = 1.4426950408889634f;

struct Tables {
    const float4* packed;
    const float* radius;
    const int32_t* node;
    const float* sigma;
    int n, max_depth;
    double x0, y0, side;
    float E;  // exp(-cutoff^2 / 2)
};

struct Dom2 {
    double x0, y0, x1, y1;
};

__global__ __launch_bounds__(256) void pack_leaves_kernel(const float* __restrict__ x, const float* __restrict__ y,
                                                          const float* __restrict__ v, const float* __restrict__ c,
                                                          const float* __restrict__ sigma, float cutoff, float side,
                                                          int max_depth, float4* __restrict__ out,
                                                          float* __restrict__ radius, int64_t n)
{
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const float sc = sigma[a] * c[a];
    out[a] = make_float4(x[a], y[a], v[a], -0.5f * LOG2E / (sc * sc));
    int l = (int)rintf(log2f(side / c[a]));
    l = min(max(l, 0), max_depth);
    const float R = cutoff * sc * 1.00001f;
    atomicMax(reinterpret_cast<int*>(radius) + l, __float_as_int(R));  // positive floats order as ints
}

__global__ void zero_floats_kernel(float* __restrict__ p, int n)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < n) p[a] = 0.0f;
}

__device__ inline bool texel_visible(const TexCascade& C, const double* rxl, const double* rxr, int j0, int i, int j)
{
    const int N = C.n;
    bool vis = false;
    for (int dj = -1; dj <= 0; ++dj) {
        const int jc = j + dj;
        if (jc < 0 || jc > N - 2) continue;
        const double xl = rxl[jc - (j0 - 1)], xr = rxr[jc - (j0 - 1)];
        for (int di = -1; di <= 0; ++di) {
            const int ic = i + di;
            if (ic < 0 || ic > N - 2) continue;
            const double xa = lattice_pos(C.x0, ic, C.hx), xb = lattice_pos(C.x0, ic + 1, C.hx);
            vis |= (xa <= xr) && (xb >= xl);
        }
    }
    return vis;
}

__device__ inline double clampd(double v, double lo, double hi) { return fmin(fmax(v, lo), hi); }

// Tile rectangle (clamped texel centres) of the wave's 8 x 8 tile.
struct TileRect {
    double x0, y0, x1, y1;
};

__device__ inline TileRect tile_rect(const TexCascade& C, const Dom2& D, int ti0, int tj0)
{
    const int N = C.n;
    const int ti1 = min(ti0 + TS - 1, N - 1), tj1 = min(tj0 + TS - 1, N - 1);
    TileRect r;
    r.x0 = clampd(lattice_pos(C.x0, ti0, C.hx), D.x0, D.x1);
    r.x1 = clampd(lattice_pos(C.x0, ti1, C.hx), D.x0, D.x1);
    r.y0 = clampd(lattice_pos(C.y0, tj0, C.hy), D.y0, D.y1);
    r.y1 = clampd(lattice_pos(C.y0, tj1, C.hy), D.y0, D.y1);
    return r;
}

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Appends to rec (and ids) the candidates with rank in [lo, lo + CAP) of the
// deterministic scan order (level, row, column); returns the total count.
template <bool WITH_IDS>
__device__ int scan_candidates(const Tables& T, const TileRect& r, int lo, float4* rec, int* ids, float* sig,
                               int lane)
{
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    int total = 0;
    for (int l = 0; l <= T.max_depth; ++l) {
        const float Rf = T.radius[l];
        if (!(Rf > 0.0f)) continue;
        const double R = Rf;
        const double c = T.side / (double)(1 << l);
        const int S = 1 << l;
        const int ia = max(0, (int)floor((r.x0 - R - T.x0) / c - 0.5));
        const int ib = min(S - 1, (int)ceil((r.x1 + R - T.x0) / c - 0.5));
        const int ja = max(0, (int)floor((r.y0 - R - T.y0) / c - 0.5));
        const int jb = min(S - 1, (int)ceil((r.y1 + R - T.y0) / c - 0.5));
        const int wi = ib - ia + 1, hj = jb - ja + 1;
        if (wi <= 0 || hj <= 0) continue;
        const int cnt = wi * hj;
        const float inv_w = 1.0f / (float)wi;
        const int64_t off = ((int64_t(1) << (2 * l)) - 1) / 3;
        for (int e0 = 0; e0 < cnt; e0 += 64) {
            const int e = e0 + lane;
            int id = -1;
            if (e < cnt) {
                int q = (int)((float)e * inv_w);
                int rem = e - q * wi;
                if (rem < 0) { --q; rem += wi; }
                if (rem >= wi) { ++q; rem -= wi; }
                const int ii = ia + rem, jj = ja + q;
                id = T.node[off + (int64_t)jj * S + ii];
                if (id >= 0) {
                    const double cx = T.x0 + (ii + 0.5) * c, cy = T.y0 + (jj + 0.5) * c;
                    const double dx = fmax(fmax(r.x0 - cx, cx - r.x1), 0.0);
                    const double dy = fmax(fmax(r.y0 - cy, cy - r.y1), 0.0);
                    if (!(dx * dx + dy * dy < R * R) || id >= T.n) id = -1;
                }
            }
            const uint64_t m = __ballot(id >= 0);
            if (m) {
                const int slot = total + __popcll(m & lt) - lo;
                if (id >= 0 && slot >= 0 && slot < CAP) {
                    const float4 p = T.packed[id];
                    rec[slot] = make_float4((float)((double)p.x - r.x0), (float)((double)p.y - r.y0), p.z, p.w);
                    if (WITH_IDS) {
                        ids[slot] = id;
                        sig[slot] = T.sigma[id];
                    }
                }
                total += __popcll(m);
            }
        }
    }
    return total;
}

__global__ __launch_bounds__(256) void discretize_kernel(Tables T, TexCascade C, Dom2 D, float* __restrict__ tex,
                                                         uint32_t* __restrict__ mask)
{
    __shared__ float4 rec_all[WAVES][CAP];
    __shared__ double rxl[TS + 1], rxr[TS + 1];
    __shared__ uint32_t mwords[TS];
    const int N = C.n;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int bi0 = blockIdx.x * (TS * WAVES), j0 = blockIdx.y * TS;
    if (threadIdx.x <= TS) {
        const int jc = j0 - 1 + (int)threadIdx.x;
        double lo = INFINITY, hi = -INFINITY;
        if (jc >= 0 && jc <= N - 2) strip_extent(C, lattice_pos(C.y0, jc, C.hy), lattice_pos(C.y0, jc + 1, C.hy), &lo, &hi);
        rxl[threadIdx.x] = lo;
        rxr[threadIdx.x] = hi;
    }
    if (threadIdx.x < TS) mwords[threadIdx.x] = 0u;
    __syncthreads();
    const int tx = lane & (TS - 1), ty = lane >> 3;
    const int ti0 = bi0 + wave * TS;
    const int i = ti0 + tx, j = j0 + ty;
    const bool inside = i < N && j < N;
    const bool vis = inside && texel_visible(C, rxl, rxr, j0, i, j);
    if (vis) atomicOr(&mwords[ty], 1u << (wave * TS + tx));
    __syncthreads();
    if (mask && threadIdx.x < TS && j0 + (int)threadIdx.x < N)
        mask[(int64_t)(j0 + threadIdx.x) * ((N + 31) / 32) + blockIdx.x] = mwords[threadIdx.x];
    // from here on each wave works alone
    if (__ballot(vis) == 0) {
        if (inside) tex[(int64_t)j * N + i] = -INFINITY;
        return;
    }
    float4* rec = rec_all[wave];
    const TileRect r = tile_rect(C, D, ti0, j0);
    const float px = (float)(clampd(lattice_pos(C.x0, i, C.hx), D.x0, D.x1) - r.x0);
    const float py = (float)(clampd(lattice_pos(C.y0, j, C.hy), D.y0, D.y1) - r.y0);
    const float E = T.E;
    float s0 = 0.0f, s1 = 0.0f;
    for (int lo = 0;; lo += CAP) {
        const int total = scan_candidates<false>(T, r, lo, rec, nullptr, nullptr, lane);
        wave_sync();
        const int nc = min(total - lo, CAP);
        if (vis) {
            int c = 0;
            for (; c + 4 <= nc; c += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const float4 q = rec[c + u];
                    const float dx = q.x - px, dy = q.y - py;
                    const float g = __builtin_amdgcn_exp2f(q.w * fmaf(dx, dx, dy * dy));
                    const float w = fmaxf(g - E, 0.0f);
                    s0 += w;
                    s1 = fmaf(w, q.z, s1);
                }
            }
            for (; c < nc; ++c) {
                const float4 q = rec[c];
                const float dx = q.x - px, dy = q.y - py;
                const float g = __builtin_amdgcn_exp2f(q.w * fmaf(dx, dx, dy * dy));
                const float w = fmaxf(g - E, 0.0f);
                s0 += w;
                s1 = fmaf(w, q.z, s1);
            }
        }
        wave_sync();
        if (lo + CAP >= total) break;
    }
    if (inside) tex[(int64_t)j * N + i] = vis ? (s0 > 0.0f ? s1 / s0 : NAN) : -INFINITY;
}

// Adjoint of Eq. 2 / Eq. 1.  Lanes first own texels (S0 of each texel), then
// own candidate leaves: for every texel of the tile with a non-zero gradient
// (a wave-uniform loop) each lane adds its leaf's share
//   g w_j / S0   and   g (v_j - v_s) / S0 * exp(-q^2/2) q^2 / sigma_j,
// and finally adds its two sums to the leaf's gradient with one atomic each.
__global__ __launch_bounds__(256) void discretize_backward_kernel(Tables T, TexCascade C, Dom2 D,
                                                                  const float* __restrict__ tex,
                                                                  const float* __restrict__ gtex,
                                                                  float* __restrict__ gv, float* __restrict__ gs)
{
    __shared__ float4 rec_all[WAVES][CAP];
    __shared__ int ids_all[WAVES][CAP];
    __shared__ float sig_all[WAVES][CAP];
    const int N = C.n;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ti0 = blockIdx.x * (TS * WAVES) + wave * TS, j0 = blockIdx.y * TS;
    const int i = ti0 + (lane & (TS - 1)), j = j0 + (lane >> 3);
    const bool inside = i < N && j < N;
    float g = 0.0f, vs = 0.0f;
    if (inside) {
        g = gtex[(int64_t)j * N + i];
        vs = tex[(int64_t)j * N + i];
    }
    const bool act = inside && g != 0.0f && isfinite(vs) && isfinite(g);
    const uint64_t active = __ballot(act);
    if (active == 0) return;
    float4* rec = rec_all[wave];
    int* ids = ids_all[wave];
    float* sig = sig_all[wave];
    const TileRect r = tile_rect(C, D, ti0, j0);
    const float px = (float)(clampd(lattice_pos(C.x0, i, C.hx), D.x0, D.x1) - r.x0);
    const float py = (float)(clampd(lattice_pos(C.y0, j, C.hy), D.y0, D.y1) - r.y0);
    const float E = T.E;
    // pass 1: S0 per texel
    float s0 = 0.0f;
    for (int lo = 0;; lo += CAP) {
        const int total = scan_candidates<true>(T, r, lo, rec, ids, sig, lane);
        wave_sync();
        const int nc = min(total - lo, CAP);
        for (int c = 0; c < nc; ++c) {
            const float4 q = rec[c];
            const float dx = q.x - px, dy = q.y - py;
            s0 += fmaxf(__builtin_amdgcn_exp2f(q.w * fmaf(dx, dx, dy * dy)) - E, 0.0f);
        }
        wave_sync();
        if (lo + CAP >= total) break;
    }
    const float gn = act && s0 > 0.0f ? g / s0 : 0.0f;
    // pass 2: lanes own candidates
    for (int lo = 0;; lo += CAP) {
        const int total = scan_candidates<true>(T, r, lo, rec, ids, sig, lane);
        wave_sync();
        const int nc = min(total - lo, CAP);
        for (int c0 = 0; c0 < nc; c0 += 64) {
            const int c = c0 + lane;
            const bool own = c < nc;
            float4 q = own ? rec[c] : make_float4(0.f, 0.f, 0.f, 0.f);
            const float sj = own ? sig[c] : 1.0f;
            float acc_v = 0.0f, acc_s = 0.0f;
            uint64_t m = active;
            while (m) {
                const int t = __ffsll((unsigned long long)m) - 1;
                m &= m - 1;
                const float tpx = __shfl(px, t), tpy = __shfl(py, t), tg = __shfl(gn, t), tv = __shfl(vs, t);
                const float dx = q.x - tpx, dy = q.y - tpy;
                const float r2 = fmaf(dx, dx, dy * dy);
                const float ex = __builtin_amdgcn_exp2f(q.w * r2);
                const float w = ex - E;
                if (own && w > 0.0f) {
                    const float q2 = r2 * q.w * (-2.0f / LOG2E);
                    acc_v = fmaf(tg, w, acc_v);
                    acc_s = fmaf(tg * (q.z - tv), ex * q2 / sj, acc_s);
                }
            }
            if (own && (acc_v != 0.0f || acc_s != 0.0f)) {
                atomicAdd(&gv[ids[c]], acc_v);
                atomicAdd(&gs[ids[c]], acc_s);
            }
        }
        wave_sync();
        if (lo + CAP >= total) break;
    }
}

hfr_status tables_of(const hfr_leaves* L, bool backward, Tables* out)
{
    HFR_REQUIRE(L != nullptr, "leaves are NULL");
    HFR_REQUIRE(L->n >= 1 && L->n <= INT32_MAX, "leaf count %lld outside [1, INT32_MAX]", (long long)L->n);
    HFR_REQUIRE(L->packed && L->level_radius && L->node, "packed records, level radii and node table are required");
    HFR_REQUIRE(!backward || L->sigma, "sigma is required");
    HFR_REQUIRE(L->max_depth >= 0 && L->max_depth <= 15, "max_depth %d outside [0, 15]", L->max_depth);
    HFR_REQUIRE(std::isfinite(L->cutoff) && L->cutoff > 0, "cutoff must be positive");
    HFR_REQUIRE(std::isfinite(L->side) && L->side > 0 && std::isfinite(L->x0) && std::isfinite(L->y0),
                "invalid lattice square");
    *out = Tables{reinterpret_cast<const float4*>(L->packed), L->level_radius, L->node, L->sigma, (int)L->n,
                  L->max_depth, L->x0, L->y0, L->side, std::exp(-0.5f * L->cutoff * L->cutoff)};
    return HFR_OK;
}

}  // namespace

extern "C" hfr_status hfr_pack_leaves(const hfr_leaves* L, hfr_stream stream)
{
    HFR_REQUIRE(L != nullptr, "leaves are NULL");
    HFR_REQUIRE(L->n >= 1 && L->n <= INT32_MAX, "leaf count %lld outside [1, INT32_MAX]", (long long)L->n);
    HFR_REQUIRE(L->x && L->y && L->v && L->c && L->sigma && L->packed && L->level_radius,
                "leaf arrays must not be NULL");
    HFR_REQUIRE(L->max_depth >= 0 && L->max_depth <= 15, "max_depth %d outside [0, 15]", L->max_depth);
    HFR_REQUIRE(std::isfinite(L->cutoff) && L->cutoff > 0, "cutoff must be positive");
    HFR_REQUIRE(std::isfinite(L->side) && L->side > 0, "side must be positive");
    hipStream_t s = (hipStream_t)stream;
    zero_floats_kernel<<<1, 64, 0, s>>>(L->level_radius, L->max_depth + 1);
    HFR_LAUNCH_CHECK("pack_leaves (radius reset)");
    const int64_t blocks = (L->n + 255) / 256;
    pack_leaves_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(
        L->x, L->y, L->v, L->c, L->sigma, L->cutoff, (float)L->side, L->max_depth,
        reinterpret_cast<float4*>(L->packed), L->level_radius, L->n);
    HFR_LAUNCH_CHECK("pack_leaves");
    return hfr_ok();
}

extern "C" hfr_status hfr_discretize(const hfr_leaves* L, const hfr_domain* dom, const hfr_cascade* cas, int32_t K,
                                     float* tex, uint32_t* mask, hfr_stream stream)
{
    Tables T;
    hfr_status st = tables_of(L, false, &T);
    if (st == HFR_OK) st = check_cascades(cas, K);
    if (st == HFR_OK) st = check_domain(dom);
    if (st != HFR_OK) return st;
    HFR_REQUIRE(tex != nullptr, "tex is NULL");
    const int N = cas[0].n;
    const Dom2 D{dom->x0, dom->y0, dom->x1, dom->y1};
    const dim3 grid((N + TS * WAVES - 1) / (TS * WAVES), (N + TS - 1) / TS);
    const int words = (N + 31) / 32;
    for (int k = 0; k < K; ++k) {
        discretize_kernel<<<grid, dim3(64 * WAVES), 0, (hipStream_t)stream>>>(
            T, tex_cascade(cas[k]), D, tex + (int64_t)k * N * N, mask ? mask + (int64_t)k * N * words : nullptr);
        HFR_LAUNCH_CHECK("discretize");
    }
    return hfr_ok();
}

extern "C" hfr_status hfr_discretize_backward(const hfr_leaves* L, const hfr_domain* dom, const hfr_cascade* cas,
                                              int32_t K, const float* tex, const float* grad_tex, float* grad_v,
                                              float* grad_sigma, hfr_stream stream)
{
    Tables T;
    hfr_status st = tables_of(L, true, &T);
    if (st == HFR_OK) st = check_cascades(cas, K);
    if (st == HFR_OK) st = check_domain(dom);
    if (st != HFR_OK) return st;
    HFR_REQUIRE(tex && grad_tex && grad_v && grad_sigma, "NULL texture or gradient buffer");
    const int N = cas[0].n;
    const Dom2 D{dom->x0, dom->y0, dom->x1, dom->y1};
    const dim3 grid((N + TS * WAVES - 1) / (TS * WAVES), (N + TS - 1) / TS);
    for (int k = 0; k < K; ++k) {
        discretize_backward_kernel<<<grid, dim3(64 * WAVES), 0, (hipStream_t)stream>>>(
            T, tex_cascade(cas[k]), D, tex + (int64_t)k * N * N, grad_tex + (int64_t)k * N * N, grad_v, grad_sigma);
        HFR_LAUNCH_CHECK("discretize_backward");
    }
    return hfr_ok();
}
