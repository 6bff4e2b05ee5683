// Discretization of the truncated-Gaussian approximation into cascade
// textures (Eq. 1 and Eq. 2), with the visibility texture fused in, and its
// adjoint.  gfx950, wave64.
//
// Work decomposition: one workgroup per 32 x 8 texel tile of one cascade
// (one launch per cascade, so the cascade polygon travels as a kernel
// argument).  A wave covers two texel rows of 32, i.e. exactly two 32-bit
// visibility words, written straight from a wave ballot.
#include <cmath>

#include "hfr_device.h"

namespace {

constexpr int TILE_X = 32;
constexpr int TILE_Y = 8;
constexpr float LOG2E = 1.4426950408889634f;

struct LeafView {
    const float4* packed;
    const float* x;
    const float* y;
    const float* c;
    const float* v;
    const float* sigma;
    const int32_t* off;
    const int32_t* idx;
    const int32_t* loc;
    int n;
    int loc_n;
    double loc_x0, loc_y0, loc_inv;
};

struct Dom2 {
    double x0, y0, x1, y1;
};

__global__ __launch_bounds__(256) void pack_leaves_kernel(const float* __restrict__ x, const float* __restrict__ y,
                                                          const float* __restrict__ v, const float* __restrict__ c,
                                                          const float* __restrict__ sigma, float4* __restrict__ out,
                                                          int64_t n)
{
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const float sc = sigma[a] * c[a];
    out[a] = make_float4(x[a], y[a], v[a], -0.5f * LOG2E / (sc * sc));
}

// Visibility of the texels of this tile: cell rows j0-1 .. j0+TILE_Y-1
// get their polygon x-extent in LDS, then each texel checks its (up to
// four) incident cells.
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

__device__ inline void fill_row_extents(const TexCascade& C, int j0, double* rxl, double* rxr)
{
    const int t = threadIdx.y * TILE_X + threadIdx.x;
    if (t <= TILE_Y) {
        const int jc = j0 - 1 + t;
        double lo = INFINITY, hi = -INFINITY;
        if (jc >= 0 && jc <= C.n - 2)
            strip_extent(C, lattice_pos(C.y0, jc, C.hy), lattice_pos(C.y0, jc + 1, C.hy), &lo, &hi);
        rxl[t] = lo;
        rxr[t] = hi;
    }
}

// Texel centre clamped into the domain, and the leaf containing it.
__device__ inline int locate(const LeafView& L, const TexCascade& C, const Dom2& D, int i, int j, double* px,
                             double* py)
{
    double x = fmin(fmax(lattice_pos(C.x0, i, C.hx), D.x0), D.x1);
    double y = fmin(fmax(lattice_pos(C.y0, j, C.hy), D.y0), D.y1);
    int ix = (int)floor((x - L.loc_x0) * L.loc_inv);
    int iy = (int)floor((y - L.loc_y0) * L.loc_inv);
    ix = min(max(ix, 0), L.loc_n - 1);
    iy = min(max(iy, 0), L.loc_n - 1);
    *px = x;
    *py = y;
    return L.loc[(int64_t)iy * L.loc_n + ix];
}

__global__ __launch_bounds__(256) void discretize_kernel(LeafView L, TexCascade C, Dom2 D, float E,
                                                         float* __restrict__ tex, uint32_t* __restrict__ mask)
{
    __shared__ double rxl[TILE_Y + 1], rxr[TILE_Y + 1];
    const int N = C.n;
    const int i0 = blockIdx.x * TILE_X, j0 = blockIdx.y * TILE_Y;
    fill_row_extents(C, j0, rxl, rxr);
    __syncthreads();
    const int i = i0 + threadIdx.x, j = j0 + threadIdx.y;
    const bool inside = i < N && j < N;
    const bool vis = inside && texel_visible(C, rxl, rxr, j0, i, j);
    if (mask) {
        // a wave holds rows (2w, 2w+1) of the tile: lanes 0-31 and 32-63
        const uint64_t bits = __ballot(vis);
        const int lane = (threadIdx.y & 1) * TILE_X + threadIdx.x;
        if (inside && (lane & 31) == 0) {
            const int words = (N + 31) / 32;
            mask[(int64_t)j * words + blockIdx.x] = (uint32_t)(bits >> (lane & 32));
        }
    }
    if (!inside) return;
    float out = -INFINITY;
    if (vis) {
        double px, py;
        const int leaf = locate(L, C, D, i, j, &px, &py);
        const float fx = (float)px, fy = (float)py;
        float s0 = 0.0f, s1 = 0.0f;
        const bool ok = (unsigned)leaf < (unsigned)L.n;
        const int b = ok ? L.off[leaf] : 0, e = ok ? L.off[leaf + 1] : 0;
        for (int q = b; q < e; ++q) {
            const int jl = L.idx[q];
            if ((unsigned)jl >= (unsigned)L.n) continue;
            const float4 r = L.packed[jl];
            const float dx = r.x - fx, dy = r.y - fy;
            const float g = __builtin_amdgcn_exp2f(r.w * (dx * dx + dy * dy));
            const float w = fmaxf(g - E, 0.0f);
            s0 += w;
            s1 = fmaf(w, r.z, s1);
        }
        out = s0 > 0.0f ? s1 / s0 : NAN;
    }
    tex[(int64_t)j * N + i] = out;
}

// Adjoint of Eq. 2 / Eq. 1 for one texel: recompute S0 and scatter
// g w_j / S0 and g (v_j - v_s) / S0 * dw_j/dsigma_j.
__global__ __launch_bounds__(256) void discretize_backward_kernel(LeafView L, TexCascade C, Dom2 D, float cutoff,
                                                                  const float* __restrict__ tex,
                                                                  const float* __restrict__ gtex,
                                                                  float* __restrict__ gv, float* __restrict__ gs)
{
    const int N = C.n;
    const int i = blockIdx.x * TILE_X + threadIdx.x, j = blockIdx.y * TILE_Y + threadIdx.y;
    if (i >= N || j >= N) return;
    const int64_t s = (int64_t)j * N + i;
    const float g = gtex[s];
    const float vs = tex[s];
    if (g == 0.0f || !isfinite(vs)) return;
    double px, py;
    const int leaf = locate(L, C, D, i, j, &px, &py);
    if ((unsigned)leaf >= (unsigned)L.n) return;
    const float fx = (float)px, fy = (float)py;
    const float E = expf(-0.5f * cutoff * cutoff);
    const int b = L.off[leaf], e = L.off[leaf + 1];
    float s0 = 0.0f;
    for (int q = b; q < e; ++q) {
        const int jl = L.idx[q];
        if ((unsigned)jl >= (unsigned)L.n) continue;
        const float dx = L.x[jl] - fx, dy = L.y[jl] - fy;
        const float sc = L.sigma[jl] * L.c[jl];
        const float q2 = (dx * dx + dy * dy) / (sc * sc);
        s0 += fmaxf(expf(-0.5f * q2) - E, 0.0f);
    }
    if (!(s0 > 0.0f)) return;
    const float gn = g / s0;
    for (int q = b; q < e; ++q) {
        const int jl = L.idx[q];
        if ((unsigned)jl >= (unsigned)L.n) continue;
        const float dx = L.x[jl] - fx, dy = L.y[jl] - fy;
        const float sig = L.sigma[jl];
        const float sc = sig * L.c[jl];
        const float q2 = (dx * dx + dy * dy) / (sc * sc);
        const float ex = expf(-0.5f * q2);
        const float w = ex - E;
        if (!(w > 0.0f)) continue;
        atomicAdd(&gv[jl], gn * w);
        atomicAdd(&gs[jl], gn * (L.v[jl] - vs) * ex * q2 / sig);
    }
}

hfr_status leaf_view(const hfr_leaves* L, bool need_packed, LeafView* out)
{
    HFR_REQUIRE(L != nullptr, "leaves are NULL");
    HFR_REQUIRE(L->n >= 1 && L->n <= INT32_MAX, "leaf count %lld outside [1, INT32_MAX]", (long long)L->n);
    HFR_REQUIRE(L->nbr_off && L->nbr_idx && L->loc, "influence lists and locator are required");
    HFR_REQUIRE(!need_packed || L->packed, "packed leaves are required (hfr_pack_leaves)");
    HFR_REQUIRE(L->loc_n >= 1 && L->loc_n <= (1 << 16), "loc_n = %d outside [1, 65536]", L->loc_n);
    HFR_REQUIRE(std::isfinite(L->loc_cell) && L->loc_cell > 0 && std::isfinite(L->loc_x0) && std::isfinite(L->loc_y0),
                "invalid locator lattice");
    *out = LeafView{reinterpret_cast<const float4*>(L->packed), L->x, L->y, L->c, L->v, L->sigma,
                    L->nbr_off, L->nbr_idx, L->loc, (int)L->n, L->loc_n, L->loc_x0, L->loc_y0, 1.0 / L->loc_cell};
    return HFR_OK;
}

}  // namespace

extern "C" hfr_status hfr_pack_leaves(const hfr_leaves* L, hfr_stream stream)
{
    HFR_REQUIRE(L != nullptr, "leaves are NULL");
    HFR_REQUIRE(L->n >= 1 && L->n <= INT32_MAX, "leaf count %lld outside [1, INT32_MAX]", (long long)L->n);
    HFR_REQUIRE(L->x && L->y && L->v && L->c && L->sigma && L->packed, "leaf arrays must not be NULL");
    const int64_t blocks = (L->n + 255) / 256;
    pack_leaves_kernel<<<dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream>>>(
        L->x, L->y, L->v, L->c, L->sigma, reinterpret_cast<float4*>(L->packed), L->n);
    HFR_LAUNCH_CHECK("pack_leaves");
    return hfr_ok();
}

extern "C" hfr_status hfr_discretize(const hfr_leaves* L, const hfr_domain* dom, const hfr_cascade* cas,
                                     int32_t K, float cutoff, float* tex, uint32_t* mask, hfr_stream stream)
{
    LeafView lv;
    hfr_status st = leaf_view(L, true, &lv);
    if (st == HFR_OK) st = check_cascades(cas, K);
    if (st == HFR_OK) st = check_domain(dom);
    if (st != HFR_OK) return st;
    HFR_REQUIRE(tex != nullptr, "tex is NULL");
    HFR_REQUIRE(std::isfinite(cutoff) && cutoff > 0, "cutoff must be positive");
    const int N = cas[0].n;
    const float E = std::exp(-0.5f * cutoff * cutoff);
    const Dom2 D{dom->x0, dom->y0, dom->x1, dom->y1};
    const dim3 grid((N + TILE_X - 1) / TILE_X, (N + TILE_Y - 1) / TILE_Y);
    const int words = (N + 31) / 32;
    for (int k = 0; k < K; ++k) {
        discretize_kernel<<<grid, dim3(TILE_X, TILE_Y), 0, (hipStream_t)stream>>>(
            lv, tex_cascade(cas[k]), D, E, tex + (int64_t)k * N * N, mask ? mask + (int64_t)k * N * words : nullptr);
        HFR_LAUNCH_CHECK("discretize");
    }
    return hfr_ok();
}

extern "C" hfr_status hfr_discretize_backward(const hfr_leaves* L, const hfr_domain* dom, const hfr_cascade* cas,
                                              int32_t K, float cutoff, const float* tex, const float* grad_tex,
                                              float* grad_v, float* grad_sigma, hfr_stream stream)
{
    LeafView lv;
    hfr_status st = leaf_view(L, false, &lv);
    if (st == HFR_OK) st = check_cascades(cas, K);
    if (st == HFR_OK) st = check_domain(dom);
    if (st != HFR_OK) return st;
    HFR_REQUIRE(L->x && L->y && L->c && L->v && L->sigma, "leaf arrays must not be NULL");
    HFR_REQUIRE(tex && grad_tex && grad_v && grad_sigma, "NULL texture or gradient buffer");
    HFR_REQUIRE(std::isfinite(cutoff) && cutoff > 0, "cutoff must be positive");
    const int N = cas[0].n;
    const Dom2 D{dom->x0, dom->y0, dom->x1, dom->y1};
    const dim3 grid((N + TILE_X - 1) / TILE_X, (N + TILE_Y - 1) / TILE_Y);
    for (int k = 0; k < K; ++k) {
        discretize_backward_kernel<<<grid, dim3(TILE_X, TILE_Y), 0, (hipStream_t)stream>>>(
            lv, tex_cascade(cas[k]), D, cutoff, tex + (int64_t)k * N * N, grad_tex + (int64_t)k * N * N, grad_v,
            grad_sigma);
        HFR_LAUNCH_CHECK("discretize_backward");
    }
    return hfr_ok();
}
