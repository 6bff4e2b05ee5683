// Maximum mipmap over the cascade textures (Tevs et al. 2008, the
// acceleration structure of Section 5).  gfx950, wave64.
//
// Level 0 is indexed by texture cell: the max of the cell's four corner
// texels, -inf when one is invisible, -inf on the padding row and column;
// each further level is the 2 x 2 max of the one below.  The ray caster
// forms the level-0 maxima from the four texels it loads for the patch test
// anyway, so level 0 is not stored: its slot at the start of each pyramid is
// left as the caller had it, and the pass writes levels 1 .. log2 N.
//
// N >= 128, pass A: one workgroup per 64 x 64 cells.  The 65 x 65 texels they
// need are staged in LDS with 16-byte loads (the texture is read once); each
// thread forms the 16 cells under one level-2 node in registers, writes its
// four level-1 nodes and the level-2 node, and levels 3 .. 6
// follow in LDS.  Pass B: one workgroup per cascade reduces level 6 (at most
// 128 x 128) to the top.  Per texel: 4 B read, 4/3 B written.
// N <= 64: one workgroup per cascade does every level.
#include <type_traits>

#include "hfr_device.h"

namespace {

constexpr int MT = 64;  // cells per tile side in pass A

__device__ __host__ inline int64_t level_offset(int N, int l)
{
    const int64_t n = N, s = N >> l;
    return (4 * n * n - 4 * s * s) / 3;
}

__device__ inline int ilog2(int n)
{
    return 31 - __clz(n);
}

// Cell maximum of four texels: -inf when one of them is not visible (finite).
__device__ __forceinline__ float cell_max(float a, float b, float c, float d)
{
    return (isfinite(a) && isfinite(b) && isfinite(c) && isfinite(d)) ? fmaxf(fmaxf(a, b), fmaxf(c, d)) : -INFINITY;
}

// Levels lin + 1 .. top of one cascade from level lin, held in LDS buffer
// src (side S = N >> lin, row stride S); ping-pongs between src and dst.  Every
// thread of the workgroup takes part.
__device__ void reduce_in_lds(float* __restrict__ mk, int N, int lin, int top, float* src, float* dst)
{
    int S = N >> lin;
    for (int l = lin + 1; l <= top; ++l) {
        const int So = S >> 1;
        const int64_t off = level_offset(N, l);
        __syncthreads();
        for (int e = threadIdx.x; e < So * So; e += blockDim.x) {
            const int a = e % So, b = e / So;
            const float r = fmaxf(fmaxf(src[(2 * b) * S + 2 * a], src[(2 * b) * S + 2 * a + 1]),
                                  fmaxf(src[(2 * b + 1) * S + 2 * a], src[(2 * b + 1) * S + 2 * a + 1]));
            dst[e] = r;
            mk[off + e] = r;
        }
        float* t = src;
        src = dst;
        dst = t;
        S = So;
    }
}

struct alignas(16) TileShared {
    float tx[MT + 1][MT + 4];  // texels (rows j, columns i) of the tile, -inf beyond the texture
    float l2[2][(MT / 4) * (MT / 4)];
};

struct SmallShared {
    float buf[2][32 * 32];
};

struct TopShared {
    float buf[2][64 * 64];
};

// Pass A: cells [bx 64, bx 64 + 64) x [by 64, by 64 + 64) of one cascade (N >= 128).
__device__ void tile_body(const float* __restrict__ tk, float* __restrict__ mk, int N, int bx, int by, TileShared& sh)
{
    const int ti = bx * MT, tj = by * MT;
    // stage texel rows tj .. tj + 64 and columns ti .. ti + 64
    for (int e = threadIdx.x; e < (MT + 1) * (MT / 4); e += blockDim.x) {
        const int r = e / (MT / 4), q = e % (MT / 4);
        const int j = tj + r;
        float4 v = make_float4(-INFINITY, -INFINITY, -INFINITY, -INFINITY);
        if (j < N) v = *reinterpret_cast<const float4*>(tk + (int64_t)j * N + ti + 4 * q);
        *reinterpret_cast<float4*>(&sh.tx[r][4 * q]) = v;
    }
    for (int r = threadIdx.x; r <= MT; r += blockDim.x) {
        const int j = tj + r, i = ti + MT;
        sh.tx[r][MT] = (j < N && i < N) ? tk[(int64_t)j * N + i] : -INFINITY;
    }
    __syncthreads();
    // thread (a, b) owns level-2 node (a, b) of the tile: cells 4a .. 4a + 3, 4b .. 4b + 3
    const int a = threadIdx.x % (MT / 4), b = threadIdx.x / (MT / 4);
    float t[5][5];
#pragma unroll
    for (int y = 0; y < 5; ++y) {
        const float4 v = *reinterpret_cast<const float4*>(&sh.tx[4 * b + y][4 * a]);
        t[y][0] = v.x;
        t[y][1] = v.y;
        t[y][2] = v.z;
        t[y][3] = v.w;
        t[y][4] = sh.tx[4 * b + y][4 * a + 4];
    }
    float n1[2][2];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            float m = -INFINITY;
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int x = 0; x < 2; ++x) {
                    const int cx = 2 * p + x, cy = 2 * q + y;
                    m = fmaxf(m, cell_max(t[cy][cx], t[cy][cx + 1], t[cy + 1][cx], t[cy + 1][cx + 1]));
                }
            n1[q][p] = m;
        }
    const int S1 = N >> 1, S2 = N >> 2;
    const int64_t o1 = level_offset(N, 1), o2 = level_offset(N, 2);
    // (a pyramid of an odd cascade starts at an odd float offset: 4-byte stores)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        float* row = mk + o1 + (int64_t)(tj / 2 + 2 * b + q) * S1 + ti / 2 + 2 * a;
        row[0] = n1[q][0];
        row[1] = n1[q][1];
    }
    const float n2 = fmaxf(fmaxf(n1[0][0], n1[0][1]), fmaxf(n1[1][0], n1[1][1]));
    mk[o2 + (int64_t)(tj / 4 + b) * S2 + ti / 4 + a] = n2;
    sh.l2[0][threadIdx.x] = n2;
    // levels 3 .. 6 of the tile (16 x 16 level-2 nodes down to one level-6 node)
    float* src = sh.l2[0];
    float* dst = sh.l2[1];
    int S = MT / 4;
    for (int l = 3; l <= 6; ++l) {
        const int So = S >> 1;
        __syncthreads();
        if ((int)threadIdx.x < So * So) {
            const int u = threadIdx.x % So, w = threadIdx.x / So;
            const float r = fmaxf(fmaxf(src[(2 * w) * S + 2 * u], src[(2 * w) * S + 2 * u + 1]),
                                  fmaxf(src[(2 * w + 1) * S + 2 * u], src[(2 * w + 1) * S + 2 * u + 1]));
            dst[threadIdx.x] = r;
            const int Sl = N >> l;
            mk[level_offset(N, l) + (int64_t)((tj >> l) + w) * Sl + (ti >> l) + u] = r;
        }
        float* tmp = src;
        src = dst;
        dst = tmp;
        S = So;
    }
}

// Pass B (N >= 128): levels 7 .. log2 N of one cascade from level 6.
__device__ void top_body(float* __restrict__ mk, int N, TopShared& sh)
{
    float (*buf)[64 * 64] = sh.buf;
    const int L = ilog2(N);
    const int S6 = N >> 6, S7 = N >> 7;
    const int64_t o6 = level_offset(N, 6), o7 = level_offset(N, 7);
    for (int e = threadIdx.x; e < S7 * S7; e += blockDim.x) {
        const int a = e % S7, b = e / S7;
        const float* p = mk + o6 + (int64_t)(2 * b) * S6 + 2 * a;
        const float r = fmaxf(fmaxf(p[0], p[1]), fmaxf(p[S6], p[S6 + 1]));
        buf[0][e] = r;
        mk[o7 + e] = r;
    }
    reduce_in_lds(mk, N, 7, L, buf[0], buf[1]);
}

// N <= 64: every level of one cascade (level 1 from the texels).
__device__ void small_body(const float* __restrict__ tk, float* __restrict__ mk, int N, SmallShared& sh)
{
    float (*buf)[32 * 32] = sh.buf;
    const int L = ilog2(N);
    const int S1 = N >> 1;
    const int64_t o1 = level_offset(N, 1);
    auto texel = [&](int i, int j) { return (i < N && j < N) ? tk[(int64_t)j * N + i] : -INFINITY; };
    for (int e = threadIdx.x; e < S1 * S1; e += blockDim.x) {
        const int a = e % S1, b = e / S1;
        float m = -INFINITY;
        for (int y = 0; y < 2; ++y)
            for (int x = 0; x < 2; ++x) {
                const int i = 2 * a + x, j = 2 * b + y;
                m = fmaxf(m, cell_max(texel(i, j), texel(i + 1, j), texel(i, j + 1), texel(i + 1, j + 1)));
            }
        buf[0][e] = m;
        mk[o1 + e] = m;
    }
    reduce_in_lds(mk, N, 1, L, buf[0], buf[1]);
}

__device__ inline int64_t pyramid_size(int N) { return (4 * (int64_t)N * N - 1) / 3; }

// One workgroup per 64 x 64-cell tile of the K cascades, stacked as K * N / 64
// tile rows.  The XCD-aware mapping hands each XCD a contiguous run of tile
// rows: the texel column and row a tile shares with its right and lower
// neighbours (its 65th) then sit in the same L2 as the neighbour's own read.
__global__ __launch_bounds__(256) void maxmip_tile_kernel(const float* __restrict__ tex, float* __restrict__ mip,
                                                          int N, int K)
{
    __shared__ TileShared sh;
    const int g = N / MT;
    int tx, trow;
    xcd_tile(blockIdx.x, g, g * K, &tx, &trow);
    const int k = trow / g;
    tile_body(tex + (int64_t)k * N * N, mip + k * pyramid_size(N), N, tx, trow - k * g, sh);
}

__global__ __launch_bounds__(256) void maxmip_top_kernel(float* __restrict__ mip, int N)
{
    __shared__ TopShared sh;
    top_body(mip + blockIdx.x * pyramid_size(N), N, sh);
}

__global__ __launch_bounds__(256) void maxmip_small_kernel(const float* __restrict__ tex, float* __restrict__ mip,
                                                           int N)
{
    __shared__ SmallShared sh;
    small_body(tex + (int64_t)blockIdx.x * N * N, mip + blockIdx.x * pyramid_size(N), N, sh);
}

// Tiles per side of pass p for texture size N: pass 0 is pass A (or the whole
// pyramid when N <= 64), pass 1 is pass B.
__device__ __host__ inline int pass_tiles(int N, int p)
{
    if (p == 0) return N > MT ? N / MT : 1;
    return N > MT ? 1 : 0;
}

// Pass p over every cascade of a batch: workgroup b takes run r of MIP_GRAIN
// consecutive tiles [r MIP_GRAIN, (r + 1) MIP_GRAIN) of the pass's tile list
// (one search, then a forward walk over the cascades), where r runs
// contiguously within each XCD (the tile pass's neighbours share an L2).
constexpr int MIP_GRAIN = 4;

union Pass0Shared {
    TileShared tile;
    SmallShared small;
};

template <int PASS>
__global__ __launch_bounds__(256) void maxmip_batch_kernel(BatchDev P, int total)
{
    __shared__ typename std::conditional<PASS == 0, Pass0Shared, TopShared>::type sh;
    const int* start = P.mip_start + PASS * (P.n_tex + 1);
    int run, unused;
    xcd_tile(blockIdx.x, gridDim.x, 1, &run, &unused);
    const int w0 = run * MIP_GRAIN, w1 = min(w0 + MIP_GRAIN, total);
    int item = find_item(start, P.n_tex, w0);
    int lo = start[item], hi = start[item + 1];
    for (int w = w0; w < w1; ++w) {
        while (w >= hi) {  // w < total, so this stops at a cascade that holds w
            ++item;
            lo = hi;
            hi = start[item + 1];
        }
        const BatchTex& it = as_constant(P.tex, item);
        const int N = it.C.n;
        const int local = w - lo;
        if (w > w0) __syncthreads();  // LDS is reused
        if constexpr (PASS == 0) {
            const int tiles = pass_tiles(N, 0);
            if (N > MT) tile_body(it.tex, it.mip, N, local % tiles, local / tiles, sh.tile);
            else small_body(it.tex, it.mip, N, sh.small);
        } else {
            top_body(it.mip, N, sh);
        }
    }
}

}  // namespace

// Host view of the pass schedule (the same rule as the kernels use): tiles per side.
void maxmip_pass_shape(int N, int p, int* tiles) { *tiles = pass_tiles(N, p); }

hfr_status launch_maxmip_batch(const BatchDev& P, const int* pass_blocks, hipStream_t s)
{
    if (pass_blocks[0] > 0) {
        maxmip_batch_kernel<0><<<dim3((pass_blocks[0] + MIP_GRAIN - 1) / MIP_GRAIN), dim3(256), 0, s>>>(P,
                                                                                                  pass_blocks[0]);
        HFR_LAUNCH_CHECK("build_maxmip (batch)");
    }
    if (pass_blocks[1] > 0) {
        maxmip_batch_kernel<1><<<dim3((pass_blocks[1] + MIP_GRAIN - 1) / MIP_GRAIN), dim3(256), 0, s>>>(P,
                                                                                                  pass_blocks[1]);
        HFR_LAUNCH_CHECK("build_maxmip (batch, top levels)");
    }
    return HFR_OK;
}

extern "C" hfr_status hfr_build_maxmip(const float* tex, int32_t K, int32_t N, float* mip, hfr_stream stream)
{
    HFR_REQUIRE(tex != nullptr && mip != nullptr, "tex and mip must not be NULL");
    HFR_REQUIRE(K >= 1 && K <= HFR_MAX_CASCADES, "K = %d outside [1, %d]", K, HFR_MAX_CASCADES);
    HFR_REQUIRE(hfr_is_pow2(N) && N >= 2 && N <= HFR_MAX_TEX_N, "N = %d is not a power of two in [2, %d]", N,
                HFR_MAX_TEX_N);
    HFR_REQUIRE(reinterpret_cast<uintptr_t>(tex) % 16 == 0, "tex must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    if (N <= MT) {
        maxmip_small_kernel<<<dim3(K), dim3(256), 0, s>>>(tex, mip, N);
        HFR_LAUNCH_CHECK("build_maxmip");
        return hfr_ok();
    }
    maxmip_tile_kernel<<<dim3((N / MT) * (N / MT) * K), dim3(256), 0, s>>>(tex, mip, N, K);
    HFR_LAUNCH_CHECK("build_maxmip");
    maxmip_top_kernel<<<dim3(K), dim3(256), 0, s>>>(mip, N);
    HFR_LAUNCH_CHECK("build_maxmip (top levels)");
    return hfr_ok();
}
