// Maximum mipmap over the cascade textures (Tevs et al. 2008, the
// acceleration structure of Section 5).  gfx950, wave64.
//
// Level 0 is indexed by texture cell (the max of the cell's four corner
// texels, -inf when one is invisible, -inf on the padding row/column);
// each further level is a 2x2 max.  One pass reads a 32 x 32 tile of
// level `lin` (computing it from the texels when lin == 0), keeps it in LDS
// and writes the next five levels, so N = 2048 takes three launches and the
// texture is read once.
#include "hfr_device.h"

namespace {

__device__ __host__ inline int64_t level_offset(int N, int l)
{
    const int64_t n = N, s = N >> l;
    return (4 * n * n - 4 * s * s) / 3;
}

// Tile (bx, by) of one pass over one cascade: reads level `lin` (or the
// texels when lin == 0) and writes levels lin + 1 .. lin + nlev.
__device__ __forceinline__ void maxmip_tile(const float* __restrict__ tk, float* __restrict__ mk, int N, int lin,
                                            int nlev, int bx, int by, float (*buf)[33])
{
    const int S = N >> lin;
    const int T = S < 32 ? S : 32;
    const int ti = bx * T, tj = by * T;
    const int64_t off_in = level_offset(N, lin);
    for (int e = threadIdx.x; e < T * T; e += blockDim.x) {
        const int li = e % T, lj = e / T;
        const int i = ti + li, j = tj + lj;
        float v;
        if (lin == 0) {
            v = -INFINITY;
            if (i < N - 1 && j < N - 1) {
                const float a = tk[(int64_t)j * N + i], b = tk[(int64_t)j * N + i + 1];
                const float c = tk[(int64_t)(j + 1) * N + i], d = tk[(int64_t)(j + 1) * N + i + 1];
                if (isfinite(a) && isfinite(b) && isfinite(c) && isfinite(d)) v = fmaxf(fmaxf(a, b), fmaxf(c, d));
            }
            mk[off_in + (int64_t)j * S + i] = v;
        } else {
            v = mk[off_in + (int64_t)j * S + i];
        }
        buf[lj][li] = v;
    }
    __syncthreads();
    int cur = T;
    for (int m = 1; m <= nlev; ++m) {
        const int nt = cur >> 1;
        const int So = S >> m;
        const int64_t off_out = level_offset(N, lin + m);
        float r = -INFINITY;
        const int e = threadIdx.x;
        const int a = e % (nt > 0 ? nt : 1), b = e / (nt > 0 ? nt : 1);
        const bool act = e < nt * nt;
        if (act) r = fmaxf(fmaxf(buf[2 * b][2 * a], buf[2 * b][2 * a + 1]), fmaxf(buf[2 * b + 1][2 * a], buf[2 * b + 1][2 * a + 1]));
        __syncthreads();
        if (act) {
            buf[b][a] = r;
            mk[off_out + (int64_t)((tj >> m) + b) * So + (ti >> m) + a] = r;
        }
        __syncthreads();
        cur = nt;
    }
}

__global__ __launch_bounds__(256) void maxmip_kernel(const float* __restrict__ tex, float* __restrict__ mip, int N,
                                                     int lin, int nlev)
{
    __shared__ float buf[32][33];
    const int k = blockIdx.z;
    maxmip_tile(tex + (int64_t)k * N * N, mip + (int64_t)k * ((4 * (int64_t)N * N - 1) / 3), N, lin, nlev,
                blockIdx.x, blockIdx.y, buf);
}

// Levels of pass p (lin = 5 p) and the tile side of that pass for N.
__device__ __host__ inline void pass_shape(int N, int p, int* lin, int* nlev, int* tiles)
{
    int L = 0;
    while ((1 << L) < N) ++L;
    *lin = 5 * p;
    const int S = N >> *lin, T = S < 32 ? S : 32;
    int lt = 0;
    while ((1 << lt) < T) ++lt;
    *nlev = *lin < L ? (lt < L - *lin ? lt : L - *lin) : 0;
    *tiles = *nlev > 0 ? S / T : 0;
}

// Pass p over every cascade of a batch: workgroup b takes the MIP_GRAIN
// consecutive tiles [b MIP_GRAIN, (b + 1) MIP_GRAIN) of the pass's tile list
// (one search, then a forward walk over the cascades).
constexpr int MIP_GRAIN = 4;

__global__ __launch_bounds__(256) void maxmip_batch_kernel(BatchDev P, int p, int total)
{
    __shared__ float buf[32][33];
    const int* start = P.mip_start + p * (P.n_tex + 1);
    const int w0 = blockIdx.x * MIP_GRAIN, w1 = min(w0 + MIP_GRAIN, total);
    int item = find_item(start, P.n_tex, w0);
    int lo = start[item], hi = start[item + 1];
    for (int w = w0; w < w1; ++w) {
        while (w >= hi) {  // w < total, so this stops at a cascade that holds w
            ++item;
            lo = hi;
            hi = start[item + 1];
        }
        const BatchTex& it = as_constant(P.tex, item);
        int lin, nlev, tiles;
        pass_shape(it.C.n, p, &lin, &nlev, &tiles);
        const int local = w - lo;
        if (w > w0) __syncthreads();  // buf is reused
        maxmip_tile(it.tex, it.mip, it.C.n, lin, nlev, local % tiles, local / tiles, buf);
    }
}

}  // namespace

// Host view of the pass schedule (the same rule as the kernels use).
void maxmip_pass_shape(int N, int p, int* lin, int* nlev, int* tiles) { pass_shape(N, p, lin, nlev, tiles); }

hfr_status launch_maxmip_batch(const BatchDev& P, const int* pass_blocks, hipStream_t s)
{
    for (int p = 0; p < HFR_MIP_PASSES; ++p) {
        if (pass_blocks[p] == 0) continue;
        maxmip_batch_kernel<<<dim3((pass_blocks[p] + MIP_GRAIN - 1) / MIP_GRAIN), dim3(256), 0, s>>>(P, p,
                                                                                                  pass_blocks[p]);
        HFR_LAUNCH_CHECK("build_maxmip (batch)");
    }
    return HFR_OK;
}

extern "C" hfr_status hfr_build_maxmip(const float* tex, int32_t K, int32_t N, float* mip, hfr_stream stream)
{
    HFR_REQUIRE(tex != nullptr && mip != nullptr, "tex and mip must not be NULL");
    HFR_REQUIRE(K >= 1 && K <= HFR_MAX_CASCADES, "K = %d outside [1, %d]", K, HFR_MAX_CASCADES);
    HFR_REQUIRE(hfr_is_pow2(N) && N >= 2 && N <= HFR_MAX_TEX_N, "N = %d is not a power of two in [2, %d]", N,
                HFR_MAX_TEX_N);
    const int L = hfr_log2i(N);
    int lin = 0;
    while (true) {
        const int S = N >> lin;
        const int T = S < 32 ? S : 32;
        const int nlev = std::min(hfr_log2i(T), L - lin);
        maxmip_kernel<<<dim3(S / T, S / T, K), dim3(256), 0, (hipStream_t)stream>>>(tex, mip, N, lin, nlev);
        HFR_LAUNCH_CHECK("build_maxmip");
        if (lin + nlev >= L) break;
        lin += nlev;
    }
    return hfr_ok();
}
