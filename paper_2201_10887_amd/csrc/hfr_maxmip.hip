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

__global__ __launch_bounds__(256) void maxmip_kernel(const float* __restrict__ tex, float* __restrict__ mip, int N,
                                                     int lin, int nlev)
{
    __shared__ float buf[32][33];
    const int k = blockIdx.z;
    const int S = N >> lin;
    const int T = S < 32 ? S : 32;
    const int ti = blockIdx.x * T, tj = blockIdx.y * T;
    const float* tk = tex + (int64_t)k * N * N;
    float* mk = mip + (int64_t)k * ((4 * (int64_t)N * N - 1) / 3);
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

}  // namespace

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
