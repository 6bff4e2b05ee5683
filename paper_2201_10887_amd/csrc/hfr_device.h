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
