// Ray casting of the cascade textures (Section 5) and its adjoint.
// gfx950, wave64.
//
// One thread per pixel; 16 x 16 pixel workgroups keep the rays of a wave
// spatially coherent.  All geometry is FP64: gfx950 issues FP64 FMA at the
// same rate as non-packed FP32, and FP64 makes the cell walk and the
// patch root agree with an exact evaluation except on measure-zero ties.
// Inside a cascade the ray descends the maximum mipmap: a node is skipped
// when the ray's lowest z over its part of the node is above the node's
// maximum; a level-0 cell whose four texels are visible is intersected
// with the bilinear patch in closed form (its four texels also give the
// level-0 maximum, so level 0 reads no pyramid).  After each step the walk
// climbs at most one level, and not at all after a cell whose patch it had to
// test: the frame time is set by the longest rays, which graze the surface
// and gain nothing from larger nodes.
#include "hfr_device.h"

namespace {



struct Ray {
    double o[3], d[3], inv_d[2];
};

struct Hit {
    int k, i, j, start;
    double t, u, v, fp;
};

// Offset of level l in a max-mipmap of N = 2^L texels per side: the sizes of
// the finer levels, 4^L + ... + 4^(L-l+1) = P(L+1) - P(L-l+1) with P(n) =
// (4^n - 1) / 3, the base-4 repunit 0x55...5 of n digits.  For N <= 8192 it
// fits in 32 bits.
__device__ inline int level_offset(int L, int l)
{
    return (int)((0x55555555u >> (30 - 2 * L)) - (0x55555555u >> (30 - 2 * (L - l))));
}

__device__ inline void slab(double o, double d, double lo, double hi, double& t0, double& t1)
{
    if (d == 0.0) {
        if (o < lo || o > hi) {
            t0 = INFINITY;
            t1 = -INFINITY;
        }
        return;
    }
    const double a = (lo - o) / d, b = (hi - o) / d;
    t0 = fmax(t0, fmin(a, b));
    t1 = fmin(t1, fmax(a, b));
}

// t-range of the ray where lo <= d(t) <= hi and inside the texture rectangle,
// intersected with [tin, tout].
__device__ inline void segment(const Ray& r, const RayCas& c, double lo, double hi, double tin, double tout,
                               double& ta, double& tb)
{
    ta = tin;
    tb = tout;
    const double d0 = (r.o[0] - c.ox) * c.vx + (r.o[1] - c.oy) * c.vy;
    const double dd = r.d[0] * c.vx + r.d[1] * c.vy;
    if (dd > 0.0) {
        ta = fmax(ta, (lo - d0) / dd);
        tb = fmin(tb, (hi - d0) / dd);
    } else if (dd < 0.0) {
        ta = fmax(ta, (hi - d0) / dd);
        tb = fmin(tb, (lo - d0) / dd);
    } else if (d0 < lo || d0 > hi) {
        ta = INFINITY;
        tb = -INFINITY;
    }
    slab(r.o[0], r.d[0], c.x0, lattice_pos(c.x0, c.n - 1, c.hx), ta, tb);
    slab(r.o[1], r.d[1], c.y0, lattice_pos(c.y0, c.n - 1, c.hy), ta, tb);
}

__device__ inline double offset_at(const Ray& r, const RayCas& c, double t)
{
    return ((r.o[0] + t * r.d[0]) - c.ox) * c.vx + ((r.o[1] + t * r.d[1]) - c.oy) * c.vy;
}

// First t' > t at which one coordinate crosses a texel line base + m h.
__device__ inline double next_crossing(double o, double d, double inv_d, double base, double h, double inv_h, double t)
{
    if (d == 0.0) return INFINITY;
    const double w = ((o + t * d) - base) * inv_h;
    double m = d > 0.0 ? floor(w) + 1.0 : ceil(w) - 1.0;
    const double step = d > 0.0 ? 1.0 : -1.0;
    for (int g = 0; g < 4; ++g) {
        const double tm = (add_rn(base, mul_rn(m, h)) - o) * inv_d;
        if (tm > t) return tm;
        m += step;
    }
    return INFINITY;
}

__device__ inline double piece_end(const Ray& r, const RayCas& c, double t, double tb)
{
    return fmin(tb, fmin(next_crossing(r.o[0], r.d[0], r.inv_d[0], c.x0, c.hx, c.inv_hx, t),
                         next_crossing(r.o[1], r.d[1], r.inv_d[1], c.y0, c.hy, c.inv_hy, t)));
}

__device__ inline void cell_at(const Ray& r, const RayCas& c, double t, int& i, int& j)
{
    i = (int)floor(((r.o[0] + t * r.d[0]) - c.x0) * c.inv_hx);
    j = (int)floor(((r.o[1] + t * r.d[1]) - c.y0) * c.inv_hy);
    i = min(max(i, 0), c.n - 2);
    j = min(max(j, 0), c.n - 2);
}

// Smallest tau in [0, tau1] with a tau^2 + b tau + c <= 0, given c > 0.
__device__ inline bool smallest_root(double a, double b, double c, double tau1, double& tau)
{
    // Division-free rejection first (most cells a grazing ray tests hold no root).  With
    // f(0) = c > 0 a root in [0, tau1] needs f(tau1) <= 0, or, for a convex f (a > 0), a
    // minimum inside the interval with a non-negative discriminant.  The margins are far
    // above FP64 rounding, so every case near the boundary takes the exact path below.
    const double f1 = (a * tau1 + b) * tau1 + c;
    if (f1 > 1e-12 * ((fabs(a) * tau1 + fabs(b)) * tau1 + fabs(c))) {
        if (!(a > 0.0 && b < 0.0 && -b < 2.0 * a * tau1)) return false;
        if (b * b - 4.0 * a * c < -1e-12 * (b * b + 4.0 * fabs(a * c))) return false;
    }
    double best = INFINITY;
    if (a == 0.0) {
        if (b < 0.0) {
            const double q = -c / b;
            if (q <= tau1) best = q;
        }
    } else {
        const double D = b * b - 4.0 * a * c;
        if (D >= 0.0) {
            const double q = -0.5 * (b + copysign(sqrt(D), b));
            const double r1 = q / a, r2 = c / q;
            if (r1 >= 0.0 && r1 <= tau1) best = fmin(best, r1);
            if (r2 >= 0.0 && r2 <= tau1) best = fmin(best, r2);
        }
    }
    if (best == INFINITY) return false;
    tau = best;
    return true;
}

// Node of level l holding cell (ci, cj): exit parameter along the ray.
__device__ inline double node_exit(const Ray& r, const RayCas& c, int ci, int cj, int l, double tb)
{
    // the boundary the ray leaves through on each axis: (I + 1) << l moving up, I << l moving down
    const int bx = ((ci >> l) + (r.d[0] > 0.0 ? 1 : 0)) << l;
    const int by = ((cj >> l) + (r.d[1] > 0.0 ? 1 : 0)) << l;
    const double tx = (lattice_pos(c.x0, bx, c.hx) - r.o[0]) * r.inv_d[0];
    const double ty = (lattice_pos(c.y0, by, c.hy) - r.o[1]) * r.inv_d[1];
    double te = tb;
    if (r.d[0] != 0.0) te = fmin(te, tx);
    if (r.d[1] != 0.0) te = fmin(te, ty);
    return te;
}

__device__ bool first_hit(const Ray& r, const RayCas& c, int k, const float* __restrict__ tex,
                          const float* __restrict__ mip, double ta, double tb, Hit& h)
{
    if (!(ta < tb)) return false;
    const int N = c.n, L = c.levels;
    double t = ta;
    double t1 = piece_end(r, c, t, tb);
    int ci, cj;
    cell_at(r, c, 0.5 * (t + t1), ci, cj);
    int l = L;
    // every iteration either descends a level or moves to a later piece
    const int max_iter = 8 * N * (L + 2) + 64;
    for (int it = 0; it < max_iter; ++it) {
        // Node maximum: from the max-mipmap above level 0; at level 0 from the cell's own four
        // texels (the same value the pyramid holds there), which the patch test needs anyway,
        // so a cell costs one round of loads instead of two.
        float M, t00 = 0.f, t10 = 0.f, t01 = 0.f, t11 = 0.f;
        if (l > 0) {
            M = mip[level_offset(L, l) + (cj >> l) * (N >> l) + (ci >> l)];
        } else {
            const int64_t b = (int64_t)cj * N + ci;
            t00 = tex[b];
            t10 = tex[b + 1];
            t01 = tex[b + N];
            t11 = tex[b + N + 1];
            M = (isfinite(t00) && isfinite(t10) && isfinite(t01) && isfinite(t11))
                    ? fmaxf(fmaxf(t00, t10), fmaxf(t01, t11)) : -INFINITY;
        }
        const double te = fmax(node_exit(r, c, ci, cj, l, tb), t1);
        const double za = r.o[2] + t * r.d[2], zb = r.o[2] + te * r.d[2];
        bool advance = false, close = false;
        if (fmin(za, zb) > (double)M) {
            advance = true;
        } else if (l > 0) {
            --l;
        } else {
            const double h00 = t00, h10 = t10, h01 = t01, h11 = t11;
            const double u0 = ((r.o[0] + t * r.d[0]) - c.x0) * c.inv_hx - ci;
            const double v0 = ((r.o[1] + t * r.d[1]) - c.y0) * c.inv_hy - cj;
            const double du = r.d[0] * c.inv_hx, dv = r.d[1] * c.inv_hy;
            const double A = h10 - h00, B = h01 - h00, C = (h00 - h10) - (h01 - h11);
            const double cc = za - (h00 + A * u0 + B * v0 + C * u0 * v0);
            const double bb = r.d[2] - A * du - B * dv - C * (u0 * dv + v0 * du);
            const double aa = -C * du * dv;
            double tau = 0.0;
            if (cc <= 0.0 || smallest_root(aa, bb, cc, te - t, tau)) {
                h.k = k;
                h.i = ci;
                h.j = cj;
                h.t = t + tau;
                h.u = u0 + tau * du;
                h.v = v0 + tau * dv;
                h.fp = 2.0 * aa * tau + bb;
                h.start = (cc <= 0.0 && t == ta);
                return true;
            }
            advance = true;
            close = true;  // the ray passed below this cell's highest texel
        }
        if (advance) {
            if (te >= tb) return false;
            t = te;
            t1 = piece_end(r, c, t, tb);
            int ni, nj;
            cell_at(r, c, 0.5 * (t + t1), ni, nj);
            const unsigned diff = (unsigned)((ni ^ ci) | (nj ^ cj));
            ci = ni;
            cj = nj;
            // climb at most one level per step, and none after a cell the ray passed below
            // the top of: a ray running close to the surface stays on level 0 instead of
            // testing (and descending from) a larger node at every cell
            if (diff) l = min(31 - __clz(diff), l + (close ? 0 : 1));
        }
    }
    return false;
}

// Pixel (col, row) of one view.  In the adjoint every lane of the wave must
// call it (the gradient scatter uses wave-wide shuffles), also lanes
// outside the image.
template <bool BACKWARD>
__device__ __forceinline__ void raycast_pixel(const RayArgs& A, int col, int row, const float* __restrict__ tex,
                                              const float* __restrict__ mip, float* __restrict__ depth,
                                              int32_t* __restrict__ hit, const float* __restrict__ gdepth,
                                              float* __restrict__ gtex)
{
    const bool in_image = col < A.W && row < A.H;
    if (!BACKWARD && !in_image) return;
    const int64_t p = (int64_t)row * A.W + col;
    float g = 0.0f;
    if (BACKWARD && in_image) g = gdepth[p];
    // in the adjoint every lane stays to the end (the scatter uses wave-wide shuffles)
    const bool live = in_image && (!BACKWARD || (g != 0.0f && isfinite(g)));
    const double sx = ((col + 0.5) / A.W) * 2.0 - 1.0;
    const double sy = 1.0 - ((row + 0.5) / A.H) * 2.0;
    Ray r;
    double n2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        r.o[a] = A.o[a];
        r.d[a] = A.fwd[a] + (sx * A.tx) * A.right[a] + (sy * A.ty) * A.up[a];
        n2 += r.d[a] * r.d[a];
    }
    const double inv_n = 1.0 / sqrt(n2);
    for (int a = 0; a < 3; ++a) r.d[a] *= inv_n;
    r.inv_d[0] = 1.0 / r.d[0];
    r.inv_d[1] = 1.0 / r.d[1];

    // clip to the domain box: xy slabs and z <= zmax
    double tin = 0.0, tout = INFINITY;
    slab(r.o[0], r.d[0], A.X0, A.X1, tin, tout);
    slab(r.o[1], r.d[1], A.Y0, A.Y1, tin, tout);
    if (r.d[2] > 0.0) tout = fmin(tout, (A.zmax - r.o[2]) / r.d[2]);
    else if (r.d[2] < 0.0) tin = fmax(tin, (A.zmax - r.o[2]) / r.d[2]);
    else if (r.o[2] > A.zmax) tin = INFINITY;

    double out_t = INFINITY, cA = 0.0, cB = 0.0;
    int hid = -1;
    Hit HA, HB;
    HB.k = -1;
    bool found = false;
    const double dd = r.d[0] * A.c[0].vx + r.d[1] * A.c[0].vy;
    const bool fwd = dd >= 0.0;
    // Cascades in the order the ray's offset sweeps them: increasing k when the offset
    // grows along the ray, decreasing otherwise.  The two sweep directions run as two
    // passes so that the cascade index is the same on every lane of a pass (the cascade
    // constants then stay in scalar registers); a lane takes part in the pass of its
    // direction and stops at its first hit.
    for (int pass = 0; pass < 2; ++pass) {
        const bool up = pass == 0;
        const bool mine = live && tin < tout && fwd == up;
        if (__ballot(mine) == 0) continue;
        for (int s = 0; s < A.K; ++s) {
            if (!mine || found) continue;
            const int k = up ? s : A.K - 1 - s;
            const RayCas& ck = A.c[k];
            double ta, tb;
            segment(r, ck, ck.near_d, ck.far_d, tin, tout, ta, tb);
            const int64_t NN = (int64_t)A.N * A.N, MM = (4 * NN - 1) / 3;
            if (!first_hit(r, ck, k, tex + k * NN, mip + k * MM, ta, tb, HA)) continue;
            found = true;
            hid = (HA.k << 26) | (HA.j << 13) | HA.i;
            out_t = HA.t;
            cA = 1.0;
            const int pk = up ? k + 1 : k - 1;
            if (pk >= 0 && pk < A.K) {
                const RayCas& cov = A.c[up ? k : pk];
                const double lo = cov.split_d, hi = cov.far_d;
                const double dA = offset_at(r, ck, HA.t);
                if (up ? dA >= lo : dA <= hi) {
                    double tb0, tb1;
                    segment(r, A.c[pk], lo, hi, tin, tout, tb0, tb1);
                    if (first_hit(r, A.c[pk], pk, tex + pk * NN, mip + pk * MM, tb0, tb1, HB)) {
                        const double delta = hi - lo;
                        double al = (dA - lo) / delta, dal = dd / delta;
                        if (al <= 0.0) { al = 0.0; dal = 0.0; }
                        if (al >= 1.0) { al = 1.0; dal = 0.0; }
                        if (up) {
                            out_t = (1.0 - al) * HA.t + al * HB.t;
                            cA = (1.0 - al) + (HB.t - HA.t) * dal;
                            cB = al;
                        } else {
                            out_t = (1.0 - al) * HB.t + al * HA.t;
                            cA = al + (HA.t - HB.t) * dal;
                            cB = 1.0 - al;
                        }
                    } else {
                        HB.k = -1;
                    }
                }
            }
        }
    }
    if (!BACKWARD) {
        depth[p] = (float)out_t;
        hit[p] = hid;
        return;
    }
    // gradient scatter: wave-combined for lanes that share a cell (common near
    // the camera, where many pixels land in one texture cell), direct atomics
    // for the rest
    const int N = A.N;
    for (int x = 0; x < 2; ++x) {
        const Hit& H = x ? HB : HA;
        const double cf = x ? cB : cA;
        const bool has = found && H.k >= 0 && !H.start && H.fp < 0.0 && cf != 0.0;
        float w[4] = {0.f, 0.f, 0.f, 0.f};
        int key = -1;
        if (has) {
            const double sc = (double)g * cf / H.fp;
            const double u = H.u, v = H.v;
            w[0] = (float)(sc * (1.0 - u) * (1.0 - v));
            w[1] = (float)(sc * u * (1.0 - v));
            w[2] = (float)(sc * (1.0 - u) * v);
            w[3] = (float)(sc * u * v);
            key = (H.k << 26) | (H.j << 13) | H.i;
        }
        const int lane = __lane_id();
        uint64_t pending = __ballot(has);
        for (int it = 0; it < 4 && pending; ++it) {
            const int leader = __ffsll((unsigned long long)pending) - 1;
            const int lkey = __shfl(key, leader);
            const uint64_t match = __ballot(has && key == lkey) & pending;
            if (__popcll(match) < 4) break;  // little sharing left: plain atomics are cheaper
            const bool mine = (match >> lane) & 1;
            float sum[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                float t = mine ? w[c] : 0.0f;
                for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
                sum[c] = t;
            }
            if (lane == leader) {
                float* gk = gtex + (int64_t)(lkey >> 26) * N * N;
                const int64_t b = (int64_t)((lkey >> 13) & 8191) * N + (lkey & 8191);
                atomicAdd(&gk[b], sum[0]);
                atomicAdd(&gk[b + 1], sum[1]);
                atomicAdd(&gk[b + N], sum[2]);
                atomicAdd(&gk[b + N + 1], sum[3]);
            }
            pending &= ~match;
        }
        if (has && ((pending >> lane) & 1)) {
            float* gk = gtex + (int64_t)H.k * N * N;
            const int64_t b = (int64_t)H.j * N + H.i;
            atomicAdd(&gk[b], w[0]);
            atomicAdd(&gk[b + 1], w[1]);
            atomicAdd(&gk[b + N], w[2]);
            atomicAdd(&gk[b + N + 1], w[3]);
        }
    }
}

template <bool BACKWARD>
__global__ __launch_bounds__(256) void raycast_kernel(RayArgs A, const float* __restrict__ tex,
                                                      const float* __restrict__ mip, float* __restrict__ depth,
                                                      int32_t* __restrict__ hit, const float* __restrict__ gdepth,
                                                      float* __restrict__ gtex)
{
    raycast_pixel<BACKWARD>(A, blockIdx.x * 16 + threadIdx.x, blockIdx.y * 16 + threadIdx.y, tex, mip, depth, hit,
                            gdepth, gtex);
}

// Persistent form over every view of a batch: each wave takes runs of
// 64-pixel tiles (tile_w x 64 / tile_w; guided: up to 32 early, down to 1 at
// the end) from the queues until all are done; waves never wait for each other.

template <bool BACKWARD>
__global__ __launch_bounds__(256) void raycast_batch_kernel(BatchDev P)
{
    int* q = P.queues + (BACKWARD ? HFR_QUEUE_RAY_BWD : HFR_QUEUE_RAY);
    const int total = P.ray_start[P.n_views];
    const int xcd = blockIdx.x & 7;
    const int lane = __lane_id();
    const int tw = P.tile_w, th = 64 / tw;
    for (;;) {
        int w0 = -1, w1 = -1, v = 0;
        if (lane == 0 && queue_grab(q, total, xcd, 1, 32, max(1, (int)gridDim.x / 2), &w0, &w1))
            v = find_item(P.ray_start, P.n_views, w0);
        // every lane is active here, so the first active lane is lane 0: the
        // values become wave-uniform (scalar registers, scalar descriptor loads)
        w0 = __builtin_amdgcn_readfirstlane(w0);
        if (w0 < 0) break;
        w1 = __builtin_amdgcn_readfirstlane(w1);
        v = __builtin_amdgcn_readfirstlane(v);
        int v_lo = P.ray_start[v], v_hi = P.ray_start[v + 1];
        for (int w = w0; w < w1; ++w) {
            while (w >= v_hi) {  // w < total, so this stops at a view that holds w
                ++v;
                v_lo = v_hi;
                v_hi = P.ray_start[v + 1];
            }
            const BatchView& V = as_constant(P.views, v);
            const int local = w - v_lo;
            const int tx = local % V.tiles_x, ty = local / V.tiles_x;
            raycast_pixel<BACKWARD>(V.A, tx * tw + lane % tw, ty * th + lane / tw, V.tex, V.mip, V.depth, V.hit,
                                    V.gdepth, V.gtex);
        }
    }
}

}  // namespace

hfr_status ray_args(const hfr_camera* cam, const hfr_domain* dom, const hfr_cascade* cas, int32_t K, RayArgs* A)
{
    HFR_REQUIRE(cam != nullptr, "camera is NULL");
    hfr_status st = check_cascades(cas, K);
    if (st == HFR_OK) st = check_domain(dom);
    if (st != HFR_OK) return st;
    HFR_REQUIRE(cam->width >= 1 && cam->width <= 16384 && cam->height >= 1 && cam->height <= 16384,
                "image size %dx%d outside [1, 16384]", cam->width, cam->height);
    HFR_REQUIRE(std::isfinite(cam->pos[0]) && std::isfinite(cam->pos[1]) && std::isfinite(cam->pos[2]) &&
                    std::isfinite(cam->yaw) && std::isfinite(cam->pitch) && cam->vfov > 0 && cam->vfov < M_PI,
                "invalid camera");
    const double cy = std::cos(cam->yaw), sy = std::sin(cam->yaw);
    const double cp = std::cos(cam->pitch), sp = std::sin(cam->pitch);
    const double f[3] = {sy * cp, cy * cp, sp}, rt[3] = {cy, -sy, 0.0};
    const double up[3] = {rt[1] * f[2] - rt[2] * f[1], rt[2] * f[0] - rt[0] * f[2], rt[0] * f[1] - rt[1] * f[0]};
    for (int a = 0; a < 3; ++a) {
        A->o[a] = cam->pos[a];
        A->fwd[a] = f[a];
        A->right[a] = rt[a];
        A->up[a] = up[a];
    }
    A->ty = std::tan(0.5 * cam->vfov);
    A->tx = A->ty * cam->width / cam->height;
    A->W = cam->width;
    A->H = cam->height;
    A->K = K;
    A->N = cas[0].n;
    A->X0 = dom->x0;
    A->Y0 = dom->y0;
    A->X1 = dom->x1;
    A->Y1 = dom->y1;
    A->zmax = dom->zmax;
    for (int k = 0; k < HFR_MAX_CASCADES; ++k) {
        RayCas& c = A->c[k];
        const hfr_cascade& s = cas[k < K ? k : 0];
        c = RayCas{s.near_d, s.far_d, s.split_d, s.origin[0], s.origin[1], s.vhat[0], s.vhat[1],
                   s.x0, s.y0, s.hx, s.hy, 1.0 / s.hx, 1.0 / s.hy, s.n, hfr_log2i(s.n)};
    }
    return HFR_OK;
}


extern "C" hfr_status hfr_raycast(const hfr_camera* cam, const hfr_domain* dom, const hfr_cascade* cas, int32_t K,
                                  const float* tex, const float* mip, float* depth, int32_t* hit, hfr_stream stream)
{
    RayArgs A;
    hfr_status st = ray_args(cam, dom, cas, K, &A);
    if (st != HFR_OK) return st;
    HFR_REQUIRE(tex && mip && depth && hit, "NULL texture, mipmap or output");
    const dim3 grid((A.W + 15) / 16, (A.H + 15) / 16);
    raycast_kernel<false><<<grid, dim3(16, 16), 0, (hipStream_t)stream>>>(A, tex, mip, depth, hit, nullptr, nullptr);
    HFR_LAUNCH_CHECK("raycast");
    return hfr_ok();
}

extern "C" hfr_status hfr_raycast_backward(const hfr_camera* cam, const hfr_domain* dom, const hfr_cascade* cas,
                                           int32_t K, const float* tex, const float* mip, const float* grad_depth,
                                           float* grad_tex, hfr_stream stream)
{
    RayArgs A;
    hfr_status st = ray_args(cam, dom, cas, K, &A);
    if (st != HFR_OK) return st;
    HFR_REQUIRE(tex && mip && grad_depth && grad_tex, "NULL texture, mipmap or gradient");
    const dim3 grid((A.W + 15) / 16, (A.H + 15) / 16);
    raycast_kernel<true><<<grid, dim3(16, 16), 0, (hipStream_t)stream>>>(A, tex, mip, nullptr, nullptr, grad_depth,
                                                                         grad_tex);
    HFR_LAUNCH_CHECK("raycast_backward");
    return hfr_ok();
}

hfr_status launch_raycast_batch(const BatchDev& P, int blocks, bool backward, hipStream_t s)
{
    if (backward) raycast_batch_kernel<true><<<dim3(blocks), dim3(256), 0, s>>>(P);
    else raycast_batch_kernel<false><<<dim3(blocks), dim3(256), 0, s>>>(P);
    HFR_LAUNCH_CHECK(backward ? "raycast_backward (batch)" : "raycast (batch)");
    return HFR_OK;
}
