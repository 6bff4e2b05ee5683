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
//
// Long rays.  Those few rays come in clusters (whole waves just below the
// horizon) and spend their steps walking node after node a little above the
// surface.  The frame kernel gives every ray a budget of RAY_BUDGET steps;
// rays that exhaust it go to a queue in the caller's workspace, and a second,
// persistent kernel walks each queued ray with RAY_SPLIT lanes, which test
// the next RAY_SPLIT nodes of the current level along the ray at once.
#include <climits>
#include <mutex>

#include "hfr_device.h"

namespace {

constexpr int RAY_BUDGET = 64;  // cell-walk steps a pixel may take in the frame kernel
constexpr int RAY_SPLIT = 16;   // lanes that share one queued ray

// Which surface a ray cast draws when a frame holds several heightfields.
struct SurfaceArgs {
    int tag;                       // surface index, written into bits 29-30 of every hit
    bool nearer;                   // forward: clip each ray at depth[p], write only a nearer hit
    const int32_t* __restrict__ filter;  // adjoint: only pixels whose hit carries this tag (NULL: all)
    int* limit_count;              // rays stopped by the walk's iteration cap are counted here (NULL: not counted)
};

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

// Root of the bilinear patch of cell (ci, cj) (texels t00 .. t11) along the
// ray piece [t, te] whose start height is za: true with the hit in h.
__device__ inline bool patch_hit(const Ray& r, const RayCas& c, int k, int ci, int cj, double t, double te, double za,
                                 double ta, float t00, float t10, float t01, float t11, Hit& h)
{
    const double h00 = t00, h10 = t10, h01 = t01, h11 = t11;
    const double u0 = ((r.o[0] + t * r.d[0]) - c.x0) * c.inv_hx - ci;
    const double v0 = ((r.o[1] + t * r.d[1]) - c.y0) * c.inv_hy - cj;
    const double du = r.d[0] * c.inv_hx, dv = r.d[1] * c.inv_hy;
    const double A = h10 - h00, B = h01 - h00, C = (h00 - h10) - (h01 - h11);
    const double cc = za - (h00 + A * u0 + B * v0 + C * u0 * v0);
    const double bb = r.d[2] - A * du - B * dv - C * (u0 * dv + v0 * du);
    const double aa = -C * du * dv;
    double tau = 0.0;
    if (!(cc <= 0.0 || smallest_root(aa, bb, cc, te - t, tau))) return false;
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

// The cell's four texels and its maximum (-inf when one is invisible).
__device__ inline float cell_texels(const float* __restrict__ tex, int N, int ci, int cj, float& t00, float& t10,
                                    float& t01, float& t11)
{
    const int64_t b = (int64_t)cj * N + ci;
    t00 = tex[b];
    t10 = tex[b + 1];
    t01 = tex[b + N];
    t11 = tex[b + N + 1];
    return (isfinite(t00) && isfinite(t10) && isfinite(t01) && isfinite(t11))
               ? fmaxf(fmaxf(t00, t10), fmaxf(t01, t11)) : -INFINITY;
}

// First root of the ray in [ta, tb] of cascade k: 1 with the hit in h, 0 when
// there is none, -1 when the step budget runs out first, -2 when the walk
// reaches its iteration cap (every iteration descends a level or moves to a
// later piece, so a walk never needs that many; the cap only guards against
// a fault in that reasoning, and the caller reports the ray instead of
// treating it as a miss).  G > 1: the G lanes
// of an aligned group hold the same ray and call this together, and every
// step tests the next G nodes of the current level along the ray at once
// (lane s the s-th: entered after the s-th crossing of the merged x- and
// y-boundary sequences, found by a co-rank search, with the boundary
// arithmetic of node_exit).  The walk descends into the first node the ray
// reaches below the maximum of, skips all G when it passes above them, and at
// level 0 keeps the earliest cell that holds a root.
template <int G>
__device__ int first_hit(const Ray& r, const RayCas& c, int k, const float* __restrict__ tex,
                         const float* __restrict__ mip, double ta, double tb, Hit& h, int& budget, int s)
{
    if (!(ta < tb)) return 0;
    const int N = c.n, L = c.levels;
    double t = ta;
    double t1 = piece_end(r, c, t, tb);
    int ci, cj;
    cell_at(r, c, 0.5 * (t + t1), ci, cj);
    int l = L;
    bool probe = true;  // G > 1: the first step looks down through the levels at ta
    // every iteration either descends a level or moves to a later piece
    const int max_iter = 8 * N * (L + 2) + 64;
    for (int it = 0; it < max_iter; ++it) {
        if (--budget < 0) return -1;
        if constexpr (G > 1) {
            // A probe tests the node holding t on levels l, l - 1, ..., lane s level l - s; a
            // march tests the next G nodes of level l along the ray, lane s the s-th: entered
            // after a crossings of the level's x-boundaries and b of its y-boundaries, a + b = s.
            int ls = l, qx, qy;
            double p0, p1;
            bool valid;
            if (probe) {
                ls = l - s;
                valid = ls >= 0;
                ls = max(ls, 0);
                qx = ci >> ls;
                qy = cj >> ls;
                p0 = t;
                p1 = fmax(node_exit(r, c, ci, cj, ls, tb), t1);
            } else {
                const int nx = ci >> l, ny = cj >> l;
                auto TX = [&](int a) {
                    return r.d[0] == 0.0
                               ? INFINITY
                               : (lattice_pos(c.x0, (r.d[0] > 0.0 ? nx + 1 + a : nx - a) << l, c.hx) - r.o[0]) *
                                     r.inv_d[0];
                };
                auto TY = [&](int b) {
                    return r.d[1] == 0.0
                               ? INFINITY
                               : (lattice_pos(c.y0, (r.d[1] > 0.0 ? ny + 1 + b : ny - b) << l, c.hy) - r.o[1]) *
                                     r.inv_d[1];
                };
                int lo = 0, hi = s;
                while (lo < hi) {  // smallest a whose next x-crossing comes after the (s - a)-th y-crossing
                    const int mid = (lo + hi) >> 1;
                    if (TX(mid) <= TY(s - mid - 1)) lo = mid + 1;
                    else hi = mid;
                }
                const int a = lo, b = s - a;
                p0 = s == 0 ? t : fmax(a > 0 ? TX(a - 1) : -INFINITY, b > 0 ? TY(b - 1) : -INFINITY);
                p1 = fmin(fmin(TX(a), TY(b)), tb);
                valid = p0 < tb;
                qx = nx + (r.d[0] > 0.0 ? a : -a);
                qy = ny + (r.d[1] > 0.0 ? b : -b);
            }
            const int last = ls > 0 ? (N >> ls) - 1 : N - 2;
            qx = min(max(qx, 0), last);
            qy = min(max(qy, 0), last);
            bool stop = false, hit = false;
            Hit hs;
            if (valid) {
                float M, t00 = 0.f, t10 = 0.f, t01 = 0.f, t11 = 0.f;
                if (ls > 0) M = mip[level_offset(L, ls) + qy * (N >> ls) + qx];
                else M = cell_texels(tex, N, qx, qy, t00, t10, t01, t11);
                const double za = r.o[2] + p0 * r.d[2], zb = r.o[2] + p1 * r.d[2];
                if (!(fmin(za, zb) > (double)M)) {
                    stop = true;  // the ray reaches below the node's maximum
                    if (ls == 0) hit = patch_hit(r, c, k, qx, qy, p0, p1, za, ta, t00, t10, t01, t11, hs);
                }
            }
            const int lane = __lane_id(), base = lane & ~(G - 1);
            const uint64_t gmask = (G == 64 ? ~0ull : ((1ull << (G & 63)) - 1)) << base;
            const uint64_t hits = __ballot(hit) & gmask;
            if (hits) {
                const int src = __ffsll((unsigned long long)hits) - 1;
                h.k = __shfl(hs.k, src);
                h.i = __shfl(hs.i, src);
                h.j = __shfl(hs.j, src);
                h.start = __shfl(hs.start, src);
                h.t = __shfl(hs.t, src);
                h.u = __shfl(hs.u, src);
                h.v = __shfl(hs.v, src);
                h.fp = __shfl(hs.fp, src);
                return 1;
            }
            const uint64_t stops = __ballot(stop) & gmask;
            int up = -1;  // after an advance: the level to climb to, before the node-change cap
            if (probe) {
                // the highest level whose node the ray passes above: continue past it
                const uint64_t above = __ballot(valid && !stop) & gmask;
                if (above) {
                    const int src = __ffsll((unsigned long long)above) - 1;
                    t = __shfl(p1, src);
                    up = l - (src - base) + 1;
                    probe = false;
                } else if (l - (G - 1) > 0) {
                    l -= G;  // below the maxima of all probed levels: probe further down
                    continue;
                } else {
                    t = __shfl(p1, base + l);  // the level-0 cell had no root
                    up = 0;
                    probe = false;
                }
            } else if (l > 0 && stops) {
                // descend into the first node the ray dips into, at the point it enters it
                t = __shfl(p0, __ffsll((unsigned long long)stops) - 1);
                l -= 1;
                probe = true;
            } else {
                // every node of the batch passed (at level 0: no cell held a root)
                t = __shfl(p1, base + G - 1);
                up = (l == 0 && stops) ? 0 : l + 1;  // climb again unless the ray ran below cell tops
            }
            if (t >= tb) return 0;
            t1 = piece_end(r, c, t, tb);
            int ni, nj;
            cell_at(r, c, 0.5 * (t + t1), ni, nj);
            if (up >= 0) {
                // as in the single-lane walk, never climb into a node that holds the previous
                // cell: that node's maximum was just found above the ray
                const unsigned diff = (unsigned)((ni ^ ci) | (nj ^ cj));
                l = min(min(up, L), diff ? 31 - __clz(diff) : 0);
            }
            ci = ni;
            cj = nj;
            continue;
        }
        // Node maximum: from the max-mipmap above level 0; at level 0 from the cell's own four
        // texels (the same value the pyramid holds there), which the patch test needs anyway,
        // so a cell costs one round of loads instead of two.
        float M, t00 = 0.f, t10 = 0.f, t01 = 0.f, t11 = 0.f;
        if (l > 0) M = mip[level_offset(L, l) + (cj >> l) * (N >> l) + (ci >> l)];
        else M = cell_texels(tex, N, ci, cj, t00, t10, t01, t11);
        const double te = fmax(node_exit(r, c, ci, cj, l, tb), t1);
        const double za = r.o[2] + t * r.d[2], zb = r.o[2] + te * r.d[2];
        bool advance = false, close = false;
        if (fmin(za, zb) > (double)M) {
            advance = true;
        } else if (l > 0) {
            --l;
        } else {
            if (patch_hit(r, c, k, ci, cj, t, te, za, ta, t00, t10, t01, t11, h)) return 1;
            advance = true;
            close = true;  // the ray passed below this cell's highest texel
        }
        if (advance) {
            if (te >= tb) return 0;
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
    return -2;
}

// Pixel (col, row) of one view.  In the adjoint every lane of the wave must
// call it (the gradient scatter uses wave-wide shuffles), also lanes
// outside the image.  G lanes (an aligned group, s = 0 .. G - 1) may share a
// pixel (see first_hit); lane s = 0 writes its results.  Returns true when
// the step budget ran out: nothing is written for the pixel then.
template <bool BACKWARD, int G, bool NEARER = false>
__device__ __forceinline__ bool raycast_pixel(const RayArgs& A, int col, int row, const float* __restrict__ tex,
                                              const float* __restrict__ mip, float* __restrict__ depth,
                                              int32_t* __restrict__ hit, const float* __restrict__ gdepth,
                                              float* __restrict__ gtex, int s, int budget, const SurfaceArgs& S)
{
    const bool in_image = col < A.W && row < A.H;
    if (!BACKWARD && !in_image) return false;
    const int64_t p = (int64_t)row * A.W + col;
    float g = 0.0f;
    if (BACKWARD && in_image) g = gdepth[p];
    if (BACKWARD && in_image && S.filter) {
        const int32_t hf = S.filter[p];
        if (hf < 0 || ((hf >> 29) & 3) != S.tag) g = 0.0f;  // another surface is nearer, or none is hit
    }
    // the nearer pass sees only what lies in front of the surfaces drawn so far
    const float clip = (!BACKWARD && NEARER) ? depth[p] : INFINITY;
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
    // the nearer pass clips the search for the first hit only: the second hit of an overlap
    // blend is this surface's own, wherever the surfaces drawn so far lie (the adjoint, which
    // walks unclipped, finds the same pair)
    const double tfull = tout;
    tout = fmin(tout, (double)clip);

    double out_t = INFINITY, cA = 0.0, cB = 0.0;
    int hid = -1;
    Hit HA, HB;
    HB.k = -1;
    bool found = false, deferred = false, limited = false;
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
        for (int step = 0; step < A.K; ++step) {
            if (!mine || found) continue;
            const int k = up ? step : A.K - 1 - step;
            const RayCas& ck = A.c[k];
            double ta, tb;
            segment(r, ck, ck.near_d, ck.far_d, tin, tout, ta, tb);
            const int64_t NN = (int64_t)A.N * A.N, MM = (4 * NN - 1) / 3;
            const int sa = first_hit<G>(r, ck, k, tex + k * NN, mip + k * MM, ta, tb, HA, budget, s);
            if (sa == 0) continue;
            found = true;
            if (sa < 0) {
                deferred = sa == -1;
                limited = sa == -2;
                continue;
            }
            hid = (S.tag << 29) | (HA.k << 26) | (HA.j << 13) | HA.i;
            out_t = HA.t;
            cA = 1.0;
            const int pk = up ? k + 1 : k - 1;
            if (pk >= 0 && pk < A.K) {
                const RayCas& cov = A.c[up ? k : pk];
                const double lo = cov.split_d, hi = cov.far_d;
                const double dA = offset_at(r, ck, HA.t);
                if (up ? dA >= lo : dA <= hi) {
                    double tb0, tb1;
                    segment(r, A.c[pk], lo, hi, tin, tfull, tb0, tb1);
                    const int sb = first_hit<G>(r, A.c[pk], pk, tex + pk * NN, mip + pk * MM, tb0, tb1, HB,
                                                      budget, s);
                    if (sb == -1) {
                        deferred = true;
                    } else if (sb == -2) {
                        limited = true;
                    } else if (sb > 0) {
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
    if (limited && !deferred && s == 0 && S.limit_count != nullptr) atomicAdd(S.limit_count, 1);
    if (!BACKWARD) {
        // a nearer pass replaces only what it finds in front (a blend may land a little behind);
        // a ray stopped by the iteration cap is reported (NaN, HFR_HIT_LIMIT), never taken for a miss
        if (!deferred && s == 0 && limited) {
            depth[p] = NAN;
            hit[p] = -2;
        } else if (!deferred && s == 0 && (!NEARER || (found && (float)out_t < clip))) {
            depth[p] = (float)out_t;
            hit[p] = hid;
        }
        return deferred;
    }
    found = found && !limited;
    // gradient scatter: wave-combined for lanes that share a cell (common near
    // the camera, where many pixels land in one texture cell), direct atomics
    // for the rest
    const int N = A.N;
    for (int x = 0; x < 2; ++x) {
        const Hit& H = x ? HB : HA;
        const double cf = x ? cB : cA;
        const bool has = found && !deferred && s == 0 && H.k >= 0 && !H.start && H.fp < 0.0 && cf != 0.0;
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
    return deferred;
}

// Frame kernel: one lane per pixel (6 waves per SIMD for the forward pass:
// at most 80 VGPRs).  With a workspace (work[0] = queue length, work[1] =
// rays stopped by the iteration cap, work[2 ..] = pixel indices) a pixel whose walk exceeds RAY_BUDGET
// steps is queued instead of finished.
template <bool BACKWARD, bool NEARER>
__global__ __launch_bounds__(256, BACKWARD ? 4 : 6) void raycast_kernel(RayArgs A, const float* __restrict__ tex,
                                                      const float* __restrict__ mip, float* __restrict__ depth,
                                                      int32_t* __restrict__ hit, const float* __restrict__ gdepth,
                                                      float* __restrict__ gtex, int* __restrict__ work, SurfaceArgs S,
                                                      int row0)
{
    const int col = blockIdx.x * 16 + threadIdx.x, row = row0 + blockIdx.y * 16 + threadIdx.y;
    const bool deferred = raycast_pixel<BACKWARD, 1, NEARER>(A, col, row, tex, mip, depth, hit, gdepth, gtex, 0,
                                                     work ? RAY_BUDGET : INT_MAX, S);
    if (!work) return;
    const uint64_t m = __ballot(deferred);  // one queue reservation per wave
    if (!m) return;
    const int lane = __lane_id(), leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(&work[0], __popcll(m));
    base = __shfl(base, leader);
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    if (deferred) work[2 + base + __popcll(m & lt)] = row * A.W + col;
}

// Queued pixels, RAY_SPLIT lanes each.  The queue is complete when this
// kernel starts, so wave w takes entries (w + j W) 64 / RAY_SPLIT onwards for
// j = 0, 1, ... (W waves in the grid): no atomics on a shared counter.  The
// loop condition is wave-uniform; a lane group whose entry lies past the
// queue's end walks nothing but stays with its wave (the adjoint's scatter
// uses wave-wide shuffles).
template <bool BACKWARD, bool NEARER>
__global__ __launch_bounds__(256) void raycast_tail_kernel(RayArgs A, const float* __restrict__ tex,
                                                           const float* __restrict__ mip, float* __restrict__ depth,
                                                           int32_t* __restrict__ hit, const float* __restrict__ gdepth,
                                                           float* __restrict__ gtex, int* __restrict__ work,
                                                           SurfaceArgs S)
{
    constexpr int G = RAY_SPLIT, PER_WAVE = 64 / G;
    const int lane = __lane_id(), s = lane & (G - 1);
    const int count = __builtin_amdgcn_readfirstlane(work[0]);
    const int waves = (int)(gridDim.x * (blockDim.x / 64));
    const int wave = (int)(blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64);
    for (int first = wave * PER_WAVE; first < count; first += waves * PER_WAVE) {
        const int idx = first + lane / G;
        const bool has = idx < count;
        const int p = has ? work[2 + idx] : 0;
        raycast_pixel<BACKWARD, G, NEARER>(A, has ? p % A.W : A.W, has ? p / A.W : 0, tex, mip, depth, hit, gdepth, gtex, s,
                                   INT_MAX, S);
    }
}

__global__ void zero_queue_kernel(int* __restrict__ work)
{
    if (threadIdx.x < 2) work[threadIdx.x] = 0;  // queue length, rays stopped by the iteration cap
}

// The second launch of a split frame: workgroups [0, tail_blocks) walk the
// queue that the first launch filled from the rows above rest_row0 (as
// raycast_tail_kernel, over tail_blocks workgroups); the others walk rows
// rest_row0 .. H - 1, one 16 x 16 tile each, every ray to its end on its own
// lane.  The queued rays, which set the first launch's tail, then run beside
// the bulk of the image instead of after it.  Lane l of a tile takes pixel
// (l mod 16, l / 16) of it, as the frame kernel's 16 x 16 workgroup does.
template <bool BACKWARD, bool NEARER>
__global__ __launch_bounds__(256) void raycast_split_kernel(
    RayArgs A, const float* __restrict__ tex, const float* __restrict__ mip, float* __restrict__ depth,
    int32_t* __restrict__ hit, const float* __restrict__ gdepth, float* __restrict__ gtex, int* __restrict__ work,
    SurfaceArgs S, int tail_blocks, int rest_row0)
{
    if ((int)blockIdx.x < tail_blocks) {
        constexpr int G = RAY_SPLIT, PER_WAVE = 64 / G;
        const int lane = __lane_id(), s = lane & (G - 1);
        const int count = __builtin_amdgcn_readfirstlane(work[0]);
        const int waves = tail_blocks * (int)(blockDim.x / 64);
        const int wave = (int)(blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64);
        for (int first = wave * PER_WAVE; first < count; first += waves * PER_WAVE) {
            const int idx = first + lane / G;
            const bool has = idx < count;
            const int p = has ? work[2 + idx] : 0;
            raycast_pixel<BACKWARD, G, NEARER>(A, has ? p % A.W : A.W, has ? p / A.W : 0, tex, mip, depth, hit, gdepth,
                                               gtex, s, INT_MAX, S);
        }
        return;
    }
    const int b = (int)blockIdx.x - tail_blocks;
    const int tiles_x = (A.W + 15) / 16;
    const int tx = b % tiles_x, ty = b / tiles_x;
    const int col = tx * 16 + (int)(threadIdx.x & 15), row = rest_row0 + ty * 16 + (int)(threadIdx.x >> 4);
    raycast_pixel<BACKWARD, 1, NEARER>(A, col, row, tex, mip, depth, hit, gdepth, gtex, 0, INT_MAX, S);
}

// Persistent form over every view of a batch: each wave takes runs of
// 64-pixel tiles (tile_w x 64 / tile_w; guided: up to P.ray_grain early, down
// to 1 at the end) from HFR_CHUNKS queues, eight per XCD, until all are
// done; waves never wait for each other.
// With P.ray_queue a pixel whose walk exceeds RAY_BUDGET steps goes to its
// view's slice of the long-ray queue (one reservation per wave and tile, as
// in the frame kernel); a pixel that finds the slice full is walked again to
// the end by the whole wave at once (lanes without such a pixel walk
// nothing), so the adjoint's shuffles see every lane.

template <bool BACKWARD>
__global__ __launch_bounds__(256) void raycast_batch_kernel(BatchDev P)
{
    int* q = P.queues + (BACKWARD ? HFR_QUEUE_RAY_BWD : HFR_QUEUE_RAY);
    const int total = P.ray_start[P.n_views];
    const int lane = __lane_id();
    const int tw = P.tile_w, th = 64 / tw;
    // home chunk: the workgroup's XCD (blockIdx.x & 7), then one of its eight
    // chunks by the wave's slot on that XCD
    const int home = (int)(blockIdx.x & 7) * 8 + (int)(((blockIdx.x >> 3) * (blockDim.x / 64) + threadIdx.x / 64) & 7);
    const int consumers = max(1, (int)(gridDim.x * (blockDim.x / 64)) / HFR_CHUNKS);
    bool scan = false;
    for (;;) {
        int w0 = -1, w1 = -1, v = 0;
        // every lane is active here: the grab is wave-wide, its result uniform
        if (!queue_grab_wave(q, HFR_CHUNKS, total, home, 1, P.ray_grain, consumers, &scan, &w0, &w1)) break;
        if (lane == 0) v = find_item(P.ray_start, P.n_views, w0);
        // the first active lane is lane 0: the values become wave-uniform
        // (scalar registers, scalar descriptor loads)
        w0 = __builtin_amdgcn_readfirstlane(w0);
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
            const int col = tx * tw + lane % tw, row = ty * th + lane / tw;
            const SurfaceArgs S{0, false, nullptr, nullptr};
            const bool deferred = raycast_pixel<BACKWARD, 1>(V.A, col, row, V.tex, V.mip, V.depth, V.hit, V.gdepth,
                                                             V.gtex, 0, P.ray_queue ? RAY_BUDGET : INT_MAX, S);
            const uint64_t m = __ballot(deferred);
            if (!m) continue;
            const int leader = __ffsll((unsigned long long)m) - 1;
            int base = 0;
            if (lane == leader) base = atomicAdd(&P.rayq_count[v], __popcll(m));
            base = __shfl(base, leader);
            const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
            const int slot = base + __popcll(m & lt);
            const bool fits = slot < V.q_cap;
            if (deferred && fits) P.rayq[V.q_off + slot] = row * V.A.W + col;
            const bool again = deferred && !fits;
            if (__ballot(again))
                raycast_pixel<BACKWARD, 1>(V.A, again ? col : V.A.W, again ? row : V.A.H, V.tex, V.mip, V.depth, V.hit,
                                           V.gdepth, V.gtex, 0, INT_MAX, S);
        }
    }
}

// The batch's queued long rays, RAY_SPLIT lanes each (as raycast_tail_kernel):
// the queue is complete when this kernel starts.  Views are taken in order,
// every wave walking each view's entries with a grid stride; the entries of
// all views are numbered consecutively (each view's count rounded up to whole
// waves' worth), so the waves' shares stay even across views.
template <bool BACKWARD>
__global__ __launch_bounds__(256) void raycast_batch_tail_kernel(BatchDev P)
{
    constexpr int G = RAY_SPLIT, PER_WAVE = 64 / G;
    const int lane = __lane_id(), s = lane & (G - 1);
    const int waves = (int)(gridDim.x * (blockDim.x / 64));
    const int wave = (int)(blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64);
    const int stride = waves * PER_WAVE;
    int64_t before = 0;  // entries of the views already passed, in whole waves' worth
    for (int v = 0; v < P.n_views; ++v) {
        const BatchView& V = as_constant(P.views, v);
        const int count = min(__builtin_amdgcn_readfirstlane(P.rayq_count[v]), V.q_cap);
        if (count == 0) continue;
        int first = (int)((((int64_t)wave * PER_WAVE - before) % stride + stride) % stride);
        for (; first < count; first += stride) {
            const int idx = first + lane / G;
            const bool has = idx < count;
            const int p = has ? P.rayq[V.q_off + idx] : 0;
            raycast_pixel<BACKWARD, G>(V.A, has ? p % V.A.W : V.A.W, has ? p / V.A.W : 0, V.tex, V.mip, V.depth,
                                       V.hit, V.gdepth, V.gtex, s, INT_MAX, SurfaceArgs{0, false, nullptr, nullptr});
        }
        before += (count + PER_WAVE - 1) / PER_WAVE * PER_WAVE;
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


namespace {

// The frame kernel, then (with a workspace) the queue of long rays.  With
// band_rows < H (a workspace given) the frame is split: the frame kernel
// walks rows 0 .. band_rows - 1 (rounded up to whole 16-row tiles) and
// queues their long rays; raycast_split_kernel then walks the queue beside
// the remaining rows.
template <bool BACKWARD>
void launch_raycast(const RayArgs& A, const float* tex, const float* mip, float* depth, int32_t* hit,
                    const float* gdepth, float* gtex, int32_t* work, const SurfaceArgs& S0, hipStream_t s,
                    int band_rows = INT_MAX)
{
    SurfaceArgs S = S0;
    S.limit_count = work ? work + 1 : nullptr;
    if (work) zero_queue_kernel<<<1, 64, 0, s>>>(work);
    const int tiles_x = (A.W + 15) / 16, tiles_y = (A.H + 15) / 16;
    const int band_tiles = work ? (int)std::min<int64_t>(tiles_y, (std::max(band_rows, 0) + 15LL) / 16) : tiles_y;
    // the nearer pass is its own instantiation: the plain walk keeps no clip depth in registers
    bool nearer = false;
    if constexpr (!BACKWARD) nearer = S.nearer;
    if (band_tiles > 0) {
        const dim3 grid(tiles_x, band_tiles);
        if constexpr (!BACKWARD) {
            if (nearer)
                raycast_kernel<false, true><<<grid, dim3(16, 16), 0, s>>>(A, tex, mip, depth, hit, gdepth, gtex, work,
                                                                         S, 0);
        }
        if (!nearer)
            raycast_kernel<BACKWARD, false><<<grid, dim3(16, 16), 0, s>>>(A, tex, mip, depth, hit, gdepth, gtex, work,
                                                                         S, 0);
    }
    if (!work) return;
    // persistent: enough lane groups that a typical queue is taken in one round
    const int64_t pixels = (int64_t)A.W * A.H;
    const int blocks = (int)std::min<int64_t>(2048, std::max<int64_t>(64, pixels / 1024));
    if (band_tiles < tiles_y) {
        const int rest = tiles_x * (tiles_y - band_tiles);
        const int rest_row0 = band_tiles * 16;
        if constexpr (!BACKWARD) {
            if (nearer)
                raycast_split_kernel<false, true><<<dim3(blocks + rest), dim3(256), 0, s>>>(
                    A, tex, mip, depth, hit, gdepth, gtex, work, S, blocks, rest_row0);
        }
        if (!nearer)
            raycast_split_kernel<BACKWARD, false><<<dim3(blocks + rest), dim3(256), 0, s>>>(
                A, tex, mip, depth, hit, gdepth, gtex, work, S, blocks, rest_row0);
        return;
    }
    if constexpr (!BACKWARD) {
        if (nearer)
            raycast_tail_kernel<false, true><<<dim3(blocks), dim3(256), 0, s>>>(A, tex, mip, depth, hit, gdepth, gtex,
                                                                               work, S);
    }
    if (!nearer)
        raycast_tail_kernel<BACKWARD, false><<<dim3(blocks), dim3(256), 0, s>>>(A, tex, mip, depth, hit, gdepth, gtex,
                                                                               work, S);
}

}  // namespace

extern "C" hfr_status hfr_raycast(const hfr_camera* cam, const hfr_domain* dom, const hfr_cascade* cas, int32_t K,
                                  const float* tex, const float* mip, float* depth, int32_t* hit, int32_t* work,
                                  hfr_stream stream)
{
    RayArgs A;
    hfr_status st = ray_args(cam, dom, cas, K, &A);
    if (st != HFR_OK) return st;
    HFR_REQUIRE(tex && mip && depth && hit, "NULL texture, mipmap or output");
    launch_raycast<false>(A, tex, mip, depth, hit, nullptr, nullptr, work, SurfaceArgs{0, false, nullptr, nullptr},
                          (hipStream_t)stream);
    HFR_LAUNCH_CHECK("raycast");
    return hfr_ok();
}

extern "C" hfr_status hfr_raycast_split(const hfr_camera* cam, const hfr_domain* dom, const hfr_cascade* cas,
                                        int32_t K, const float* tex, const float* mip, float* depth, int32_t* hit,
                                        int32_t* work, int32_t band_rows, hfr_stream stream)
{
    RayArgs A;
    hfr_status st = ray_args(cam, dom, cas, K, &A);
    if (st != HFR_OK) return st;
    HFR_REQUIRE(tex && mip && depth && hit && work, "NULL texture, mipmap, output or workspace");
    HFR_REQUIRE(band_rows >= 0, "band_rows %d is negative", band_rows);
    launch_raycast<false>(A, tex, mip, depth, hit, nullptr, nullptr, work, SurfaceArgs{0, false, nullptr, nullptr},
                          (hipStream_t)stream, band_rows);
    HFR_LAUNCH_CHECK("raycast_split");
    return hfr_ok();
}

extern "C" hfr_status hfr_raycast_backward_split(const hfr_camera* cam, const hfr_domain* dom,
                                                 const hfr_cascade* cas, int32_t K, const float* tex,
                                                 const float* mip, const float* grad_depth, float* grad_tex,
                                                 int32_t* work, int32_t band_rows, hfr_stream stream)
{
    RayArgs A;
    hfr_status st = ray_args(cam, dom, cas, K, &A);
    if (st != HFR_OK) return st;
    HFR_REQUIRE(tex && mip && grad_depth && grad_tex && work, "NULL texture, mipmap, gradient or workspace");
    HFR_REQUIRE(band_rows >= 0, "band_rows %d is negative", band_rows);
    launch_raycast<true>(A, tex, mip, nullptr, nullptr, grad_depth, grad_tex, work,
                         SurfaceArgs{0, false, nullptr, nullptr}, (hipStream_t)stream, band_rows);
    HFR_LAUNCH_CHECK("raycast_backward_split");
    return hfr_ok();
}

extern "C" hfr_status hfr_raycast_nearer(const hfr_camera* cam, const hfr_domain* dom, const hfr_cascade* cas,
                                         int32_t K, const float* tex, const float* mip, int32_t surface, float* depth,
                                         int32_t* hit, int32_t* work, hfr_stream stream)
{
    RayArgs A;
    hfr_status st = ray_args(cam, dom, cas, K, &A);
    if (st != HFR_OK) return st;
    HFR_REQUIRE(tex && mip && depth && hit, "NULL texture, mipmap or output");
    HFR_REQUIRE(surface >= 1 && surface <= HFR_MAX_SURFACES - 1, "surface %d outside [1, %d]", surface,
                HFR_MAX_SURFACES - 1);
    launch_raycast<false>(A, tex, mip, depth, hit, nullptr, nullptr, work, SurfaceArgs{surface, true, nullptr, nullptr},
                          (hipStream_t)stream);
    HFR_LAUNCH_CHECK("raycast_nearer");
    return hfr_ok();
}

extern "C" hfr_status hfr_raycast_backward(const hfr_camera* cam, const hfr_domain* dom, const hfr_cascade* cas,
                                           int32_t K, const float* tex, const float* mip, const float* grad_depth,
                                           float* grad_tex, int32_t* work, hfr_stream stream)
{
    RayArgs A;
    hfr_status st = ray_args(cam, dom, cas, K, &A);
    if (st != HFR_OK) return st;
    HFR_REQUIRE(tex && mip && grad_depth && grad_tex, "NULL texture, mipmap or gradient");
    launch_raycast<true>(A, tex, mip, nullptr, nullptr, grad_depth, grad_tex, work, SurfaceArgs{0, false, nullptr, nullptr},
                         (hipStream_t)stream);
    HFR_LAUNCH_CHECK("raycast_backward");
    return hfr_ok();
}

extern "C" hfr_status hfr_raycast_backward_surface(const hfr_camera* cam, const hfr_domain* dom,
                                                   const hfr_cascade* cas, int32_t K, const float* tex,
                                                   const float* mip, int32_t surface, const int32_t* hit,
                                                   const float* grad_depth, float* grad_tex, int32_t* work,
                                                   hfr_stream stream)
{
    RayArgs A;
    hfr_status st = ray_args(cam, dom, cas, K, &A);
    if (st != HFR_OK) return st;
    HFR_REQUIRE(tex && mip && hit && grad_depth && grad_tex, "NULL texture, mipmap, hit or gradient");
    HFR_REQUIRE(surface >= 0 && surface <= HFR_MAX_SURFACES - 1, "surface %d outside [0, %d]", surface,
                HFR_MAX_SURFACES - 1);
    launch_raycast<true>(A, tex, mip, nullptr, nullptr, grad_depth, grad_tex, work,
                         SurfaceArgs{surface, false, hit, nullptr}, (hipStream_t)stream);
    HFR_LAUNCH_CHECK("raycast_backward_surface");
    return hfr_ok();
}

// ------------------------------------------------------------------------
// hfr_raycast_static: hfr_raycast with the long-ray queue in a library-owned
// device array instead of a caller workspace, so the call allocates nothing.

namespace {

constexpr int64_t STATIC_QUEUE_PIXELS = int64_t(1) << 22;  // W x H at most (1920 x 1080, 2560 x 1600 fit)

// The queue (count, unused word, pixel indices) of every hfr_raycast_static
// call on a device: 16 MiB + 8 B, held by each device the library runs on
// until the process ends.  Host code never names it directly: its device
// address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) int32_t scratch[STATIC_QUEUE_PIXELS + 2];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mutex;
int32_t* scratch_ptr[MAX_DEVICES] = {};

// Device address of this device's scratch array (looked up on the first call).
hfr_status scratch_address(hipStream_t stream, int32_t** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return hfr_fail(HFR_EDEVICE, "raycast_static: hipGetDevice failed");
    HFR_REQUIRE(dev >= 0 && dev < MAX_DEVICES, "raycast_static: device %d beyond the %d supported", dev, MAX_DEVICES);
    if (stream != nullptr) {
        hipDevice_t sd = -1;
        if (hipStreamGetDevice(stream, &sd) != hipSuccess)
            return hfr_fail(HFR_EDEVICE, "raycast_static: hipStreamGetDevice failed");
        HFR_REQUIRE(sd == dev, "raycast_static: the stream belongs to device %d, the current device is %d", (int)sd,
                    dev);
    }
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return hfr_fail(HFR_EDEVICE, "raycast_static: hipGetSymbolAddress: %s", hipGetErrorString(e));
        scratch_ptr[dev] = static_cast<int32_t*>(p);
    }
    *out = scratch_ptr[dev];
    return HFR_OK;
}

}  // namespace

extern "C" hfr_status hfr_raycast_static_max_pixels(int64_t* pixels)
{
    HFR_REQUIRE(pixels != nullptr, "NULL output");
    *pixels = STATIC_QUEUE_PIXELS;
    return hfr_ok();
}

extern "C" hfr_status hfr_raycast_static(const hfr_camera* cam, const hfr_domain* dom, const hfr_cascade* cas,
                                         int32_t K, const float* tex, const float* mip, float* depth, int32_t* hit,
                                         hfr_stream stream)
{
    RayArgs A;
    hfr_status st = ray_args(cam, dom, cas, K, &A);
    if (st != HFR_OK) return st;
    HFR_REQUIRE(tex && mip && depth && hit, "NULL texture, mipmap or output");
    HFR_REQUIRE((int64_t)A.W * A.H <= STATIC_QUEUE_PIXELS,
                "raycast_static: %d x %d pixels exceed the static queue's %lld (use hfr_raycast with a workspace)",
                A.W, A.H, (long long)STATIC_QUEUE_PIXELS);
    int32_t* work = nullptr;
    st = scratch_address((hipStream_t)stream, &work);
    if (st != HFR_OK) return st;
    // the frame kernel appends to the queue after zero_queue_kernel has cleared its count
    launch_raycast<false>(A, tex, mip, depth, hit, nullptr, nullptr, work, SurfaceArgs{0, false, nullptr, nullptr},
                          (hipStream_t)stream);
    HFR_LAUNCH_CHECK("raycast_static");
    return hfr_ok();
}

hfr_status launch_raycast_batch(const BatchDev& P, int blocks, int tail_blocks, bool backward, hipStream_t s)
{
    if (backward) raycast_batch_kernel<true><<<dim3(blocks), dim3(256), 0, s>>>(P);
    else raycast_batch_kernel<false><<<dim3(blocks), dim3(256), 0, s>>>(P);
    HFR_LAUNCH_CHECK(backward ? "raycast_backward (batch)" : "raycast (batch)");
    if (!P.ray_queue) return HFR_OK;
    if (backward) raycast_batch_tail_kernel<true><<<dim3(tail_blocks), dim3(256), 0, s>>>(P);
    else raycast_batch_tail_kernel<false><<<dim3(tail_blocks), dim3(256), 0, s>>>(P);
    HFR_LAUNCH_CHECK(backward ? "raycast_backward long rays (batch)" : "raycast long rays (batch)");
    return HFR_OK;
}
