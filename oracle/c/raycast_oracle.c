/*
 * FP64 reference ray caster over cascade textures.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the oracle's Python wrapper, which only
 * the tests, the smoke check and the benchmark's CPU-baseline leg use.  It
 * shares no code or header with the HIP library.
 *
 * What it computes (paper Section 5, plus the readings stated here):
 *  - A ray o + t d (|d| = 1) is clipped to the domain's xy box and to
 *    z <= zmax; t >= 0.  Leaving that box ends the ray (a miss).
 *  - The offset d(t) = (o_xy + t d_xy - origin) . vhat sweeps the cascades;
 *    they are visited in the order the ray sweeps them (nearest first when
 *    d grows along the ray).  Cascade k covers near_k <= d <= far_k and its
 *    texture rectangle [x0, x0 + (N-1) hx] x [y0, y0 + (N-1) hy].
 *  - Inside a cascade the ray is cut at every texel-column and texel-row
 *    crossing; each piece lies in one texture cell, found from the piece's
 *    midpoint.  In a cell whose four corner texels are visible the surface
 *    is the bilinear patch of those texels, and along the piece
 *    f(t) = z(t) - B(u(t), v(t)) is a quadratic in t.  The hit is the
 *    smallest t of the piece with f(t) <= 0: its start when f(start) <= 0,
 *    else the smallest root (stable quadratic formula, linear when the
 *    quadratic coefficient is zero).  The first hit over the pieces in
 *    ray order is the cascade's hit.
 *  - Overlaps: if the first hit A (cascade k) lies in the overlap shared
 *    with the next cascade visited, that cascade is searched over the
 *    overlap part only; if it has a hit B there the depth is the convex
 *    combination (1 - a) t_nearer + a t_farther with
 *    a = clamp((d(t_A) - split) / (far - split), 0, 1) of the nearer
 *    cascade's split and far offsets.  Without B the depth is t_A.
 *  - For each hit the derivative of the returned depth with respect to
 *    t_A and t_B is reported, and the derivative of t_X with respect to its
 *    four corner heights is phi_c(u, v) / f'(t_X) (implicit function
 *    theorem on f(t_X) = 0); a hit at the very start of a cascade segment
 *    does not move with the heights.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    double near_d, far_d, split_d, ox, oy, vx, vy, x0, y0, hx, hy;
    int n;
} ocas;

typedef struct {
    int found, k, i, j, at_start;
    double t, u, v, fp;
} ohit;

static double dmin(double a, double b) { return a < b ? a : b; }
static double dmax(double a, double b) { return a > b ? a : b; }

static void slab(double o, double d, double lo, double hi, double* t0, double* t1)
{
    if (d == 0.0) {
        if (o < lo || o > hi) { *t0 = INFINITY; *t1 = -INFINITY; }
        return;
    }
    double a = (lo - o) / d, b = (hi - o) / d;
    *t0 = dmax(*t0, dmin(a, b));
    *t1 = dmin(*t1, dmax(a, b));
}

static void box_clip(const double* o, const double* d, const double* dom, double* t0, double* t1)
{
    *t0 = 0.0;
    *t1 = INFINITY;
    slab(o[0], d[0], dom[0], dom[2], t0, t1);
    slab(o[1], d[1], dom[1], dom[3], t0, t1);
    if (d[2] > 0.0) *t1 = dmin(*t1, (dom[5] - o[2]) / d[2]);
    else if (d[2] < 0.0) *t0 = dmax(*t0, (dom[5] - o[2]) / d[2]);
    else if (o[2] > dom[5]) { *t0 = INFINITY; *t1 = -INFINITY; }
}

/* t-range where lo <= d(t) <= hi, intersected into [t0, t1]. */
static void offset_range(const double* o, const double* d, const ocas* c, double lo, double hi,
                         double* t0, double* t1)
{
    double d0 = (o[0] - c->ox) * c->vx + (o[1] - c->oy) * c->vy;
    double dd = d[0] * c->vx + d[1] * c->vy;
    if (dd > 0.0) {
        *t0 = dmax(*t0, (lo - d0) / dd);
        *t1 = dmin(*t1, (hi - d0) / dd);
    } else if (dd < 0.0) {
        *t0 = dmax(*t0, (hi - d0) / dd);
        *t1 = dmin(*t1, (lo - d0) / dd);
    } else if (d0 < lo || d0 > hi) {
        *t0 = INFINITY;
        *t1 = -INFINITY;
    }
}

static double offset_at(const double* o, const double* d, const ocas* c, double t)
{
    return ((o[0] + t * d[0]) - c->ox) * c->vx + ((o[1] + t * d[1]) - c->oy) * c->vy;
}

static void segment(const double* o, const double* d, const ocas* c, double lo, double hi,
                    double tin, double tout, double* ta, double* tb)
{
    *ta = tin;
    *tb = tout;
    offset_range(o, d, c, lo, hi, ta, tb);
    slab(o[0], d[0], c->x0, c->x0 + (c->n - 1) * c->hx, ta, tb);
    slab(o[1], d[1], c->y0, c->y0 + (c->n - 1) * c->hy, ta, tb);
}

/* Next t > t at which coordinate o + t d crosses a lattice line base + m h. */
static double next_crossing(double o, double d, double base, double h, double t)
{
    if (d == 0.0) return INFINITY;
    double w = (o + t * d - base) / h;
    double m = d > 0.0 ? floor(w) + 1.0 : ceil(w) - 1.0;
    for (int guard = 0; guard < 4; ++guard) {
        double tm = ((base + m * h) - o) / d;
        if (tm > t) return tm;
        m += d > 0.0 ? 1.0 : -1.0;
    }
    return INFINITY;
}

/* Smallest tau in [0, tau1] with a tau^2 + b tau + c <= 0, given c > 0. */
static int smallest_root(double a, double b, double c, double tau1, double* tau)
{
    double best = INFINITY;
    if (a == 0.0) {
        if (b < 0.0) {
            double r = -c / b;
            if (r <= tau1) best = r;
        }
    } else {
        double D = b * b - 4.0 * a * c;
        if (D >= 0.0) {
            double q = -0.5 * (b + copysign(sqrt(D), b));
            double r1 = q / a, r2 = c / q;
            if (r1 >= 0.0 && r1 <= tau1) best = dmin(best, r1);
            if (r2 >= 0.0 && r2 <= tau1) best = dmin(best, r2);
        }
    }
    if (best == INFINITY) return 0;
    *tau = best;
    return 1;
}

static int first_hit(const double* o, const double* d, const ocas* c, int k, const double* tex,
                     double ta, double tb, ohit* h)
{
    h->found = 0;
    if (!(ta < tb)) return 0;
    const int N = c->n;
    double t = ta;
    while (t < tb) {
        double t1 = dmin(tb, dmin(next_crossing(o[0], d[0], c->x0, c->hx, t),
                                  next_crossing(o[1], d[1], c->y0, c->hy, t)));
        double tm = 0.5 * (t + t1);
        int i = (int)floor(((o[0] + tm * d[0]) - c->x0) / c->hx);
        int j = (int)floor(((o[1] + tm * d[1]) - c->y0) / c->hy);
        i = i < 0 ? 0 : (i > N - 2 ? N - 2 : i);
        j = j < 0 ? 0 : (j > N - 2 ? N - 2 : j);
        double h00 = tex[(size_t)j * N + i], h10 = tex[(size_t)j * N + i + 1];
        double h01 = tex[(size_t)(j + 1) * N + i], h11 = tex[(size_t)(j + 1) * N + i + 1];
        if (isfinite(h00) && isfinite(h10) && isfinite(h01) && isfinite(h11)) {
            double u0 = ((o[0] + t * d[0]) - c->x0) / c->hx - i;
            double v0 = ((o[1] + t * d[1]) - c->y0) / c->hy - j;
            double du = d[0] / c->hx, dv = d[1] / c->hy;
            double z0 = o[2] + t * d[2];
            double A = h10 - h00, B = h01 - h00, C = (h00 - h10) - (h01 - h11);
            double cc = z0 - (h00 + A * u0 + B * v0 + C * u0 * v0);
            double bb = d[2] - A * du - B * dv - C * (u0 * dv + v0 * du);
            double aa = -C * du * dv;
            double tau = 0.0;
            int hit = cc <= 0.0 ? 1 : smallest_root(aa, bb, cc, t1 - t, &tau);
            if (hit) {
                h->found = 1;
                h->k = k;
                h->i = i;
                h->j = j;
                h->t = t + tau;
                h->u = u0 + tau * du;
                h->v = v0 + tau * dv;
                h->fp = 2.0 * aa * tau + bb;
                h->at_start = (cc <= 0.0 && t == ta);
                return 1;
            }
        }
        t = t1;
    }
    return 0;
}

typedef struct {
    const double *orig, *dir, *dom, *cas;
    const double* tex;
    int K, n_rays;
    double* depth;
    int32_t* hit;
    int32_t* rec;  /* per ray: kA iA jA startA kB iB jB startB */
    double* val;   /* per ray: tA uA vA fpA tB uB vB fpB */
    double* coef;  /* per ray: dDepth/dtA, dDepth/dtB */
    int begin, end;
} job;

static void cast_one(const job* J, int r)
{
    const double* o = J->orig + 3 * (size_t)r;
    const double* d = J->dir + 3 * (size_t)r;
    ocas cs[16];
    const int K = J->K;
    size_t NN = 0;
    for (int k = 0; k < K; ++k) {
        const double* p = J->cas + 12 * k;
        cs[k] = (ocas){p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7], p[8], p[9], p[10], (int)p[11]};
        NN = (size_t)cs[k].n * cs[k].n;
    }
    int32_t* rec = J->rec + 8 * (size_t)r;
    double* val = J->val + 8 * (size_t)r;
    double* coef = J->coef + 2 * (size_t)r;
    for (int a = 0; a < 8; ++a) { rec[a] = -1; val[a] = NAN; }
    coef[0] = coef[1] = 0.0;
    J->depth[r] = INFINITY;
    J->hit[r] = -1;

    double tin, tout;
    box_clip(o, d, J->dom, &tin, &tout);
    if (!(tin < tout)) return;
    const double dd = d[0] * cs[0].vx + d[1] * cs[0].vy;
    const int fwd = dd >= 0.0;
    for (int s = 0; s < K; ++s) {
        const int k = fwd ? s : K - 1 - s;
        double ta, tb;
        segment(o, d, &cs[k], cs[k].near_d, cs[k].far_d, tin, tout, &ta, &tb);
        ohit A;
        if (!first_hit(o, d, &cs[k], k, J->tex + NN * k, ta, tb, &A)) continue;
        rec[0] = A.k; rec[1] = A.i; rec[2] = A.j; rec[3] = A.at_start;
        val[0] = A.t; val[1] = A.u; val[2] = A.v; val[3] = A.fp;
        J->hit[r] = (A.k << 26) | (A.j << 13) | A.i;
        double depth = A.t, cA = 1.0, cB = 0.0;
        const int p = fwd ? k + 1 : k - 1;
        if (p >= 0 && p < K) {
            const int ov = fwd ? k : p;           /* nearer cascade of the pair */
            const double lo = cs[ov].split_d, hi = cs[ov].far_d;
            const double dA = offset_at(o, d, &cs[k], A.t);
            if (fwd ? dA >= lo : dA <= hi) {
                double tb0, tb1;
                segment(o, d, &cs[p], lo, hi, tin, tout, &tb0, &tb1);
                ohit B;
                if (first_hit(o, d, &cs[p], p, J->tex + NN * p, tb0, tb1, &B)) {
                    rec[4] = B.k; rec[5] = B.i; rec[6] = B.j; rec[7] = B.at_start;
                    val[4] = B.t; val[5] = B.u; val[6] = B.v; val[7] = B.fp;
                    const double delta = hi - lo;
                    double al = (dA - lo) / delta, dal = dd / delta;
                    if (al <= 0.0) { al = 0.0; dal = 0.0; }
                    if (al >= 1.0) { al = 1.0; dal = 0.0; }
                    if (fwd) {  /* A nearer, B farther */
                        depth = (1.0 - al) * A.t + al * B.t;
                        cA = (1.0 - al) + (B.t - A.t) * dal;
                        cB = al;
                    } else {    /* B nearer, A farther */
                        depth = (1.0 - al) * B.t + al * A.t;
                        cA = al + (A.t - B.t) * dal;
                        cB = 1.0 - al;
                    }
                }
            }
        }
        J->depth[r] = depth;
        coef[0] = cA;
        coef[1] = cB;
        return;
    }
}

static void* run_job(void* arg)
{
    job* J = (job*)arg;
    for (int r = J->begin; r < J->end; ++r) cast_one(J, r);
    return NULL;
}

/* Cast n_rays rays.  cas holds 12 doubles per cascade:
 * near far split origin_x origin_y vhat_x vhat_y x0 y0 hx hy N.
 * tex holds K textures of N*N doubles (row j, column i), -inf = invisible. */
int oracle_raycast(int n_rays, const double* orig, const double* dir, const double* dom, int K,
                   const double* cas, const double* tex, double* depth, int32_t* hit, int32_t* rec,
                   double* val, double* coef, int n_threads)
{
    if (K < 1 || K > 16 || n_rays < 0) return -1;
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    job jobs[256];
    pthread_t th[256];
    int per = (n_rays + n_threads - 1) / n_threads;
    for (int a = 0; a < n_threads; ++a) {
        jobs[a] = (job){orig, dir, dom, cas, tex, K, n_rays, depth, hit, rec, val, coef, 0, 0};
        jobs[a].begin = a * per < n_rays ? a * per : n_rays;
        jobs[a].end = (a + 1) * per < n_rays ? (a + 1) * per : n_rays;
    }
    for (int a = 1; a < n_threads; ++a) pthread_create(&th[a], NULL, run_job, &jobs[a]);
    run_job(&jobs[0]);
    for (int a = 1; a < n_threads; ++a) pthread_join(th[a], NULL);
    return 0;
}

/* First root of one ray in one given cell (i, j) of a cascade, over the whole
 * piece of the ray inside that cell (no cascade-range restriction). */
int oracle_cell_root(const double* o, const double* d, const double* cas, const double* tex_k, int i,
                     int j, double* t_out)
{
    ocas c = {cas[0], cas[1], cas[2], cas[3], cas[4], cas[5], cas[6], cas[7], cas[8], cas[9], cas[10],
              (int)cas[11]};
    double ta = -INFINITY, tb = INFINITY;
    slab(o[0], d[0], c.x0 + i * c.hx, c.x0 + (i + 1) * c.hx, &ta, &tb);
    slab(o[1], d[1], c.y0 + j * c.hy, c.y0 + (j + 1) * c.hy, &ta, &tb);
    ta = dmax(ta, 0.0);
    if (!(ta <= tb)) return 0;
    const int N = c.n;
    double h00 = tex_k[(size_t)j * N + i], h10 = tex_k[(size_t)j * N + i + 1];
    double h01 = tex_k[(size_t)(j + 1) * N + i], h11 = tex_k[(size_t)(j + 1) * N + i + 1];
    if (!(isfinite(h00) && isfinite(h10) && isfinite(h01) && isfinite(h11))) return 0;
    double u0 = ((o[0] + ta * d[0]) - c.x0) / c.hx - i;
    double v0 = ((o[1] + ta * d[1]) - c.y0) / c.hy - j;
    double du = d[0] / c.hx, dv = d[1] / c.hy;
    double A = h10 - h00, B = h01 - h00, C = (h00 - h10) - (h01 - h11);
    double cc = (o[2] + ta * d[2]) - (h00 + A * u0 + B * v0 + C * u0 * v0);
    double bb = d[2] - A * du - B * dv - C * (u0 * dv + v0 * du);
    double aa = -C * du * dv;
    double tau = 0.0;
    if (cc > 0.0 && !smallest_root(aa, bb, cc, tb - ta, &tau)) return 0;
    *t_out = ta + tau;
    return 1;
}
