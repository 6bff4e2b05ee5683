/*
 * FP64 reference of the truncated radial-basis approximation (Eq. 1 and
 * Eq. 2) and of its adjoint, for workloads too large for the NumPy form.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the oracle's Python wrapper, which only
 * the tests, the smoke check and the benchmark's CPU-baseline leg use.  It
 * shares no code or header with the HIP library.
 *
 * What it computes, per point p (already clamped into the domain by the
 * caller):
 *   w_j(p) = exp(-(r / (sigma_j c_j))^2 / 2) - exp(-k^2 / 2), r = |p_j - p|
 *            (Eq. 1; Wendland's (1 - u)^4 (4u + 1) with u = r / (k sigma_j c_j)
 *            when basis = 1), and leaf j influences p iff w_j(p) > 0;
 *   v(p)   = sum_j w_j v_j / sum_j w_j over the influencing leaves (Eq. 2).
 * The adjoint adds, for every point s with texel gradient g_s,
 *   g_s w_j / S0 to d/dv_j  and  g_s (v_j - v_s) / S0 * dw_j/dsigma_j to d/dsigma_j.
 *
 * Finding the influencing leaves: leaves are grouped by cell size (every
 * quadtree level has one), and each group is bucketed on a square grid
 * whose bucket side is at least the group's largest truncation radius
 * k sigma c.  A leaf can influence p only if it lies within that radius,
 * so it lies in p's bucket or one of the eight around it; every leaf in
 * those buckets is tested with its own weight.  This is a search structure
 * only: the sum is the definition's sum over every leaf with w > 0.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double c;         /* cell size of the group */
    double reach;     /* bucket side: the group's largest truncation radius */
    double bx0, by0;  /* bucket grid origin */
    int64_t nb;       /* buckets per side */
    int64_t* start;   /* [nb * nb + 1] first entry of each bucket */
    int64_t* ids;     /* leaf indices, bucket by bucket */
} group_t;

typedef struct {
    int64_t n;
    const double *x, *y, *c, *v, *sigma;
    double cutoff, E;
    int basis;
    int n_groups;
    group_t* g;
} field_t;

static int cmp_double(const void* a, const void* b)
{
    const double x = *(const double*)a, y = *(const double*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static void free_field(field_t* f)
{
    for (int a = 0; a < f->n_groups; ++a) {
        free(f->g[a].start);
        free(f->g[a].ids);
    }
    free(f->g);
}

/* Groups by cell size and buckets each group.  0 on success. */
static int build_field(field_t* f)
{
    double* sizes = malloc(sizeof(double) * (size_t)f->n);
    if (!sizes) return -1;
    memcpy(sizes, f->c, sizeof(double) * (size_t)f->n);
    qsort(sizes, (size_t)f->n, sizeof(double), cmp_double);
    int m = 0;
    for (int64_t a = 0; a < f->n; ++a)
        if (a == 0 || sizes[a] != sizes[a - 1]) sizes[m++] = sizes[a];
    f->n_groups = m;
    f->g = calloc((size_t)m, sizeof(group_t));
    if (!f->g) { free(sizes); return -1; }
    double xmin = INFINITY, ymin = INFINITY, xmax = -INFINITY, ymax = -INFINITY;
    for (int64_t a = 0; a < f->n; ++a) {
        xmin = fmin(xmin, f->x[a]); xmax = fmax(xmax, f->x[a]);
        ymin = fmin(ymin, f->y[a]); ymax = fmax(ymax, f->y[a]);
    }
    for (int q = 0; q < m; ++q) {
        group_t* g = &f->g[q];
        g->c = sizes[q];
        double smax = 0.0;
        for (int64_t a = 0; a < f->n; ++a)
            if (f->c[a] == g->c && f->sigma[a] > smax) smax = f->sigma[a];
        g->reach = f->cutoff * smax * g->c;
        const double span = fmax(xmax - xmin, ymax - ymin);
        g->nb = (int64_t)floor(span / g->reach) + 1;
        if (g->nb > 8192) { /* a finer grid than this only saves tests */
            g->nb = 8192;
            g->reach = span / 8191.0;
            if (g->reach < f->cutoff * smax * g->c) g->reach = f->cutoff * smax * g->c;
        }
        g->bx0 = xmin;
        g->by0 = ymin;
        const int64_t nbb = g->nb * g->nb;
        g->start = calloc((size_t)(nbb + 1), sizeof(int64_t));
        if (!g->start) { free(sizes); return -1; }
        int64_t count = 0;
        for (int64_t a = 0; a < f->n; ++a) {
            if (f->c[a] != g->c) continue;
            int64_t bi = (int64_t)floor((f->x[a] - g->bx0) / g->reach);
            int64_t bj = (int64_t)floor((f->y[a] - g->by0) / g->reach);
            bi = bi < 0 ? 0 : (bi >= g->nb ? g->nb - 1 : bi);
            bj = bj < 0 ? 0 : (bj >= g->nb ? g->nb - 1 : bj);
            g->start[bj * g->nb + bi + 1]++;
            count++;
        }
        for (int64_t b = 0; b < nbb; ++b) g->start[b + 1] += g->start[b];
        g->ids = malloc(sizeof(int64_t) * (size_t)(count ? count : 1));
        int64_t* fill = malloc(sizeof(int64_t) * (size_t)nbb);
        if (!g->ids || !fill) { free(fill); free(sizes); return -1; }
        memcpy(fill, g->start, sizeof(int64_t) * (size_t)nbb);
        for (int64_t a = 0; a < f->n; ++a) {
            if (f->c[a] != g->c) continue;
            int64_t bi = (int64_t)floor((f->x[a] - g->bx0) / g->reach);
            int64_t bj = (int64_t)floor((f->y[a] - g->by0) / g->reach);
            bi = bi < 0 ? 0 : (bi >= g->nb ? g->nb - 1 : bi);
            bj = bj < 0 ? 0 : (bj >= g->nb ? g->nb - 1 : bj);
            g->ids[fill[bj * g->nb + bi]++] = a;
        }
        free(fill);
    }
    free(sizes);
    return 0;
}

/* Eq. 1 (or Wendland's function) and its sigma-derivative for leaf j at p. */
static double weight(const field_t* f, int64_t j, double px, double py, double* dw_dsigma)
{
    const double r = hypot(f->x[j] - px, f->y[j] - py);
    const double q = r / (f->sigma[j] * f->c[j]);
    if (f->basis == 1) {
        const double u = q / f->cutoff;
        if (!(u < 1.0)) { *dw_dsigma = 0.0; return 0.0; }
        const double t = 1.0 - u;
        *dw_dsigma = 20.0 * u * u * t * t * t / f->sigma[j];
        return t * t * t * t * (4.0 * u + 1.0);
    }
    const double g = exp(-0.5 * q * q);
    *dw_dsigma = g * q * q / f->sigma[j];
    return g - f->E;
}

/* Calls visit(j, w, dw/dsigma) for every leaf with w > 0 at p. */
typedef void (*visit_fn)(void* ctx, int64_t j, double w, double dw);

static void for_each_influencer(const field_t* f, double px, double py, visit_fn visit, void* ctx)
{
    for (int q = 0; q < f->n_groups; ++q) {
        const group_t* g = &f->g[q];
        const int64_t ci = (int64_t)floor((px - g->bx0) / g->reach);
        const int64_t cj = (int64_t)floor((py - g->by0) / g->reach);
        for (int64_t bj = cj - 1; bj <= cj + 1; ++bj) {
            if (bj < 0 || bj >= g->nb) continue;
            for (int64_t bi = ci - 1; bi <= ci + 1; ++bi) {
                if (bi < 0 || bi >= g->nb) continue;
                const int64_t b = bj * g->nb + bi;
                for (int64_t e = g->start[b]; e < g->start[b + 1]; ++e) {
                    const int64_t j = g->ids[e];
                    double dw;
                    const double w = weight(f, j, px, py, &dw);
                    if (w > 0.0) visit(ctx, j, w, dw);
                }
            }
        }
    }
}

typedef struct {
    const field_t* f;
    double s0, s1;
} sum_ctx;

static void add_sum(void* ctx, int64_t j, double w, double dw)
{
    (void)dw;
    sum_ctx* s = ctx;
    s->s0 += w;
    s->s1 += w * s->f->v[j];
}

typedef struct {
    const field_t* f;
    const double *px, *py;
    double *val, *s0;
    int64_t a0, a1;
} eval_job;

static void* eval_range(void* arg)
{
    eval_job* J = arg;
    for (int64_t a = J->a0; a < J->a1; ++a) {
        sum_ctx s = {J->f, 0.0, 0.0};
        for_each_influencer(J->f, J->px[a], J->py[a], add_sum, &s);
        J->s0[a] = s.s0;
        J->val[a] = s.s1 / s.s0;
    }
    return NULL;
}

/* Eq. 2 at n_pts points: val[a] = v(p_a), s0[a] = sum of the weights.
 * Returns 0, or -1 on bad arguments or allocation failure. */
int oracle_rbf_eval(int64_t n, const double* x, const double* y, const double* c, const double* v,
                    const double* sigma, double cutoff, int basis, int64_t n_pts, const double* px,
                    const double* py, double* val, double* s0, int threads)
{
    if (n < 1 || cutoff <= 0.0 || (basis != 0 && basis != 1) || n_pts < 0) return -1;
    field_t f = {n, x, y, c, v, sigma, cutoff, exp(-0.5 * cutoff * cutoff), basis, 0, NULL};
    if (basis == 1) f.E = 0.0;
    if (build_field(&f) != 0) { free_field(&f); return -1; }
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t tid[256];
    eval_job jobs[256];
    for (int t = 0; t < threads; ++t) {
        jobs[t] = (eval_job){&f, px, py, val, s0, n_pts * t / threads, n_pts * (t + 1) / threads};
        if (threads > 1) pthread_create(&tid[t], NULL, eval_range, &jobs[t]);
    }
    if (threads == 1) eval_range(&jobs[0]);
    else for (int t = 0; t < threads; ++t) pthread_join(tid[t], NULL);
    free_field(&f);
    return 0;
}

typedef struct {
    const field_t* f;
    double g, vs, s0;  /* texel gradient, texel value, weight sum */
    double *gv, *gs;
} grad_ctx;

static void add_grad(void* ctx, int64_t j, double w, double dw)
{
    grad_ctx* G = ctx;
    G->gv[j] += G->g * w / G->s0;
    G->gs[j] += G->g * (G->f->v[j] - G->vs) / G->s0 * dw;
}

/* Adjoint of Eq. 2 at n_pts points with gradients g[a]: accumulates
 * d loss / d v into gv[n] and d loss / d sigma into gs[n] (v_s and S0 are
 * recomputed here).  Single thread, points in order.  0 or -1. */
int oracle_rbf_adjoint(int64_t n, const double* x, const double* y, const double* c, const double* v,
                       const double* sigma, double cutoff, int basis, int64_t n_pts, const double* px,
                       const double* py, const double* g, double* gv, double* gs)
{
    if (n < 1 || cutoff <= 0.0 || (basis != 0 && basis != 1) || n_pts < 0) return -1;
    field_t f = {n, x, y, c, v, sigma, cutoff, exp(-0.5 * cutoff * cutoff), basis, 0, NULL};
    if (basis == 1) f.E = 0.0;
    if (build_field(&f) != 0) { free_field(&f); return -1; }
    for (int64_t a = 0; a < n_pts; ++a) {
        if (g[a] == 0.0) continue;
        sum_ctx s = {&f, 0.0, 0.0};
        for_each_influencer(&f, px[a], py[a], add_sum, &s);
        grad_ctx G = {&f, g[a], s.s1 / s.s0, s.s0, gv, gs};
        for_each_influencer(&f, px[a], py[a], add_grad, &G);
    }
    free_field(&f);
    return 0;
}
