// Host side of libhfr: error reporting, start-up structures (adaptive
// quadtree, influence lists, point-location lattice) and per-frame cascade
// fitting.  Everything here is plain C++17 in FP64.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "hfr_internal.h"

// ------------------------------------------------------------------ errors

static thread_local std::string g_last_error;

hfr_status hfr_fail(hfr_status code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

hfr_status hfr_ok()
{
    g_last_error.clear();
    return HFR_OK;
}

extern "C" int hfr_abi_version(void) { return HFR_ABI_VERSION; }

extern "C" const char* hfr_last_error(void) { return g_last_error.c_str(); }

extern "C" hfr_status hfr_runtime_version(int* version)
{
    HFR_REQUIRE(version != nullptr, "version is NULL");
    hipError_t e = hipRuntimeGetVersion(version);
    if (e != hipSuccess) return hfr_fail(HFR_EDEVICE, "hipRuntimeGetVersion: %s", hipGetErrorString(e));
    return hfr_ok();
}

static unsigned worker_count(int64_t work)
{
    unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    hw = std::min(hw, 64u);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(hw, work / 4096 + 1));
}

template <class F>
static void parallel_for(int64_t n, F&& body)
{
    unsigned T = worker_count(n);
    if (T == 1) {
        body(0, n, 0u);
        return;
    }
    std::vector<std::thread> th;
    int64_t per = (n + T - 1) / T;
    for (unsigned t = 0; t < T; ++t) {
        int64_t a = std::min<int64_t>(n, t * per), b = std::min<int64_t>(n, (t + 1) * per);
        th.emplace_back([=, &body] { body(a, b, t); });
    }
    for (auto& x : th) x.join();
}

// ------------------------------------------------------------------ quadtree

struct hfr_quadtree {
    std::vector<float> x, y, c, v;
    std::vector<int32_t> level, i, j;
};

extern "C" hfr_status hfr_build_quadtree(const float* dem, int64_t n, double side, double x0, double y0,
                                         int32_t max_depth, double tau, hfr_quadtree** out)
{
    HFR_REQUIRE(dem != nullptr && out != nullptr, "dem and out must not be NULL");
    HFR_REQUIRE(hfr_is_pow2(n) && n <= 65536, "raster side %lld must be a power of two <= 65536", (long long)n);
    const int D = hfr_log2i(n);
    HFR_REQUIRE(max_depth >= 0 && max_depth <= D, "max_depth %d outside [0, %d]", max_depth, D);
    HFR_REQUIRE(std::isfinite(side) && side > 0 && std::isfinite(x0) && std::isfinite(y0),
                "side must be positive and the origin finite");
    HFR_REQUIRE(!std::isnan(tau), "tau is NaN");
    *out = nullptr;
    for (int64_t a = 0; a < n * n; ++a)
        HFR_REQUIRE(std::isfinite(dem[a]), "raster sample %lld is not finite", (long long)a);

    hfr_quadtree* q = new (std::nothrow) hfr_quadtree;
    if (!q) return hfr_fail(HFR_ENOMEM, "out of host memory");
    try {
        // mean pyramid, levels 0 .. max_depth (finer levels only feed the next coarser one)
        std::vector<std::vector<double>> M(D + 1);
        M[D].assign(dem, dem + n * n);
        for (int l = D - 1; l >= 0; --l) {
            const int64_t s = int64_t(1) << l, s2 = s * 2;
            M[l].resize(s * s);
            const std::vector<double>& f = M[l + 1];
            for (int64_t jj = 0; jj < s; ++jj)
                for (int64_t ii = 0; ii < s; ++ii) {
                    double a = f[(2 * jj) * s2 + 2 * ii], b = f[(2 * jj) * s2 + 2 * ii + 1];
                    double c = f[(2 * jj + 1) * s2 + 2 * ii], d = f[(2 * jj + 1) * s2 + 2 * ii + 1];
                    M[l][jj * s + ii] = ((a + b) + (c + d)) * 0.25;
                }
        }
        auto crit = [&](int l, int64_t ii, int64_t jj) {
            const int L = l + 1;
            const int64_t s = int64_t(1) << L;
            const std::vector<double>& m = M[L];
            double best = 0.0;
            for (int64_t cj = 2 * jj; cj <= 2 * jj + 1; ++cj)
                for (int64_t ci = 2 * ii; ci <= 2 * ii + 1; ++ci) {
                    const double ctr = m[cj * s + ci];
                    const double lf = m[cj * s + std::max<int64_t>(ci - 1, 0)];
                    const double rt = m[cj * s + std::min<int64_t>(ci + 1, s - 1)];
                    const double dn = m[std::max<int64_t>(cj - 1, 0) * s + ci];
                    const double up = m[std::min<int64_t>(cj + 1, s - 1) * s + ci];
                    const double d2x = (lf + rt) - 2.0 * ctr;
                    const double d2y = (dn + up) - 2.0 * ctr;
                    best = std::max(best, std::max(std::fabs(d2x), std::fabs(d2y)));
                }
            return best;
        };
        struct Node { int32_t l, i, j; };
        std::vector<Node> stack{{0, 0, 0}};
        while (!stack.empty()) {
            Node nd = stack.back();
            stack.pop_back();
            if (nd.l < max_depth && crit(nd.l, nd.i, nd.j) > tau) {
                // push children so that (0,0), (1,0), (0,1), (1,1) pop in that order
                for (int dj = 1; dj >= 0; --dj)
                    for (int di = 1; di >= 0; --di)
                        stack.push_back({nd.l + 1, 2 * nd.i + di, 2 * nd.j + dj});
            } else {
                const double c = side / std::ldexp(1.0, nd.l);
                q->x.push_back((float)(x0 + (nd.i + 0.5) * c));
                q->y.push_back((float)(y0 + (nd.j + 0.5) * c));
                q->c.push_back((float)c);
                q->v.push_back((float)M[nd.l][(int64_t)nd.j * (int64_t(1) << nd.l) + nd.i]);
                q->level.push_back(nd.l);
                q->i.push_back(nd.i);
                q->j.push_back(nd.j);
            }
        }
    } catch (const std::bad_alloc&) {
        delete q;
        return hfr_fail(HFR_ENOMEM, "out of host memory building the quadtree");
    }
    *out = q;
    return hfr_ok();
}

extern "C" hfr_status hfr_quadtree_size(const hfr_quadtree* q, int64_t* n_leaves)
{
    HFR_REQUIRE(q && n_leaves, "NULL argument");
    *n_leaves = (int64_t)q->x.size();
    return hfr_ok();
}

extern "C" hfr_status hfr_quadtree_export(const hfr_quadtree* q, float* x, float* y, float* c, float* v,
                                          int32_t* level, int32_t* i, int32_t* j)
{
    HFR_REQUIRE(q != nullptr, "quadtree is NULL");
    const size_t n = q->x.size();
    if (x) std::memcpy(x, q->x.data(), n * sizeof(float));
    if (y) std::memcpy(y, q->y.data(), n * sizeof(float));
    if (c) std::memcpy(c, q->c.data(), n * sizeof(float));
    if (v) std::memcpy(v, q->v.data(), n * sizeof(float));
    if (level) std::memcpy(level, q->level.data(), n * sizeof(int32_t));
    if (i) std::memcpy(i, q->i.data(), n * sizeof(int32_t));
    if (j) std::memcpy(j, q->j.data(), n * sizeof(int32_t));
    return hfr_ok();
}

extern "C" void hfr_quadtree_destroy(hfr_quadtree* q) { delete q; }

// ------------------------------------------------------- lattice bookkeeping

namespace {

struct LatticeLeaves {
    std::vector<int8_t> level;
    std::vector<int32_t> i, j;
};

// Recovers (level, i, j) of each leaf from its centre and size.
hfr_status lattice_of(int64_t n, const float* x, const float* y, const float* c, double x0, double y0,
                      double side, int max_depth, LatticeLeaves& out)
{
    HFR_REQUIRE(n >= 1 && x && y && c, "need n >= 1 leaves with x, y, c");
    HFR_REQUIRE(std::isfinite(side) && side > 0 && std::isfinite(x0) && std::isfinite(y0),
                "side must be positive and the origin finite");
    HFR_REQUIRE(max_depth >= 0 && max_depth <= 24, "max_depth %d outside [0, 24]", max_depth);
    out.level.resize(n);
    out.i.resize(n);
    out.j.resize(n);
    for (int64_t a = 0; a < n; ++a) {
        const double ca = c[a];
        HFR_REQUIRE(std::isfinite(ca) && ca > 0, "leaf %lld has an invalid size", (long long)a);
        const int l = (int)std::lround(std::log2(side / ca));
        const double cl = side / std::ldexp(1.0, l);
        HFR_REQUIRE(l >= 0 && l <= max_depth && std::fabs(ca - cl) <= 1e-6 * cl,
                    "leaf %lld size %g is not side / 2^l with l <= %d", (long long)a, ca, max_depth);
        const double fi = (x[a] - x0) / cl - 0.5, fj = (y[a] - y0) / cl - 0.5;
        const int64_t ii = std::llround(fi), jj = std::llround(fj);
        const int64_t s = int64_t(1) << l;
        HFR_REQUIRE(std::fabs(fi - ii) <= 1e-4 && std::fabs(fj - jj) <= 1e-4 && ii >= 0 && jj >= 0 && ii < s && jj < s,
                    "leaf %lld centre (%g, %g) is off the level-%d lattice", (long long)a, x[a], y[a], l);
        out.level[a] = (int8_t)l;
        out.i[a] = (int32_t)ii;
        out.j[a] = (int32_t)jj;
    }
    return HFR_OK;
}

}  // namespace

// ------------------------------------------------------------ influence lists

struct hfr_neighbours {
    std::vector<int32_t> off, idx;
};

extern "C" hfr_status hfr_build_neighbours(int64_t n, const float* x, const float* y, const float* c,
                                           const float* sigma, double x0, double y0, double side,
                                           int32_t max_depth, float cutoff, float slack, hfr_neighbours** out)
{
    HFR_REQUIRE(out != nullptr && sigma != nullptr, "out and sigma must not be NULL");
    HFR_REQUIRE(std::isfinite(cutoff) && cutoff > 0, "cutoff must be positive");
    HFR_REQUIRE(std::isfinite(slack) && slack >= 0, "slack must be >= 0");
    *out = nullptr;
    LatticeLeaves lat;
    hfr_status st = lattice_of(n, x, y, c, x0, y0, side, max_depth, lat);
    if (st != HFR_OK) return st;
    for (int64_t a = 0; a < n; ++a)
        HFR_REQUIRE(std::isfinite(sigma[a]) && sigma[a] > 0, "leaf %lld has an invalid sigma", (long long)a);

    hfr_neighbours* nb = new (std::nothrow) hfr_neighbours;
    if (!nb) return hfr_fail(HFR_ENOMEM, "out of host memory");
    try {
        // dense per-level index: leaf id at (level, i, j) or -1
        int top = 0;
        for (int64_t a = 0; a < n; ++a) top = std::max(top, (int)lat.level[a]);
        std::vector<std::vector<int32_t>> grid(top + 1);
        std::vector<double> rmax(top + 1, 0.0);
        std::vector<char> present(top + 1, 0);
        for (int64_t a = 0; a < n; ++a) {
            const int l = lat.level[a];
            if (!present[l]) {
                present[l] = 1;
                grid[l].assign((size_t)1 << (2 * l), -1);
            }
            grid[l][((size_t)lat.j[a] << l) + lat.i[a]] = (int32_t)a;
            const double R = (((double)cutoff * (double)sigma[a]) * (double)c[a]) * (1.0 + (double)slack);
            rmax[l] = std::max(rmax[l], R);
        }
        const unsigned T = worker_count(n);
        std::vector<std::vector<int32_t>> part_idx(T);
        std::vector<std::vector<int64_t>> part_cnt(T);
        std::vector<int64_t> begin(T + 1, 0);
        parallel_for(n, [&](int64_t lo, int64_t hi, unsigned t) {
            std::vector<int32_t>& out_idx = part_idx[t];
            std::vector<int64_t>& cnt = part_cnt[t];
            std::vector<int32_t> cand;
            for (int64_t a = lo; a < hi; ++a) {
                cand.clear();
                const double xa = x[a], ya = y[a], ha = 0.5 * (double)c[a];
                for (int l = 0; l <= top; ++l) {
                    if (!present[l]) continue;
                    const double cl = side / std::ldexp(1.0, l);
                    const int64_t s = int64_t(1) << l;
                    const double reach = ha + rmax[l];
                    const int64_t i0 = std::max<int64_t>(0, (int64_t)std::floor((xa - reach - x0) / cl - 0.5) - 1);
                    const int64_t i1 = std::min<int64_t>(s - 1, (int64_t)std::ceil((xa + reach - x0) / cl - 0.5) + 1);
                    const int64_t j0 = std::max<int64_t>(0, (int64_t)std::floor((ya - reach - y0) / cl - 0.5) - 1);
                    const int64_t j1 = std::min<int64_t>(s - 1, (int64_t)std::ceil((ya + reach - y0) / cl - 0.5) + 1);
                    const int32_t* g = grid[l].data();
                    for (int64_t jj = j0; jj <= j1; ++jj)
                        for (int64_t ii = i0; ii <= i1; ++ii) {
                            const int32_t b = g[(jj << l) + ii];
                            if (b < 0) continue;
                            const double dx = std::max(std::fabs((double)x[b] - xa) - ha, 0.0);
                            const double dy = std::max(std::fabs((double)y[b] - ya) - ha, 0.0);
                            const double R = (((double)cutoff * (double)sigma[b]) * (double)c[b]) * (1.0 + (double)slack);
                            if (dx * dx + dy * dy < R * R) cand.push_back(b);
                        }
                }
                std::sort(cand.begin(), cand.end());
                out_idx.insert(out_idx.end(), cand.begin(), cand.end());
                cnt.push_back((int64_t)cand.size());
            }
        });
        int64_t total = 0;
        for (unsigned t = 0; t < T; ++t) total += (int64_t)part_idx[t].size();
        if (total > INT32_MAX) {
            delete nb;
            return hfr_fail(HFR_ECAPACITY, "influence lists hold %lld entries, above the INT32_MAX that the 32-bit offsets hold (hfr_build_neighbours_device has 64-bit offsets)", (long long)total);
        }
        nb->off.resize(n + 1);
        nb->idx.reserve(total);
        int64_t pos = 0, a = 0;
        nb->off[0] = 0;
        for (unsigned t = 0; t < T; ++t) {
            for (int64_t k : part_cnt[t]) {
                pos += k;
                nb->off[++a] = (int32_t)pos;
            }
            nb->idx.insert(nb->idx.end(), part_idx[t].begin(), part_idx[t].end());
            std::vector<int32_t>().swap(part_idx[t]);
        }
    } catch (const std::bad_alloc&) {
        delete nb;
        return hfr_fail(HFR_ENOMEM, "out of host memory building influence lists");
    }
    *out = nb;
    return hfr_ok();
}

extern "C" hfr_status hfr_neighbours_size(const hfr_neighbours* nb, int64_t* nnz)
{
    HFR_REQUIRE(nb && nnz, "NULL argument");
    *nnz = (int64_t)nb->idx.size();
    return hfr_ok();
}

extern "C" hfr_status hfr_neighbours_export(const hfr_neighbours* nb, int32_t* off, int32_t* idx)
{
    HFR_REQUIRE(nb && off && idx, "NULL argument");
    std::memcpy(off, nb->off.data(), nb->off.size() * sizeof(int32_t));
    std::memcpy(idx, nb->idx.data(), nb->idx.size() * sizeof(int32_t));
    return hfr_ok();
}

extern "C" void hfr_neighbours_destroy(hfr_neighbours* nb) { delete nb; }

// ------------------------------------------------------------ node table

extern "C" hfr_status hfr_build_level_index(int64_t n, const float* x, const float* y, const float* c, double x0,
                                            double y0, double side, int32_t max_depth, int32_t* rank, int32_t* order)
{
    HFR_REQUIRE(rank != nullptr && order != nullptr, "rank and order must not be NULL");
    HFR_REQUIRE(max_depth >= 0 && max_depth <= 15, "max_depth %d outside [0, 15]", max_depth);
    HFR_REQUIRE(n <= INT32_MAX, "leaf count %lld above INT32_MAX", (long long)n);
    LatticeLeaves lat;
    hfr_status st = lattice_of(n, x, y, c, x0, y0, side, max_depth, lat);
    if (st != HFR_OK) return st;
    const int64_t total = ((int64_t(1) << (2 * (max_depth + 1))) - 1) / 3 + max_depth + 1;
    std::fill(rank, rank + total, 0);
    // coverage count on the finest lattice detects gaps and overlaps
    const int64_t S = int64_t(1) << max_depth;
    std::vector<uint8_t> cover;
    try {
        cover.assign(S * S, 0);
    } catch (const std::bad_alloc&) {
        return hfr_fail(HFR_ENOMEM, "out of host memory");
    }
    auto level_off = [](int l) { return ((int64_t(1) << (2 * l)) - 1) / 3 + l; };
    for (int64_t a = 0; a < n; ++a) {
        const int l = lat.level[a];
        int32_t& cnt = rank[level_off(l) + ((int64_t)lat.j[a] << l) + lat.i[a] + 1];
        HFR_REQUIRE(cnt == 0, "leaf %lld shares its lattice node with another leaf", (long long)a);
        cnt = 1;
        const int sh = max_depth - l;
        const int64_t i0 = (int64_t)lat.i[a] << sh, j0 = (int64_t)lat.j[a] << sh, w = int64_t(1) << sh;
        for (int64_t jj = j0; jj < j0 + w; ++jj)
            for (int64_t ii = i0; ii < i0 + w; ++ii) {
                HFR_REQUIRE(cover[jj * S + ii] == 0, "leaf %lld overlaps another leaf", (long long)a);
                cover[jj * S + ii] = 1;
            }
    }
    for (int64_t a = 0; a < S * S; ++a) HFR_REQUIRE(cover[a], "lattice cell %lld is not covered", (long long)a);
    // exclusive prefix counts, level after level: rank[off_l + q] = leaves before (l, q)
    int64_t acc = 0;
    for (int l = 0; l <= max_depth; ++l) {
        int32_t* r = rank + level_off(l);
        const int64_t cells = int64_t(1) << (2 * l);
        r[0] = (int32_t)acc;
        for (int64_t q = 1; q <= cells; ++q) {
            acc += r[q];
            r[q] = (int32_t)acc;
        }
    }
    for (int64_t a = 0; a < n; ++a) {
        const int l = lat.level[a];
        order[rank[level_off(l) + ((int64_t)lat.j[a] << l) + lat.i[a]]] = (int32_t)a;
    }
    return hfr_ok();
}

// ------------------------------------------------------------ cascade fitting

namespace {

struct V3 { double x, y, z; };
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

struct P2 { double x, y; };

struct Plane { V3 a; double h; };  // a . p >= h

// Convex polygon (3-D) clipped to a half-space (Sutherland-Hodgman, one plane).
std::vector<V3> clip3(const std::vector<V3>& poly, const Plane& pl)
{
    std::vector<V3> out;
    const size_t m = poly.size();
    for (size_t k = 0; k < m; ++k) {
        const V3 p = poly[k], q = poly[(k + 1) % m];
        const double gp = dot(pl.a, p) - pl.h, gq = dot(pl.a, q) - pl.h;
        if (gp >= 0) out.push_back(p);
        if ((gp >= 0) != (gq >= 0)) out.push_back(p + (gp / (gp - gq)) * (q - p));
    }
    return out;
}

// Convex polygon (2-D) restricted to where g(p) = s * ((p - o) . v - lim) >= 0.
std::vector<P2> clip2(const std::vector<P2>& poly, P2 o, P2 v, double lim, double s)
{
    std::vector<P2> out;
    const size_t m = poly.size();
    auto g = [&](P2 p) { return s * (((p.x - o.x) * v.x + (p.y - o.y) * v.y) - lim); };
    for (size_t k = 0; k < m; ++k) {
        const P2 p = poly[k], q = poly[(k + 1) % m];
        const double gp = g(p), gq = g(q);
        if (gp >= 0) out.push_back(p);
        if ((gp >= 0) != (gq >= 0) && m > 1) {
            const double t = gp / (gp - gq);
            out.push_back({p.x + t * (q.x - p.x), p.y + t * (q.y - p.y)});
        }
    }
    std::vector<P2> res;
    for (const P2& p : out)
        if (res.empty() || p.x != res.back().x || p.y != res.back().y) res.push_back(p);
    if (res.size() > 1 && res.front().x == res.back().x && res.front().y == res.back().y) res.pop_back();
    return res;
}

double cross2(P2 o, P2 a, P2 b) { return (a.x - o.x) * (b.y - o.y) - (a.y - o.y) * (b.x - o.x); }

// Counter-clockwise convex hull (monotone chain), collinear points dropped.
std::vector<P2> hull2(std::vector<P2> pts)
{
    std::sort(pts.begin(), pts.end(), [](P2 a, P2 b) { return a.x < b.x || (a.x == b.x && a.y < b.y); });
    pts.erase(std::unique(pts.begin(), pts.end(), [](P2 a, P2 b) { return a.x == b.x && a.y == b.y; }), pts.end());
    if (pts.size() <= 2) return pts;
    std::vector<P2> h(2 * pts.size());
    size_t k = 0;
    for (size_t a = 0; a < pts.size(); ++a) {
        while (k >= 2 && cross2(h[k - 2], h[k - 1], pts[a]) <= 0) --k;
        h[k++] = pts[a];
    }
    for (size_t a = pts.size() - 1, t = k + 1; a-- > 0;) {
        while (k >= t && cross2(h[k - 2], h[k - 1], pts[a]) <= 0) --k;
        h[k++] = pts[a];
    }
    h.resize(k - 1);
    return h;
}

const double kSnapTol = 1e-9;

void snap_axis(double lo, double hi, double origin, double c_min, int N, double* x0, double* h)
{
    *x0 = origin + std::floor((lo - origin) / c_min + kSnapTol) * c_min;
    const double ext = std::max(1.0, std::ceil((hi - *x0) / (2.0 * c_min) - kSnapTol)) * 2.0 * c_min;
    *h = ext / (N - 1);
}

// Fixed-lattice form: the spacing is the smallest c_min 2^(e/4) (integer e) whose lattice,
// anchored at a whole number of spacings from the origin, covers [lo, hi].
void snap_axis_aligned(double lo, double hi, double origin, double c_min, int N, double* x0, double* h)
{
    static const double quarter[4] = {1.0, 1.189207115002721, 1.4142135623730951, 1.681792830507429};
    const double need = std::max(hi - lo, 0.0) / (N - 1);
    int e = need > 0 ? (int)std::floor(4.0 * std::log2(need / c_min)) - 1 : -64;
    for (;; ++e) {
        const int q = (int)std::floor(e / 4.0), r = e - 4 * q;
        *h = std::ldexp(c_min * quarter[r], q);
        *x0 = origin + std::floor((lo - origin) / *h + kSnapTol) * *h;
        if (*x0 + (N - 1) * *h >= hi - kSnapTol * *h) return;
    }
}

hfr_status fit_cascades(const hfr_camera* cam, const hfr_domain* dom, int32_t K, int32_t N, double lambda,
                        double overlap, double c_min, bool aligned, hfr_cascade* out);

}  // namespace

extern "C" hfr_status hfr_fit_cascades(const hfr_camera* cam, const hfr_domain* dom, int32_t K, int32_t N,
                                       double lambda, double overlap, double c_min, hfr_cascade* out)
{
    return fit_cascades(cam, dom, K, N, lambda, overlap, c_min, false, out);
}

extern "C" hfr_status hfr_fit_cascades_aligned(const hfr_camera* cam, const hfr_domain* dom, int32_t K, int32_t N,
                                               double lambda, double overlap, double c_min, hfr_cascade* out)
{
    return fit_cascades(cam, dom, K, N, lambda, overlap, c_min, true, out);
}

namespace {

hfr_status fit_cascades(const hfr_camera* cam, const hfr_domain* dom, int32_t K, int32_t N, double lambda,
                        double overlap, double c_min, bool aligned, hfr_cascade* out)
{
    HFR_REQUIRE(cam && dom && out, "NULL argument");
    HFR_REQUIRE(K >= 1 && K <= HFR_MAX_CASCADES, "K = %d outside [1, %d]", K, HFR_MAX_CASCADES);
    HFR_REQUIRE(hfr_is_pow2(N) && N >= 2 && N <= HFR_MAX_TEX_N, "N = %d is not a power of two in [2, %d]", N,
                HFR_MAX_TEX_N);
    HFR_REQUIRE(std::isfinite(c_min) && c_min > 0, "c_min must be positive");
    HFR_REQUIRE(lambda >= 0 && lambda <= 1, "lambda must lie in [0, 1]");
    HFR_REQUIRE(std::isfinite(overlap) && overlap >= 0, "overlap must be >= 0");
    const double vals[] = {cam->pos[0], cam->pos[1], cam->pos[2], cam->yaw, cam->pitch, cam->vfov, cam->znear,
                           dom->x0, dom->y0, dom->x1, dom->y1, dom->zmin, dom->zmax};
    for (double v : vals) HFR_REQUIRE(std::isfinite(v), "camera and domain must be finite");
    HFR_REQUIRE(cam->width >= 1 && cam->height >= 1, "image size must be positive");
    HFR_REQUIRE(cam->vfov > 0 && cam->vfov < M_PI, "vfov must lie in (0, pi)");
    HFR_REQUIRE(cam->znear > 0, "znear must be positive");
    HFR_REQUIRE(dom->x1 > dom->x0 && dom->y1 > dom->y0 && dom->zmax >= dom->zmin, "empty domain");

    const double cy = std::cos(cam->yaw), sy = std::sin(cam->yaw);
    const double cp = std::cos(cam->pitch), sp = std::sin(cam->pitch);
    const V3 fwd{sy * cp, cy * cp, sp}, right{cy, -sy, 0.0};
    const V3 up = cross(right, fwd);
    const double hl = std::hypot(fwd.x, fwd.y);
    HFR_REQUIRE(hl >= 1e-12, "the view direction has no horizontal component");
    const P2 vhat{fwd.x / hl, fwd.y / hl};
    const V3 o{cam->pos[0], cam->pos[1], cam->pos[2]};
    const P2 o2{o.x, o.y};
    const double ty = std::tan(0.5 * cam->vfov), tx = ty * cam->width / cam->height;

    // frustum half-spaces: near plane and four side planes through the eye
    const Plane fr[5] = {{fwd, dot(fwd, o) + cam->znear},
                         {tx * fwd - right, dot(tx * fwd - right, o)},
                         {tx * fwd + right, dot(tx * fwd + right, o)},
                         {ty * fwd - up, dot(ty * fwd - up, o)},
                         {ty * fwd + up, dot(ty * fwd + up, o)}};
    // vertices of (box intersected with frustum): clipped box faces and near-plane corners inside the box
    const double X[2] = {dom->x0, dom->x1}, Y[2] = {dom->y0, dom->y1}, Z[2] = {dom->zmin, dom->zmax};
    std::vector<std::vector<V3>> faces;
    for (int s = 0; s < 2; ++s) {
        faces.push_back({{X[s], Y[0], Z[0]}, {X[s], Y[1], Z[0]}, {X[s], Y[1], Z[1]}, {X[s], Y[0], Z[1]}});
        faces.push_back({{X[0], Y[s], Z[0]}, {X[1], Y[s], Z[0]}, {X[1], Y[s], Z[1]}, {X[0], Y[s], Z[1]}});
        faces.push_back({{X[0], Y[0], Z[s]}, {X[1], Y[0], Z[s]}, {X[1], Y[1], Z[s]}, {X[0], Y[1], Z[s]}});
    }
    std::vector<P2> pts;
    for (auto& f : faces) {
        std::vector<V3> p = f;
        for (const Plane& pl : fr) {
            if (p.empty()) break;
            p = clip3(p, pl);
        }
        for (const V3& v : p) pts.push_back({v.x, v.y});
    }
    const double tol = 1e-9 * std::max({1.0, std::fabs(dom->x0), std::fabs(dom->x1), std::fabs(dom->y0),
                                        std::fabs(dom->y1), std::fabs(dom->zmin), std::fabs(dom->zmax)});
    for (int sa = -1; sa <= 1; sa += 2)
        for (int sb = -1; sb <= 1; sb += 2) {
            const V3 p = o + cam->znear * (fwd + (sa * tx) * right + (sb * ty) * up);
            if (p.x >= dom->x0 - tol && p.x <= dom->x1 + tol && p.y >= dom->y0 - tol && p.y <= dom->y1 + tol &&
                p.z >= dom->zmin - tol && p.z <= dom->zmax + tol)
                pts.push_back({p.x, p.y});
        }
    const std::vector<P2> hull = hull2(pts);

    for (int k = 0; k < K; ++k) {
        hfr_cascade& c = out[k];
        std::memset(&c, 0, sizeof c);
        c.origin[0] = o2.x;
        c.origin[1] = o2.y;
        c.vhat[0] = vhat.x;
        c.vhat[1] = vhat.y;
        c.n = N;
        c.x0 = dom->x0;
        c.y0 = dom->y0;
        c.hx = c.hy = 2.0 * c_min / (N - 1);
    }
    if (hull.empty()) return hfr_ok();

    double n = INFINITY, f = -INFINITY;
    for (const P2& p : hull) {
        const double d = (p.x - o2.x) * vhat.x + (p.y - o2.y) * vhat.y;
        n = std::min(n, d);
        f = std::max(f, d);
    }
    const double np = std::max({n, cam->znear, c_min});
    std::vector<double> s(K);
    for (int k = 1; k < K; ++k) {
        const double uni = n + (f - n) * k / K;
        const double lg = f > np ? np * std::pow(f / np, (double)k / K) : uni;
        s[k - 1] = lambda * lg + (1.0 - lambda) * uni;
    }
    for (int k = 0; k < K; ++k) {
        hfr_cascade& c = out[k];
        const double near_d = k == 0 ? n : s[k - 1];
        const double split_d = k < K - 1 ? s[k] : f;
        const double far_d = k < K - 1 ? split_d + overlap * (split_d - near_d) : f;
        c.near_d = near_d;
        c.split_d = split_d;
        c.far_d = far_d;
        std::vector<P2> poly = clip2(clip2(hull, o2, vhat, near_d, 1.0), o2, vhat, far_d, -1.0);
        if (poly.size() > HFR_MAX_POLY)
            return hfr_fail(HFR_EUNSUPPORTED, "cascade %d polygon has %zu vertices (max %d)", k, poly.size(),
                            HFR_MAX_POLY);
        c.n_poly = (int32_t)poly.size();
        if (poly.empty()) continue;
        double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
        for (size_t a = 0; a < poly.size(); ++a) {
            c.poly[a][0] = poly[a].x;
            c.poly[a][1] = poly[a].y;
            xmin = std::min(xmin, poly[a].x);
            xmax = std::max(xmax, poly[a].x);
            ymin = std::min(ymin, poly[a].y);
            ymax = std::max(ymax, poly[a].y);
        }
        auto snap = aligned ? snap_axis_aligned : snap_axis;
        snap(xmin, xmax, dom->x0, c_min, N, &c.x0, &c.hx);
        snap(ymin, ymax, dom->y0, c_min, N, &c.y0, &c.hy);
    }
    return hfr_ok();
}

}  // namespace
