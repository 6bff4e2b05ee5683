// Adaptive quadtree of a raster built on the device (the adaptive grid of
// Section 2, built at start-up in the paper), producing the leaves directly
// in level-index order together with their rank table.  gfx950, wave64.
//
// The decisions are those of hfr_build_quadtree, made with the same FP64
// arithmetic: a mean pyramid of 2 x 2 averages ((a + b) + (c + d)) / 4, and a
// node splits (below max_depth) when the largest |second difference| of its
// four children's means (neighbours replicated at the raster edge) exceeds
// tau.  Instead of a depth-first walk every lattice node is classified at
// once, level after level: a node is present when its parent is present and
// splits, and a leaf when it is present and does not split.  The leaf flags,
// written one slot late into the rank-table layout with a 0 opening every
// level, become the rank table under one inclusive scan; each leaf is then
// written at its rank, so the leaves come out sorted by (level, row, column).
#include <algorithm>

#include "hfr_device.h"

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__host__ __device__ inline int64_t pyramid_offset(int l) { return ((int64_t(1) << (2 * l)) - 1) / 3; }
__host__ __device__ inline int64_t rank_offset(int l) { return pyramid_offset(l) + l; }

__global__ void raster_to_double_kernel(const float* __restrict__ dem, double* __restrict__ out, int64_t count)
{
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < count; a += (int64_t)gridDim.x * blockDim.x)
        out[a] = (double)dem[a];
}

// Level of side s from the level of side 2s below it.
__global__ void mean_level_kernel(const double* __restrict__ fine, double* __restrict__ coarse, int s)
{
    const int64_t count = (int64_t)s * s;
    const int64_t s2 = 2 * (int64_t)s;
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < count; a += (int64_t)gridDim.x * blockDim.x) {
        const int64_t jj = a / s, ii = a - jj * s;
        const double p = fine[(2 * jj) * s2 + 2 * ii], q = fine[(2 * jj) * s2 + 2 * ii + 1];
        const double r = fine[(2 * jj + 1) * s2 + 2 * ii], t = fine[(2 * jj + 1) * s2 + 2 * ii + 1];
        coarse[a] = __dmul_rn(__dadd_rn(__dadd_rn(p, q), __dadd_rn(r, t)), 0.25);
    }
}

// split[q] for the nodes of a level of side s, from the means of the level below (side 2s).
__global__ void split_kernel(const double* __restrict__ m, int s, double tau, uint8_t* __restrict__ split)
{
    const int64_t count = (int64_t)s * s;
    const int64_t S = 2 * (int64_t)s;
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < count; a += (int64_t)gridDim.x * blockDim.x) {
        const int64_t jj = a / s, ii = a - jj * s;
        double best = 0.0;
        for (int64_t cj = 2 * jj; cj <= 2 * jj + 1; ++cj)
            for (int64_t ci = 2 * ii; ci <= 2 * ii + 1; ++ci) {
                const double ctr = m[cj * S + ci];
                const double lf = m[cj * S + (ci > 0 ? ci - 1 : 0)];
                const double rt = m[cj * S + (ci + 1 < S ? ci + 1 : S - 1)];
                const double dn = m[(cj > 0 ? cj - 1 : 0) * S + ci];
                const double up = m[(cj + 1 < S ? cj + 1 : S - 1) * S + ci];
                // 2 ctr is exact, so a fused subtract rounds like the separate one
                const double d2x = __dsub_rn(__dadd_rn(lf, rt), __dmul_rn(2.0, ctr));
                const double d2y = __dsub_rn(__dadd_rn(dn, up), __dmul_rn(2.0, ctr));
                best = fmax(best, fmax(fabs(d2x), fabs(d2y)));
            }
        split[a] = best > tau ? 1 : 0;
    }
}

// Presence and leaf flags of level l (side s): flags go to rank[off_l + q + 1],
// with rank[off_l] = 0 opening the level.
__global__ void leaf_flags_kernel(int l, int max_depth, const uint8_t* __restrict__ split_l,
                                  const uint8_t* __restrict__ present_up, const uint8_t* __restrict__ split_up,
                                  uint8_t* __restrict__ present_l, int32_t* __restrict__ rank_l)
{
    const int s = 1 << l;
    const int64_t count = (int64_t)s * s;
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < count; a += (int64_t)gridDim.x * blockDim.x) {
        const int64_t jj = a >> l, ii = a & (s - 1);
        bool present = true;
        if (l > 0) {
            const int64_t pq = (jj >> 1) * (s >> 1) + (ii >> 1);
            present = present_up[pq] && split_up[pq];
        }
        const bool splits = l < max_depth && split_l[a];
        present_l[a] = present ? 1 : 0;
        rank_l[a + 1] = (present && !splits) ? 1 : 0;
        if (a == 0) rank_l[0] = 0;
    }
}

// In-place inclusive scan of each SCAN_TILE-element tile; the tile's total
// goes to sums[tile].
template <typename T>
__global__ __launch_bounds__(SCAN_THREADS) void scan_tiles_kernel(T* __restrict__ data, int64_t n, T* __restrict__ sums)
{
    __shared__ T buf[SCAN_TILE];
    __shared__ T wsum[SCAN_THREADS / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int e = k * SCAN_THREADS + t;
        buf[e] = base + e < n ? data[base + e] : 0;
    }
    __syncthreads();
    T run = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        run += buf[t * SCAN_ITEMS + k];
        buf[t * SCAN_ITEMS + k] = run;
    }
    T incl = run;
    for (int o = 1; o < 64; o <<= 1) {
        const T y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    T before = incl - run;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    for (int k = 0; k < SCAN_ITEMS; ++k) buf[t * SCAN_ITEMS + k] += before;
    __syncthreads();
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int e = k * SCAN_THREADS + t;
        if (base + e < n) data[base + e] = buf[e];
    }
    if (t == SCAN_THREADS - 1) sums[blockIdx.x] = buf[SCAN_TILE - 1];
}

// Adds the inclusive prefix of the earlier tiles' totals to every tile but the first.
template <typename T>
__global__ void add_tile_offsets_kernel(T* __restrict__ data, int64_t n, const T* __restrict__ sums)
{
    const int64_t tile = (int64_t)blockIdx.x + 1;
    const T add = sums[tile - 1];
    for (int64_t e = tile * SCAN_TILE + threadIdx.x; e < std::min<int64_t>(n, (tile + 1) * SCAN_TILE);
         e += blockDim.x)
        data[e] += add;
}

// Leaves of level l written at their ranks.
__global__ void emit_leaves_kernel(int l, double side, double x0, double y0, const double* __restrict__ mean_l,
                                   const int32_t* __restrict__ rank_l, float* __restrict__ x, float* __restrict__ y,
                                   float* __restrict__ c, float* __restrict__ v, int32_t* __restrict__ level,
                                   int32_t* __restrict__ li, int32_t* __restrict__ lj, int64_t n_leaves)
{
    const int s = 1 << l;
    const int64_t count = (int64_t)s * s;
    const double cs = ldexp(side, -l);
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < count; a += (int64_t)gridDim.x * blockDim.x) {
        const int32_t p = rank_l[a];
        if (rank_l[a + 1] - p != 1 || p < 0 || p >= n_leaves) continue;
        const int64_t jj = a >> l, ii = a & (s - 1);
        x[p] = (float)__dadd_rn(x0, __dmul_rn((double)ii + 0.5, cs));
        y[p] = (float)__dadd_rn(y0, __dmul_rn((double)jj + 0.5, cs));
        c[p] = (float)cs;
        v[p] = (float)mean_l[a];
        if (level) level[p] = l;
        if (li) li[p] = (int32_t)ii;
        if (lj) lj[p] = (int32_t)jj;
    }
}

// Per-leaf lists of the leaves whose truncation radius (widened by slack)
// reaches the leaf's closed square, in level-index (sorted position) space:
// thread p handles the leaf at sorted position p and walks, level by level,
// the window rows around its square through the rank table, testing each
// leaf there exactly as hfr_build_neighbours does (FP64, unfused).  With
// FILL = false it writes the list length to counts[p + 1]; with FILL = true
// it writes the sorted positions of the list from off[p] on.
template <bool FILL>
__global__ void neighbours_kernel(const float* __restrict__ x, const float* __restrict__ y,
                                  const float* __restrict__ c, const float* __restrict__ sigma,
                                  const int32_t* __restrict__ rank, const int32_t* __restrict__ order,
                                  const float* __restrict__ level_radius, int64_t n, int max_depth, double cutoff,
                                  double widen, double x0, double y0, double side, int64_t* __restrict__ off,
                                  int32_t* __restrict__ idx)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = order[p];
        const double xa = x[a], ya = y[a], ha = __dmul_rn(0.5, (double)c[a]);
        int64_t k = 0, base = 0, cap = 0;
        if (FILL) {
            base = off[p];
            cap = off[p + 1] - base;
        }
        for (int l = 0; l <= max_depth; ++l) {
            const double Rl = (double)level_radius[l];
            if (!(Rl > 0.0)) continue;
            const int64_t S = int64_t(1) << l;
            const double cl = ldexp(side, -l);
            const double reach = ha + Rl * widen;
            const int64_t i0 = max((int64_t)0, (int64_t)floor((xa - reach - x0) / cl - 0.5) - 1);
            const int64_t i1 = min(S - 1, (int64_t)ceil((xa + reach - x0) / cl - 0.5) + 1);
            const int64_t j0 = max((int64_t)0, (int64_t)floor((ya - reach - y0) / cl - 0.5) - 1);
            const int64_t j1 = min(S - 1, (int64_t)ceil((ya + reach - y0) / cl - 0.5) + 1);
            if (i0 > i1 || j0 > j1) continue;
            const int32_t* rk = rank + rank_offset(l);
            for (int64_t jj = j0; jj <= j1; ++jj) {
                const int32_t lo = rk[jj * S + i0], hi = rk[jj * S + i1 + 1];
                for (int32_t q = lo; q < hi; ++q) {
                    const int32_t b = order[q];
                    const double dx = fmax(__dsub_rn(fabs(__dsub_rn((double)x[b], xa)), ha), 0.0);
                    const double dy = fmax(__dsub_rn(fabs(__dsub_rn((double)y[b], ya)), ha), 0.0);
                    const double R = __dmul_rn(__dmul_rn(__dmul_rn(cutoff, (double)sigma[b]), (double)c[b]), widen);
                    if (__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)) < __dmul_rn(R, R)) {
                        if (FILL && k < cap) idx[base + k] = q;
                        ++k;
                    }
                }
            }
        }
        if (!FILL) off[p + 1] = k;
        if (!FILL && p == 0) off[0] = 0;
    }
}

struct Layout {
    int64_t pyramid;  // double, levels 0 .. D
    int64_t split;    // uint8, levels 0 .. max_depth - 1
    int64_t present;  // uint8, levels 0 .. max_depth
    int64_t sums;     // int32, the scan's tile totals, every recursion level
    int64_t bytes;
};

int64_t scan_sums_count(int64_t n)
{
    int64_t total = 0;
    while (n > 1) {
        n = (n + SCAN_TILE - 1) / SCAN_TILE;
        total += n;
    }
    return total + 1;
}

Layout layout_of(int D, int max_depth)
{
    auto up = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    Layout L{};
    L.pyramid = 0;
    L.split = up(L.pyramid + pyramid_offset(D + 1) * 8);
    L.present = up(L.split + pyramid_offset(max_depth));
    L.sums = up(L.present + pyramid_offset(max_depth + 1));
    L.bytes = up(L.sums + scan_sums_count(rank_offset(max_depth + 1)) * 4);
    return L;
}

int grid_for(int64_t count) { return (int)std::min<int64_t>((count + 255) / 256, 8192); }

// Inclusive scan of data[0, n) in place; sums has scan_sums_count(n) entries.
template <typename T>
void scan_inclusive(T* data, int64_t n, T* sums, hipStream_t s)
{
    const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    scan_tiles_kernel<T><<<dim3((unsigned)tiles), dim3(SCAN_THREADS), 0, s>>>(data, n, sums);
    if (tiles > 1) {
        scan_inclusive<T>(sums, tiles, sums + tiles, s);
        add_tile_offsets_kernel<T><<<dim3((unsigned)(tiles - 1)), dim3(256), 0, s>>>(data, n, sums);
    }
}

hfr_status check_args(int64_t n, double side, double x0, double y0, int32_t max_depth, int* D)
{
    HFR_REQUIRE(hfr_is_pow2(n) && n <= 32768, "raster side %lld must be a power of two <= 32768", (long long)n);
    *D = hfr_log2i(n);
    HFR_REQUIRE(max_depth >= 0 && max_depth <= *D && max_depth <= 15, "max_depth %d outside [0, min(%d, 15)]",
                max_depth, *D);
    HFR_REQUIRE(std::isfinite(side) && side > 0 && std::isfinite(x0) && std::isfinite(y0),
                "side must be positive and the origin finite");
    return HFR_OK;
}

}  // namespace

extern "C" hfr_status hfr_quadtree_device_workspace(int64_t n, int32_t max_depth, int64_t* bytes)
{
    HFR_REQUIRE(bytes != nullptr, "bytes is NULL");
    int D = 0;
    hfr_status st = check_args(n, 1.0, 0.0, 0.0, max_depth, &D);
    if (st != HFR_OK) return st;
    *bytes = layout_of(D, max_depth).bytes;
    return hfr_ok();
}

extern "C" hfr_status hfr_build_quadtree_device(const float* dem, int64_t n, double side, double x0, double y0,
                                                int32_t max_depth, double tau, void* work, int32_t* rank,
                                                int64_t* n_leaves, hfr_stream stream)
{
    HFR_REQUIRE(dem && work && rank && n_leaves, "NULL raster, workspace, rank table or count");
    HFR_REQUIRE(!std::isnan(tau), "tau is NaN");
    int D = 0;
    hfr_status st = check_args(n, side, x0, y0, max_depth, &D);
    if (st != HFR_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const Layout lay = layout_of(D, max_depth);
    char* w = static_cast<char*>(work);
    double* pyr = reinterpret_cast<double*>(w + lay.pyramid);
    uint8_t* split = reinterpret_cast<uint8_t*>(w + lay.split);
    uint8_t* present = reinterpret_cast<uint8_t*>(w + lay.present);
    int32_t* sums = reinterpret_cast<int32_t*>(w + lay.sums);
    raster_to_double_kernel<<<grid_for(n * n), 256, 0, s>>>(dem, pyr + pyramid_offset(D), n * n);
    for (int l = D - 1; l >= 0; --l) {
        const int64_t side_l = int64_t(1) << l;
        mean_level_kernel<<<grid_for(side_l * side_l), 256, 0, s>>>(pyr + pyramid_offset(l + 1),
                                                                      pyr + pyramid_offset(l), (int)side_l);
    }
    for (int l = 0; l < max_depth; ++l) {
        const int64_t side_l = int64_t(1) << l;
        split_kernel<<<grid_for(side_l * side_l), 256, 0, s>>>(pyr + pyramid_offset(l + 1), (int)side_l, tau,
                                                                 split + pyramid_offset(l));
    }
    for (int l = 0; l <= max_depth; ++l) {
        const int64_t side_l = int64_t(1) << l;
        leaf_flags_kernel<<<grid_for(side_l * side_l), 256, 0, s>>>(
            l, max_depth, l < max_depth ? split + pyramid_offset(l) : nullptr,
            l > 0 ? present + pyramid_offset(l - 1) : nullptr, l > 0 ? split + pyramid_offset(l - 1) : nullptr,
            present + pyramid_offset(l), rank + rank_offset(l));
    }
    const int64_t total = rank_offset(max_depth + 1);
    scan_inclusive<int32_t>(rank, total, sums, s);
    HFR_LAUNCH_CHECK("build_quadtree_device");
    int32_t count = 0;
    HFR_REQUIRE(hipMemcpyAsync(&count, rank + total - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s) == hipSuccess &&
                    hipStreamSynchronize(s) == hipSuccess,
                "reading the leaf count failed");
    *n_leaves = count;
    return hfr_ok();
}

extern "C" hfr_status hfr_quadtree_device_leaves(int64_t n, double side, double x0, double y0, int32_t max_depth,
                                                 const void* work, const int32_t* rank, int64_t n_leaves, float* x,
                                                 float* y, float* c, float* v, int32_t* level, int32_t* i, int32_t* j,
                                                 hfr_stream stream)
{
    HFR_REQUIRE(work && rank && x && y && c && v, "NULL workspace, rank table or leaf array");
    HFR_REQUIRE(n_leaves >= 1 && n_leaves <= INT32_MAX, "leaf count %lld outside [1, INT32_MAX]",
                (long long)n_leaves);
    int D = 0;
    hfr_status st = check_args(n, side, x0, y0, max_depth, &D);
    if (st != HFR_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const Layout lay = layout_of(D, max_depth);
    const double* pyr = reinterpret_cast<const double*>(static_cast<const char*>(work) + lay.pyramid);
    for (int l = 0; l <= max_depth; ++l) {
        const int64_t side_l = int64_t(1) << l;
        emit_leaves_kernel<<<grid_for(side_l * side_l), 256, 0, s>>>(l, side, x0, y0, pyr + pyramid_offset(l),
                                                                       rank + rank_offset(l), x, y, c, v, level, i, j,
                                                                       n_leaves);
    }
    HFR_LAUNCH_CHECK("quadtree_device_leaves");
    return hfr_ok();
}

extern "C" hfr_status hfr_neighbours_device_workspace(int64_t n, int64_t* bytes)
{
    HFR_REQUIRE(bytes != nullptr, "bytes is NULL");
    HFR_REQUIRE(n >= 1 && n <= INT32_MAX, "leaf count %lld outside [1, INT32_MAX]", (long long)n);
    *bytes = scan_sums_count(n + 1) * (int64_t)sizeof(int64_t);
    return hfr_ok();
}

namespace {

hfr_status check_neighbour_args(const hfr_leaves* L, float slack)
{
    HFR_REQUIRE(L != nullptr, "leaves are NULL");
    HFR_REQUIRE(L->n >= 1 && L->n <= INT32_MAX, "leaf count %lld outside [1, INT32_MAX]", (long long)L->n);
    HFR_REQUIRE(L->x && L->y && L->c && L->sigma && L->rank && L->order && L->level_radius,
                "leaf arrays, the level index and the level radii must not be NULL");
    HFR_REQUIRE(L->max_depth >= 0 && L->max_depth <= 15, "max_depth %d outside [0, 15]", L->max_depth);
    HFR_REQUIRE(std::isfinite(L->cutoff) && L->cutoff > 0, "cutoff must be positive");
    HFR_REQUIRE(std::isfinite(slack) && slack >= 0, "slack must be >= 0");
    HFR_REQUIRE(std::isfinite(L->side) && L->side > 0 && std::isfinite(L->x0) && std::isfinite(L->y0),
                "invalid lattice square");
    return HFR_OK;
}

}  // namespace

extern "C" hfr_status hfr_build_neighbours_device(const hfr_leaves* L, float slack, void* work, int64_t* off,
                                                  int64_t* nnz, hfr_stream stream)
{
    hfr_status st = check_neighbour_args(L, slack);
    if (st != HFR_OK) return st;
    HFR_REQUIRE(work && off && nnz, "NULL workspace, offsets or count");
    hipStream_t s = (hipStream_t)stream;
    const double widen = 1.0 + (double)slack;
    neighbours_kernel<false><<<grid_for(L->n), 256, 0, s>>>(L->x, L->y, L->c, L->sigma, L->rank, L->order,
                                                             L->level_radius, L->n, L->max_depth, (double)L->cutoff,
                                                             widen, L->x0, L->y0, L->side, off, nullptr);
    scan_inclusive<int64_t>(off, L->n + 1, static_cast<int64_t*>(work), s);
    HFR_LAUNCH_CHECK("build_neighbours_device");
    int64_t total = 0;
    HFR_REQUIRE(hipMemcpyAsync(&total, off + L->n, sizeof(int64_t), hipMemcpyDeviceToHost, s) == hipSuccess &&
                    hipStreamSynchronize(s) == hipSuccess,
                "reading the entry count failed");
    *nnz = total;
    return hfr_ok();
}

extern "C" hfr_status hfr_neighbours_device_fill(const hfr_leaves* L, float slack, const int64_t* off, int32_t* idx,
                                                 hfr_stream stream)
{
    hfr_status st = check_neighbour_args(L, slack);
    if (st != HFR_OK) return st;
    HFR_REQUIRE(off && idx, "NULL offsets or entries");
    hipStream_t s = (hipStream_t)stream;
    neighbours_kernel<true><<<grid_for(L->n), 256, 0, s>>>(L->x, L->y, L->c, L->sigma, L->rank, L->order,
                                                            L->level_radius, L->n, L->max_depth, (double)L->cutoff,
                                                            1.0 + (double)slack, L->x0, L->y0, L->side,
                                                            const_cast<int64_t*>(off), idx);
    HFR_LAUNCH_CHECK("neighbours_device_fill");
    return hfr_ok();
}
