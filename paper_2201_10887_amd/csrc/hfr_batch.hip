// Batched rendering: many views (camera + cascade set) of many heightfields
// rendered by one set of launches.  The paper renders one view per frame;
// batching is this library's addition.  The per-view work is exactly that of
// hfr_discretize / hfr_build_maxmip / hfr_raycast and their adjoints (the
// batch kernels call the same block and pixel bodies); what the plan adds is
// the work distribution:
//  - discretize and its adjoint: one persistent launch over all 16 x 16
//    texel blocks of all cascades of all views (64 chunk queues, eight per XCD);
//  - max-mipmap: one launch over the 64 x 64-cell tiles of all cascades, one for their top levels;
//  - ray casting and its adjoint: one persistent launch over all 64-pixel
//    tiles of all views, taken wave by wave; optionally (tuning.ray_queue)
//    the long rays of every view finish in a second launch, 16 lanes each.
// Every per-camera value (cascades, ray setup) lives in device memory, so
// the launch sequence can be captured once and replayed for new cameras.
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "hfr_device.h"

void maxmip_pass_shape(int N, int p, int* tiles);

namespace {

__global__ void zero_ints_kernel(int* __restrict__ p, int n)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < n) p[a] = 0;
}

// Row y < n_tex of the grid zeroes cascade y's texel gradients; row
// n_tex + f zeroes field f's leaf gradients.
__global__ __launch_bounds__(256) void zero_grads_kernel(BatchDev P, int n_fields)
{
    const int y = blockIdx.y;
    float* a = nullptr;
    float* b = nullptr;
    int64_t n = 0;
    if (y < P.n_tex) {
        const BatchTex& it = P.tex[y];
        a = it.gtex;
        n = (int64_t)it.C.n * it.C.n;
    } else if (y - P.n_tex < n_fields) {
        const BatchField& F = P.fields[y - P.n_tex];
        a = F.gv;
        b = F.gs;
        n = F.T.n;
    }
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        a[e] = 0.0f;
        if (b) b[e] = 0.0f;
    }
}

template <class T>
hfr_status dev_alloc(T** p, size_t count)
{
    *p = nullptr;
    if (count == 0) return HFR_OK;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) return hfr_fail(HFR_EDEVICE, "hipMalloc of %zu bytes: %s", count * sizeof(T), hipGetErrorString(e));
    return HFR_OK;
}

hfr_status check_tuning(const hfr_batch_tuning& t)
{
    HFR_REQUIRE(t.disc_blocks_per_cu >= 1 && t.disc_blocks_per_cu <= 16, "disc_blocks_per_cu %d outside [1, 16]",
                t.disc_blocks_per_cu);
    HFR_REQUIRE(t.ray_blocks_per_cu >= 1 && t.ray_blocks_per_cu <= 16, "ray_blocks_per_cu %d outside [1, 16]",
                t.ray_blocks_per_cu);
    HFR_REQUIRE(t.ray_tile_w == 8 || t.ray_tile_w == 16 || t.ray_tile_w == 32 || t.ray_tile_w == 64,
                "ray_tile_w %d is not 8, 16, 32 or 64", t.ray_tile_w);
    HFR_REQUIRE(t.disc_grain >= 1 && t.disc_grain <= 64, "disc_grain %d outside [1, 64]", t.disc_grain);
    HFR_REQUIRE(t.ray_queue == 0 || t.ray_queue == 1, "ray_queue %d is not 0 or 1", t.ray_queue);
    HFR_REQUIRE(t.ray_grain >= 1 && t.ray_grain <= 32, "ray_grain %d outside [1, 32]", t.ray_grain);
    return HFR_OK;
}

constexpr int64_t MAX_WORK = int64_t(1) << 30;

}  // namespace

struct hfr_batch_plan {
    int device = 0, cus = 0;
    std::vector<hfr_batch_field> fields;
    std::vector<hfr_batch_view> views;
    std::vector<int> cas_off;       // first cascade of each view in `cas`
    std::vector<hfr_cascade> cas;   // from the last hfr_batch_set_cameras
    std::vector<int> tex_start, mip_start, ray_start;
    int pass_blocks[HFR_MIP_PASSES] = {};
    hfr_batch_tuning tuning{4, 4, 32, 8, 0, 8};
    int tail_blocks = 64;            // workgroups of the long-ray launch
    bool cameras_set = false, backward_ok = false, upload_pending = false;
    // pinned staging of the per-camera descriptors
    BatchTex* tex_h = nullptr;
    BatchView* views_h = nullptr;
    hipEvent_t upload_done = nullptr;
    // device copies
    BatchField* fields_d = nullptr;
    BatchTex* tex_d = nullptr;
    BatchView* views_d = nullptr;
    int *tex_start_d = nullptr, *mip_start_d = nullptr, *ray_start_d = nullptr, *queues_d = nullptr;
    int *rayq_d = nullptr, *rayq_count_d = nullptr;
    BatchDev P{};
};

namespace {

void release(hfr_batch_plan* q)
{
    if (q->upload_pending && q->upload_done) (void)hipEventSynchronize(q->upload_done);
    (void)hipFree(q->fields_d);
    (void)hipFree(q->tex_d);
    (void)hipFree(q->views_d);
    (void)hipFree(q->tex_start_d);
    (void)hipFree(q->mip_start_d);
    (void)hipFree(q->ray_start_d);
    (void)hipFree(q->queues_d);
    (void)hipFree(q->rayq_d);
    (void)hipFree(q->rayq_count_d);
    if (q->tex_h) (void)hipHostFree(q->tex_h);
    if (q->views_h) (void)hipHostFree(q->views_h);
    if (q->upload_done) (void)hipEventDestroy(q->upload_done);
    delete q;
}

hfr_status wait_upload(hfr_batch_plan* q)
{
    if (!q->upload_pending) return HFR_OK;
    hipError_t e = hipEventSynchronize(q->upload_done);
    if (e != hipSuccess) return hfr_fail(HFR_EDEVICE, "waiting for the descriptor upload: %s", hipGetErrorString(e));
    q->upload_pending = false;
    return HFR_OK;
}

// Tile counts for the current tuning (host staging and prefix sums).
hfr_status layout_rays(hfr_batch_plan* q)
{
    const int tw = q->tuning.ray_tile_w, th = 64 / tw;
    q->ray_start.assign(q->views.size() + 1, 0);
    int64_t total = 0;
    for (size_t v = 0; v < q->views.size(); ++v) {
        const hfr_batch_view& V = q->views[v];
        const int tx = (V.width + tw - 1) / tw, ty = (V.height + th - 1) / th;
        q->views_h[v].tiles_x = tx;
        total += (int64_t)tx * ty;
        HFR_REQUIRE(total < MAX_WORK, "too many pixel tiles in the batch");
        q->ray_start[v + 1] = (int)total;
    }
    return HFR_OK;
}

}  // namespace

extern "C" hfr_status hfr_batch_plan_create(const hfr_batch_field* fields, int32_t n_fields,
                                            const hfr_batch_view* views, int32_t n_views, hfr_batch_plan** out)
{
    HFR_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    HFR_REQUIRE(fields != nullptr && views != nullptr, "fields or views are NULL");
    HFR_REQUIRE(n_fields >= 1 && n_fields <= 4096, "n_fields %d outside [1, 4096]", n_fields);
    HFR_REQUIRE(n_views >= 1 && n_views <= 4096, "n_views %d outside [1, 4096]", n_views);
    std::vector<Tables> tables(n_fields);
    std::vector<bool> field_bwd(n_fields);
    for (int f = 0; f < n_fields; ++f) {
        const hfr_batch_field& F = fields[f];
        hfr_status st = leaf_tables(&F.leaves, false, &tables[f]);
        if (st == HFR_OK) st = check_domain(&F.dom);
        if (st != HFR_OK) return hfr_fail(st, "field %d: %s", f, hfr_last_error());
        field_bwd[f] = F.grad_v && F.grad_sigma && F.leaves.sigma;
    }
    bool bwd = true;
    int64_t tex_blocks = 0, n_tex = 0;
    int64_t pass_total[HFR_MIP_PASSES] = {};
    for (int v = 0; v < n_views; ++v) {
        const hfr_batch_view& V = views[v];
        HFR_REQUIRE(V.field >= 0 && V.field < n_fields, "view %d names field %d of %d", v, V.field, n_fields);
        HFR_REQUIRE(V.K >= 1 && V.K <= HFR_MAX_CASCADES, "view %d: K = %d outside [1, %d]", v, V.K, HFR_MAX_CASCADES);
        HFR_REQUIRE(hfr_is_pow2(V.N) && V.N >= 2 && V.N <= HFR_MAX_TEX_N, "view %d: N = %d is not a power of two in [2, %d]",
                    v, V.N, HFR_MAX_TEX_N);
        HFR_REQUIRE(V.width >= 1 && V.width <= 16384 && V.height >= 1 && V.height <= 16384,
                    "view %d: image size %dx%d outside [1, 16384]", v, V.width, V.height);
        HFR_REQUIRE(V.tex && V.mip && V.depth && V.hit, "view %d: NULL texture, pyramid or image buffer", v);
        HFR_REQUIRE(reinterpret_cast<uintptr_t>(V.tex) % 16 == 0, "view %d: textures must be 16-byte aligned", v);
        HFR_REQUIRE(V.split_lambda >= 0 && V.split_lambda <= 1 && V.overlap >= 0 && V.c_min > 0 &&
                        std::isfinite(V.overlap) && std::isfinite(V.c_min),
                    "view %d: invalid split_lambda, overlap or c_min", v);
        bwd = bwd && V.grad_depth && V.grad_tex && field_bwd[V.field];
        const int64_t gx = (V.N + 15) / 16;
        tex_blocks += V.K * gx * gx;
        n_tex += V.K;
        for (int p = 0; p < HFR_MIP_PASSES; ++p) {
            int tiles;
            maxmip_pass_shape(V.N, p, &tiles);
            pass_total[p] += (int64_t)V.K * tiles * tiles;
        }
    }
    HFR_REQUIRE(tex_blocks < MAX_WORK, "too many texel blocks in the batch");
    HFR_REQUIRE(pass_total[0] < MAX_WORK, "too many max-mipmap tiles in the batch");

    hfr_batch_plan* q = new (std::nothrow) hfr_batch_plan();
    if (!q) return hfr_fail(HFR_ENOMEM, "plan allocation failed");
    q->fields.assign(fields, fields + n_fields);
    q->views.assign(views, views + n_views);
    q->backward_ok = bwd;
    hipError_t e = hipGetDevice(&q->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&q->cus, hipDeviceAttributeMultiprocessorCount, q->device);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&q->upload_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void**)&q->tex_h, n_tex * sizeof(BatchTex), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&q->views_h, n_views * sizeof(BatchView), hipHostMallocDefault);
    if (e != hipSuccess) {
        release(q);
        return hfr_fail(HFR_EDEVICE, "plan set-up: %s", hipGetErrorString(e));
    }
    std::memset(q->tex_h, 0, n_tex * sizeof(BatchTex));
    std::memset(q->views_h, 0, n_views * sizeof(BatchView));

    // static parts of the descriptors
    std::vector<BatchField> fd(n_fields);
    for (int f = 0; f < n_fields; ++f) {
        const hfr_batch_field& F = fields[f];
        fd[f] = BatchField{tables[f], Dom2{F.dom.x0, F.dom.y0, F.dom.x1, F.dom.y1}, F.grad_v, F.grad_sigma,
                           F.leaves.basis};
    }
    q->tex_start.assign(n_tex + 1, 0);
    q->mip_start.assign(HFR_MIP_PASSES * (n_tex + 1), 0);
    q->cas_off.assign(n_views + 1, 0);
    int64_t rayq_total = 0;  // long-ray queue: a quarter of each view's pixels (a ray past that finishes in place)
    int t = 0;
    for (int v = 0; v < n_views; ++v) {
        const hfr_batch_view& V = views[v];
        q->cas_off[v + 1] = q->cas_off[v] + V.K;
        const int64_t NN = (int64_t)V.N * V.N, MM = (4 * NN - 1) / 3;
        const int gx = (V.N + 15) / 16;
        for (int k = 0; k < V.K; ++k, ++t) {
            BatchTex& it = q->tex_h[t];
            it.C.n = V.N;
            it.field = V.field;
            it.gx = gx;
            it.tex = V.tex + k * NN;
            it.mask = V.mask ? reinterpret_cast<uint16_t*>(V.mask + k * (int64_t)V.N * ((V.N + 31) / 32)) : nullptr;
            it.mip = V.mip + k * MM;
            it.gtex = V.grad_tex ? V.grad_tex + k * NN : nullptr;
            q->tex_start[t + 1] = q->tex_start[t] + gx * gx;
            for (int p = 0; p < HFR_MIP_PASSES; ++p) {
                int tiles;
                maxmip_pass_shape(V.N, p, &tiles);
                int* ms = &q->mip_start[p * (n_tex + 1)];
                ms[t + 1] = ms[t] + tiles * tiles;
            }
        }
        BatchView& bv = q->views_h[v];
        bv.q_off = (int)rayq_total;
        bv.q_cap = (int)std::max<int64_t>(64, (int64_t)V.width * V.height / 4);
        rayq_total += bv.q_cap;
        bv.tex = V.tex;
        bv.mip = V.mip;
        bv.depth = V.depth;
        bv.hit = V.hit;
        bv.gdepth = V.grad_depth;
        bv.gtex = V.grad_tex;
    }
    for (int p = 0; p < HFR_MIP_PASSES; ++p) q->pass_blocks[p] = (int)pass_total[p];
    q->cas.assign(q->cas_off[n_views], hfr_cascade{});
    hfr_status st = layout_rays(q);
    if (st != HFR_OK) {
        release(q);
        return st;
    }
    st = dev_alloc(&q->fields_d, n_fields);
    if (st == HFR_OK) st = dev_alloc(&q->tex_d, n_tex);
    if (st == HFR_OK) st = dev_alloc(&q->views_d, n_views);
    if (st == HFR_OK) st = dev_alloc(&q->tex_start_d, q->tex_start.size());
    if (st == HFR_OK) st = dev_alloc(&q->mip_start_d, q->mip_start.size());
    if (st == HFR_OK) st = dev_alloc(&q->ray_start_d, q->ray_start.size());
    if (st == HFR_OK) st = dev_alloc(&q->queues_d, HFR_QUEUE_WORDS);
    if (st == HFR_OK && rayq_total >= MAX_WORK) st = hfr_fail(HFR_EINVAL, "too many pixels in the batch");
    if (st == HFR_OK) st = dev_alloc(&q->rayq_d, rayq_total);
    if (st == HFR_OK) st = dev_alloc(&q->rayq_count_d, n_views);
    if (st != HFR_OK) {
        release(q);
        return st;
    }
    e = hipMemcpy(q->fields_d, fd.data(), n_fields * sizeof(BatchField), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(q->tex_start_d, q->tex_start.data(), q->tex_start.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(q->mip_start_d, q->mip_start.data(), q->mip_start.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(q->ray_start_d, q->ray_start.data(), q->ray_start.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        release(q);
        return hfr_fail(HFR_EDEVICE, "plan upload: %s", hipGetErrorString(e));
    }
    q->P = BatchDev{q->fields_d, q->tex_d, q->tex_start_d, q->mip_start_d, q->views_d, q->ray_start_d, q->queues_d,
                    q->rayq_d, q->rayq_count_d, (int)n_tex, n_views, q->tuning.ray_tile_w, q->tuning.disc_grain,
                    q->tuning.ray_queue, q->tuning.ray_grain, 0};
    for (int f = 0; f < n_fields; ++f) q->P.any_wendland |= fields[f].leaves.basis == HFR_BASIS_WENDLAND;
    // the long-ray launch: enough lane groups that a typical queue is taken in one round
    int64_t pixels = 0;
    for (int v = 0; v < n_views; ++v) pixels += (int64_t)views[v].width * views[v].height;
    q->tail_blocks = (int)std::min<int64_t>(2048, std::max<int64_t>(64, pixels / 1024));
    *out = q;
    return hfr_ok();
}

extern "C" void hfr_batch_plan_destroy(hfr_batch_plan* plan)
{
    if (plan) release(plan);
}

extern "C" hfr_status hfr_batch_set_tuning(hfr_batch_plan* plan, const hfr_batch_tuning* tuning)
{
    HFR_REQUIRE(plan != nullptr && tuning != nullptr, "plan or tuning is NULL");
    hfr_status st = check_tuning(*tuning);
    if (st != HFR_OK) return st;
    st = wait_upload(plan);
    if (st != HFR_OK) return st;
    const hfr_batch_tuning old = plan->tuning;
    plan->tuning = *tuning;
    st = layout_rays(plan);
    if (st != HFR_OK) {
        plan->tuning = old;
        (void)layout_rays(plan);
        return st;
    }
    // launches already queued may still read the old layout
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess)
        e = hipMemcpy(plan->ray_start_d, plan->ray_start.data(), plan->ray_start.size() * sizeof(int),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && plan->cameras_set)
        e = hipMemcpy(plan->views_d, plan->views_h, plan->views.size() * sizeof(BatchView), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hfr_fail(HFR_EDEVICE, "tuning upload: %s", hipGetErrorString(e));
    plan->P.tile_w = tuning->ray_tile_w;
    plan->P.disc_grain = tuning->disc_grain;
    plan->P.ray_queue = tuning->ray_queue;
    plan->P.ray_grain = tuning->ray_grain;
    return hfr_ok();
}

extern "C" hfr_status hfr_batch_set_cameras(hfr_batch_plan* plan, const hfr_camera* cams, hfr_stream stream)
{
    HFR_REQUIRE(plan != nullptr && cams != nullptr, "plan or cameras are NULL");
    const int nv = (int)plan->views.size();
    std::vector<hfr_cascade> cas(plan->cas.size());
    std::vector<RayArgs> args(nv);
    for (int v = 0; v < nv; ++v) {
        const hfr_batch_view& V = plan->views[v];
        HFR_REQUIRE(cams[v].width == V.width && cams[v].height == V.height,
                    "camera %d is %dx%d, its view is %dx%d", v, cams[v].width, cams[v].height, V.width, V.height);
        const hfr_domain& dom = plan->fields[V.field].dom;
        hfr_cascade* cv = &cas[plan->cas_off[v]];
        hfr_status st = hfr_fit_cascades(&cams[v], &dom, V.K, V.N, V.split_lambda, V.overlap, V.c_min, cv);
        if (st == HFR_OK) st = ray_args(&cams[v], &dom, cv, V.K, &args[v]);
        if (st != HFR_OK) return hfr_fail(st, "camera %d: %s", v, hfr_last_error());
    }
    hfr_status st = wait_upload(plan);
    if (st != HFR_OK) return st;
    int t = 0;
    for (int v = 0; v < nv; ++v) {
        const hfr_batch_view& V = plan->views[v];
        for (int k = 0; k < V.K; ++k, ++t) plan->tex_h[t].C = tex_cascade(cas[plan->cas_off[v] + k]);
        plan->views_h[v].A = args[v];
    }
    plan->cas = cas;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(plan->tex_d, plan->tex_h, (size_t)t * sizeof(BatchTex), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(plan->views_d, plan->views_h, nv * sizeof(BatchView), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(plan->upload_done, s);
    if (e != hipSuccess) return hfr_fail(HFR_EDEVICE, "descriptor upload: %s", hipGetErrorString(e));
    plan->upload_pending = true;
    plan->cameras_set = true;
    return hfr_ok();
}

extern "C" hfr_status hfr_batch_cascades(const hfr_batch_plan* plan, int32_t view, hfr_cascade* out)
{
    HFR_REQUIRE(plan != nullptr && out != nullptr, "plan or out is NULL");
    HFR_REQUIRE(view >= 0 && view < (int)plan->views.size(), "view %d outside [0, %d)", view, (int)plan->views.size());
    HFR_REQUIRE(plan->cameras_set, "no cameras set");
    for (int k = 0; k < plan->views[view].K; ++k) out[k] = plan->cas[plan->cas_off[view] + k];
    return hfr_ok();
}

extern "C" hfr_status hfr_batch_long_rays(const hfr_batch_plan* plan, int32_t* out)
{
    HFR_REQUIRE(plan != nullptr && out != nullptr, "plan or out is NULL");
    const int nv = plan->P.n_views;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(out, plan->rayq_count_d, nv * sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hfr_fail(HFR_EDEVICE, "reading the long-ray counts: %s", hipGetErrorString(e));
    return hfr_ok();
}

extern "C" hfr_status hfr_batch_launch(const hfr_batch_plan* plan, hfr_stream stream)
{
    HFR_REQUIRE(plan != nullptr, "plan is NULL");
    HFR_REQUIRE(plan->cameras_set, "no cameras set");
    hipStream_t s = (hipStream_t)stream;
    zero_ints_kernel<<<(HFR_QUEUE_WORDS + 255) / 256, 256, 0, s>>>(plan->queues_d, HFR_QUEUE_WORDS);
    HFR_LAUNCH_CHECK("batch queue reset");
    if (plan->P.ray_queue) {
        const int nv = plan->P.n_views;
        zero_ints_kernel<<<(nv + 255) / 256, 256, 0, s>>>(plan->rayq_count_d, nv);
        HFR_LAUNCH_CHECK("batch long-ray queue reset");
    }
    hfr_status st = launch_discretize_batch(plan->P, plan->cus * plan->tuning.disc_blocks_per_cu, false, s);
    if (st == HFR_OK) st = launch_maxmip_batch(plan->P, plan->pass_blocks, s);
    if (st == HFR_OK)
        st = launch_raycast_batch(plan->P, plan->cus * plan->tuning.ray_blocks_per_cu, plan->tail_blocks, false, s);
    return st == HFR_OK ? hfr_ok() : st;
}

extern "C" hfr_status hfr_batch_launch_backward(const hfr_batch_plan* plan, hfr_stream stream)
{
    HFR_REQUIRE(plan != nullptr, "plan is NULL");
    HFR_REQUIRE(plan->cameras_set, "no cameras set");
    HFR_REQUIRE(plan->backward_ok, "the plan has no backward pass (a view lacks grad_depth / grad_tex, or a field "
                                   "lacks grad_v / grad_sigma / sigma)");
    hipStream_t s = (hipStream_t)stream;
    zero_ints_kernel<<<(HFR_QUEUE_WORDS + 255) / 256, 256, 0, s>>>(plan->queues_d, HFR_QUEUE_WORDS);
    HFR_LAUNCH_CHECK("batch queue reset");
    const int nf = (int)plan->fields.size();
    zero_grads_kernel<<<dim3(64, plan->P.n_tex + nf), dim3(256), 0, s>>>(plan->P, nf);
    HFR_LAUNCH_CHECK("batch gradient reset");
    if (plan->P.ray_queue) {
        const int nv = plan->P.n_views;
        zero_ints_kernel<<<(nv + 255) / 256, 256, 0, s>>>(plan->rayq_count_d, nv);
        HFR_LAUNCH_CHECK("batch long-ray queue reset");
    }
    hfr_status st =
        launch_raycast_batch(plan->P, plan->cus * plan->tuning.ray_blocks_per_cu, plan->tail_blocks, true, s);
    if (st == HFR_OK) st = launch_discretize_batch(plan->P, plan->cus * plan->tuning.disc_blocks_per_cu, true, s);
    return st == HFR_OK ? hfr_ok() : st;
}
