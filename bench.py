"""Benchmark of the per-frame path on one MI355X.

Workload (default): the medium scene -- 40.96 km fBm terrain, ~4M quadtree
leaves, sigma 1 and a 3.5 sigma cutoff, 4 cascades of 2048^2 FP32 texels
(split lambda 0.5), 1920x1080 rays.  One forward step = cascade fit (host),
discretize (+ visibility), max-mipmap, ray cast; one training step adds the
ray-cast adjoint and the discretize adjoint.  Inputs are resident in HBM
before timing.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
DISC_CASCADES_PER_LAUNCH = 4  # cascades of one view per discretize launch
VALU_CLOCK_HZ = 2.4e9  # MI355X peak engine clock


def recorded_figure(kernel_source: str, summary: str, key: str):
    """A per-launch figure from a committed counter summary (`key`: e.g. traffic_bytes_per_launch,
    FETCH_SIZE and WRITE_SIZE each scaled by what the counter reads for a copy of known size, or
    valu_instructions_per_launch).  The figure is only valid for the kernel source it was taken on,
    so it is returned only when the summary's recorded SHA-256 matches."""
    try:
        with open(os.path.join(ROOT, summary)) as f:
            text = f.read()
        with open(os.path.join(ROOT, kernel_source), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ":" in line and line.lstrip("- `").split(":")[0] in ("source_sha256", key):
            k, v = line.lstrip("- `").split(":", 1)
            fields[k] = v.strip().strip("`")
    if fields.get("source_sha256") != sha or key not in fields:
        return None
    return int(float(fields[key]))


def recorded_traffic(kernel_source: str, summary: str):
    """HBM bytes per launch recorded with the counters (see recorded_figure)."""
    return recorded_figure(kernel_source, summary, "traffic_bytes_per_launch")


def build_scene(name: str):
    from paper_2201_10887_amd import api, synth
    w = synth.WORKLOADS[name]
    t0 = time.time()
    # rasters above 4096^2 take minutes in NumPy; the same generator runs in torch on the GPU
    dev = "cuda" if w.dem_n > 4096 else None
    dem = synth.fbm_dem(w.dem_n, w.octaves, w.hurst, w.seed, mountains=w.mountains, device=dev)
    t1 = time.perf_counter()
    leaves = api.build_quadtree(dem, w.side, w.max_depth, w.tau)
    build_scene.quadtree_host_ms = (time.perf_counter() - t1) * 1e3
    leaves["sigma"] = np.full(len(leaves["x"]), w.sigma, np.float32)
    cam = synth.camera_of(w, dem)
    print(f"[bench] scene {name}: {len(leaves['x'])} leaves, built in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    return w, dem, leaves, cam


def startup_ms(R, dem, w) -> dict:
    """Start-up costs: the quadtree on the host and on the device (the raster already resident,
    the leaf count read back once), the host level index, and the per-leaf influence lists on the
    device and (while their offsets fit 32 bits) on the host."""
    import torch
    from paper_2201_10887_amd import api
    d = torch.as_tensor(np.ascontiguousarray(dem, np.float32), device="cuda")
    api.build_quadtree_device(d, w.side, w.max_depth, w.tau)  # first call: allocator warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    q = api.build_quadtree_device(d, w.side, w.max_depth, w.tau)
    torch.cuda.synchronize()
    t_dev = (time.perf_counter() - t0) * 1e3
    if q["x"].numel() != R.L.n:
        raise RuntimeError("device and host quadtrees differ in leaf count")
    # the paper's per-leaf influence lists, on the device over the device-built leaves
    Lq = api.DeviceLeaves.from_device(q, w.sigma, w.side, w.max_depth, w.cutoff)
    api.pack_leaves(Lq)
    del q, d
    off, idx = api.build_neighbours_device(Lq)
    del off, idx
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    off, idx = api.build_neighbours_device(Lq)
    torch.cuda.synchronize()
    t_nb = (time.perf_counter() - t0) * 1e3
    nnz = int(idx.numel())
    del off, idx, Lq
    leaves = {"x": R.L.x.cpu().numpy(), "y": R.L.y.cpu().numpy(), "c": R.L.c.cpu().numpy()}
    t0 = time.perf_counter()
    api.build_level_index(leaves, w.side, w.max_depth)
    t_index = (time.perf_counter() - t0) * 1e3
    torch.cuda.empty_cache()
    out = {"quadtree_host": round(build_scene.quadtree_host_ms, 1), "quadtree_device": round(t_dev, 2),
           "level_index_host": round(t_index, 1), "neighbours_device": round(t_nb, 2), "neighbour_entries": nnz}
    if nnz < 2 ** 31:  # the host lists use 32-bit offsets
        leaves["sigma"] = np.full(len(leaves["x"]), w.sigma, np.float32)
        t0 = time.perf_counter()
        api.build_neighbours(leaves, w.side, w.max_depth, w.cutoff)
        out["neighbours_host"] = round((time.perf_counter() - t0) * 1e3, 1)
        out["neighbours_host_threads"] = min(os.cpu_count() or 1, 64)
    return out


def texel_reuse_flight(R, cam, depth, hit, frames=32, step=2.0, yaw_step=0.05) -> dict:
    """Forward frames along a flight (``step`` m per frame along the view, turning ``yaw_step`` deg per
    frame): the stable fit with every texel computed, the fixed-lattice fit with every texel computed,
    and the fixed-lattice fit copying the blocks the previous frame holds.  ms per frame over the
    whole flight (host fits included), and the share of visible blocks copied."""
    import torch
    from paper_2201_10887_amd import api, synth
    path = synth.camera_path(cam, frames, step, yaw_step)
    aligned = [api.fit_cascades(c, R.dom, R.K, R.N, R.lam, R.overlap, R.c_min, aligned=True) for c in path]

    def flight(fn):
        fn(0)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for f in range(frames):
            fn(f)
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / frames

    R.set_texel_reuse(False)
    ms_stable = flight(lambda f: R.forward(path[f], None, depth, hit))
    ms_aligned = flight(lambda f: R.forward(path[f], aligned[f], depth, hit))
    R.set_texel_reuse(True)
    ms_reuse = flight(lambda f: R.forward(path[f], None, depth, hit))
    # copied share: one more flight, counting visible 16 x 16 blocks per frame from the masks
    R.set_texel_reuse(True)
    R.count_reused = True
    R.reused_blocks.zero_()
    visible = 0
    for f in range(frames):
        R.forward(path[f], None, depth, hit)
        if f > 0:
            for _, _, mask, _ in R.surfaces():
                m = mask.view(torch.int16).reshape(R.K, R.N // 16, 16, -1)
                visible += int((m != 0).any(dim=2).sum())
    copied = int(R.reused_blocks.item())
    R.count_reused = False
    R.set_texel_reuse(False)
    return {"frames": frames, "step_m": step, "yaw_step_deg": yaw_step, "ms_per_frame_stable_fit": round(ms_stable, 4),
            "ms_per_frame_fixed_lattice": round(ms_aligned, 4), "ms_per_frame_reuse": round(ms_reuse, 4),
            "copied_block_fraction": round(copied / max(visible, 1), 4)}


def timed(fn, steps, stream):
    import torch
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def copy_bandwidth_gbs(stream, nbytes=1 << 30, reps=5):
    """HBM bandwidth a plain device-to-device copy reaches (bytes read + written per second), over
    buffers four times the 256 MB last-level cache, median of ``reps`` copies after two untimed."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        dst.copy_(src)
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    del src, dst
    return 2 * nbytes / (float(np.median(ts)) * 1e-3) / 1e9


def frame_times(fn, frames, warmup, stream):
    """Each of ``frames`` calls timed on its own (HIP events on the stream, after ``warmup``
    untimed calls): the median and the 10th / 90th percentiles in ms."""
    import torch
    for _ in range(warmup):
        fn()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(frames + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for f in range(frames):
        fn()
        ev[f + 1].record(stream)
    torch.cuda.synchronize()
    ts = np.sort([ev[f].elapsed_time(ev[f + 1]) for f in range(frames)])
    return {"frames": frames, "median": round(float(np.median(ts)), 4), "p10": round(float(ts[frames // 10]), 4),
            "p90": round(float(ts[(9 * frames) // 10]), 4)}


def discretize_work(R, cas, leaves, w, samples=20000) -> dict:
    """Algorithmic work of one discretize pass (all K cascades), for the roofline.

    FLOPs: 12 per (visible texel, leaf with w > 0) pair -- two differences,
    two products and a fused multiply-add for r^2, the exponent scale, one
    exp2, the truncation subtraction and clamp, and a fused multiply-add plus
    an add for the two sums.  The pair count is the visible-texel count times
    the mean number of influencing leaves of a seeded sample of visible
    texels (counted in FP64 over lattice windows of the level index, level by level).
    Bytes: every texel's FP32 value and visibility bit written once, and the
    16-byte record of every leaf within reach of a cascade's polygon read once.
    """
    import torch
    from paper_2201_10887_amd import api
    K, N = R.K, R.N
    words = (N + 31) // 32
    m = R.mask.cpu().numpy().view(np.uint32)
    vis = ((m[:, :, :, None] >> np.arange(32, dtype=np.uint32)) & 1).reshape(K, N, words * 32)[:, :, :N].astype(bool)
    n_vis = int(vis.sum())
    x = leaves["x"].astype(np.float64)
    y = leaves["y"].astype(np.float64)
    c = leaves["c"].astype(np.float64)
    sg = leaves["sigma"].astype(np.float64)
    rank, order = R.L.rank.cpu().numpy(), R.L.order.cpu().numpy()
    rng = np.random.default_rng(11)
    kk, jj, ii = np.nonzero(vis)
    pick = rng.choice(len(kk), min(samples, len(kk)), replace=False)
    px = np.empty(len(pick))
    py = np.empty(len(pick))
    for a, p in enumerate(pick):
        cv = api.CascadeView(cas[kk[p]])
        px[a] = min(max(cv.x0 + ii[p] * cv.hx, 0.0), w.side)
        py[a] = min(max(cv.y0 + jj[p] * cv.hy, 0.0), w.side)
    # influencers of each sample point: per quadtree level, every leaf node of that level
    # within the level's largest reach, tested with the leaf's own weight (w > 0)
    counts = np.zeros(len(pick), dtype=np.int64)
    E = np.exp(-0.5 * w.cutoff ** 2)
    for l in range(w.max_depth + 1):
        S = 1 << l
        cl = w.side / S
        at = leaves["level"] == l
        if not at.any():
            continue
        r = int(np.ceil(w.cutoff * float(sg[at].max()))) + 1
        gi = np.minimum((px / cl).astype(np.int64), S - 1)
        gj = np.minimum((py / cl).astype(np.int64), S - 1)
        off = np.arange(-r, r + 1)
        I = gi[:, None, None] + off[None, None, :]
        J = gj[:, None, None] + off[None, :, None]
        ok = (I >= 0) & (I < S) & (J >= 0) & (J < S)
        cell = api.rank_offset(l) + np.clip(J, 0, S - 1) * S + np.clip(I, 0, S - 1)
        leaf_at = ok & (rank[cell + 1] > rank[cell])
        ids = np.where(leaf_at, order[np.minimum(rank[cell], len(order) - 1)], -1)
        a_idx, lst = np.nonzero(ids.reshape(len(pick), -1) >= 0)
        lid = ids.reshape(len(pick), -1)[a_idx, lst]
        q = np.hypot(x[lid] - px[a_idx], y[lid] - py[a_idx]) / (sg[lid] * c[lid])
        counts += np.bincount(a_idx, weights=(np.exp(-0.5 * q * q) - E > 0), minlength=len(pick)).astype(np.int64)
    counts = counts.tolist()
    pairs = n_vis * float(np.mean(counts))
    nbytes = K * N * N * 4 + K * N * words * 4
    for k in range(K):
        cv = api.CascadeView(cas[k])
        if len(cv.poly) == 0:
            continue
        reach = w.cutoff * sg * c
        inside = ((x > cv.poly[:, 0].min() - reach) & (x < cv.poly[:, 0].max() + reach)
                  & (y > cv.poly[:, 1].min() - reach) & (y < cv.poly[:, 1].max() + reach))
        nbytes += 16 * int(inside.sum())
    return {"flops": 12.0 * pairs, "bytes": float(nbytes), "pairs": pairs, "visible_texels": n_vis,
            "mean_influencers": float(np.mean(counts))}


def cpu_baseline(w, leaves, cam, R, cas, vis_texels, reps=3):
    """The FP64 oracle's whole frame on the host cores: its own cascade fit, Eq. 2 at every visible
    texel of every cascade (the plain-C form, one thread per core), and the ray cast of every pixel
    over those textures (the plain-C walk).  Median of ``reps`` frames."""
    from oracle import cascades as ocas, discretize as odisc, raycast as oray
    threads = _host_threads()
    times, stage = [], []
    c_min = float(leaves["c"].min())
    dom = R.dom
    for _ in range(reps):
        t0 = time.perf_counter()
        cs = ocas.fit_cascades(cam, dom, R.K, R.N, w.split_lambda, w.overlap, c_min)
        t1 = time.perf_counter()
        tex = [odisc.discretize_c(c, leaves, dom, w.cutoff, threads=threads) for c in cs]
        t2 = time.perf_counter()
        oray.raycast(cam, dom, cs, np.stack(tex), threads=threads)
        t3 = time.perf_counter()
        times.append(t3 - t0)
        stage.append((t1 - t0, t2 - t1, t3 - t2))
    order = np.argsort(times)
    mid = int(order[len(order) // 2])
    surfaces = 1 + len(R.extra)
    ms = surfaces * times[mid] * 1e3
    return {"value": round(ms, 1), "unit": "ms/frame", "cores": threads, "kind": "oracle",
            "cpu": _cpu_model(), "cpu_count": os.cpu_count(),
            "stage_s": {"fit": round(stage[mid][0], 4), "discretize": round(stage[mid][1], 3),
                        "raycast": round(stage[mid][2], 3)},
            "sample": f"the whole {cam.width}x{cam.height} frame ({vis_texels} visible texels over {R.K} x {R.N}^2, "
                      f"every pixel), FP64 oracle: NumPy fit and visibility, plain-C Eq. 2 and ray walk on "
                      f"{threads} threads; median of {reps} frames" + (f", times {surfaces} surfaces"
                                                                        if surfaces > 1 else "")}


def _host_threads() -> int:
    """Host threads for the oracle: the CPUs this process may run on, at most 16 (one GPU's share of a box)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def fit_tau(dem, side, depth, target, rel=0.15, iters=24):
    """Refinement threshold (bisected on a log scale) whose quadtree has about ``target`` leaves."""
    from paper_2201_10887_amd import api
    lo, hi, best = 1e-3, 1e3, None
    for _ in range(iters):
        tau = math.sqrt(lo * hi)
        n = api.quadtree_leaf_count(dem, side, depth, tau)
        if best is None or abs(n - target) < abs(best[1] - target):
            best = (tau, n)
        if abs(n - target) <= rel * target:
            break
        if n > target:
            lo = tau
        else:
            hi = tau
    return best[0]


def build_batch_fields(n_fields=8, n_views=64, seed=1004):
    """8 fBm heightfields of uneven size and 64 cameras on them (seeded)."""
    from paper_2201_10887_amd import api, synth
    from paper_2201_10887_amd.batch import Field
    t0 = time.time()
    fspecs = synth.batch_fields(n_fields, seed)
    vspecs = synth.batch_views(n_views, n_fields, seed)
    dems, fields = [], []
    for f, tau in zip(fspecs, synth.BATCH_TAU):
        dem = synth.fbm_dem(f.dem_n, f.octaves, 0.8, f.seed)
        leaves = api.build_quadtree(dem, f.side, f.depth, tau)
        leaves["sigma"] = np.ones(len(leaves["x"]), np.float32)
        dems.append(dem)
        fields.append(Field(leaves, f.side, f.depth, 3.5))
    cams = synth.batch_cameras(dems, fspecs, vspecs, seed)
    print(f"[bench] batch fields: {', '.join(str(f.n) for f in fields)} leaves, {n_views} views, built in "
          f"{time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    return fields, vspecs, cams


def batch_renderer(fields, vspecs, budget_texels):
    """The batch's buffers and plan with N per view from the texel budget."""
    from paper_2201_10887_amd import autotune
    from paper_2201_10887_amd.batch import BatchRenderer, ViewSpec
    ns = autotune.texel_budget([(v.width, v.height, v.K) for v in vspecs], budget_texels)
    specs = [ViewSpec(v.field, v.K, n, v.width, v.height, 0.5, 0.05) for v, n in zip(vspecs, ns)]
    return BatchRenderer(fields, specs, backward=True)


def batch_main(args):
    """Many views of many heightfields: one batched launch set (captured as a graph) against
    the same views rendered one by one through the per-view entry points.  The texel budget is
    chosen by measurement (the largest whose tuned forward + backward step fits the target)."""
    import torch
    from paper_2201_10887_amd import api, autotune
    fields, vspecs, cams = build_batch_fields()
    gen = torch.Generator(device="cuda").manual_seed(1004)
    log = (lambda m: print(m, file=sys.stderr, flush=True)) if args.verbose else None

    def build(budget):
        R = batch_renderer(fields, vspecs, budget)
        R.set_cameras(cams)
        R.forward()
        for b in R.bufs:
            d = b["depth"]
            b["grad_depth"].copy_(torch.where(torch.isfinite(d), torch.randn(d.shape, generator=gen, device="cuda"),
                                              torch.zeros_like(d)))
        return R

    chosen = autotune.tune_budget(build, cams, args.batch_target_ms, backward=True, log=log)
    R = chosen["renderer"]
    tuned = {"tuning": R.tuning}
    print(f"[bench] texel budget {chosen['budget']} ({chosen['curve']}), tuning {R.tuning}", file=sys.stderr,
          flush=True)
    stream = torch.cuda.current_stream()

    def train():
        R.forward()
        R.backward()

    for _ in range(args.warmup):
        train()
    ms = {"batch_fwd": timed(R.forward, args.steps, stream), "batch_fwd_bwd": timed(train, args.steps, stream)}
    g_fwd, g_train = R.capture(backward=False), R.capture(backward=True)
    ms["graph_fwd"] = timed(g_fwd.replay, args.steps, stream)
    ms["graph_fwd_bwd"] = timed(g_train.replay, args.steps, stream)

    cas = [R.cascades(v) for v in range(R.n_views)]
    works = [api.ray_workspace(cams[v], "cuda") for v in range(R.n_views)]

    def per_view_fwd():
        for v, b in enumerate(R.bufs):
            f = R.fields[R.specs[v].field]
            api.discretize(f.L, f.dom, cas[v], b["tex"])
            api.build_maxmip(b["tex"], b["mip"])
            api.raycast(cams[v], f.dom, cas[v], b["tex"], b["mip"], b["depth"], b["hit"], None, works[v])

    def per_view_train():
        for f in R.fields:
            f.grad_v.zero_()
            f.grad_sigma.zero_()
        for v, b in enumerate(R.bufs):
            f = R.fields[R.specs[v].field]
            api.discretize(f.L, f.dom, cas[v], b["tex"])
            api.build_maxmip(b["tex"], b["mip"])
            api.raycast(cams[v], f.dom, cas[v], b["tex"], b["mip"], b["depth"], b["hit"], None, works[v])
            b["grad_tex"].zero_()
            api.raycast_backward(cams[v], f.dom, cas[v], b["tex"], b["mip"], b["grad_depth"], b["grad_tex"], None,
                                 works[v])
            api.discretize_backward(f.L, f.dom, cas[v], b["tex"], b["grad_tex"], f.grad_v, f.grad_sigma)

    per_view_train()
    ms["per_view_fwd"] = timed(per_view_fwd, args.steps, stream)
    ms["per_view_fwd_bwd"] = timed(per_view_train, args.steps, stream)
    texels = sum(s.K * s.N * s.N for s in R.specs)
    rays = sum(s.width * s.height for s in R.specs)
    out = {
        "metric": "batched views: ms per batch step (forward + backward), vs the same views rendered one by one",
        "value": round(ms["graph_fwd_bwd"], 4),
        "unit": "ms/batch",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms["graph_fwd_bwd"], 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 texels, f64 ray geometry",
        "data": "synthetic (seeded fBm terrain)",
        "config": {"workload": f"batch: 8 fBm heightfields (9k-1.64M leaves, depth 8-12), 64 views "
                               f"(256^2 to 1080p, K 2-4), texel budget tuned to a {args.batch_target_ms} ms step",
                   "fields": [f.n for f in R.fields], "views": R.n_views, "texels": texels, "rays": rays},
        "ms": {k: round(v, 4) for k, v in ms.items()},
        "speedup_vs_per_view": {"fwd": round(ms["per_view_fwd"] / ms["graph_fwd"], 3),
                                "fwd_bwd": round(ms["per_view_fwd_bwd"] / ms["graph_fwd_bwd"], 3)},
        "grays_per_s_fwd": round(rays / (ms["graph_fwd"] * 1e-3) / 1e9, 3),
        "texel_budget": {"chosen": chosen["budget"], "target_ms": chosen["target_ms"], "curve": chosen["curve"]},
        "tuning": tuned["tuning"],
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="medium")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-reps", type=int, default=3, help="oracle frames timed for the CPU baseline (median)")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--batch-target-ms", type=float, default=33.3,
                    help="batch workload: time target of one forward + backward step for the texel budget tuner")
    ap.add_argument("--skip-flight", action="store_true",
                    help="skip the texel-reuse flight (profiled runs: its launches differ from a frame's)")
    ap.add_argument("--skip-startup", action="store_true",
                    help="skip the start-up measurements (device quadtree, influence lists)")
    ap.add_argument("--per-cascade", action="store_true",
                    help="also time discretize with each cascade launched alone (counter runs per cascade)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 256 MiB device copy (known traffic) to calibrate hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (each frame runs on one device)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        return batch_main(args)
    import torch
    from paper_2201_10887_amd import api, synth
    from paper_2201_10887_amd.renderer import Renderer

    w, dem, leaves, cam = build_scene(args.workload)
    build_scene.dem_cache = dem
    t0 = time.time()
    R = Renderer(leaves, w.side, w.max_depth, w.cutoff, w.cascades, w.tex_n, w.split_lambda, w.overlap)
    if w.water_seed:  # a second surface on the same cells, drawn where nearer
        R.add_surface(synth.water_surface(leaves, w.side, w.water_seed, w.water_wet))
    torch.cuda.synchronize()
    print(f"[bench] renderer ready in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    H, W = cam.height, cam.width
    depth = torch.empty((H, W), dtype=torch.float32, device="cuda")
    hit = torch.empty((H, W), dtype=torch.int32, device="cuda")
    gtex = torch.zeros_like(R.tex)
    gv = torch.zeros(R.L.n, dtype=torch.float32, device="cuda")
    gs = torch.zeros_like(gv)

    def forward():
        return R.forward(cam, None, depth, hit)

    tuned = R.tune_raycast(cam)
    print(f"[bench] long-ray queue: forward {R.long_ray_queue} (split {R.ray_band_deg}), adjoint "
          f"{R.long_ray_queue_backward} (split {R.ray_band_deg_backward}) {tuned}",
          file=sys.stderr, flush=True)
    _, _, cas = forward()
    torch.cuda.synchronize()
    gen = torch.Generator(device="cuda").manual_seed(1003)
    grad_depth = torch.where(torch.isfinite(depth), torch.randn(depth.shape, generator=gen, device="cuda"),
                             torch.zeros_like(depth)).contiguous()

    def train_step():
        _, _, c = forward()
        gtex.zero_()
        gv.zero_()
        gs.zero_()
        R.backward(cam, c, grad_depth, gtex, gv, gs, hit=hit)

    for _ in range(args.warmup):
        forward()
        train_step()
    ms_fwd = timed(forward, args.steps, stream)
    ms_train = timed(train_step, args.steps, stream)
    print(f"[bench] forward {ms_fwd:.3f} ms, forward+backward {ms_train:.3f} ms", file=sys.stderr, flush=True)
    # the frame time as a distribution: 100 frames after 10 warm-up frames, each timed on its own
    per_frame = frame_times(forward, 100, 10, stream)
    copy_gbs = copy_bandwidth_gbs(stream)

    # per-stage times on the same stream
    stage = {
        "discretize": lambda: api.discretize(R.L, R.dom, cas, R.tex, R.mask),
        "build_maxmip": lambda: api.build_maxmip(R.tex, R.mip),
        "raycast": lambda: api.raycast(cam, R.dom, cas, R.tex, R.mip, depth, hit, None, R.ray_work(cam),
                                       R.ray_band_rows(cam)),
        "raycast_backward": lambda: api.raycast_backward(cam, R.dom, cas, R.tex, R.mip, grad_depth, gtex, None,
                                                         R.ray_work(cam, backward=True),
                                                         R.ray_band_rows(cam, backward=True)),
        "discretize_backward": lambda: api.discretize_backward(R.L, R.dom, cas, R.tex, gtex, gv, gs),
    }
    # the same frame's textures with the other basis (Wendland C2 on the same support)
    Lw = R.L.with_basis("wendland")
    api.pack_leaves(Lw)
    tex_w = torch.empty_like(R.tex)
    stage["discretize_wendland"] = lambda: api.discretize(Lw, R.dom, cas, tex_w)
    if R.extra:
        X = R.extra[0]
        d_ter, h_ter = api.raycast(cam, R.dom, cas, R.tex, R.mip, None, None, None, R.ray_work(cam))

        def nearer():  # from the terrain-only image each time (two 8 MB copies included)
            depth.copy_(d_ter)
            hit.copy_(h_ter)
            api.raycast_nearer(cam, R.dom, cas, X["tex"], X["mip"], 1, depth, hit, None, R.ray_work(cam))

        stage.update({
            "discretize_water": lambda: api.discretize(X["L"], R.dom, cas, X["tex"], X["mask"]),
            "build_maxmip_water": lambda: api.build_maxmip(X["tex"], X["mip"]),
            "raycast_nearer_water": nearer,
        })
    if args.per_cascade:  # each cascade in a launch of its own
        for k in range(R.K):
            one = (api.Cascade * 1)(cas[k])
            stage[f"discretize_cascade{k}"] = (lambda one=one, k=k: api.discretize(R.L, R.dom, one, R.tex[k:k + 1],
                                                                                   R.mask[k:k + 1]))
    def stage_time(f):
        # two warm-up calls (the clocks settle after the host-side set-up above), then the median of
        # three timing loops of `steps` calls each
        f()
        f()
        return float(np.median([timed(f, args.steps, stream) for _ in range(3)]))

    stage_ms = {k: stage_time(f) for k, f in stage.items()}
    del Lw, tex_w
    api.discretize(R.L, R.dom, cas, R.tex, R.mask)
    torch.cuda.synchronize()
    t_host = time.perf_counter()
    for _ in range(100):
        R.fit(cam)
    fit_us = (time.perf_counter() - t_host) * 1e4

    startup = None if args.skip_startup else startup_ms(R, dem, w)
    work = discretize_work(R, cas, leaves, w)
    reuse = None if args.skip_flight else texel_reuse_flight(R, cam, depth, hit)
    print(f"[bench] texel reuse along a flight: {reuse}", file=sys.stderr, flush=True)
    vis_texels, pairs = work["visible_texels"], work["pairs"]
    forward()  # leave the full frame (every surface) in depth / hit
    torch.cuda.synchronize()
    hits = int(torch.isfinite(depth).sum())
    water_px = int(((hit >= 0) & ((hit >> 29) == 1)).sum()) if R.extra else 0
    K = R.K
    t_disc = stage_ms["discretize"] * 1e-3
    t_alu_floor = work["flops"] / (FP32_PEAK_TFLOPS * 1e12)
    t_hbm_floor = work["bytes"] / (HBM_PEAK_GBS * 1e9)
    if t_alu_floor >= t_hbm_floor:
        roof = {"bound": "alu", "achieved": round(work["flops"] / t_disc / 1e12, 3), "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(t_alu_floor / t_disc, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(work["bytes"] / t_disc / 1e9, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(t_hbm_floor / t_disc, 4)}
    traffic = None
    if args.workload == "medium":
        traffic = recorded_traffic("paper_2201_10887_amd/csrc/hfr_discretize.hip",
                                   "profiles/discretize_kernel_medium_hbm_counters.md")
    launches = -(-K // DISC_CASCADES_PER_LAUNCH)  # the library discretizes up to four cascades per launch
    # VALU issue: a CU issues at most one wave64 VALU instruction per cycle (four SIMDs, four cycles each)
    valu = recorded_figure("paper_2201_10887_amd/csrc/hfr_discretize.hip",
                           "profiles/discretize_kernel_medium_valu_counters.md",
                           "valu_instructions_per_launch") if args.workload == "medium" else None
    if valu is not None:
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        roof["valu_instructions_per_launch"] = valu
        roof["valu_issue_frac"] = round(valu / (cus * VALU_CLOCK_HZ) / (stage_ms["discretize"] / launches * 1e-3), 4)
    roof.update({"traffic": traffic, "kernel": "discretize_kernel<0>", "launches": launches,
                 "per_launch_ms": round(stage_ms["discretize"] / launches, 4),
                 "algorithmic_flops_per_launch": round(work["flops"] / launches), "algorithmic_bytes_per_launch":
                 round(work["bytes"] / launches), "hbm_frac": round(t_hbm_floor / t_disc, 4),
                 "alu_frac": round(t_alu_floor / t_disc, 4)})
    # max-mipmap: each texel read once (4 B), levels 1 .. log2 N written (level 0 is not stored)
    mip_bytes = K * (R.N * R.N * 4 + (api.mip_size(R.N) - R.N * R.N) * 4)
    dominant = max(("discretize", "build_maxmip", "raycast"), key=lambda k: stage_ms[k])
    out = {
        "metric": "ms/frame at 1080p (Gtexel/s, Grays/s, %HBM roofline); fwd+bwd vs fwd time",
        "value": round(ms_fwd, 4),
        "unit": "ms/frame",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_fwd, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 texels, f64 ray geometry",
        "data": "synthetic (seeded fBm terrain)",
        "config": {"workload": w.name, "leaves": int(R.L.n), "cascades": K, "tex_n": R.N,
                   "resolution": f"{W}x{H}", "sigma": w.sigma, "cutoff": w.cutoff, "split_lambda": w.split_lambda},
        "frame_ms": per_frame,
        "fwd_bwd_ms": round(ms_train, 4),
        "fwd_bwd_over_fwd": round(ms_train / ms_fwd, 3),
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "long_ray_queue": {"forward": R.long_ray_queue, "adjoint": R.long_ray_queue_backward,
                           "split_deg_forward": R.ray_band_deg, "split_deg_adjoint": R.ray_band_deg_backward,
                           "tuning_ms": tuned},
        "fit_cascades_host_us": round(fit_us, 1),
        "startup_ms": startup,
        "texel_reuse_flight": reuse,
        "gtexel_per_s": round(vis_texels / (stage_ms["discretize"] * 1e-3) / 1e9, 3),
        "gtexel_per_s_all": round(K * R.N * R.N / (stage_ms["discretize"] * 1e-3) / 1e9, 3),
        "grays_per_s": round(W * H / (stage_ms["raycast"] * 1e-3) / 1e9, 3),
        "hit_fraction": round(hits / (W * H), 4),
        "surfaces": 1 + len(R.extra),
        "water_pixel_fraction": round(water_px / (W * H), 4) if R.extra else None,
        "visible_texels": vis_texels,
        "pairs": round(pairs),
        "mean_influencers": round(work["mean_influencers"], 2),
        "maxmip_hbm_frac": round(mip_bytes / (stage_ms["build_maxmip"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "maxmip_roofline": {"bound": "hbm", "achieved": round(mip_bytes / (stage_ms["build_maxmip"] * 1e-3) / 1e9, 1),
                            "peak": HBM_PEAK_GBS, "unit": "GB/s", "algorithmic_bytes": mip_bytes,
                            "frac": round(mip_bytes / (stage_ms["build_maxmip"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                            "frac_of_copy": round(mip_bytes / (stage_ms["build_maxmip"] * 1e-3) / 1e9 / copy_gbs, 4),
                            "traffic": (recorded_traffic("paper_2201_10887_amd/csrc/hfr_maxmip.hip",
                                                         "profiles/maxmip_kernel_medium_hbm_counters.md")
                                        if args.workload == "medium" else None)},
        "hbm_copy_gbs": round(copy_gbs, 1),
        "dominant_stage": dominant,
        "roofline": roof,
    }
    if args.copy_probe:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 2 * src.numel() * 4
    if args.workload == "large":
        out["cpu_baseline"] = {"skipped": "the oracle's range-query trees over 64M leaves take minutes and tens "
                                          "of GB; the per-texel and per-ray oracle costs are those of the medium scene"}
    elif not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(w, leaves, cam, R, cas, vis_texels, args.cpu_reps)
        except Exception as e:  # the baseline is reported, not required
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
