#!/usr/bin/env python3
"""Forward+backward SAR images/s of the SDGR hot path on one MI355X.

Workload (default "vehicle_200k"): 200,000 Gaussians on a seeded composite of
boxes and cylinders inside a 6 x 3 x 2.5 m envelope, 72 views (azimuth 0-355
deg in 5 deg steps, incidence alternating 30/45 deg), 256 x 256 images at
0.1 m. One step = plan (pair counts) + forward of all 72 views + L1-loss
cotangent against a target rendered from a copy with means jittered by
N(0, 0.1 m) + backward to all Gaussian parameters + the overflow check,
everything resident in HBM. Pair capacities come from an exact count taken
before the timed region plus 10 % headroom. In the timed steps the overflow
check is ORed into a device flag on the stream and read once after the loop
(an overflow would invalidate the run, which is then repeated with a fresh
count); the per-stage times come from a separate pass with HIP events. Prints one JSON line, which also carries the roofline
object of the dominant kernel (HBM bytes of the algorithm per launch over its
measured launch time), the forward-only 1k-Gaussian and the 50k-Gaussian
building workloads as sub-objects, the reconstruction of a synthetic vehicle
with the paper's 30k-iteration schedule (iterations/s and its image and point
metrics), the served-vs-plain stream and the FP64 oracle timed on the host.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import ctypes
import hashlib
import json
import math
import os
import sys
import time
import types

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
# FP32 VALU issue rate without packed instructions: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz = 39.3e12 lane-operations/s (an FMA counts once); the
# transcendental unit runs at a quarter of that rate.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

WORKLOADS = ("vehicle_200k", "building_50k", "fwd_1k", "large_2m")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="vehicle_200k", choices=WORKLOADS)
    ap.add_argument("--cpu-rows", type=int, default=64,
                    help="range rows of one view the CPU oracle baseline times")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the per-stage HIP event timing")
    ap.add_argument("--serving-requests", type=int, default=1000,
                    help="requests of the served-vs-plain stream (0 skips it)")
    ap.add_argument("--no-work-count", action="store_true",
                    help="skip the untimed step that counts footprint hits (profiler runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of MIB MiB and one gather of "
                         "MIB MiB in random 64-byte rows (the reference kernels that scale "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE to bytes)")
    ap.add_argument("--no-other-workloads", action="store_true",
                    help="skip the short runs of the 1k-Gaussian and building workloads")
    ap.add_argument("--no-deterministic", action="store_true",
                    help="skip the short run of the same workload in the deterministic mode")
    ap.add_argument("--no-reconstruction", action="store_true",
                    help="skip the 30k-iteration reconstruction of the synthetic vehicle")
    ap.add_argument("--recon-iterations", type=int, default=30_000)
    ap.add_argument("--with-large", action="store_true",
                    help="also time the 2M-Gaussian recompute workload (a few seconds)")
    return ap.parse_args()


def workload(name):
    from paper_2506_21633_amd import scenes
    if name == "vehicle_200k":
        sc = scenes.vehicle(303, 200_000)
        views = scenes.vehicle_views()
        target = scenes.jitter(sc, 306)
        cfg = dict(workload=name, gaussians=sc.n, views=len(views), image="256x256",
                   pixel_m=0.1, incidence_deg=[30, 45], loss="L1 vs jittered target")
    elif name == "building_50k":
        sc = scenes.building(202, 50_000)
        views = scenes.building_views()
        target = scenes.jitter(sc, 203)
        cfg = dict(workload=name, gaussians=sc.n, views=len(views), image="128x128",
                   pixel_m=0.15, incidence_deg=[40], loss="L1 vs jittered target")
    elif name == "large_2m":
        sc = scenes.large_block(505, 2_000_000)
        views = scenes.large_views()
        target = scenes.jitter(sc, 506)
        cfg = dict(workload=name, gaussians=sc.n, views=len(views), image="1024x1024",
                   pixel_m=0.1, incidence_deg=[35], loss="L1 vs jittered target",
                   recompute=True)
    else:
        sc, views = scenes.fwd_1k()
        target = scenes.jitter(sc, 102)
        cfg = dict(workload=name, gaussians=sc.n, views=len(views), image="64x64",
                   pixel_m=0.15, incidence_deg=[45], loss="L1 vs jittered target")
    return sc, views, target, cfg


def source_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2506_21633_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel, launches_per_step, src_hash):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    rec = d.get(kernel)
    if not rec or rec.get("source_hash") != src_hash:
        return None
    return rec.get("bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sc, views, rows):
    """The FP64 oracle (untuned) on a bounded sample: the central `rows`
    range rows of view 0 (image and computation plane), all Gaussians,
    forward + backward (the oracle's backward runs its forward first, so one
    backward call is the whole step) with a fixed random cotangent; scaled
    to whole images."""
    import numpy as np
    import oracle
    from paper_2506_21633_amd import scenes
    v = views[0]
    band = scenes.View(azimuth=v.azimuth, grazing=v.grazing, img_w=v.img_w, img_h=rows,
                       d_az=v.d_az, d_rg=v.d_rg, comp_w=v.img_w, comp_h=rows,
                       comp_d_az=v.d_az, comp_d_el=v.d_rg * math.tan(v.grazing))
    G = np.random.default_rng(0).standard_normal((rows, v.img_w))
    t0 = time.perf_counter()
    oracle.backward_view(sc, band, G)
    dt = time.perf_counter() - t0
    per_image = dt * (v.img_h / rows)
    return {"value": 1.0 / per_image, "unit": "images/s", "cores": oracle.threads(),
            "cpu": cpu_model(), "kind": "oracle",
            "sample": f"forward+backward of the central {rows} of {v.img_h} range rows of "
                      f"view 0 ({v.img_w} columns, {sc.n} Gaussians), {dt:.1f} s, "
                      f"scaled x{v.img_h / rows:g} to one image"}


def serving_bench(dev, n_requests, seed=404, loads=(0.5, 0.8, 1.2, 2.0)):
    """Served (continuous batching, 2 launch slots, admission by exact
    workspace bytes, plans counted on planner threads) vs plain (one request
    per launch, FIFO) on the same Poisson arrival stream over 8 resident
    scenes of 1e4-5e5 Gaussians, at arrival rates of `loads` times the plain
    form's measured capacity, n_requests per point. Requests: 1-16 views of
    64^2-512^2 at 0.1 m, azimuth U[0, 360), incidence 30 or 45 deg; half ask
    for the L1 gradient against a zero target as well."""
    import numpy as np
    import torch
    from paper_2506_21633_amd import api, scenes
    from paper_2506_21633_amd.serve import GpuExecutor, Request, Server, percentile
    sc = scenes.serving_scenes(seed)
    resident = {f"s{k}": api.GaussianTensors.from_numpy(x, dev) for k, x in enumerate(sc)}
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(n_requests):
        sid = f"s{int(rng.integers(0, len(sc)))}"
        size = int(rng.choice([64, 128, 256, 512]))
        vs = [scenes.View.from_degrees(float(rng.uniform(0, 360)), float(rng.choice([30.0, 45.0])),
                                       size, 0.1) for _ in range(int(rng.integers(1, 17)))]
        want = bool(rng.integers(0, 2))
        tgt = torch.zeros(size * size * len(vs), device=dev) if want else None
        reqs.append((sid, vs, want, tgt))
    images = sum(len(r[1]) for r in reqs)

    def run(batching, rate):
        ex = GpuExecutor(resident, dev)
        srv = Server(ex, hbm_budget=96 << 30, max_views=96, slots=2, batching=batching)
        arrivals = np.cumsum(np.random.default_rng(seed + 1).exponential(1.0 / rate, len(reqs)))
        t0 = time.perf_counter()
        futs = []
        for a, (sid, vs, want, tgt) in zip(arrivals, reqs):
            while time.perf_counter() - t0 < a:
                time.sleep(2e-4)
            futs.append(srv.submit(Request(sid, vs, want, tgt)))
        lat = [f.result(600).latency_s for f in futs]
        dt = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        return {"p50_ms": round(percentile(lat, 50) * 1e3, 3),
                "p99_ms": round(percentile(lat, 99) * 1e3, 3),
                "images_per_s": round(images / dt, 1),
                "launches": len(srv.batch_sizes),
                "mean_batch_requests": round(st["mean_batch_requests"], 3)}

    # capacity of the plain form: back-to-back requests
    ex = GpuExecutor(resident, dev)
    warm = Server(ex, hbm_budget=96 << 30, batching=False)
    for sid, vs, want, tgt in reqs[:8]:
        warm.submit(Request(sid, vs, want, tgt)).result(600)
    k = min(64, len(reqs))
    t0 = time.perf_counter()
    futs = [warm.submit(Request(sid, vs, want, tgt)) for sid, vs, want, tgt in reqs[:k]]
    for f in futs:
        f.result(600)
    service = (time.perf_counter() - t0) / k
    warm.close()
    points = []
    for load in loads:
        rate = load / service
        points.append({"load": load, "qps": round(rate, 1), "served": run(True, rate),
                       "plain": run(False, rate)})
    return {"plain_capacity_qps": round(1.0 / service, 1), "requests_per_point": len(reqs),
            "points": points,
            "workload": "8 resident vehicle scenes (1e4-5e5 Gaussians), Poisson arrivals, "
                        "1-16 views of 64^2-512^2, half with L1 gradient"}


def calibration_kernels(dev, mib):
    """Reference kernels of known HBM bytes for scaling the rocprofv3
    FETCH_SIZE / WRITE_SIZE counters: a device-to-device copy of `mib` MiB
    (streaming) and a gather of `mib` MiB in random 64-byte rows (the access
    shape of the record gathers); reads and writes `mib` MiB each, plus 8 B
    of index per row for the gather."""
    import torch
    nf = mib * (1 << 20) // 4
    src = torch.ones(nf, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize(dev)
    dst.copy_(src)
    rows = src.view(-1, 16)
    perm = torch.randperm(rows.shape[0], device=dev)
    torch.cuda.synchronize(dev)
    torch.index_select(rows, 0, perm, out=dst.view(-1, 16))
    torch.cuda.synchronize(dev)
    del src, dst, perm


def make_step(r, target_images, forward_only=False, flags=None):
    """One step: forward with pair capacities from the last exact count
    plus 10 % headroom, L1 cotangent, backward, overflow check. Without
    `flags` the check synchronises and an overflowing step is redone with a
    new count; with `flags` (a device int32) it is ORed in on the stream and
    the caller reads it once after its loop (no host sync per step)."""
    import torch
    from paper_2506_21633_amd import _capi
    numel = float(target_images.numel())

    def step():
        while True:
            res = r.forward(r.planned(0.1))
            if not forward_only:
                G = torch.sign(res.images - target_images) / numel
                r.backward(res, G)
            if flags is not None:
                r.status_into(res, flags)
                return res
            try:
                r.status(res)
                return res
            except _capi.SDGRError as exc:
                if exc.code != _capi.SDGR_EOVERFLOW:
                    raise
                r.replan()
    return step


def timed_steps(dev, r, target_images, steps, forward_only=False):
    """Seconds for `steps` steps bracketed by synchronisation, the overflow
    checks deferred to one read after the loop (an overflow invalidates the
    run, which is then repeated once with a fresh count)."""
    import torch
    for attempt in range(2):
        flags = torch.zeros(1, dtype=torch.int32, device=dev)
        step = make_step(r, target_images, forward_only, flags)
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize(dev)
        dt = time.perf_counter() - t0
        if int(flags.item()) == 0:
            return dt
        r.replan()
    raise RuntimeError("pair counts overflowed the plan in two timed runs")


def time_workload(name, dev, steps, warmup, forward_only=False):
    """Short timed run of one more workload: images/s and ms per step."""
    import torch
    from paper_2506_21633_amd import api
    sc, views, target, cfg = workload(name)
    opts = api.RenderOptions(recompute=bool(cfg.get("recompute", False)))
    r = api.Renderer([api.GaussianTensors.from_numpy(sc, dev)], views, opts)
    timg = api.Renderer([api.GaussianTensors.from_numpy(target, dev)], views,
                        opts).forward().images.clone()
    step = make_step(r, timg, forward_only)
    for _ in range(warmup):
        step()
    dt = timed_steps(dev, r, timg, steps, forward_only)
    cfg = dict(cfg, mode="forward only" if forward_only else "forward+backward",
               steps=steps, warmup=warmup)
    if forward_only:
        cfg.pop("loss", None)
    return {"value": len(views) * steps / dt, "unit": "images/s",
            "ms_per_step": dt * 1e3 / steps, "config": cfg}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}, WORLD_SIZE {world}); "
              "multi-GPU view sharding is not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2506_21633_amd import _capi, api

    dev = torch.device("cuda:0")
    if args.copy_calibration > 0:
        calibration_kernels(dev, args.copy_calibration)
    sc, views, target, cfg = workload(args.workload)
    g = api.GaussianTensors.from_numpy(sc, dev)
    tgt = api.GaussianTensors.from_numpy(target, dev)
    opts = api.RenderOptions(recompute=bool(cfg.get("recompute", False)))
    r = api.Renderer([g], views, opts)
    target_images = api.Renderer([tgt], views, opts).forward().images.clone()
    step = make_step(r, target_images)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize(dev)
    res = step()
    exact = r._last_exact          # the exact pair counts (capacities add 10 %)
    torch.cuda.synchronize(dev)
    # pairs the step actually sorted and rasterized: all computation-plane
    # pairs, and imaging-plane pairs of the Gaussians with nonzero intensity;
    # records pass A used (the backward's work list)
    st = res.state[:64].view(torch.int32).cpu()
    used = types.SimpleNamespace(records=exact.records, rays=exact.rays,
                                 pairs_c=int(st[1]), pairs_i=int(st[2]), active=int(st[5]),
                                 pixels=sum(v.img_w * v.img_h for v in views), n=sc.n)

    lib = _capi.lib()
    work = [0] * 16
    if not args.no_work_count:
        # one untimed step with the work counters on
        api.count_work(True)
        res = step()
        torch.cuda.synchronize(dev)
        api.count_work(False)
        work = list(r.work_counters(res).values())
        del res
    dt = timed_steps(dev, r, target_images, args.steps)
    stages = {}
    if not args.no_profile:
        # per-stage times (HIP events on the launching stream) from a separate
        # pass, so that the event records do not load the timed steps
        _capi.profile_read()
        lib.sdgr_profile_enable(1)
        for _ in range(min(args.steps, 10)):
            step()
        torch.cuda.synchronize(dev)
        lib.sdgr_profile_enable(0)
        stages = _capi.profile_read()

    nv = len(views)
    ms_step = dt * 1e3 / args.steps
    out = {
        "metric": ("fwd+bwd SAR images/s at 200k Gaussians 256^2" if args.workload == "vehicle_200k"
                   else f"fwd+bwd SAR images/s ({args.workload})"),
        "value": nv * args.steps / dt,
        "unit": "images/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": dict(cfg, parallelism="single GPU", pairs_c=used.pairs_c,
                       pairs_i=used.pairs_i, pairs_i_all=exact.pairs_i, tiles_c=exact.tiles_c,
                       tiles_i=exact.tiles_i, records=used.records, records_used=used.active),
    }
    out["work"] = dict(zip(api.WORK_NAMES[:14], work[:14]))
    out["path_hbm"] = path_hbm(used, ms_step)
    if stages:
        per = {k: v[0] / max(v[1], 1) for k, v in stages.items() if v[1]}
        out["stages_ms"] = {k: round(v, 4) for k, v in per.items()}
        dom = max(per, key=per.get)
        out["roofline"] = roofline(dom, per[dom], used, work)
        out["kernels_hbm"] = {k: kernel_hbm(k, per[k], used) for k in ALGO_BYTES if k in per}
    if not args.no_deterministic:
        # the same step with ordered sums instead of float atomics
        rd = api.Renderer([g], views, api.RenderOptions(recompute=opts.recompute,
                                                        deterministic=True))
        dstep = make_step(rd, target_images)
        for _ in range(2):
            dstep()
        ddt = timed_steps(dev, rd, target_images, 5) / 5
        out["deterministic"] = {"value": nv / ddt, "unit": "images/s",
                                "ms_per_step": ddt * 1e3, "steps": 5}
        del rd, dstep
    if not args.no_other_workloads:
        out["workloads"] = {
            "fwd_1k": time_workload("fwd_1k", dev, 50, 5, forward_only=True),
            "building_50k": time_workload("building_50k", dev, 10, 3),
        }
        if args.with_large:
            out["workloads"]["large_2m"] = time_workload("large_2m", dev, 3, 1)
    if not args.no_reconstruction:
        out["reconstruction"] = reconstruction_bench(dev, args.recon_iterations)
    if args.serving_requests > 0:
        out["serving"] = serving_bench(dev, args.serving_requests)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, views, args.cpu_rows)
    print(json.dumps(out), flush=True)


def reconstruction_bench(dev, iterations):
    """Synthetic reconstruction (Sec. III-B): a 20k-Gaussian vehicle renders
    the 72 training views (incidence 15/45/75 deg, azimuth every 15 deg, 64 x
    64 at 0.2 m); 15k Gaussians start on a hemispherical shell and run the
    paper's schedule (SH degree + 1 every 2,500 iterations, densify from 10k
    to 25k) in batches of 8 views. Reports iterations/s over the whole run and
    the metrics on 24 held-out views and against the ground-truth centres
    (F1 at 0.2 m, one resolution cell)."""
    import torch
    from paper_2506_21633_amd import api, scenes, train
    gt = scenes.vehicle(909, 20_000)
    views = scenes.reconstruction_views(64, 0.2)
    tviews = scenes.reconstruction_test_views(64, 0.2)
    gtt = api.GaussianTensors.from_numpy(gt, dev)
    targets = api.Renderer([gtt], views).forward().stacked().clone()
    ttargets = api.Renderer([gtt], tviews).forward().stacked().clone()
    truth = torch.as_tensor(gt.means, device=dev)
    init = scenes.hemisphere_init(15_000, 4.0, seed=910, center=(0.0, 0.0, -1.25))
    cfg = train.TrainConfig(iterations=iterations)
    rec = train.Reconstruction(init, views, targets, cfg, device=dev)

    def metrics():
        img = api.Renderer([rec.gaussians()], tviews).forward().stacked()
        im = train.image_metrics(img, ttargets)
        pm = train.point_metrics(rec.p["means"], truth, tau=0.2)
        return {"gaussians": rec.n, "psnr": round(im["psnr"], 3), "ssim": round(im["ssim"], 4),
                "cd": round(pm["cd"], 4), "precision": round(pm["precision"], 4),
                "recall": round(pm["recall"], 4), "f1": round(pm["f1"], 4)}

    start = metrics()
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    rec.run()
    torch.cuda.synchronize(dev)
    dt = time.perf_counter() - t0
    return {"iterations": iterations, "seconds": round(dt, 2),
            "iterations_per_s": round(iterations / dt, 1),
            "images_per_s": round(iterations * cfg.batch_views / dt, 1),
            "densify_calls": rec.densify_calls, "start": start, "end": metrics()}


HIT_KERNELS = {"raster_a_fwd": 0, "raster_a_bwd": 1, "raster_b_fwd": 2, "raster_b_bwd": 3}
ENTRY_KERNELS = {"raster_a_fwd": 4, "raster_a_bwd": 5, "raster_b_fwd": 6}
# the sources of each stage's kernels (the stored counters are taken on them)
SOURCES = {"raster_a_fwd": ("raster.hip",), "raster_b_fwd": ("raster.hip",),
           "raster_b_bwd": ("raster.hip",), "raster_a_bwd": ("raster.hip", "sort.hip"),
           "pair_sort": ("sort.hip",), "depth_sort": ("sort.hip",), "bin_pairs": ("sort.hip",),
           "preprocess": ("preprocess.hip",), "plan_query": ("preprocess.hip",),
           "params_bwd": ("preprocess.hip",)}

# Lane-operations the definition needs per footprint hit ((cell, Gaussian)
# evaluation with q < q_max), each exp weighted 4 (quarter-rate unit):
#   pass A fwd: quadratic form 8, exp 5, footprint 2, kappa f 1, exp 5,
#               alpha 1, alpha T 1, A += 1, T *= 1, tau += 1           = 26
#   pass B fwd: quadratic form 8, exp 5, footprint 2, x I 1, S += 1      = 17
#   pass B bwd: quadratic form 8, exp 5, footprint 2, dI 2, dq 2,
#               centre 8, conic 10                                      = 37
#   pass A bwd: quadratic form 8, exp 5, footprint 2, x 1, exp 5,
#               tau -= 1, exp 5, dalpha 2, U 3, dx 1, dkappa 2, dq 3,
#               centre 8, conic 10                                      = 56
OPS_PER_HIT = {"raster_a_fwd": 26, "raster_b_fwd": 17, "raster_b_bwd": 37,
               "raster_a_bwd": 56}

# Algorithmic HBM bytes per launch of each stage: the compulsory traffic of
# the binned method, split from the per-unit figures of the whole step
# (per pair 4 B read in each rasterizer pass, 12 B emitted, 24 B per sort
# pass; per used record its 24 B plane record read in each pass that needs
# it and 8 B per float accumulated read-modify-write; per ray and pixel 4 B
# per array written or read). u: Kc, Ki (pairs of the two planes), R
# (records), Nu (records pass A used), rays, pixels, N (Gaussians).
ALGO_BYTES = {
    # pass A forward: pair ids, plane-C records, A accumulated, tau written
    "raster_a_fwd": lambda u: 4 * u.pairs_c + (24 + 8) * u.active + 4 * u.rays,
    # pass A backward: pair ids, plane-C records, c = P dL/dI, six
    # plane-C gradient sums accumulated, tau read
    "raster_a_bwd": lambda u: 4 * u.pairs_c + (24 + 4 + 48) * u.active + 4 * u.rays,
    # pass B forward: pair ids, plane-I records, image written
    "raster_b_fwd": lambda u: 4 * u.pairs_i + 24 * u.active + 4 * u.pixels,
    # pass B backward: plane-I records, dL/dS read once, six plane-I sums
    # and c written, six plane-C sums cleared
    "raster_b_bwd": lambda u: (24 + 28 + 24) * u.active + 4 * u.pixels,
    # parameter adjoint: parameters read and gradients written per Gaussian,
    # 12 plane gradients and A read per used record
    "params_bwd": lambda u: 96 * u.n + 52 * u.active,
    # projection: parameters read, 48 B record and 8 B pair count per record
    "preprocess": lambda u: 48 * u.n + 56 * u.records,
    # one 24 B pass over the computation-plane pairs
    "pair_sort": lambda u: 24 * u.pairs_c,
    # emission of the computation-plane pairs
    "bin_pairs": lambda u: 12 * u.pairs_c,
}


def kernel_hbm(stage, ms, u):
    byts = ALGO_BYTES[stage](u)
    gbs = byts / (ms * 1e-3) / 1e9
    return {"bytes": byts, "ms": round(ms, 4), "GBps": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4)}


def roofline(kernel, ms, u, work):
    """Roofline object of the dominant stage against HBM: achieved = its
    algorithmic bytes per launch (ALGO_BYTES) / its mean launch time from
    HIP events on the launching stream. The lane-operation count of the
    rasterizers against the VALU peak is a secondary figure."""
    src = SOURCES.get(kernel)
    traffic = stored_traffic(kernel, 1, source_hash(*src)) if src else None
    out = {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": None, "traffic": traffic, "kernel": kernel, "ms": ms}
    if kernel in ALGO_BYTES:
        h = kernel_hbm(kernel, ms, u)
        out.update(achieved=h["GBps"], frac=h["GBps"] / HBM_PEAK_GBS,
                   algorithmic_bytes=h["bytes"])
    if kernel in HIT_KERNELS and work[HIT_KERNELS[kernel]]:
        hits = work[HIT_KERNELS[kernel]]
        ops = hits * OPS_PER_HIT[kernel] / (ms * 1e-3) / 1e12
        out["alu"] = {"achieved": ops, "peak": VALU_PEAK_TOPS, "unit": "Tlane-op/s",
                      "frac": ops / VALU_PEAK_TOPS,
                      "work": f"{hits} footprint hits x {OPS_PER_HIT[kernel]} lane-ops"}
        if kernel in ENTRY_KERNELS:
            out["alu"]["evaluated_over_hits"] = work[ENTRY_KERNELS[kernel]] * 64 / hits
    return out


def path_hbm(u, ms_step):
    """Compulsory HBM bytes of one fwd+bwd step of the binned method (per
    Gaussian: parameters read and gradients written, 96 B; per used record:
    the projected record written once and read in forward and backward plus
    the per-record reductions, 256 B; per pair: emission, one sort pass, one
    read in forward and one in backward, 44 B; per pixel and per ray: image
    and dL/dS, optical depth written and read, 8 B each) against 8 TB/s."""
    byts = (96 * u.n + 256 * u.active + 44 * (u.pairs_c + u.pairs_i) + 8 * u.pixels
            + 8 * u.rays)
    gbs = byts / (ms_step * 1e-3) / 1e9
    return {"bytes_per_step": byts, "achieved_GBps": gbs, "peak_GBps": HBM_PEAK_GBS,
            "frac": gbs / HBM_PEAK_GBS}


if __name__ == "__main__":
    main()
