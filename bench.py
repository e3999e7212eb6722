"""Throughput benchmark of the in-scattering hot path on one GPU.

A step is one whole frame: rebuild the density pyramid of the 256^3 fBm cloud
from the resident grid, apply the light (the transmittance sweep runs again),
trace the 1920x1080 camera rays to their first delta-tracking collision and
compact them (about 1.2M shading points), then gather, CNN + attention,
backbone and decode for every point, and write the image.  Nothing crosses
PCIe inside the timed region; the collision count stays on the device.

Prints one JSON line: shading points/s (whole job), ms per frame, frames/s,
per-kernel times from HIP events the library records on the stream its
kernels run on, the roofline of the dominant kernel, the radiance error of
each precision against the FP64 oracle on a seeded sample of the frame, the
oracle's own throughput on the host cores, and a serving run (Poisson frame
requests over media of 64^3..512^3 and three resolutions) with p50/p99 frame
latency.
"""

import argparse
import json
import os
import queue
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}
VALU_FP32_TFLOPS = 78.6   # 256 CUs x 64 lanes x 2 FLOP x 2.4 GHz, without packed FP32
G_SWEEP = (0.0, 0.5, 0.85, 0.95)   # HG asymmetries of the precision workload

# Algorithmic FP32 vector work of the gather per shading point: 12 layers x 225
# sites, each two trilinear interpolations (7 lerps of 2 FLOP), one exponent
# (2) and four running statistics (4); plus 225 phase features (12 each).
GATHER_FLOP_PER_POINT = 12 * 225 * (2 * 14 + 2 + 4) + 225 * 12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="bf16", choices=["fp32", "bf16", "fp8"])
    ap.add_argument("--workload", default="frame", choices=["frame", "large", "small"])
    ap.add_argument("--cpu-sample", type=int, default=32768,
                    help="points of the frame the oracle is timed on, per run (0 = skip)")
    ap.add_argument("--cpu-runs", type=int, default=3, help="oracle timing runs (the median is reported)")
    ap.add_argument("--parity-sample", type=int, default=262144,
                    help="seeded subset of the frame's collisions checked against the oracle at the workload's g")
    ap.add_argument("--parity-sample-by-g", type=int, default=16384,
                    help="seeded subset checked at each g of the precision workload")
    ap.add_argument("--paper-path", action="store_true", default=True,
                    help="also time the paper's templates and backbone modules on the frame's collisions")
    ap.add_argument("--no-paper-path", dest="paper_path", action="store_false")
    ap.add_argument("--paper-sample", type=int, default=16384,
                    help="seeded subset of the collisions checked against the oracle on the paper's path")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this size (for scaling HBM counters)")
    ap.add_argument("--compare-fp32", action="store_true", default=True)
    ap.add_argument("--no-compare-fp32", dest="compare_fp32", action="store_false")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="measured length of the Poisson request trace of the serving run (0 = skip)")
    ap.add_argument("--serve-warmup", type=float, default=5.0,
                    help="seconds of the trace before the measured part (requests not recorded)")
    ap.add_argument("--serve-sustained-seconds", type=float, default=30.0,
                    help="length of the second trace, at 70%% of the rate the device sustained")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-inflight", type=int, default=4)
    ap.add_argument("--serve-budget-gb", type=int, default=200)
    return ap.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_work(wl, levels, level_geom, npix, npts, width, n_linear, prec):
    """Algorithmic bytes / FLOPs of each kernel per frame (one launch per frame
    for the frame workload; the large one runs the features and backbone in
    passes of at most 2^21 points)."""
    row_bytes = {"fp32": 1088 * 4, "bf16": 1088 * 2, "fp8": 1152}[prec]   # stored descriptor row
    # bytes per stored transmittance feature: the FP8 path runs the CNN on BF16
    b_t = {"fp32": 4, "bf16": 2, "fp8": 2}[prec]
    n0 = wl.n
    vox = [(n0 >> m) ** 3 for m in range(levels)]
    samples = sum(nu * nv * n for (nu, nv, n) in level_geom)          # rays x slices of every level
    pairs_v = sum(nu * (nv + 1) * n for (nu, nv, n) in level_geom)
    conv_flop = 2 * 12 * (504 * 27 + 80 * 216) + 2 * 12 * (64 + 64)  # per point: conv1, conv2, attention
    mlp_flop = 2 * (1057 * width + (n_linear - 2) * width * width + width)
    # the transmittance fields as the method defines them: the density pyramid
    # read and one FP32 path density per ray sample written
    fields = 4 * sum(vox) + 4 * samples
    return {
        "pyramid": {"bytes": 4 * sum(vox[:-1]) + 4 * sum(vox[1:])},
        # reads the pyramid, writes the path density; this library writes it
        # as its pairs along V (the gather's layout), counted as layout bytes
        "sweep": {"bytes": fields, "layout_bytes": 4 * sum(vox) + 8 * pairs_v},
        "site_tables": {"bytes": 225 * 16},
        # rays: flag, point and direction per pixel; scan; compacted copies
        "raygen": {"bytes": npix * (4 + 12 + 12) + npix * 8 + npts * (12 + 12 + 4)},
        # the gather of the method: per point its position and direction in,
        # 12 x 225 graded transmittances (b_t bytes each) and 12 x 8 squeeze
        # statistics and the two scalars out, plus the fields read once
        "features": {"bytes": npts * (24 + 2700 * b_t + 208) + fields, "flops": npts * conv_flop,
                     "valu_flops": npts * GATHER_FLOP_PER_POINT},
        "backbone": {"bytes": npts * (row_bytes + 8), "flops": npts * mlp_flop},
        "image": {"bytes": npix * 4 + npts * 12},
    }


TPL_COUNTS = (6, 8, 12, 16, 24, 32, 48, 48, 32, 16, 16, 8)


def module_flop_per_point():
    """Useful FLOPs of the paper's backbone modules per point: per type, each
    step's excitation (S1 2x8, S2 (n+2)x2), FC-1 (n'x(n+2)) and FC-2 (n'xn'),
    then the 64x56 merge; two FLOPs per multiply-add."""
    macs = 0
    for k in list(range(0, 7)) + list(range(8, 11)):
        a, b = TPL_COUNTS[k] + 2, TPL_COUNTS[k + 1]
        macs += 16 + 2 * a + b * a + b * b
    return 2 * 3 * (macs + 64 * 56)


def paper_path(ctx, mid, wl, params, pts, dirs, tp, td, stream, prec, om, sample, rng):
    """The frame's collisions through the paper's templates, then either the
    MLP directly or the six backbone modules and the MLP: per-kernel times,
    algorithmic rates, and the radiance against the FP64 oracle on a seeded
    subset."""
    import torch
    from workloads import weights
    mods = weights.he_init_modules(seed=2)
    ctx.set_weights(params, modules=mods)
    out = {}
    f32 = lambda x: float(np.float32(x))
    op = dict(params)
    op["lam"] = f32(params["lam"])
    op["gamma"] = f32(params["gamma"])
    sidx = np.sort(rng.choice(len(pts), min(sample, len(pts)), replace=False))
    sp = torch.from_numpy(np.ascontiguousarray(pts[sidx], np.float32)).cuda()
    sd = torch.from_numpy(np.ascontiguousarray(dirs[sidx], np.float32)).cuda()
    tl = torch.empty(len(pts), dtype=torch.float32, device="cuda")
    b_row = {"fp32": 4, "bf16": 2, "fp8": 1}[prec]
    ctx.set_templates("paper")
    for name, bb in (("templates_mlp", "mlp"), ("templates_modules_mlp", "paper")):
        ctx.set_backbone(bb)
        ent = {}
        for pr in sorted({prec, "fp32"}):
            if pr == "fp8":
                ctx.calibrate_fp8(mid, sp[:65536], sd[:65536])
            ctx.set_precision(pr)
            for _ in range(2):
                ctx.query_device(mid, tp, td, tl, stream=stream.cuda_stream)
            torch.cuda.synchronize()
            ctx.profile(True)
            for _ in range(5):
                ctx.query_device(mid, tp, td, tl, stream=stream.cuda_stream)
            torch.cuda.synchronize()
            rep = ctx.profile_report()
            ctx.profile(False)
            ks = {k: v[1] / 5 for k, v in rep.items()}
            sl = torch.empty(len(sidx), dtype=torch.float32, device="cuda")
            ctx.query_device(mid, sp, sd, sl)
            _, y = ctx.network(mid, sp, sd, want_desc=False)
            torch.cuda.synchronize()
            ent[pr] = {"ms": sum(ks.values()), "kernels_ms": ks, "L": sl.cpu().numpy().astype(np.float64),
                       "y": y.cpu().numpy().astype(np.float64)}
        if bb == "mlp":
            ref = om.tpl_query(op, pts[sidx], dirs[sidx], f32(wl.sigma_t), f32(wl.albedo), f32(wl.g), f32(wl.radiance))
        else:
            ref = om.tpl_modules_query(op, mods, pts[sidx], dirs[sidx], f32(wl.sigma_t), f32(wl.albedo), f32(wl.g),
                                       f32(wl.radiance))
        res = {}
        for pr, e in ent.items():
            res[pr] = {"ms": e["ms"], "kernels_ms": e["kernels_ms"],
                       "points_per_s": len(pts) / (e["ms"] * 1e-3),
                       "rel_l2_vs_fp64_oracle": float(np.linalg.norm(e["L"] - ref["L"]) / np.linalg.norm(ref["L"])),
                       "max_abs_dy": float(np.abs(e["y"] - ref["y"]).max())}
        # algorithmic rates at the headline precision
        ks = ent[prec]["kernels_ms"]
        n = len(pts)
        if "features" in ks:
            row = (894 * 4) if bb == "paper" else 894 * b_row
            byt = n * (24 + row + 4)
            valu = n * (266 * (2 * 14 + 2 + 4 + 12))
            t = ks["features"] * 1e-3
            res["template_features_rates"] = {"bytes_per_point": 24 + row + 4, "GBps": byt / t / 1e9,
                                              "hbm_frac": byt / t / 1e9 / HBM_PEAK_GBS,
                                              "valu_flop_per_point": valu / n,
                                              "valu_frac": valu / t / 1e12 / VALU_FP32_TFLOPS}
        if "modules" in ks:
            fl = n * module_flop_per_point()
            t = ks["modules"] * 1e-3
            res["modules_rates"] = {"flop_per_point": module_flop_per_point(), "TFLOPs": fl / t / 1e12,
                                    "mfma_frac_fp32": fl / t / 1e12 / MFMA_PEAK_TFLOPS["fp32"]}
        out[name] = res
        log("paper path %s: %s" % (name, {pr: round(r["ms"], 3) for pr, r in res.items() if "ms" in r}))
    ctx.set_templates("lattice")
    ctx.set_backbone("mlp")
    ctx.set_precision(prec)
    ctx.set_weights(params)
    out["sample_points"] = int(len(sidx))
    out["weights"] = "He-normal backbone (workload's) and modules (seed 2); FP8 scales calibrated on the sample"
    return out


def measured_traffic(kernel, prec, workload):
    """HBM bytes per launch from the committed counter summary of this kernel,
    if it was taken on the current source; else None."""
    from paper_2401_14051_amd import rocprof_summary
    path = os.path.join(ROOT, "profiles", "%s_%s_%s_traffic.json" % (kernel, workload, prec))
    if not os.path.exists(path) or kernel not in rocprof_summary.KERNEL_SOURCES:
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != rocprof_summary.source_hash(kernel):
        return None
    return rec["traffic_bytes_per_launch"]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            return next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        return "unknown CPU"


def cpu_baseline(args, om, op, wl, pts, dirs, rng):
    """The FP64 oracle timed on the host cores (median of args.cpu_runs runs):
    the full-resolution sweep, then the gather alone and the whole query on a
    seeded subset of the frame's collisions, scaled to the frame; the small
    workload (32^3, all points) also on one core."""
    from oracle import oracle
    from workloads import configs
    f32 = lambda x: float(np.float32(x))
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    oracle.set_threads(threads)
    cidx = np.sort(rng.choice(len(pts), min(args.cpu_sample, len(pts)), replace=False))
    cp, cd = pts[cidx], dirs[cidx]
    t_sweep, t_gather, t_query = [], [], []
    for _ in range(args.cpu_runs):
        t = time.perf_counter()
        om.set_light(np.asarray(wl.light, np.float32))
        t_sweep.append(time.perf_counter() - t)
        t = time.perf_counter()
        om.features(f32(wl.sigma_t), f32(wl.g), op["lam"], cp, cd, outputs=("stats", "f0"))
        t_gather.append(time.perf_counter() - t)
        t = time.perf_counter()
        om.query(op, cp, cd, f32(wl.sigma_t), f32(wl.albedo), f32(wl.g), f32(wl.radiance))
        t_query.append(time.perf_counter() - t)
    sw, ga, qu = (float(np.median(v)) for v in (t_sweep, t_gather, t_query))
    frame_s = sw + qu * len(pts) / len(cidx)
    # the small workload on one core, all of its points
    sm = configs.SMALL
    sd = sm.density()
    sp, sdir, _ = sm.points(sd)
    sop = dict(sm.params())
    sop["lam"] = f32(sop["lam"])
    oracle.set_threads(1)
    t_small = []
    for _ in range(args.cpu_runs):
        t = time.perf_counter()
        smm = oracle.Medium(sd)
        smm.set_light(np.asarray(sm.light, np.float32))
        smm.query(sop, sp, sdir, f32(sm.sigma_t), f32(sm.albedo), f32(sm.g), f32(sm.radiance))
        t_small.append(time.perf_counter() - t)
    oracle.set_threads(threads)
    ts = float(np.median(t_small))
    log("oracle: sweep %.2fs, gather %.2fs and query %.2fs for %d points on %d threads; small workload "
        "%.2fs on 1 thread" % (sw, ga, qu, len(cidx), threads, ts))
    return {"value": len(pts) / frame_s, "unit": "shading points/s", "cores": threads, "kind": "oracle",
            "sample": "FP64 oracle (C, OpenMP) on %s, %d threads (%d logical CPUs visible), median of %d runs: "
                      "full-resolution sweep plus a seeded %d-point subset of the frame's %d collisions, scaled to "
                      "the frame" % (cpu_model(), threads, os.cpu_count() or 0, args.cpu_runs, len(cidx), len(pts)),
            "per_stage_s": {"sweep_per_light": sw, "gather_per_point": ga / len(cidx),
                            "network_per_point": (qu - ga) / len(cidx), "query_per_point": qu / len(cidx)},
            "small_workload_1_core": {"points": len(sp), "seconds": ts, "points_per_s": len(sp) / ts,
                                      "includes": "pyramid, sweep and query of the 32^3 workload"}}


def frame_camera(nis, wl):
    if wl.cam == "ortho":
        return nis.camera(wl.res[0], wl.res[0], vfov_deg=0.0, ortho_z=1.0)
    return nis.camera(wl.res[0], wl.res[1], 45.0, eye=wl.eye)


def serving(ctx, nis, args):
    """Poisson frame requests through the frame server: media of 64^3..512^3
    (pyramids resident), resolutions 256^2 / 720p / 1080p, a random light and
    g per request, BF16 network.  Returns the offered and achieved rates and
    the latency percentiles (submission to observed completion)."""
    from workloads import configs, medium
    t0 = time.time()
    # media seeds 101..104 for the four sizes
    mids = {n: ctx.load_medium(medium.fbm_cloud(n, seed=101 + i), 8.0, 0.99, 0.85)
            for i, n in enumerate((64, 128, 256, 512))}
    log("serving: media loaded (%.1fs)" % (time.time() - t0))
    cams = {res: nis.camera(res[0], res[1], 45.0, eye=configs.FRAME_EYE)
            for res in ((256, 256), (1280, 720), (1920, 1080))}

    def run(trace, t_from=0.0):
        """Submits the trace in real time; requests arriving before t_from
        (the warm-up) run but are not recorded."""
        q = queue.Queue()
        recs = []

        def submit():
            base = time.perf_counter()
            for r in trace:
                dt = r["t"] - (time.perf_counter() - base)
                if dt > 0:
                    time.sleep(dt)
                q.put((ctx.submit(mids[r["n"]], cams[r["res"]], r["light"], 1.0, r["g"], r["seed"]), r))
            q.put(None)

        def collect():
            while True:
                item = q.get()
                if item is None:
                    return
                fid, r = item
                res = ctx.wait(fid)
                if r["t"] >= t_from:
                    recs.append((res.status, res.t_submit, res.t_start, res.t_done, res.n_points, r["n"],
                                 r["res"]))
                ctx.release(fid)

        ts, tc = threading.Thread(target=submit), threading.Thread(target=collect)
        ts.start()
        tc.start()
        ts.join()
        tc.join()
        ok = [x for x in recs if x[0] == 0]
        lat = np.array([x[3] - x[1] for x in ok]) * 1e3
        span = max(x[3] for x in ok) - min(x[1] for x in ok)
        measured = [r for r in trace if r["t"] >= t_from]
        out = {"requests": len(measured), "completed": len(ok), "failed": len(recs) - len(ok),
               "offered_rps": len(measured) / max(trace[-1]["t"] - t_from, 1e-9),
               "frames_per_s": len(ok) / span, "points_per_s": sum(x[4] for x in ok) / span,
               "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
               "mean_ms": float(np.mean(lat)),
               "mean_queue_ms": float(np.mean([(x[2] - x[1]) * 1e3 for x in ok])),
               "mean_service_ms": float(np.mean([(x[3] - x[2]) * 1e3 for x in ok])),
               "service_mean_s": float(np.mean([x[3] - x[2] for x in ok])),
               "service_m2_s2": float(np.mean([(x[3] - x[2]) ** 2 for x in ok])),
               "service_p99_ms": float(np.percentile([(x[3] - x[2]) * 1e3 for x in ok], 99))}
        # latency by request class (medium edge, resolution): queueing
        # (submission to admission) and service (admission to completion)
        by = {}
        for key in sorted({(x[5], tuple(x[6])) for x in ok}):
            sel = [x for x in ok if (x[5], tuple(x[6])) == key]
            ql = np.array([x[2] - x[1] for x in sel]) * 1e3
            sv = np.array([x[3] - x[2] for x in sel]) * 1e3
            by["%d^3 %dx%d" % (key[0], key[1][0], key[1][1])] = {
                "n": len(sel), "queue_p50_ms": float(np.percentile(ql, 50)),
                "queue_p99_ms": float(np.percentile(ql, 99)), "service_p50_ms": float(np.percentile(sv, 50)),
                "service_p99_ms": float(np.percentile(sv, 99))}
        out["by_class"] = by
        return out

    ctx.server_start(args.serve_budget_gb << 30, "bf16", args.serve_inflight)
    try:
        # warm every slot with a 1080p frame of the largest medium (allocations)
        warm = [dict(t=0.0, n=512, res=(1920, 1080), light=(0.3, 0.9, 0.3), g=0.85, seed=i)
                for i in range(args.serve_inflight)]
        run(warm)
        # service times of requests that never share the device (one every
        # 50 ms, the same mix): the moments of the M/G/1 estimate below
        iso = configs.serving_trace(4.0, rate=60.0, seed=9)
        for i, r in enumerate(iso):
            r["t"] = 0.05 * i
        isolated = run(iso)
        trace = configs.serving_trace(args.serve_warmup + args.serve_seconds, rate=args.serve_rate, seed=7)
        log("serving: %d requests over %.1fs (%.1fs warm-up) at %.0f req/s"
            % (len(trace), args.serve_warmup + args.serve_seconds, args.serve_warmup, args.serve_rate))
        offered = run(trace, args.serve_warmup)
        log("serving: offered %s" % json.dumps(offered))
        # the same mix at 70% of the rate the device sustained, for latency
        # percentiles that are not dominated by a growing queue
        rate = 0.7 * offered["frames_per_s"]
        trace2 = configs.serving_trace(args.serve_warmup + args.serve_sustained_seconds, rate=rate, seed=8)
        sustained = run(trace2, args.serve_warmup)
        log("serving: sustained %s" % json.dumps(sustained))
        # Pollaczek-Khinchine: a single server fed Poisson arrivals at rate
        # lambda waits lambda E[S^2] / (2 (1 - rho)) on average, rho = lambda E[S]
        es, es2 = isolated["service_mean_s"], isolated["service_m2_s2"]
        rho = rate * es
        mg1 = {"isolated_service_mean_ms": es * 1e3, "isolated_service_p99_ms": isolated["service_p99_ms"],
               "isolated_service_m2_ms2": es2 * 1e6, "rho": rho,
               "predicted_mean_wait_ms": rate * es2 / (2 * (1 - rho)) * 1e3 if rho < 1 else None,
               "measured_mean_latency_minus_isolated_service_ms": sustained["mean_ms"] - es * 1e3}
        log("serving: M/G/1 %s" % json.dumps(mg1))
    finally:
        ctx.server_stop()
    for m in mids.values():
        ctx.unload_medium(m)
    return {"config": "Poisson arrivals (trace seed 7; %gs measured after a %gs warm-up); media 64^3/128^3/256^3/"
                      "512^3 fBm, seeds 101-104 (resident); 256^2/720p/1080p pinhole; random light and g in "
                      "[0.3,0.95]; bf16; %d frames in flight; budget %d GB"
                      % (args.serve_seconds, args.serve_warmup, args.serve_inflight, args.serve_budget_gb),
            "latency": "submission to observed completion, host steady clock",
            "at_%g_rps" % args.serve_rate: offered,
            "at_70pct_capacity": dict(sustained, rate_rps=rate),
            "mg1_at_70pct": mg1}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the hot path runs on one GPU; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2401_14051_amd import nis
    from workloads import camera, configs

    wl = configs.BY_NAME[args.workload]
    t0 = time.time()
    density = wl.density()
    o, d = wl.rays()
    pts, dirs, pix = camera.delta_track(density, wl.sigma_t, o, d, seed=wl.point_seed)
    params = wl.params()
    npix = o.shape[0]
    log("workload %s: %d^3 medium, %d pixels, %d points (%.1fs)" % (wl.name, wl.n, npix, len(pts),
                                                                   time.time() - t0))

    ctx = nis.Context(0)
    mid = ctx.load_medium(density, wl.sigma_t, wl.albedo, wl.g)
    ctx.set_light(mid, wl.light, wl.radiance)
    ctx.set_weights(params)
    # the FP8 backbone's static activation scales, calibrated with the FP32
    # path on a seeded subset of the frame's collisions
    crng = np.random.default_rng(11)
    cidx = np.sort(crng.choice(len(pts), min(65536, len(pts)), replace=False))
    ctx.calibrate_fp8(mid, torch.from_numpy(np.ascontiguousarray(pts[cidx], np.float32)).cuda(),
                      torch.from_numpy(np.ascontiguousarray(dirs[cidx], np.float32)).cuda())
    cam = frame_camera(nis, wl)
    stream = torch.cuda.Stream()
    img = torch.empty(npix, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()

    def step():
        ctx.rebuild_pyramid(mid, stream.cuda_stream)
        ctx.set_light(mid, wl.light, wl.radiance)
        ctx.render(mid, cam, wl.point_seed, out=img, stream=stream.cuda_stream)

    def run(prec, steps, warmup):
        ctx.set_precision(prec)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        w0 = time.perf_counter()
        ev[0].record(stream)
        for i in range(steps):
            step()
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        ms = ev[0].elapsed_time(ev[steps]) / steps
        per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
        return ms, wall, per

    res = {}
    precs = [args.precision] + ([p for p in ("bf16", "fp8", "fp32") if p != args.precision]
                                if args.compare_fp32 else [])
    per_frame = {}
    for prec in precs:
        ms, wall, per_frame[prec] = run(prec, args.steps, args.warmup)
        ctx.profile(True)
        nprof = max(3, min(args.steps, 10))
        for _ in range(nprof):
            step()
        torch.cuda.synchronize()
        rep = ctx.profile_report()
        ctx.profile(False)
        # time per frame of each kernel (a frame of more points than one pass
        # holds launches the features and backbone kernels once per pass)
        res[prec] = {"ms": ms, "wall_s": wall, "kernels": {k: v[1] / nprof for k, v in rep.items()},
                     "launches_per_frame": {k: v[0] / nprof for k, v in rep.items()}}
        log("%s: %.3f ms/frame, kernels %s" % (prec, ms, {k: round(v, 4) for k, v in res[prec]["kernels"].items()}))

    # the headline precision's fps three ways: the light changed every frame
    # (the steps above), a static light (rays and query only), and the query of
    # the frame's collision points alone (no camera rays)
    ctx.set_precision(args.precision)
    tp = torch.from_numpy(np.ascontiguousarray(pts, np.float32)).cuda()
    td = torch.from_numpy(np.ascontiguousarray(dirs, np.float32)).cuda()
    tl = torch.empty(len(pts), dtype=torch.float32, device="cuda")
    nmode = max(3, min(args.steps, 10))

    def timed_mode(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(nmode):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / nmode

    ms_static = timed_mode(lambda: ctx.render(mid, cam, wl.point_seed, out=img, stream=stream.cuda_stream))
    ms_query = timed_mode(lambda: ctx.query_device(mid, tp, td, tl, stream=stream.cuda_stream))
    # the paper's own use: the network evaluated at 4129 template centres
    # sampled uniformly in the medium, with and without a light change
    cp, cd = camera.random_points(4129, seed=17, lo=0.0, hi=1.0)
    tcp = torch.from_numpy(np.ascontiguousarray(cp, np.float32)).cuda()
    tcd = torch.from_numpy(np.ascontiguousarray(cd, np.float32)).cuda()
    tcl = torch.empty(len(cp), dtype=torch.float32, device="cuda")
    ms_tpl = timed_mode(lambda: ctx.query_device(mid, tcp, tcd, tcl, stream=stream.cuda_stream))

    def tpl_light():
        ctx.set_light(mid, wl.light, wl.radiance)
        ctx.query_device(mid, tcp, tcd, tcl, stream=stream.cuda_stream)

    ms_tpl_light = timed_mode(tpl_light)
    template_batch = {"points": len(cp), "ms_static_light": ms_tpl, "ms_light_change": ms_tpl_light}
    log("4129 template centres: %.3f ms (static light), %.3f ms (light change)" % (ms_tpl, ms_tpl_light))
    # the same across media: 4129 centres in each of four media (this frame's
    # 256^3 cloud twice, with other centres, and 128^3 and 64^3 clouds, seeds
    # 102 and 101, each under its own light), as one batched query and as
    # four single queries (static lights)
    from workloads import medium as wmedium
    extra = [ctx.load_medium(wmedium.fbm_cloud(nn, seed=sd), wl.sigma_t, wl.albedo, wl.g) for nn, sd in ((128, 102), (64, 101))]
    ctx.set_light(extra[0], (-0.7, 0.2, 0.4), 1.0)
    ctx.set_light(extra[1], (0.1, -0.3, -0.95), 1.0)
    bq = []
    for i, m in enumerate([mid, extra[0], extra[1], mid]):
        q, qd = camera.random_points(4129, seed=31 + i, lo=0.0, hi=1.0)
        bq.append((m, torch.from_numpy(np.ascontiguousarray(q, np.float32)).cuda(),
                   torch.from_numpy(np.ascontiguousarray(qd, np.float32)).cuda(),
                   torch.empty(4129, dtype=torch.float32, device="cuda")))
    ms_batch = timed_mode(lambda: ctx.query_batch(bq, stream=stream.cuda_stream))

    def singles():
        for m, q, qd, o in bq:
            ctx.query_device(m, q, qd, o, stream=stream.cuda_stream)

    ms_singles = timed_mode(singles)
    template_batch["four_media"] = {"points": 4 * 4129, "ms_one_batched_query": ms_batch,
                                    "ms_four_single_queries": ms_singles}
    log("4 x 4129 centres over 4 media: %.3f ms batched, %.3f ms as single queries" % (ms_batch, ms_singles))
    for m in extra:
        ctx.unload_medium(m)
    fps_modes = {"light_change_full_frame": 1000.0 / res[args.precision]["ms"],
                 "static_light_full_frame": 1000.0 / ms_static,
                 "static_light_query_only": 1000.0 / ms_query}
    log("fps: light change %.1f, static light %.1f, query only %.1f" % tuple(fps_modes.values()))

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # parity of the rendered frame on a seeded sample of its hit pixels,
    # against the FP64 oracle at the generator's collision points
    from oracle import oracle
    f32 = lambda x: float(np.float32(x))
    om = oracle.Medium(density)
    om.set_light(np.asarray(wl.light, np.float32))
    op = dict(params)
    op["lam"] = f32(params["lam"])
    rng = np.random.default_rng(123)
    sidx = np.sort(rng.choice(len(pts), min(args.parity_sample, len(pts)), replace=False))
    t_par = time.perf_counter()
    oref = om.query(op, pts[sidx], dirs[sidx], f32(wl.sigma_t), f32(wl.albedo), f32(wl.g), f32(wl.radiance))
    log("oracle at %d sampled collisions: %.1fs" % (len(sidx), time.perf_counter() - t_par))
    ref = f32(wl.albedo) * oref["L"]
    errs, errs_f = {}, {}
    sp = torch.from_numpy(np.ascontiguousarray(pts[sidx], np.float32)).cuda()
    sd = torch.from_numpy(np.ascontiguousarray(dirs[sidx], np.float32)).cuda()
    for prec in precs:
        ctx.set_precision(prec)
        step()
        torch.cuda.synchronize()
        got = img.cpu().numpy()[pix[sidx]].astype(np.float64)
        errs[prec] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        # the network's part alone, F = albedo^gamma expm1(y)
        _, y = ctx.network(mid, sp, sd, want_desc=False)
        fh = f32(wl.albedo) ** params["gamma"] * np.expm1(y.cpu().numpy().astype(np.float64))
        errs_f[prec] = float(np.linalg.norm(fh - oref["F"]) / np.linalg.norm(oref["F"]))
    miss = np.ones(npix, bool)
    miss[pix] = False
    misses_zero = bool(np.all(img.cpu().numpy()[miss] == 0.0))

    # radiance rel-L2 per precision over the HG asymmetries of the precision
    # workload, at a smaller seeded subset of the same collisions (device
    # query, medium g changed in place; the light fields do not depend on g)
    errs_g = {}
    gidx = np.sort(rng.choice(len(sidx), min(args.parity_sample_by_g, len(sidx)), replace=False))
    gp, gd = pts[sidx][gidx], dirs[sidx][gidx]
    tgp = torch.from_numpy(np.ascontiguousarray(gp, np.float32)).cuda()
    tgd = torch.from_numpy(np.ascontiguousarray(gd, np.float32)).cuda()
    sl = torch.empty(len(gidx), dtype=torch.float32, device="cuda")
    for g in G_SWEEP:
        ctx.set_medium_params(mid, wl.sigma_t, wl.albedo, g)
        rg = om.query(op, gp, gd, f32(wl.sigma_t), f32(wl.albedo), f32(g), f32(wl.radiance))["L"]
        errs_g[str(g)] = {}
        for prec in precs:
            ctx.set_precision(prec)
            ctx.query_device(mid, tgp, tgd, sl)
            torch.cuda.synchronize()
            got = sl.cpu().numpy().astype(np.float64)
            errs_g[str(g)][prec] = float(np.linalg.norm(got - rg) / np.linalg.norm(rg))
        log("g = %s: rel-L2 %s" % (g, ", ".join("%s %.2e" % kv for kv in errs_g[str(g)].items())))
    ctx.set_medium_params(mid, wl.sigma_t, wl.albedo, wl.g)
    ctx.set_precision(args.precision)

    # the paper's own templates and backbone modules over the same collisions
    paper = None
    if args.paper_path and args.workload == "frame":
        paper = paper_path(ctx, mid, wl, params, pts, dirs, tp, td, stream, args.precision, om,
                           args.paper_sample, np.random.default_rng(321))
        if args.precision == "fp8":
            ctx.calibrate_fp8(mid, torch.from_numpy(np.ascontiguousarray(pts[cidx], np.float32)).cuda(),
                              torch.from_numpy(np.ascontiguousarray(dirs[cidx], np.float32)).cuda())

    # oracle throughput on the host cores (bounded sample, median of runs)
    cpu = None
    if args.cpu_sample > 0:
        cpu = cpu_baseline(args, om, op, wl, pts, dirs, rng)

    prec = args.precision
    ms = res[prec]["ms"]
    levels = len(ctx.pyramid(mid))
    geom = []
    for m in range(levels):
        D, (ulo, uhi, vlo, vhi) = ctx.path_density(mid, m)
        geom.append((uhi - ulo + 1, vhi - vlo + 1, D.shape[0]))
    work = kernel_work(wl, levels, geom, npix, len(pts), params["width"], params["n_linear"], prec)
    kernels = {}
    for k, t_ms in res[prec]["kernels"].items():
        w = work.get(k, {})
        ent = {"ms": t_ms}
        if "bytes" in w:
            ent["GBps"] = w["bytes"] / (t_ms * 1e-3) / 1e9
            ent["hbm_frac"] = ent["GBps"] / HBM_PEAK_GBS
        if "layout_bytes" in w:
            ent["layout_GBps"] = w["layout_bytes"] / (t_ms * 1e-3) / 1e9
        if "flops" in w:
            ent["TFLOPs"] = w["flops"] / (t_ms * 1e-3) / 1e12
            ent["mfma_frac"] = ent["TFLOPs"] / MFMA_PEAK_TFLOPS[prec]
        if "valu_flops" in w:
            ent["valu_TFLOPs"] = w["valu_flops"] / (t_ms * 1e-3) / 1e12
            ent["valu_frac"] = ent["valu_TFLOPs"] / VALU_FP32_TFLOPS
        kernels[k] = ent
    # the whole network (conv + attention inside the gather kernel, backbone):
    # its useful FLOPs over the two kernels' time
    net_ms = res[prec]["kernels"].get("features", 0.0) + res[prec]["kernels"].get("backbone", 0.0)
    net_flops = work["features"]["flops"] + work["backbone"]["flops"]
    network = {"flops_per_point": net_flops / len(pts), "ms": net_ms,
               "TFLOPs": net_flops / (net_ms * 1e-3) / 1e12,
               "mfma_frac": net_flops / (net_ms * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS[prec]}
    dom = max(res[prec]["kernels"], key=lambda k: res[prec]["kernels"][k])
    dk = kernels[dom]
    if "flops" in work.get(dom, {}) and "valu_flops" not in work.get(dom, {}):
        roof = {"kernel": dom, "bound": "mfma", "achieved": dk["TFLOPs"], "peak": MFMA_PEAK_TFLOPS[prec],
                "unit": "TFLOP/s", "frac": dk["mfma_frac"], "traffic": None}
    else:
        # the gather (and any other kernel) against HBM on its algorithmic
        # bytes; for the gather also its vector-ALU and conv MFMA fractions
        roof = {"kernel": dom, "bound": "hbm", "achieved": dk["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dk["hbm_frac"], "traffic": None}
        if "valu_frac" in dk:
            roof.update({"algorithmic_bytes": work[dom]["bytes"], "valu_achieved_TFLOPs": dk["valu_TFLOPs"],
                         "valu_peak_TFLOPs": VALU_FP32_TFLOPS, "valu_frac": dk["valu_frac"],
                         "conv_mfma_frac": dk["mfma_frac"]})
    roof["traffic"] = measured_traffic(dom, prec, args.workload)

    serve = None
    if args.serve_seconds > 0:
        ctx.set_weights(configs.FRAME.params())
        serve = serving(ctx, nis, args)

    line = {
        "metric": "shading points/sec (1080p frame of a 256^3 fBm cloud, light change every frame)",
        "value": len(pts) / (ms * 1e-3),
        "unit": "shading points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic (seeded fBm cloud, delta-tracked camera rays on the GPU, He-init weights)",
        "config": {"workload": "%s: %d^3 fBm cloud, %dx%d camera, %d shading points, backbone %dx%d, %s"
                               % (wl.name, wl.n, wl.res[0], wl.res[1] if wl.cam != "ortho" else wl.res[0],
                                  len(pts), params["n_linear"], params["width"], prec),
                   "points": len(pts), "pixels": npix},
        "fps": 1000.0 / ms,
        "rel_l2_vs_fp64_oracle": {p: errs[p] for p in precs},
        "rel_l2_F_vs_fp64_oracle": {p: errs_f[p] for p in precs},
        "rel_l2_vs_fp64_oracle_by_g": errs_g,
        "frame_ms": {p: {"median": float(np.median(per_frame[p])), "p99": float(np.percentile(per_frame[p], 99))}
                     for p in precs},
        "fps_modes": fps_modes,
        "template_batch": template_batch,
        "paper_templates_and_modules": paper,
        "misses_are_zero": misses_zero,
        "per_precision": {p: {"ms_per_step": res[p]["ms"], "points_per_s": len(pts) / (res[p]["ms"] * 1e-3),
                              "fps": 1000.0 / res[p]["ms"], "kernels_ms": res[p]["kernels"]} for p in precs},
        "kernels": kernels,
        "network": network,
        "roofline": roof,
        "cpu_baseline": cpu,
        "serving": serve,
    }
    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()
