"""Throughput benchmark of the in-scattering hot path on one GPU.

A step is one pass of the whole path over one 1080p frame of the 256^3 fBm
cloud (about 1.2M shading points, backbone 10 x 200): rebuild the density
pyramid from the resident grid, apply the light (the transmittance sweep runs
again), then gather, CNN + attention, backbone and decode for every point.
Inputs are resident in device memory before the timed region starts.

Prints one JSON line: shading points/s (whole job), ms per step, 1080p frames/s,
per-kernel times from HIP events recorded by the library on the stream its
kernels run on, the roofline of the dominant kernel, the radiance error against
the FP64 oracle on a seeded sample, and the oracle's own throughput on the host
cores.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}
VALU_FP32_TFLOPS = 78.6   # 256 CUs x 64 lanes x 2 FLOP x 2.4 GHz, without packed FP32

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
    ap.add_argument("--cpu-sample", type=int, default=131072,
                    help="points of the frame the oracle is timed on (0 = skip)")
    ap.add_argument("--parity-sample", type=int, default=2048)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this size (for scaling HBM counters)")
    ap.add_argument("--compare-fp32", action="store_true", default=True)
    ap.add_argument("--no-compare-fp32", dest="compare_fp32", action="store_false")
    return ap.parse_args()


def kernel_work(wl, levels, level_geom, npts, width, n_linear, prec):
    """Algorithmic bytes / FLOPs per launch of each kernel."""
    esize = {"fp32": 4, "bf16": 2, "fp8": 2}[prec]     # the FP8 path stores the descriptor in BF16
    n0 = wl.n
    vox = [(n0 >> m) ** 3 for m in range(levels)]
    samples = sum(nu * nv * n for (nu, nv, n) in level_geom)
    conv_flop = 2 * 12 * (504 * 27 + 80 * 216)                       # per point
    mlp_flop = 2 * (1057 * width + (n_linear - 2) * width * width + width)
    return {
        "pyramid": {"bytes": 4 * sum(vox[:-1]) + 4 * sum(vox[1:])},
        "sweep": {"bytes": 4 * sum(vox) + 4 * samples},
        "site_tables": {"bytes": 225 * 16},
        "features": {"bytes": npts * (24 + 4 + 1088 * esize), "flops": npts * conv_flop,
                     "valu_flops": npts * GATHER_FLOP_PER_POINT},
        "backbone": {"bytes": npts * (1088 * esize + 8), "flops": npts * mlp_flop},
    }


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


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2401_14051_amd import nis
    from workloads import configs

    wl = configs.BY_NAME[args.workload]
    t0 = time.time()
    density = wl.density()
    pts, dirs, _ = wl.points(density)
    params = wl.params()
    print("[bench] workload %s: %d^3 medium, %d points (%.1fs)" % (wl.name, wl.n, len(pts), time.time() - t0),
          file=sys.stderr, flush=True)

    ctx = nis.Context(0)
    mid = ctx.load_medium(density, wl.sigma_t, wl.albedo, wl.g)
    ctx.set_light(mid, wl.light, wl.radiance)
    ctx.set_weights(params)
    stream = torch.cuda.Stream()
    dp = torch.from_numpy(pts).cuda()
    dd = torch.from_numpy(dirs).cuda()
    out = torch.empty(len(pts), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()

    def step():
        ctx.rebuild_pyramid(mid, stream.cuda_stream)
        ctx.set_light(mid, wl.light, wl.radiance)
        ctx.query_device(mid, dp, dd, out, stream.cuda_stream)

    def run(prec, steps, warmup):
        ctx.set_precision(prec)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        ms = e0.elapsed_time(e1) / steps
        return ms, wall

    res = {}
    precs = [args.precision] + ([p for p in ("bf16", "fp8", "fp32") if p != args.precision]
                                if args.compare_fp32 else [])
    for prec in precs:
        ms, wall = run(prec, args.steps, args.warmup)
        ctx.profile(True)
        for _ in range(max(3, min(args.steps, 10))):
            step()
        torch.cuda.synchronize()
        rep = ctx.profile_report()
        ctx.profile(False)
        res[prec] = {"ms": ms, "wall_s": wall, "kernels": {k: v[1] / v[0] for k, v in rep.items()},
                     "launches": {k: v[0] for k, v in rep.items()}}
        print("[bench] %s: %.3f ms/step, kernels %s" % (prec, ms, {k: round(v, 4) for k, v in
                                                                 res[prec]["kernels"].items()}),
              file=sys.stderr, flush=True)

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # parity on a seeded sample, against the FP64 oracle
    from oracle import oracle
    f32 = lambda x: float(np.float32(x))
    om = oracle.Medium(density)
    t_sw = time.perf_counter()
    om.set_light(np.asarray(wl.light, np.float32))
    t_sweep = time.perf_counter() - t_sw
    op = dict(params)
    op["lam"] = f32(params["lam"])
    rng = np.random.default_rng(123)
    sidx = np.sort(rng.choice(len(pts), min(args.parity_sample, len(pts)), replace=False))
    ref = om.query(op, pts[sidx], dirs[sidx], f32(wl.sigma_t), f32(wl.albedo), f32(wl.g), f32(wl.radiance))
    errs = {}
    for prec in precs:
        ctx.set_precision(prec)
        step()
        torch.cuda.synchronize()
        got = out.cpu().numpy()[sidx].astype(np.float64)
        errs[prec] = float(np.linalg.norm(got - ref["L"]) / np.linalg.norm(ref["L"]))

    # oracle throughput on the host cores (bounded sample)
    cpu = None
    if args.cpu_sample > 0:
        cidx = np.sort(rng.choice(len(pts), min(args.cpu_sample, len(pts)), replace=False))
        tq = time.perf_counter()
        om.query(op, pts[cidx], dirs[cidx], f32(wl.sigma_t), f32(wl.albedo), f32(wl.g), f32(wl.radiance))
        tq = time.perf_counter() - tq
        frame_s = t_sweep + tq * len(pts) / len(cidx)
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cpu = {"value": len(pts) / frame_s, "unit": "shading points/s", "cores": cores, "kind": "oracle",
               "sample": "FP64 oracle: full-resolution sweep (%.2fs, 1 thread) plus a seeded %d-point subset "
                         "of the frame (%.2fs on %d threads), scaled to the frame's %d points"
                         % (t_sweep, len(cidx), tq, cores, len(pts))}

    prec = args.precision
    ms = res[prec]["ms"]
    levels = len(ctx.pyramid(mid))
    geom = []
    for m in range(levels):
        D, (ulo, uhi, vlo, vhi) = ctx.path_density(mid, m)
        geom.append((uhi - ulo + 1, vhi - vlo + 1, D.shape[0]))
    work = kernel_work(wl, levels, geom, len(pts), params["width"], params["n_linear"], prec)
    kernels = {}
    for k, t_ms in res[prec]["kernels"].items():
        w = work.get(k, {})
        ent = {"ms": t_ms}
        if "bytes" in w:
            ent["GBps"] = w["bytes"] / (t_ms * 1e-3) / 1e9
            ent["hbm_frac"] = ent["GBps"] / HBM_PEAK_GBS
        if "flops" in w:
            ent["TFLOPs"] = w["flops"] / (t_ms * 1e-3) / 1e12
            ent["mfma_frac"] = ent["TFLOPs"] / MFMA_PEAK_TFLOPS[prec]
        if "valu_flops" in w:
            ent["valu_TFLOPs"] = w["valu_flops"] / (t_ms * 1e-3) / 1e12
            ent["valu_frac"] = ent["valu_TFLOPs"] / VALU_FP32_TFLOPS
        kernels[k] = ent
    dom = max(res[prec]["kernels"], key=lambda k: res[prec]["kernels"][k])
    dk = kernels[dom]
    if dom == "features":
        # the gather's interpolation arithmetic runs on the vector ALUs; the two
        # small convolutions (conv_flop) run on MFMA and are reported beside it
        roof = {"kernel": dom, "bound": "alu", "achieved": dk["valu_TFLOPs"], "peak": VALU_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": dk["valu_frac"], "traffic": None}
    elif "flops" in work.get(dom, {}):
        roof = {"kernel": dom, "bound": "mfma", "achieved": dk["TFLOPs"], "peak": MFMA_PEAK_TFLOPS[prec],
                "unit": "TFLOP/s", "frac": dk["mfma_frac"], "traffic": None}
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": dk["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dk["hbm_frac"], "traffic": None}
    roof["traffic"] = measured_traffic(dom, prec, args.workload)

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
        "data": "synthetic (seeded fBm cloud, delta-tracked 1080p camera points, He-init weights)",
        "config": {"workload": "%s: %d^3 fBm cloud, %dx%d camera, %d shading points, backbone %dx%d, %s"
                               % (wl.name, wl.n, wl.res[0], wl.res[1], len(pts), params["n_linear"],
                                  params["width"], prec),
                   "points": len(pts)},
        "fps": 1000.0 / ms,
        "rel_l2_vs_fp64_oracle": {p: errs[p] for p in precs},
        "per_precision": {p: {"ms_per_step": res[p]["ms"], "points_per_s": len(pts) / (res[p]["ms"] * 1e-3),
                              "fps": 1000.0 / res[p]["ms"], "kernels_ms": res[p]["kernels"]} for p in precs},
        "kernels": kernels,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()
