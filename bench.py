"""Benchmark of the preconditioned NCG-MLS field-map estimator on one MI355X.

A step is one full solve of the 128x128x64, 8-coil, 3-echo field-map problem
(coil combination, the initial map of eq. (w0) and 100 NCG iterations with
IC(0) and three line-search steps each) on inputs already resident in device
memory.  value = in-mask voxels x iterations / second, whole job.

Progress goes to stderr; stdout carries exactly one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def bytes_per_voxel(kclass, precision, L, ordering, precond):
    """Algorithmic bytes per voxel of one launch of each kernel class: every
    per-voxel array the kernel must read or write once (neighbour values are
    re-used from cache and not counted again; the 1-byte neighbour code is
    counted).  t = working type size, pivots are FP64."""
    t = 4 if precision == "mix" else 8
    code = 1
    if kclass == "grad":      # read echoes (2L t), f, z; write f, g, D
        return code + 2 * L * t + 2 * t + 3 * t
    if kclass == "mls":       # read echoes, f, z
        return code + 2 * L * t + 2 * t
    if kclass == "dots":      # read g, g_prev, p
        return 3 * t
    if kclass == "dir":       # read p, z_prev, f, D; write z
        return code + 5 * t
    if precond == "ic0" and ordering == "natural":
        if kclass == "precond_a":   # read D, g; write 1/pivot (8), x
            return code + 2 * t + 8 + t
        if kclass == "precond_b":   # read x, 1/pivot; write p
            return code + t + 8 + t
    if precond == "ic0" and ordering == "redblack":
        if kclass == "precond_a":   # read D, g; write 1/pivot (8), p (black)
            return code + 2 * t + 8 + t
        if kclass == "precond_b":   # read g, 1/pivot, p; write p (red)
            return code + t + 8 + 2 * t
    if kclass == "precond_a":       # diagonal / identity: read D, g; write 1/pivot, p
        return code + 2 * t + 8 + t
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["mix", "f64"], default="mix")
    ap.add_argument("--ordering", choices=["natural", "redblack"], default="natural")
    ap.add_argument("--precond", choices=["ic0", "diag", "none"], default="ic0")
    ap.add_argument("--mask", choices=["full", "paper"], default="full")
    ap.add_argument("--shape", default="128,128,64")
    ap.add_argument("--kernel-iters", type=int, default=10)
    ap.add_argument("--cpu-iters", type=int, default=25)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2005_08661_amd import fmap, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    shape = tuple(int(s) for s in args.shape.split(","))
    log("generating %s volume (%s mask)" % (shape, args.mask))
    vol = synth.mid_fieldmap(mask=args.mask, shape=shape)
    prec = fmap.MIX if args.precision == "mix" else fmap.F64
    order = fmap.NATURAL if args.ordering == "natural" else fmap.REDBLACK
    pc = {"ic0": fmap.IC0, "diag": fmap.DIAG, "none": fmap.NONE}[args.precond]
    y, s, m = fmap.to_device(vol)
    plan = fmap.Plan(fmap.params_for(vol, precision=prec, ordering=order, precond=pc))
    out = torch.zeros(shape, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        plan.solve(y, s, m, out=out)
    torch.cuda.synchronize()
    niter = vol.niter

    log("timing %d steps" % args.steps)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        plan.solve(y, s, m, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = ev0.elapsed_time(ev1) / max(args.steps, 1)
    tr = plan.trace()
    nmask = plan.mask_count()
    value = nmask * niter / (ms_step * 1e-3)
    log("step %.3f ms (wall %.3f ms), %.3e voxel-iterations/s" % (ms_step, wall * 1e3 / args.steps, value))

    # iteration loop alone (graph replays), from the solved state
    ev0.record(stream)
    plan.iterate(niter, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_loop = ev0.elapsed_time(ev1)
    loop_rate = nmask * niter / (ms_loop * 1e-3)

    # per-kernel durations from HIP events on the launch stream
    kt = plan.time_kernels(args.kernel_iters)
    L = vol.necho
    kinfo = {}
    for k, (ms, nl) in kt.items():
        if nl == 0:
            continue
        b = bytes_per_voxel(k, args.precision, L, args.ordering, args.precond) * vol.mask.size
        avg = ms / nl
        kinfo[k] = dict(avg_us=avg * 1e3, launches=nl, total_ms=ms, bytes=b,
                        gbs=b / (avg * 1e-3) / 1e9 if avg > 0 else 0.0)
    dom = max(kinfo, key=lambda k: kinfo[k]["total_ms"])
    iter_bytes = sum(bytes_per_voxel(k, args.precision, L, args.ordering, args.precond) * kinfo[k]["launches"]
                     for k in kinfo) / args.kernel_iters * vol.mask.size
    iter_frac = iter_bytes / (ms_loop * 1e-3 / niter) / (HBM_PEAK_GBS * 1e9)
    for k, v in kinfo.items():
        log("  %-10s %9.2f us/launch  %8.1f GB/s  (%d launches)" % (k, v["avg_us"], v["gbs"], v["launches"]))
    log("loop %.3f ms for %d iterations; whole-iteration %.1f%% of HBM peak" % (ms_loop, niter, 100 * iter_frac))

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        log("cpu baseline: oracle, %d iterations" % args.cpu_iters)
        t0 = time.perf_counter()
        O.run_volume(vol, ordering=order, precond={"ic0": O.IC0, "diag": O.DIAG, "none": O.NONE}[args.precond],
                     niter=args.cpu_iters)
        tc = time.perf_counter() - t0
        cpu = {"value": nmask * args.cpu_iters / tc, "unit": "voxel-iterations/s", "cores": 1, "kind": "oracle",
               "sample": "%dx%dx%d 8 coils: coil combination, eq. (w0) start and %d NCG iterations (FP64, "
                         "single-threaded C), %.1f s" % (shape + (args.cpu_iters, tc))}
        log("cpu %.3e voxel-iterations/s" % cpu["value"])

    line = {
        "metric": "NCG+IC voxel-iterations/s and % HBM roofline at 128×128×64×8 coils",
        "value": value,
        "unit": "voxel-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mix" else "f64",
        "data": "synthetic",
        "config": {
            "workload": "field map %dx%dx%d, 8 coils, 3 echoes (0/2.2/4.4 ms), beta 2^-4, %d NCG iterations x %d "
                        "line-search steps, %s preconditioner%s, %s precision, %s mask (%d unknowns); step = "
                        "setup + eq. (w0) start + iterations" % (
                            shape + (niter, vol.nmls, args.precond.upper(),
                                     " (%s order)" % args.ordering if args.precond == "ic0" else "",
                                     args.precision.upper(), args.mask, nmask)),
            "grid": list(shape), "coils": 8, "echoes": L, "niter": niter, "nmls": vol.nmls,
            "precision": args.precision, "ordering": args.ordering, "precond": args.precond,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": kinfo[dom]["gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": kinfo[dom]["gbs"] / HBM_PEAK_GBS,
            "traffic": None,
        },
        "iteration": {
            "loop_ms": ms_loop,
            "loop_voxel_iterations_per_s": loop_rate,
            "bytes_per_iteration": iter_bytes,
            "hbm_frac": iter_frac,
            "kernels_us": {k: round(v["avg_us"], 3) for k, v in kinfo.items()},
        },
        "final_cost": float(tr[-1, 0]),
        "cpu_baseline": cpu,
    }
    plan.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
