"""Benchmark of the preconditioned NCG-MLS field-map estimator on one MI355X.

A step is one full solve of the 128x128x64, 8-coil, 3-echo field-map problem
(coil combination, the initial map of eq. (w0) and 100 NCG iterations with
IC(0) and three line-search steps each) on inputs already resident in device
memory, with the plan's default schedule (resident at this size; the
streaming schedule is timed beside it).  value = in-mask voxels x iterations
/ second, whole job.

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
    """Algorithmic bytes per voxel of one launch of each kernel class: each
    per-voxel array the step must read or write, once, for the voxels it
    concerns (neighbour values come from cache and are not counted again; the
    1-byte neighbour code is counted).  t = working type size; pivots and
    1/h are FP64."""
    t = 4 if precision == "mix" else 8
    rb = precond == "ic0" and ordering == "redblack"
    if kclass == "grad":       # read code, echoes, f, z_prev; write f, g, D (+ 1/h of red voxels)
        return 1 + 2 * L * t + 5 * t + (4 if rb else 0)
    if kclass == "mls":        # read code, echoes, f, z
        return 1 + 2 * L * t + 2 * t
    if kclass == "dir":        # read code, p, z_prev, f, D; write z
        return 1 + 5 * t
    if precond == "ic0" and ordering in ("natural", "blockrb"):  # block red-black: same arrays, one tile at a time
        if kclass == "precond_a":  # read code, D, g; write 1/P (8), x
            return 1 + 3 * t + 8
        if kclass == "precond_b":  # read code, x, 1/P (8), g, g_prev; write p
            return 1 + 4 * t + 8
    if rb:
        # black pass with both dot products: D, p of black; g, g_prev of all; 1/h of red
        if kclass == "precond_a":
            return 1 + 3 * t + 4
        # red pass fused with the direction: g, 1/h of red; p of black; z_prev, f, D of all / z
        if kclass == "precond_b":
            return 1 + 4.5 * t + 4
    if kclass == "precond_a":      # diagonal / identity: read code, D, g, g_prev; write 1/h (8), p
        return 1 + 4 * t + 8
    return 0


def alg_bytes_per_voxel(precision, L, nmls):
    """B_alg: the minimum global sweeps the method's data dependencies force per
    voxel and NCG iteration, independent of how the kernels are split: forward
    sweep (echo data, f, z_prev in; f, g, D, pivot (FP64), x out), backward
    sweep (x, pivot, g, g_prev, z_prev in; p out), direction and line-search
    setup (p, z_prev, f, D in; z out), and nmls - 1 line-search passes (echo
    data, f, z).  MIX, L = 3, nmls = 3: 168 B."""
    if precision == "mix":
        return (8 * L + 32) + 28 + 20 + (nmls - 1) * (8 * L + 8)
    return (16 * L + 56) + 48 + 40 + (nmls - 1) * (16 * L + 16)


def iteration_bytes_per_voxel(precision, L, ordering, precond, nmls):
    """Bytes per voxel of one whole iteration as this implementation's passes
    move them (sum of the per-pass model above)."""
    rb = precond == "ic0" and ordering == "redblack"
    b = bytes_per_voxel("grad", precision, L, ordering, precond) + bytes_per_voxel("precond_a", precision, L, ordering,
                                                                                  precond)
    if precond == "ic0":
        b += bytes_per_voxel("precond_b", precision, L, ordering, precond)
    if not rb:
        b += bytes_per_voxel("dir", precision, L, ordering, precond)
    return b + (nmls - 1) * bytes_per_voxel("mls", precision, L, ordering, precond)


KERNEL_SYMBOL = {"grad": "k_grad", "mls": "k_mls", "dir": "k_dir", "precond_a": None, "precond_b": None,
                 "resident": "k_resident"}


def kernel_symbol(kclass, ordering, precond, nz):
    if kclass in ("precond_a", "precond_b"):
        if precond != "ic0":
            return "k_diag"
        if ordering == "natural":
            return "k_ic_fwd_wave" if kclass == "precond_a" else "k_ic_bwd_wave"
        if ordering == "blockrb":
            return "k_icb_fwd" if kclass == "precond_a" else "k_icb_bwd"
        pair = "_pair" if nz % 2 == 0 else ""  # pair-mapped passes when every column length is even
        return ("k_rb_black" if kclass == "precond_a" else "k_rb_red_dir") + pair
    return KERNEL_SYMBOL[kclass]


def measured_traffic(kclass, args):
    """HBM bytes per launch of the kernel from the committed counter summary,
    or None if there is none for this workload or the sources changed since."""
    from paper_2005_08661_amd.prof_summary import source_hash
    path = os.path.join(ROOT, "profiles", "counters_fieldmap_%s_%s_%s.json" % (
        args.shape.replace(",", "x"), args.precision, args.ordering if args.precond == "ic0" else args.precond))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != source_hash():
        return None
    sym = kernel_symbol(kclass, args.ordering, args.precond, int(args.shape.split(",")[2]))
    for name, v in rec["kernels"].items():
        if sym and ("fm::%s<" % sym) in name:
            return v["traffic_bytes"]
    return None


def copy_rate_gbs(torch, mbytes=1024, reps=10):
    """Read + write rate of a plain device copy of mbytes MB (torch's copy kernel): the
    practical streaming ceiling of the HBM, measured beside the published peak."""
    n = mbytes * 1048576 // 4
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    del a, b
    return 2 * mbytes * 1048576 / (ms * 1e-3) / 1e9


def flip_threshold(te):
    """Half the period of the phase-wrap ambiguity of the closest echo pair, 1/(2 min |t_m - t_n|): a voxel
    that differs by more than this between two maps sits in another local minimum (a basin flip)."""
    te = np.asarray(te, dtype=np.float64)
    return 1.0 / (2.0 * min(abs(te[m] - te[n]) for m in range(len(te)) for n in range(m + 1, len(te))))


def map_diff(a, b, mask, thr):
    d = (np.asarray(a) - np.asarray(b))[mask]
    return {"rms_hz": float(np.sqrt(np.mean(d ** 2))), "max_abs_hz": float(np.abs(d).max()),
            "basin_flips": int(np.count_nonzero(np.abs(d) > thr))}


def host_threads():
    """Threads for the all-cores oracle run: the CPUs this process may run on, capped by OMP_NUM_THREADS when
    the environment sets it (the host's share of cores)."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def bench_cpu(args, vol, synth, batched_vols, headline):
    """The FP64 oracle on the host (a -O3 -march=native copy compiled here), on 1 thread and on all threads:
    the headline volume in full on all threads, which also gives the parity of the GPU maps, and a
    20-iteration sample on 1 thread; the small volume (32x32x16, 1 coil, 50 iterations, natural-order IC(0)) in
    full on both; the 16 uneven volumes for 3 iterations per volume on both.  The oracle's parallel loops
    are those over independent voxels; its sums stay sequential, so every thread count gives the same bits."""
    import tempfile

    import oracle as O
    from oracle import build as obuild

    tmp = tempfile.mkdtemp(prefix="fmo_native_")
    O.use_library(obuild.build_native(tmp))
    nall = host_threads()
    affinity = len(os.sched_getaffinity(0))
    log("cpu baseline: oracle -O3 -march=native, 1 and %d threads (%d CPUs in the affinity mask)" % (nall, affinity))
    order = {"natural": O.NATURAL, "redblack": O.REDBLACK, "blockrb": O.BLOCKRB}[args.ordering]
    pc = {"ic0": O.IC0, "diag": O.DIAG, "none": O.NONE}[args.precond]

    def run(v, nt, niter, ordering=order, precond=pc):
        O.set_threads(nt)
        t0 = time.perf_counter()
        r = O.run_volume(v, ordering=ordering, precond=precond, niter=niter)
        return r, time.perf_counter() - t0

    out = {"affinity_cpus": affinity, "threads_all": nall, "build": "gcc -O3 -march=native -fopenmp "
                                                                      "-ffp-contract=off"}
    nmask = int(vol.mask.sum())
    # the headline volume: full solve on all threads (the parity reference), 20-iteration sample on one thread
    ref, t_all = run(vol, nall, vol.niter)
    _, t_one = run(vol, 1, 20)
    out["headline"] = {"all_threads": {"value": nmask * vol.niter / t_all, "seconds": t_all, "niter": vol.niter},
                      "one_thread": {"value": nmask * 20 / t_one, "seconds": t_one, "niter": 20}}
    log("cpu headline volume: %.3e voxel-iterations/s on %d threads (100 iterations, %.1f s), %.3e on 1 thread "
        "(20 iterations, %.1f s)" % (out["headline"]["all_threads"]["value"], nall, t_all,
                                     out["headline"]["one_thread"]["value"], t_one))
    # the small volume (32x32x16, 1 coil)
    tiny = synth.tiny_fieldmap()
    n1 = int(tiny.mask.sum())
    _, t1a = run(tiny, nall, tiny.niter, O.NATURAL, O.IC0)
    _, t11 = run(tiny, 1, tiny.niter, O.NATURAL, O.IC0)
    out["small_32x32x16"] = {"voxels": n1, "niter": tiny.niter, "all_threads": n1 * tiny.niter / t1a,
                      "one_thread": n1 * tiny.niter / t11}
    log("cpu 32x32x16 volume: %.3e (all) / %.3e (1 thread) voxel-iterations/s" % (out["small_32x32x16"]["all_threads"],
                                                                        out["small_32x32x16"]["one_thread"]))
    # the 16 uneven volumes: every volume, 3 iterations
    vols4 = batched_vols if batched_vols is not None else synth.batched(16)
    n4 = sum(int(v.mask.sum()) for v in vols4)
    rates = {}
    for name, nt in (("all_threads", nall), ("one_thread", 1)):
        t = 0.0
        for v in vols4:
            t += run(v, nt, 3, O.REDBLACK, O.IC0)[1]
        rates[name] = n4 * 3 / t
    out["batch16"] = dict(voxels=n4, niter=3, **rates)
    log("cpu 16 uneven volumes: %.3e (all) / %.3e (1 thread) voxel-iterations/s" % (rates["all_threads"],
                                                                        rates["one_thread"]))
    O.set_threads(nall)
    # parity of the GPU maps against the oracle's full run (Sec. III Algorithm, same fixed iteration counts)
    m = vol.mask.astype(bool)
    thr = flip_threshold(vol.te)
    rt = ref["trace"]
    par = {"reference": "FP64 oracle, %d iterations, %s IC(0), same seeded inputs" % (vol.niter, args.ordering),
           "flip_threshold_hz": thr}
    for tag, (f, tr) in headline.items():
        d = map_diff(f, ref["f"], m, thr)
        d["restart_mismatches"] = int(np.count_nonzero(tr[:-1, 3] != rt[:-1, O.TR["restart"]]))
        d["cost_max_rel_diff"] = float(np.max(np.abs(tr[:, 0] - rt[:, O.TR["cost"]]) / np.abs(rt[:, O.TR["cost"]])))
        par[tag] = d
        log("parity %s vs oracle: rms %.3e Hz, max %.3e Hz, %d basin flips, %d restart mismatches" % (
            tag, d["rms_hz"], d["max_abs_hz"], d["basin_flips"], d["restart_mismatches"]))
    if "mix" in headline and "f64" in headline:
        par["mix_vs_f64"] = map_diff(headline["mix"][0], headline["f64"][0], m, thr)
        log("parity MIX vs F64: rms %.3e Hz" % par["mix_vs_f64"]["rms_hz"])
    cpu = {"value": out["headline"]["all_threads"]["value"], "unit": "voxel-iterations/s", "cores": nall,
           "kind": "oracle",
           "sample": "the headline problem as the GPU step (%dx%dx%d, 8 coils, coil combination, eq. (w0) start, %d NCG "
                     "iterations, FP64 C, %d threads, %.1f s); one thread: %.3e voxel-iterations/s on 20 "
                     "iterations" % (vol.shape + (vol.niter, nall, t_all, out["headline"]["one_thread"]["value"])),
           "detail": out}
    return cpu, par


def roofline_entry(kinfo, dom, traffic):
    """Roofline of the dominant kernel.  The path has no dense contraction and its arithmetic intensity is below
    the FP32 balance of the chip (157.3 TFLOP/s / 8 TB/s = 19.7 flop/B), so its roofline is the HBM one:
    achieved = algorithmic bytes per launch / average launch duration.  `limiter` says what the counters show
    limits the kernel: the bytes that crossed the L2 per launch (FETCH_SIZE + WRITE_SIZE, scaled by a plain
    copy) over the launch duration, as a fraction of the HBM peak; when that is under half of the peak the
    kernel is not waiting on HBM but on latency (grid synchronisation, dependent loads) or issue."""
    k = kinfo[dom]
    ent = {"bound": "hbm", "kernel": dom, "achieved": k["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": k["gbs"] / HBM_PEAK_GBS, "traffic": traffic}
    if traffic:
        meas = traffic / (k["avg_us"] * 1e-6) / 1e9
        ent["measured_gbs"] = meas
        ent["measured_frac"] = meas / HBM_PEAK_GBS
        ent["limiter"] = "hbm bandwidth" if meas >= 0.5 * HBM_PEAK_GBS else \
            "latency and synchronisation (measured traffic %.0f%% of the HBM peak)" % (100 * meas / HBM_PEAK_GBS)
    else:
        ent["limiter"] = None
    return ent


def time_solve(plan, fmap, y, s, m, out, steps, torch):
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        plan.solve(y, s, m, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / max(steps, 1)


def bench_batched(args, fmap, synth, torch, prec):
    """16 uneven volumes (64..160 x 64..160 x 32..96, 4 coils, TE 0/2/5 ms, beta 2^U[-6,-2]):
    one batched solve against a loop of single-volume solves, same precision and ordering."""
    log("batched: generating 16 volumes")
    vols = synth.batched(16)
    dev = [fmap.to_device(v) for v in vols]
    ys, ss, ms = [d[0] for d in dev], [d[1] for d in dev], [d[2] for d in dev]
    nvox = sum(int(v.mask.sum()) for v in vols)
    niter = vols[0].niter
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    prms = [fmap.params_for(v, precision=prec, ordering=fmap.REDBLACK) for v in vols]
    with fmap.Batch(prms) as b:
        grid, tune_ms = b.autotune(ys, ss, ms, probe_iters=3)
        log("batched: autotuned %d workgroups (%.3f ms per iteration)" % (grid, tune_ms))
        outs = b.solve(ys, ss, ms)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            outs = b.solve(ys, ss, ms)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_b = ev0.elapsed_time(ev1) / args.steps
    plans = [fmap.Plan(p) for p in prms]
    louts = [torch.zeros(v.shape, dtype=torch.float64, device="cuda") for v in vols]
    for pl, (y, s, m), o in zip(plans, dev, louts):
        pl.solve(y, s, m, out=o)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        for pl, (y, s, m), o in zip(plans, dev, louts):
            pl.solve(y, s, m, out=o)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_l = ev0.elapsed_time(ev1) / args.steps
    diff = max(float(torch.sqrt(torch.mean(((a - c)[mm.bool()]) ** 2))) for a, c, mm in zip(outs, louts, ms))
    for pl in plans:
        pl.close()
    res = {"volumes": len(vols), "voxels": nvox, "grid": grid, "niter": niter, "precision": args.precision,
           "ms_per_solve": ms_b, "value": nvox * niter / (ms_b * 1e-3),
           "loop_ms_per_solve": ms_l, "loop_value": nvox * niter / (ms_l * 1e-3),
           "speedup_vs_loop": ms_l / ms_b, "max_rms_diff_vs_loop_hz": diff,
           "shapes": [list(v.shape) for v in vols]}
    log("batched: %.3f ms per solve (%.3e voxel-iterations/s); loop of single solves %.3f ms; x%.2f; "
        "max RMS difference %.2e Hz" % (ms_b, res["value"], ms_l, res["speedup_vs_loop"], diff))
    return res, vols


def bench_convergence(args, fmap, vol, y, s, m, torch, prec, ms_iter_rb):
    """Iterations and time to reach a relative cost gap (Psi_i - Psi*) / (Psi_0 - Psi*) of 1e-3 and
    1e-4 for each preconditioner on the benchmark volume, Psi* = the least cost of the 400-iteration F64
    solves (IC(0) in natural, red-black and block red-black order, IC_t with the level-1 pattern and the
    tolerance 1e-3 x H_max in natural order, diag(H), none).  Time = iterations x the measured time of one
    iteration of that preconditioner."""
    log("convergence: 400-iteration traces per preconditioner")
    runs = {"ic0_natural": (fmap.NATURAL, fmap.IC0), "ic0_redblack": (fmap.REDBLACK, fmap.IC0),
            "ic0_blockrb": (fmap.BLOCKRB, fmap.IC0),
            "ict_natural": (fmap.NATURAL, fmap.ICT), "diag": (fmap.NATURAL, fmap.DIAG),
            "none": (fmap.NATURAL, fmap.NONE)}
    traces, ms_iter = {}, {}
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for name, (order, pc) in runs.items():
        prm = fmap.params_for(vol, precision=fmap.F64, ordering=order, precond=pc, niter=400)
        with fmap.Plan(prm) as pl:
            pl.solve(y, s, m)
            traces[name] = pl.trace()[:, 0].copy()
        # time per iteration in the benchmark's precision
        with fmap.Plan(fmap.params_for(vol, precision=prec, ordering=order, precond=pc, niter=20)) as pl:
            pl.solve(y, s, m)
            ev0.record(stream)
            pl.iterate(20)
            ev1.record(stream)
            torch.cuda.synchronize()
            ms_iter[name] = ev0.elapsed_time(ev1) / 20
    best = min(float(t.min()) for t in traces.values())
    res = {"reference_cost": best, "niter_max": 400}
    for name, tr in traces.items():
        gap = (tr - best) / (tr[0] - best)
        row = {"ms_per_iteration": ms_iter[name]}
        for tol in (1e-3, 1e-4):
            hit = np.nonzero(gap <= tol)[0]
            it = int(hit[0]) if hit.size else None
            row["iters_%g" % tol] = it
            row["ms_%g" % tol] = None if it is None else it * ms_iter[name]
        res[name] = row
        log("  %-13s %.4f ms/iteration; gap 1e-3 after %s iterations (%s ms), 1e-4 after %s (%s ms)" % (
            name, ms_iter[name], row["iters_0.001"], None if row["ms_0.001"] is None else round(row["ms_0.001"], 2),
            row["iters_0.0001"], None if row["ms_0.0001"] is None else round(row["ms_0.0001"], 2)))
    return res


def bench_paper_mask(args, fmap, synth, torch, prec):
    """The headline problem on the paper-rule mask (reading R13: the first echo's coil-combined magnitude
    thresholded at 0.1 of its maximum, its convex hull, dilated twice): same solve, in-mask unknowns only."""
    log("paper mask: generating 128x128x64 with the convex-hull mask")
    vol = synth.mid_fieldmap(mask="paper")
    y, s, m = fmap.to_device(vol)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = torch.zeros(vol.shape, dtype=torch.float64, device="cuda")
    with fmap.Plan(fmap.params_for(vol, precision=prec, ordering=fmap.REDBLACK)) as plan:
        sched = "resident" if plan.schedule() == fmap.SCHED_RESIDENT else "stream"
        plan.solve(y, s, m, out=out)
        torch.cuda.synchronize()
        ms_solve = time_solve(plan, fmap, y, s, m, out, args.steps, torch)
        ev0.record(stream)
        plan.iterate(vol.niter, out=out)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_loop = ev0.elapsed_time(ev1)
        n = plan.mask_count()
    b = alg_bytes_per_voxel(args.precision, vol.necho, vol.nmls) * n
    res = {"grid": list(vol.shape), "voxels": n, "mask_fraction": n / float(vol.mask.size), "schedule": sched,
           "ms_per_step": ms_solve, "value": n * vol.niter / (ms_solve * 1e-3), "loop_ms": ms_loop,
           "loop_voxel_iterations_per_s": n * vol.niter / (ms_loop * 1e-3),
           "hbm_frac": b / (ms_loop * 1e-3 / vol.niter) / (HBM_PEAK_GBS * 1e9)}
    log("paper mask: %d unknowns (%.1f%%), %s schedule, step %.3f ms (%.3e voxel-iterations/s), loop %.3f ms, "
        "%.1f%% of HBM peak" % (n, 100 * res["mask_fraction"], sched, ms_solve, res["value"], ms_loop,
                                100 * res["hbm_frac"]))
    return res


def bench_waterfat(args, fmap, synth, torch):
    """192x192x64, 8 coils, 6 echoes, six-peak fat: full solve (setup, sweep + PWLS start, 100
    iterations) in MIX, the iteration loop alone, and the MIX map against an F64 solve."""
    log("water-fat: generating 192x192x64, 8 coils, 6 echoes")
    vol = synth.waterfat()
    y, s, m = fmap.to_device(vol)
    nmask = int(vol.mask.sum())
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = torch.zeros(vol.shape, dtype=torch.float64, device="cuda")
    with fmap.Plan(fmap.params_for(vol, precision=fmap.MIX, ordering=fmap.REDBLACK)) as plan:
        plan.solve(y, s, m, out=out)
        torch.cuda.synchronize()
        ms_solve = time_solve(plan, fmap, y, s, m, out, args.steps, torch)
        ev0.record(stream)
        plan.setup(y, s, m)
        plan.init()
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_init = ev0.elapsed_time(ev1)
        plan.solve(y, s, m, out=out)
        ev0.record(stream)
        plan.iterate(vol.niter, out=out)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_loop = ev0.elapsed_time(ev1)
        plan.solve(y, s, m, out=out)
        f_mix = out.clone()
    with fmap.Plan(fmap.params_for(vol, precision=fmap.F64, ordering=fmap.REDBLACK)) as plan:
        f_64 = plan.solve(y, s, m)
    mb = m.bool()
    diff = float(torch.sqrt(torch.mean((f_mix - f_64)[mb] ** 2)))
    res = {"grid": list(vol.shape), "coils": vol.ncoil, "echoes": vol.necho, "pairs": vol.necho * (vol.necho - 1) // 2,
           "niter": vol.niter, "voxels": nmask, "ms_per_solve": ms_solve, "init_ms": ms_init,
           "loop_ms": ms_loop, "loop_voxel_iterations_per_s": nmask * vol.niter / (ms_loop * 1e-3),
           "rms_mix_vs_f64_hz": diff}
    log("water-fat: solve %.3f ms (init %.3f ms, loop %.3f ms, %.3e voxel-iterations/s); MIX vs F64 %.2e Hz RMS"
        % (ms_solve, ms_init, ms_loop, res["loop_voxel_iterations_per_s"], diff))
    return res


def order2_bytes_per_voxel(kclass, precision, L):
    """Algorithmic bytes per voxel of one launch of each kernel class of the
    second-order regulariser with IC(0) in three-colour order (a third of the
    voxels per colour; pivots FP64, stored inverted; the diag(C^T C) byte array
    counted).  The two forward launches share a class, and so do the two
    backward ones: the figure is their mean."""
    t = 4 if precision == "mix" else 8
    if kclass == "grad":       # read code, echoes, f, z_prev; write f, g, D
        return 1 + 2 * L * t + 5 * t
    if kclass == "mls":
        return 1 + 2 * L * t + 2 * t
    if kclass == "dir":
        return 1 + 5 * t
    if kclass == "precond_a":
        # colours 0-1: read code, D, diag, g, g_prev; write 1/D of colours 0-1, y and y' of colour 1
        fwd1 = 2 + 3 * t + 16 / 3 + 2 * t / 3
        # colour 2: read code, 1/D of colours 0-1, D and diag of colour 2, g and g_prev of colours 0 and 2,
        # y and y' of colour 1; write 1/D and p of colour 2
        fwd2 = 1 + 16 / 3 + (t + 1) / 3 + 4 * t / 3 + 2 * t / 3 + (8 + t) / 3
        return (fwd1 + fwd2) / 2
    if kclass == "precond_b":
        # colour 1: read code, 1/D of colours 0-1, y of colour 1, p of colour 2; write p of colour 1
        bwd1 = 1 + 16 / 3 + t
        # colour 0: read code, g and 1/D of colour 0, p of colours 1-2; write p of colour 0
        bwd0 = 1 + 8 / 3 + 4 * t / 3
        return (bwd1 + bwd0) / 2
    return 0


def bench_order2(args, fmap, synth, torch, prec):
    """Second-order finite differences on the benchmark volume (128x128x64, 8 coils, full mask):
    full solves with IC(0) in three-colour order and with the diagonal preconditioner, the IC(0)
    iteration loop, its per-kernel rates against the byte model above, and the iterations each
    preconditioner needs to a 1e-3 relative cost gap."""
    log("order 2: generating 128x128x64")
    vol = synth.mid_fieldmap()
    vol.reg_order = 2
    y, s, m = fmap.to_device(vol)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = torch.zeros(vol.shape, dtype=torch.float64, device="cuda")
    res = {"grid": list(vol.shape), "niter": vol.niter}
    traces = {}
    for name, order, pc in (("ic0_color3", fmap.COLOR3, fmap.IC0), ("diag", fmap.NATURAL, fmap.DIAG)):
        with fmap.Plan(fmap.params_for(vol, precision=prec, ordering=order, precond=pc)) as plan:
            plan.solve(y, s, m, out=out)
            torch.cuda.synchronize()
            ms_solve = time_solve(plan, fmap, y, s, m, out, max(1, args.steps // 2), torch)
            traces[name] = plan.trace()
            ev0.record(stream)
            plan.iterate(vol.niter, out=out)
            ev1.record(stream)
            torch.cuda.synchronize()
            ms_loop = ev0.elapsed_time(ev1)
            n = plan.mask_count()
            r = {"ms_per_solve": ms_solve, "loop_ms": ms_loop, "value": n * vol.niter / (ms_solve * 1e-3)}
            if pc == fmap.IC0:
                kt = plan.time_kernels(args.kernel_iters)
                kinfo = {}
                for k, (ms, nl) in kt.items():
                    if nl == 0:
                        continue
                    b = order2_bytes_per_voxel(k, args.precision, vol.necho) * n
                    avg = ms / nl
                    kinfo[k] = {"avg_us": round(avg * 1e3, 3), "launches": nl, "gbs": round(b / (avg * 1e-3) / 1e9, 1)}
                it_b = sum(order2_bytes_per_voxel(k, args.precision, vol.necho) * (2 if k.startswith("precond") else 1)
                           for k in ("grad", "precond_a", "precond_b", "dir")) \
                    + (vol.nmls - 1) * order2_bytes_per_voxel("mls", args.precision, vol.necho)
                r.update(kernels=kinfo, bytes_per_voxel_iteration=round(it_b, 2),
                         hbm_frac=it_b * n / (ms_loop * 1e-3 / vol.niter) / (HBM_PEAK_GBS * 1e9))
                for k, v in kinfo.items():
                    log("  order 2 %-10s %9.2f us/launch  %8.1f GB/s  (%d launches)" % (k, v["avg_us"], v["gbs"],
                                                                                        v["launches"]))
            res[name] = r
            log("order 2 %s: solve %.3f ms (%.3e voxel-iterations/s), loop %.3f ms" % (name, ms_solve, r["value"],
                                                                                      ms_loop))
    c_ic, c_d = traces["ic0_color3"][:, 0], traces["diag"][:, 0]
    final = min(c_ic[-1], c_d[-1])
    gap = lambda c: int(np.argmax(c - final <= 1e-3 * (c[0] - final))) if np.any(c - final <= 1e-3 * (c[0] - final)) \
        else None
    res["iterations_to_1e-3_gap"] = {"ic0_color3": gap(c_ic), "diag": gap(c_d)}
    log("order 2: iterations to a 1e-3 gap: IC(0) %s, diagonal %s" % (gap(c_ic), gap(c_d)))
    return res


def bench_large(args, fmap, synth, torch, prec):
    """256x256x128 (8.4 M voxels, working set well above the 256 MB Infinity Cache): the field-map
    problem of the benchmark at eight times the size, a true HBM measurement.  2 coils (the coil
    count only changes the setup, not the iteration)."""
    shape = (256, 256, 128)
    log("large: generating %s" % (shape,))
    vol = synth.fieldmap_volume(shape, 2, [0.0, 2.2e-3, 4.4e-3], 2.0 ** -4, 100, synth.SEED_BASE + 1, 8, 250.0,
                                True, 30.0, mask="full", name="fieldmap 256x256x128 2 coils 3 echoes")
    y, s, m = fmap.to_device(vol)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = torch.zeros(shape, dtype=torch.float64, device="cuda")
    with fmap.Plan(fmap.params_for(vol, precision=prec, ordering=fmap.REDBLACK)) as plan:
        sched = "resident" if plan.schedule() == fmap.SCHED_RESIDENT else "stream"
        plan.solve(y, s, m, out=out)
        torch.cuda.synchronize()
        ms_solve = time_solve(plan, fmap, y, s, m, out, 1, torch)
        ev0.record(stream)
        plan.iterate(vol.niter, out=out)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_loop = ev0.elapsed_time(ev1)
        n = plan.mask_count()
    b = alg_bytes_per_voxel(args.precision, vol.necho, vol.nmls) * n
    res = {"grid": list(shape), "voxels": n, "schedule": sched, "ms_per_solve": ms_solve, "loop_ms": ms_loop,
           "loop_voxel_iterations_per_s": n * vol.niter / (ms_loop * 1e-3),
           "hbm_frac": b / (ms_loop * 1e-3 / vol.niter) / (HBM_PEAK_GBS * 1e9)}
    log("large: %s schedule, solve %.2f ms, loop %.2f ms (%.3e voxel-iterations/s, %.1f%% of HBM peak)" % (
        sched, ms_solve, ms_loop, res["loop_voxel_iterations_per_s"], 100 * res["hbm_frac"]))
    return res


def bench_ict(args, fmap, synth, torch, prec):
    """The headline volume (128x128x64, 8 coils) preconditioned by IC with a drop tolerance (IC_t, natural
    order, fill bounded to the level-1 pattern, tolerance 1e-3 x H_max): the factor and both triangular
    solves are formed every iteration, one launch per level of the schedule (699 levels each way)."""
    log("ict: generating 128x128x64")
    vol = synth.mid_fieldmap()
    niter = 10
    y, s, m = fmap.to_device(vol)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = torch.zeros(vol.shape, dtype=torch.float64, device="cuda")
    with fmap.Plan(fmap.params_for(vol, precision=prec, ordering=fmap.NATURAL, precond=fmap.ICT, niter=niter)) as plan:
        plan.solve(y, s, m, out=out)
        torch.cuda.synchronize()
        ms_solve = time_solve(plan, fmap, y, s, m, out, 1, torch)
        ev0.record(stream)
        plan.iterate(niter, out=out)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_loop = ev0.elapsed_time(ev1)
        plan.status()
        n = plan.mask_count()
    res = {"grid": list(vol.shape), "voxels": n, "niter": niter, "ms_per_solve": ms_solve, "loop_ms": ms_loop,
           "ms_per_iteration": ms_loop / niter, "loop_voxel_iterations_per_s": n * niter / (ms_loop * 1e-3)}
    log("ict: solve %.2f ms, %.3f ms per iteration" % (ms_solve, res["ms_per_iteration"]))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["mix", "f64"], default="mix")
    ap.add_argument("--ordering", choices=["natural", "redblack", "blockrb"], default="redblack")
    ap.add_argument("--precond", choices=["ic0", "diag", "none"], default="ic0")
    ap.add_argument("--mask", choices=["full", "paper"], default="full")
    ap.add_argument("--shape", default="128,128,64")
    ap.add_argument("--workload", choices=["fieldmap", "batched", "waterfat", "order2", "large", "ict", "copy"],
                    default="fieldmap",
                    help="fieldmap: the headline line (default); batched / waterfat / order2 / large / ict: only that "
                         "workload; copy: a plain 1 GiB device copy (the calibration of the traffic counters)")
    ap.add_argument("--kernel-iters", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-natural", action="store_true", help="skip the natural-order comparison line")
    ap.add_argument("--no-batched", action="store_true", help="skip the 16-volume batched comparison")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the implicit-adjoint timing")
    ap.add_argument("--no-waterfat", action="store_true", help="skip the 192x192x64 water-fat solve")
    ap.add_argument("--no-large", action="store_true", help="skip the 256x256x128 HBM-sized field-map loop")
    ap.add_argument("--no-order2", action="store_true", help="skip the second-order regulariser solves")
    ap.add_argument("--no-paper-mask", action="store_true", help="skip the headline problem on the paper-rule mask")
    ap.add_argument("--no-convergence", action="store_true",
                    help="skip the time-to-accuracy comparison of the preconditioners")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2005_08661_amd import fmap, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "copy":
        gbs = copy_rate_gbs(torch, 1024, max(1, args.steps))
        print(json.dumps({"metric": "device copy rate (read + write)", "value": gbs, "unit": "GB/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "ms_per_step": 2 * 1024 * 1048576 / gbs / 1e6,
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                          "data": "synthetic", "config": {"workload": "copy of 1 GiB (1073741824 bytes)"}}),
              flush=True)
        return
    if args.workload != "fieldmap":
        prec = fmap.MIX if args.precision == "mix" else fmap.F64
        if args.workload == "batched":
            res, _ = bench_batched(args, fmap, synth, torch, prec)
            value, ms = res["value"], res["ms_per_solve"]
            wl = "16 field-map volumes of 64-160 x 64-160 x 32-96 voxels (%d unknowns), 4 coils, TE 0/2/5 ms, " \
                 "100 NCG iterations, one batched solve, red-black IC(0), %s" % (res["voxels"], args.precision.upper())
        elif args.workload == "order2":
            res = bench_order2(args, fmap, synth, torch, prec)
            value, ms = res["ic0_color3"]["value"], res["ic0_color3"]["ms_per_solve"]
            wl = "field map 128x128x64, 8 coils, 3 echoes, second-order finite differences, 100 NCG iterations, " \
                 "IC(0) in three-colour order, %s" % args.precision.upper()
        elif args.workload == "ict":
            res = bench_ict(args, fmap, synth, torch, prec)
            value, ms = res["loop_voxel_iterations_per_s"], res["ms_per_solve"]
            wl = "field map 128x128x64 (%d unknowns), 8 coils, 3 echoes, %d NCG iterations, IC_t (natural order, " \
                 "level-1 fill, 1e-3 H_max), %s" % (res["voxels"], res["niter"], args.precision.upper())
        elif args.workload == "large":
            res = bench_large(args, fmap, synth, torch, prec)
            value, ms = res["loop_voxel_iterations_per_s"], res["ms_per_solve"]
            wl = "field map 256x256x128 (%d unknowns), 2 coils, 3 echoes, 100 NCG iterations, red-black IC(0), " \
                 "%s schedule, %s" % (res["voxels"], res["schedule"], args.precision.upper())
        else:
            res = bench_waterfat(args, fmap, synth, torch)
            value, ms = res["loop_voxel_iterations_per_s"], res["ms_per_solve"]
            wl = "water-fat 192x192x64, 8 coils, 6 echoes, six-peak fat, 100 NCG iterations, red-black IC(0), MIX"
        print(json.dumps({"metric": "voxel-iterations/s", "value": value, "unit": "voxel-iterations/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None,
                          "dtype": "f32+f64" if args.precision == "mix" else "f64", "data": "synthetic",
                          "config": {"workload": wl}, "detail": res}), flush=True)
        return
    shape = tuple(int(s) for s in args.shape.split(","))
    log("generating %s volume (%s mask)" % (shape, args.mask))
    vol = synth.mid_fieldmap(mask=args.mask, shape=shape)
    prec = fmap.MIX if args.precision == "mix" else fmap.F64
    order = {"natural": fmap.NATURAL, "redblack": fmap.REDBLACK, "blockrb": fmap.BLOCKRB}[args.ordering]
    pc = {"ic0": fmap.IC0, "diag": fmap.DIAG, "none": fmap.NONE}[args.precond]
    y, s, m = fmap.to_device(vol)
    plan = fmap.Plan(fmap.params_for(vol, precision=prec, ordering=order, precond=pc))
    out = torch.zeros(shape, dtype=torch.float64, device="cuda")
    stream_h = torch.cuda.current_stream()

    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        plan.solve(y, s, m, out=out)
    torch.cuda.synchronize()
    niter = vol.niter

    log("timing %d steps" % args.steps)
    t0 = time.perf_counter()
    ms_step = time_solve(plan, fmap, y, s, m, out, args.steps, torch)
    wall = time.perf_counter() - t0
    tr = plan.trace()
    f_step = out.cpu().numpy()
    nmask = plan.mask_count()
    value = nmask * niter / (ms_step * 1e-3)
    log("step %.3f ms (wall %.3f ms), %.3e voxel-iterations/s" % (ms_step, wall * 1e3 / args.steps, value))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    # iteration loop alone (graph replays or one resident launch), from the solved state
    ev0.record(stream_h)
    plan.iterate(niter, out=out)
    ev1.record(stream_h)
    torch.cuda.synchronize()
    ms_loop = ev0.elapsed_time(ev1)
    loop_rate = nmask * niter / (ms_loop * 1e-3)

    # per-kernel durations from HIP events on the launch stream
    L = vol.necho
    # the roofline of the whole iteration and of the resident kernel uses B_alg; the per-pass model
    # (slightly smaller for red-black IC(0), whose fused passes skip some sweeps) is reported beside it
    it_bytes_vox = alg_bytes_per_voxel(args.precision, L, vol.nmls)
    pass_bytes_vox = iteration_bytes_per_voxel(args.precision, L, args.ordering, args.precond, vol.nmls)

    def kernel_table(kt, iters):
        kinfo = {}
        for k, (ms, nl) in kt.items():
            if nl == 0:
                continue
            if k == "resident":  # one launch runs all the iterations of the call
                b = it_bytes_vox * nmask * iters / nl
            else:
                b = bytes_per_voxel(k, args.precision, L, args.ordering, args.precond) * nmask
            avg = ms / nl
            kinfo[k] = dict(avg_us=avg * 1e3, launches=nl, total_ms=ms, bytes=b,
                            gbs=b / (avg * 1e-3) / 1e9 if avg > 0 else 0.0)
        return kinfo

    schedule = "resident" if plan.schedule() == fmap.SCHED_RESIDENT else "stream"
    # the resident kernel is timed over a whole solve's iteration count, like the launches of the solves
    kiters = niter if schedule == "resident" else args.kernel_iters
    kinfo = kernel_table(plan.time_kernels(kiters), kiters)
    dom = max(kinfo, key=lambda k: kinfo[k]["total_ms"])
    iter_bytes = it_bytes_vox * nmask
    iter_frac = iter_bytes / (ms_loop * 1e-3 / niter) / (HBM_PEAK_GBS * 1e9)
    for k, v in kinfo.items():
        log("  %-10s %9.2f us/launch  %8.1f GB/s  (%d launches)" % (k, v["avg_us"], v["gbs"], v["launches"]))
    log("%s schedule: loop %.3f ms for %d iterations; whole-iteration %.1f%% of HBM peak (algorithmic bytes)" % (
        schedule, ms_loop, niter, 100 * iter_frac))
    stream = None
    if schedule == "resident":
        # the streaming schedule on the same plan, for comparison
        plan.set_schedule(fmap.SCHED_STREAM)
        ms_s = time_solve(plan, fmap, y, s, m, out, max(1, args.steps // 2), torch)
        ev0.record(stream_h)
        plan.iterate(niter, out=out)
        ev1.record(stream_h)
        torch.cuda.synchronize()
        ms_loop_s = ev0.elapsed_time(ev1)
        ks = kernel_table(plan.time_kernels(args.kernel_iters), args.kernel_iters)
        plan.set_schedule(fmap.SCHED_AUTO)
        stream = {"ms_per_step": ms_s, "loop_ms": ms_loop_s, "value": nmask * niter / (ms_s * 1e-3),
                  "hbm_frac": iter_bytes / (ms_loop_s * 1e-3 / niter) / (HBM_PEAK_GBS * 1e9),
                  "kernels_us": {k: round(v["avg_us"], 3) for k, v in ks.items()}}
        log("stream schedule: %.3f ms per step, loop %.3f ms" % (ms_s, ms_loop_s))

    natural = None
    if not args.no_natural and args.ordering == "redblack" and args.precond == "ic0":
        log("natural-order IC(0) on the same volume")
        with fmap.Plan(fmap.params_for(vol, precision=prec, ordering=fmap.NATURAL)) as pn:
            pn.solve(y, s, m, out=out)
            ms_nat = time_solve(pn, fmap, y, s, m, out, 1, torch)
            trn = pn.trace()
        natural = {"ms_per_step": ms_nat, "value": nmask * niter / (ms_nat * 1e-3),
                   "final_cost": float(trn[-1, 0])}
        log("natural order: %.3f ms per step, %.3e voxel-iterations/s" % (ms_nat, natural["value"]))

    convergence = None
    if not args.no_convergence and args.precond == "ic0":
        convergence = bench_convergence(args, fmap, vol, y, s, m, torch, prec, ms_loop / niter)

    adjoint = None
    if not args.no_adjoint:
        # backward of L = ||f - f_true||^2 over the mask at the solved map (config of the differentiable form)
        ftrue = torch.from_numpy(vol.f_true).cuda()
        plan.solve(y, s, m, out=out)
        dldf = 2.0 * (out - ftrue) * m
        plan.adjoint(dldf, rtol=1e-6)  # workspace allocation, untimed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = plan.adjoint(dldf, rtol=1e-6)
        torch.cuda.synchronize()
        ms_adj = (time.perf_counter() - t0) * 1e3
        adjoint = {"ms": ms_adj, "cg_iterations": res["iters"], "rtol": 1e-6, "dL_dbeta": res["dbeta"],
                   "loss": "||f - f_true||^2 over the mask", "outputs": "dL/dbeta, dL/dy (complex64, 8 coils)"}
        log("adjoint: %.3f ms, %d CG iterations" % (ms_adj, res["iters"]))

    batched, batched_vols = None, None
    if not args.no_batched:
        batched, batched_vols = bench_batched(args, fmap, synth, torch, prec)

    waterfat = None
    if not args.no_waterfat:
        waterfat = bench_waterfat(args, fmap, synth, torch)

    large = None
    if not args.no_large and args.shape == "128,128,64":
        large = bench_large(args, fmap, synth, torch, prec)

    order2 = None
    if not args.no_order2 and args.shape == "128,128,64" and args.mask == "full":
        order2 = bench_order2(args, fmap, synth, torch, prec)

    paper_mask = None
    if not args.no_paper_mask and args.shape == "128,128,64" and args.mask == "full":
        paper_mask = bench_paper_mask(args, fmap, synth, torch, prec)

    copy_gbs = copy_rate_gbs(torch)
    log("device copy of 1 GB: %.0f GB/s (read + write)" % copy_gbs)

    cpu, parity = None, None
    if not args.no_cpu_baseline:
        headline = {args.precision: (f_step, tr)}
        if args.precision == "mix":
            with fmap.Plan(fmap.params_for(vol, precision=fmap.F64, ordering=order, precond=pc)) as p64:
                f64 = p64.solve(y, s, m).cpu().numpy()
                headline["f64"] = (f64, p64.trace())
        cpu, parity = bench_cpu(args, vol, synth, batched_vols, headline)

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
        "hbm_copy_gbs": copy_gbs,
        "roofline": roofline_entry(kinfo, dom, measured_traffic(dom, args)),
        "iteration": {
            "schedule": schedule,
            "loop_ms": ms_loop,
            "loop_voxel_iterations_per_s": loop_rate,
            "bytes_per_iteration": iter_bytes,
            "alg_bytes_per_voxel": it_bytes_vox,
            "pass_model_bytes_per_voxel": pass_bytes_vox,
            "hbm_frac": iter_frac,
            "kernels_us": {k: round(v["avg_us"], 3) for k, v in kinfo.items()},
            "stream_schedule": stream,
        },
        "final_cost": float(tr[-1, 0]),
        "natural_order": natural,
        "large_256x256x128": large,
        "second_order": order2,
        "paper_mask": paper_mask,
        "convergence": convergence,
        "adjoint": adjoint,
        "batched": batched,
        "waterfat": waterfat,
        "cpu_baseline": cpu,
        "parity": parity,
    }
    plan.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
