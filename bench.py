#!/usr/bin/env python3
"""Throughput benchmark: finite-source binary-lens magnifications per second.

Workload: the fit-style batch of 1024 lens/source parameter sets x 2000
epochs (tau in [-1.5, 1.5]) with log10 s ~ U[-0.5,0.5], log10 q ~ U[-5,-1],
alpha ~ U[0,2pi), u0 ~ U[-0.1,0.1], log10 rho ~ U[-4,-2] (seed 1), uniform
source, relative tolerance 1e-4, answered in one call of twk_lightcurves:
point-source test for every epoch, contour integration for the rest in one
persistent launch.  A step is one such call over the whole batch; inputs
are resident in device memory before timing starts.

Paths timed (same call, mode bits differ): plain FP64 (no learned budget),
+ mixed precision (FP32 bulk root iterations), + learned budget (the MLP's
starting grid and longest-first queue).  The headline value is the learned
+ mixed path; the others are reported beside it.

Prints one JSON line with the value, the roofline of the dominant kernel
(the persistent contour kernel, VALU-bound), and the CPU oracle timed on a
bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "finite-source magnifications/sec at \u22641e-4 rel. err, learned-batched vs plain GPU"

# Algorithmic floating-point work of the contour kernel, counted by hand
# from the device code (FMA = 2 flops, add/mul/rcp/sqrt = 1).  Units: one
# root sweep (all five roots of one limb point), one limb sample outside the
# sweeps (coefficients, lens-equation polish, residual classification,
# derivatives, angle), one interval link (assignment, area, error).
F_SWEEP64 = 925.0
F_SWEEP32 = 715.0
F_SAMPLE = 1285.0
F_INTERVAL = 300.0

# MI355X vector peak: 256 CUs x 4 SIMD x 16 lanes x 2 flops (FMA) x 2.4 GHz.
# FP64 FMA runs at full rate; FP32 without packed instructions (disabled for
# all device code here) runs at the same rate, so both paths share it.
PEAK_VALU_TFLOPS = 78.6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def flops_of(stats):
    return (stats["sweeps64"] * F_SWEEP64 + stats["sweeps32"] * F_SWEEP32 +
            stats["samples"] * F_SAMPLE + stats["intervals"] * F_INTERVAL)


def run_path(ctx, dev, c, mode, steps, warmup, label):
    import torch
    args = [torch.as_tensor(a, device=dev) for a in (c.s, c.q, c.u0, c.alpha, c.rho, c.tau)]
    out = ctx.alloc_out(c.nsets * c.nepochs)
    ctx.enable_timing(True)
    for w in range(warmup):
        ctx.lightcurves(*args, c.tol, mode=mode, out=out)
        ctx.sync()
        log(f"[{label}] warmup {w + 1}/{warmup} done")
    fs_ms = []
    tot_ms = []
    mlp_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ctx.lightcurves(*args, c.tol, mode=mode, out=out)
        kt = ctx.kernel_times()  # waits for this step
        fs_ms.append(kt["fs_ms"])
        tot_ms.append(kt["total_ms"])
        mlp_ms.append(kt["mlp_ms"])
        if "graph" in label:  # a replayed call is timed as a whole
            log(f"[{label}] step {k + 1}/{steps}: {kt['total_ms']:.2f} ms")
        else:
            log(f"[{label}] step {k + 1}/{steps}: {kt['total_ms']:.2f} ms (contour kernel {kt['fs_ms']:.2f} ms,"
                f" point pass {kt['ps_ms']:.2f} ms, learned stage {kt['mlp_ms']:.2f} ms,"
                f" rest {kt['rest_ms']:.2f} ms)")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = ctx.stats()
    ctx.enable_timing(False)
    fl = out[3].cpu().numpy()
    ns = out[2].cpu().numpy()
    nfs = ns[(fl & 1) == 0]
    hist = {f"<= {b}": int(np.sum(nfs <= b)) for b in (64, 128, 256, 512, 1024, 2048, 4096)}
    return dict(ms_per_step=1e3 * wall / steps, fs_kernel_ms=float(np.mean(fs_ms)),
                event_ms=float(np.mean(tot_ms)), mlp_ms=float(np.mean(mlp_ms)), stats=st,
                fs_fraction=float(np.mean((fl & 1) == 0)), mag=out[0],
                samples_hist=hist, samples_max=int(nfs.max()) if nfs.size else 0)


def cpu_baseline(c, seconds, seed=11):
    """The oracle as it stands: point-source test, else contour integration at
    the same tolerance, one epoch after another on one core, over a seeded
    random sample of the batch's epochs until the time budget is used."""
    from oracle import ref
    rng = np.random.default_rng(seed)
    order = rng.permutation(c.nsets * c.nepochs)
    t0 = time.perf_counter()
    done = 0
    for i in order:
        k, j = divmod(int(i), c.nepochs)
        zx, zy = ref.trajectory(c.u0[k], c.alpha[k], c.tau[j:j + 1])
        ok, mu = ref.ps_adequate(c.s[k], c.q[k], complex(zx[0], zy[0]), c.rho[k], c.tol)
        if not ok:
            ref.finite_mag(c.s[k], c.q[k], zx, zy, c.rho[k], c.tol)
        done += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    return dict(value=done / dt, unit="magnifications/s", cores=1, kind="oracle",
                sample=f"{done} epochs drawn at random (seed {seed}) from the 1024x2000 batch, "
                       f"point-source test then contour integration at tol {c.tol}, single thread, "
                       f"{dt:.1f} s")


WEIGHTS = os.path.join(HERE, "paper_2501_03322_amd", "weights", "mlp_budget.bin")
TRAFFIC = os.path.join(HERE, "profiles", "k_fs_traffic.json")


def lib_digest(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def device_code_digest(path):
    """sha256 of the library's device code: the `.hip_fatbin` section of the
    ELF shared object, which holds every kernel's gfx950 code object and no
    host code (a host-only change leaves it unchanged)."""
    import hashlib
    import struct
    with open(path, "rb") as f:
        b = f.read()
    if b[:4] != b"\x7fELF" or b[4] != 2:
        raise ValueError(f"{path}: not a 64-bit ELF file")
    shoff, = struct.unpack_from("<Q", b, 0x28)
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", b, 0x3A)
    secs = [struct.unpack_from("<IIQQQQIIQQ", b, shoff + i * shentsize) for i in range(shnum)]
    names = secs[shstrndx][4]
    for name_off, _, _, _, off, size, *_ in secs:
        end = b.index(b"\0", names + name_off)
        if b[names + name_off:end] == b".hip_fatbin":
            return hashlib.sha256(b[off:off + size]).hexdigest()
    raise ValueError(f"{path}: no .hip_fatbin section")


def measured_traffic(lib_path):
    """HBM bytes per launch of the contour kernel from the committed counter
    runs (FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known size),
    valid only while the library's device code is the one they were taken on."""
    if not os.path.exists(TRAFFIC):
        return None
    with open(TRAFFIC) as f:
        t = json.load(f)
    if t.get("device_code_sha256") != device_code_digest(lib_path):
        return None
    return t.get("hbm_bytes_per_launch")


def pmc_summary(fetch_dir, write_dir):
    """HBM traffic of one contour-kernel launch from two counter runs.
    FETCH_SIZE and WRITE_SIZE are in KiB per dispatch; each is scaled by
    what it reads for the 1 GiB device copies of the same run (the copy
    reads and writes exactly 1 GiB), and the launch is the run's last
    contour-kernel dispatch (the timed step)."""
    import csv
    import glob

    def read(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    if r["Counter_Name"] == counter:
                        rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
        per = {}
        for did, name, v in rows:
            per.setdefault(did, [name, 0.0])[1] += v
        fs = [per[k][1] for k in sorted(per) if "k_fs" in per[k][0]]
        # the probe's three 1 GiB copies are the run's largest copy dispatches
        cp = sorted(per[k][1] for k in per if "copyBuffer" in per[k][0])[-3:]
        if not fs or not cp:
            raise SystemExit(f"{d}: no contour-kernel or copy dispatch with {counter}")
        kib = float(1 << 20)  # 1 GiB in KiB
        factor = kib / float(np.median(cp))
        return fs[-1] * 1024.0 * factor, factor

    fetch, ff = read(fetch_dir, "FETCH_SIZE")
    write, wf = read(write_dir, "WRITE_SIZE")
    from paper_2501_03322_amd import twk
    return {"lib_sha256": lib_digest(twk.LIB_PATH),
            "device_code_sha256": device_code_digest(twk.LIB_PATH), "hbm_bytes_per_launch": fetch + write,
            "fetch_bytes": fetch, "write_bytes": write,
            "fetch_copy_factor": ff, "write_copy_factor": wf}


def path_summary(n, r):
    st = r["stats"]
    fs_s = r["fs_kernel_ms"] * 1e-3
    return {"value": n / (r["ms_per_step"] * 1e-3), "ms_per_step": r["ms_per_step"],
            "fs_kernel_ms": r["fs_kernel_ms"], "learned_stage_ms": r["mlp_ms"],
            "contour_mags_per_s": st["fs_tasks"] / fs_s,
            "limb_solves_per_s": st["samples"] / fs_s,
            "achieved_tflops": flops_of(st) / fs_s / 1e12,
            "samples": int(st["samples"]), "fs_tasks": int(st["fs_tasks"])}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="time only the headline path (for profiling runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 1 GiB device copy (reference for HBM counters)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (default launch parameters)")
    ap.add_argument("--no-graphs", action="store_true",
                    help="issue every call eagerly instead of replaying a captured graph")
    ap.add_argument("--tune", metavar="LDS,WAVES,SHIFT",
                    help="fixed launch tuning (LDS capacity, waves per CU, budget shift) instead "
                         "of the autotuner, e.g. to profile the configuration a bench run chose")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no run: turn two rocprofv3 --pmc output folders (FETCH_SIZE, then "
                         "WRITE_SIZE, each of a run with --copy-probe) into the traffic record "
                         "of the contour kernel, printed as JSON")
    args = ap.parse_args()
    if args.pmc_summary:
        print(json.dumps(pmc_summary(*args.pmc_summary)))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs one GPU per process; --gpus must be 1 "
                                   "(a batch shards by parameter sets, one process per GPU)"}))
        sys.exit(2)

    import torch
    from paper_2501_03322_amd import inputs, twk

    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(dev)  # default priority; a created stream can be captured
    torch.cuda.set_stream(stream)
    ctx = twk.Context(0, stream=stream)
    if not os.path.exists(WEIGHTS):
        log(f"{WEIGHTS} missing: training the learned budget first")
        from paper_2501_03322_amd import train_mlp
        train_mlp.train(WEIGHTS, log=log)
    ctx.mlp_load(WEIGHTS)
    c = inputs.batched_curves()
    n = c.nsets * c.nepochs
    log(f"workload: {c.nsets} sets x {c.nepochs} epochs = {n} magnifications, tol {c.tol}")

    head_mode = twk.MODE_MLP | twk.MODE_MIXED
    if args.tune:
        lds, waves, shift = args.tune.split(",")
        ctx.set_tuning(lds_cap=int(lds), waves_per_cu=int(waves), budget_shift=float(shift))
        log(f"fixed tuning: {ctx.get_tuning().as_dict()}")
    elif not args.no_tune:
        t0 = time.perf_counter()
        tuned = ctx.autotune(c.s, c.q, c.u0, c.alpha, c.rho, c.tau, c.tol, mode=head_mode, trials=1)
        log(f"autotuned on the workload in {time.perf_counter() - t0:.1f} s: {tuned.as_dict()}")
    tuning = ctx.get_tuning().as_dict()
    best = run_path(ctx, dev, c, head_mode, args.steps, args.warmup, "learned+mixed")
    graph = None
    if not args.no_graphs:
        # the same path replayed from a captured graph (timed as whole calls)
        ctx.set_tuning(graphs=1)
        g = run_path(ctx, dev, c, head_mode, args.steps, args.warmup, "learned+mixed, graph replay")
        ctx.set_tuning(graphs=0)
        graph = {"ms_per_step": g["ms_per_step"], "event_ms": g["event_ms"],
                 "value": n / (g["ms_per_step"] * 1e-3),
                 "bitwise_equal_to_eager": bool(torch.equal(g["mag"], best["mag"]))}
    others = {}
    if not args.no_plain:
        others["mixed"] = run_path(ctx, dev, c, twk.MODE_MIXED, args.steps, args.warmup, "mixed")
        others["plain_fp64"] = run_path(ctx, dev, c, twk.MODE_FP64, args.steps, args.warmup, "fp64")
        for k, r in others.items():
            rel = (best["mag"] / r["mag"] - 1).abs().max().item()
            log(f"max relative difference learned+mixed vs {k} over the batch: {rel:.3g}")
            r["max_rel_diff_vs_headline"] = rel

    if args.copy_probe:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy probe: 3 x 1 GiB device-to-device copies done")

    st = best["stats"]
    flops = flops_of(st)
    achieved = flops / (best["fs_kernel_ms"] * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": n / (best["ms_per_step"] * 1e-3),
        "unit": "magnifications/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": best["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "batched light curves: 1024 parameter sets x 2000 epochs, uniform source, "
                               "tol 1e-4, one persistent launch (seed 1)",
                   "nsets": c.nsets, "nepochs": c.nepochs, "tol": c.tol,
                   "path": "learned budget + batched persistent + mixed precision"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_VALU_TFLOPS,
                     "traffic": measured_traffic(twk.LIB_PATH),
                     "kernel": f"k_fs<{tuning['lds_cap']}, mixed>",
                     "flops_per_launch": flops, "kernel_ms": best["fs_kernel_ms"]},
        "work": {"fs_fraction": best["fs_fraction"], **{k: int(v) for k, v in st.items()},
                 "samples_per_source_cumulative": best["samples_hist"],
                 "samples_per_source_max": best["samples_max"]},
        "paths": {"learned+mixed": path_summary(n, best)},
        "tuning": tuning,
        "graph_replay": graph,
        "paper_context": "the paper reports ~1e2 speedup of its GPU code (RTX 4090) over one CPU core "
                         "(EPYC 7H12, VBBL) on its own benchmarks; other hardware and workload",
    }
    for k, r in others.items():
        out["paths"][k] = path_summary(n, r)
        out["paths"][k]["max_rel_diff_vs_headline"] = r["max_rel_diff_vs_headline"]
    if "plain_fp64" in others:
        out["speedup_vs_plain_fp64"] = others["plain_fp64"]["ms_per_step"] / best["ms_per_step"]
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle for about {args.cpu_seconds:.0f} s")
        out["cpu_baseline"] = cpu_baseline(c, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
