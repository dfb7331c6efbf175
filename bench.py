"""Benchmark: cell-ordinate sweep updates/s of ROM source iteration on one MI355X, and batched ROM
against plain DOM in time to a fixed error.

One step = one pass of the whole hot path over the workload's synthetic input, inputs resident in
HBM: ordinate ingestion, source iteration to convergence (sweeps + partial-flux combine + FP64
residual, replayed from captured HIP graphs), FP64 ensemble moments where the workload has samples,
and the results left in HBM.  The default workload is c5, the largest single-GPU configuration: 200
independent problems (grid sides 64..1024, 16..512 ordinates, random 8 x 8 block maps of cross
sections) solved together, one persistent sweep launch per iteration.  The sweep shape the headline
is timed with is pinned per workload (the fastest in full-solve timings), so that the timed work does
not depend on a timing-based choice made in the same process.

The JSON line carries, besides the contract fields:
  * roofline -- the dominant kernel (the sweep): its achieved rate from its own launch durations
    (the device real-time clock, summed by the combine step over the launches that did work),
    against the FP32 vector peak (157.3 TFLOP/s) and against the unpacked FP32 rate this build
    issues (78.6 TFLOP/s; packed FP32 is switched off); or, for the angular-flux-storing sweep of a
    dense kernel, HBM bytes against 8 TB/s.  `traffic` is the HBM bytes per launch from rocprofv3
    FETCH_SIZE / WRITE_SIZE counters of the committed profile of this kernel shape (null once the
    kernel sources differ from the profiled ones), with its bandwidth against the datasheet peak and
    against a copy measured in this run, and its ratio to the algorithmic bytes;
  * cpu_baseline -- the FP64 oracle on this host: median of 3 runs on all cores and on one core,
    the CPU model, and the sample it was timed on (a bounded sample of the same workload);
  * tte -- time to a fixed error on the 64 x 64 isotropic problem (bench_tte.py's protocol):
    FP64 DOM against batched FP32 ROM, median over five seed blocks.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c5|c1|c2|c3|c4] [--no-cpu] [--no-tte]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import rom_inputs as RI  # noqa: E402

# Algorithmic work of one upwind cell-ordinate update: w*S (1 mul), + a*x and + b*y (2 fma = 4
# flops), sigma_t + a + b (1 add), the division (1), and the scalar-flux accumulation (1 add).
FLOPS_PER_UPDATE = 8
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X datasheet, FP32 vector (packed FP32 instructions)
FP32_UNPACKED_TFLOPS = 78.6       # the same units issuing one FP32 operation per lane per cycle
FP64_VECTOR_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per update.  Flux-only sweep: a wavefront pass over the grid reads
# sigma_t and the isotropic source and writes one partial flux per cell for its 64 lanes, and the
# combine step reads the partials, sigma_s, q and the old flux and writes the flux and the next
# source: about 20 bytes per cell per 64 updates.  Angular-flux-storing sweep: the FP32
# per-ordinate source read and the BF16 angular flux written, 6 bytes per update.
BYTES_PER_ISO_UPDATE = 20.0 / 64.0
BYTES_PER_ANG_UPDATE = 6.0

# The sweep shape each workload's headline is timed with: the fastest in full-solve timings on
# MI355X (c3's band of 7 strips lies between the autotuner's candidates 4 and 8).
PINNED = {
    "c1": {"sweep": "diag", "diag_rows": 64, "diag_k": 1, "band": 2, "tile": "0x0"},
    "c2": {"sweep": "diag", "diag_rows": 64, "diag_k": 2, "band": 4, "tile": "0x0"},
    "c3": {"sweep": "strip", "tile": "16x16", "band": 7, "diag_rows": 0, "diag_k": 0},
    "c4": {"sweep": "diag", "diag_rows": 16, "diag_k": 4, "band": 4, "tile": "0x0"},
    "c5": {"sweep": "strip", "tile": "16x16", "band": 4, "diag_rows": 0, "diag_k": 0},
}

# HBM bytes per sweep launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (scaled by a 256 MiB copy:
# 1 FETCH_SIZE KiB = 2 KiB read, 1 WRITE_SIZE KiB = 1 KiB written), for the pinned kernel shape of
# each workload.  Reported only while the kernel sources hash to what was profiled and the run
# used that shape; otherwise `traffic` is null.
KERNEL_SOURCES = {
    "row-lane": ["rom_common.h", "rom_device.h", "rom_diag.h", "rom_diag_f32.hip", "rom_diag_f32_ang.hip",
                 "rom_diag_f64.hip"],
    "strip": ["rom_common.h", "rom_device.h", "rom_sweep.h", "rom_sweep_f32_16x16.hip", "rom_sweep_f32_16x8.hip",
              "rom_sweep_f32_8x4.hip", "rom_sweep_f32_8x8.hip", "rom_sweep_f64.hip"],
}
MEASURED_TRAFFIC = {  # workload: [(kernel family, shape as in config, source hash, bytes per launch), ...]
    "c2": [("row-lane", {"rows_per_block": 64, "ordinates_per_lane": 2, "waves_per_group": 4}, "0598a01edc4a0c77", 38940000)],
    "c1": [("row-lane", {"rows_per_block": 64, "ordinates_per_lane": 1, "waves_per_group": 2}, "0598a01edc4a0c77", 1690000)],
    "c3": [("strip", {"sweep_tile": "16x16", "band": 7}, "1ae15ac46a2bed53", 827140000)],
    "c4": [("row-lane", {"rows_per_block": 16, "ordinates_per_lane": 4, "waves_per_group": 4}, "0598a01edc4a0c77", 459540000)],
    "c5": [("strip", {"sweep_tile": "16x16", "band": 4}, "1ae15ac46a2bed53", 3162290000)],
}


def kernel_hash(family):
    import hashlib
    m = hashlib.sha256()
    for f in KERNEL_SOURCES[family]:
        with open(os.path.join(ROOT, "paper_2407_12527_amd", "csrc", f), "rb") as fh:
            m.update(fh.read())
    return m.hexdigest()[:16]


def measured_traffic(workload, config):
    """HBM bytes per launch of the profiled kernel, if this run used a profiled shape and the
    kernel sources still hash to the profiled ones (else None)."""
    for family, shape, digest, nbytes in MEASURED_TRAFFIC.get(workload, []):
        if config.get("sweep_kernel") == family and all(config.get(k) == v for k, v in shape.items()):
            return nbytes if kernel_hash(family) == digest else None
    return None


DESCR = {
    "c1": "c1: 64x64, 32 iid sphere ordinates, sigma_t 1, sigma_s 0.5 iso, FP64, tol 1e-8",
    "c2": "c2: 256x256 7x7 checkerboard, 256 stratified random ordinates (seed 0), FP32 sweeps, tol 1e-6",
    "c3": "c3: 512x512, ensemble of 64 samples x 128 stratified random ordinates, FP32, tol 1e-6, FP64 mean/var",
    "c4": "c4: 256x256, HG g=0.8, 1024 stratified random ordinates, FP32 sweeps + BF16 MFMA contraction, tol 1e-6",
    "c5": "c5: 200 independent problems, sides in {64..1024}, n = 4m with m in 4..128, random 8x8 block maps, FP32, "
          "tol 1e-6, one persistent sweep launch per iteration",
}


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0, help="timed steps (0: a workload default of about 3 s)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c5", choices=sorted(DESCR))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-tte", action="store_true", help="skip the time-to-error measurement")
    ap.add_argument("--autotune", action="store_true", help="let the autotuner pick the sweep shape")
    ap.add_argument("--tile", default=None, help="sweep chunk x strip size, e.g. 8x4 (default: pinned)")
    ap.add_argument("--band", type=int, default=None,
                    help="strips (strip sweep) or row blocks (row-lane sweep) per workgroup (default: pinned)")
    ap.add_argument("--sweep", default=None, choices=["auto", "strip", "diag"], help="sweep kernel (default: pinned)")
    ap.add_argument("--diag-rows", type=int, default=None, help="row-lane sweep: rows per lane block (16, 64)")
    ap.add_argument("--diag-k", type=int, default=None, help="row-lane sweep: ordinates per lane (1, 2, 4)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a device-to-device copy of BYTES (reference for HBM byte counters)")
    a = ap.parse_args(argv)
    pin = {"sweep": "auto", "tile": "0x0", "band": 0, "diag_rows": 0, "diag_k": 0} if a.autotune else PINNED[a.workload]
    for k in ("sweep", "tile", "band", "diag_rows", "diag_k"):
        if getattr(a, k) is None:
            setattr(a, k, pin[k])
    if a.steps <= 0:
        a.steps = {"c1": 200, "c2": 200, "c3": 40, "c4": 20, "c5": 40}[a.workload]
    return a


def solve_opts(a, R, wl, precision=None):
    kind = {"auto": R.ROM_SWEEP_AUTO, "strip": R.ROM_SWEEP_STRIP, "diag": R.ROM_SWEEP_DIAG}[a.sweep]
    tile = tuple(int(v) for v in a.tile.lower().split("x"))
    prec = precision if precision is not None else (R.ROM_PREC_FP64 if wl.precision == "fp64" else R.ROM_PREC_FP32)
    return R.si_opts(tol=wl.tol, max_iter=wl.max_iter, precision=prec, tile=tile, band=a.band, sweep=kind,
                     diag_rows=a.diag_rows, diag_k=a.diag_k)


def sweep_shape(shape):
    """The sweep kernel and shape a solve ran with (as rom_si_stats reports them)."""
    tx, ty, band, lanes, kind = shape
    if kind == 2:
        return {"sweep_kernel": "row-lane", "rows_per_block": ty, "ordinates_per_lane": tx, "waves_per_group": band}
    return {"sweep_kernel": "strip", "sweep_tile": f"{tx}x{ty}", "band": band, "lanes_per_group": lanes}


def calibrate_copy(nbytes):
    """A plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE counters give the scale
    factor between the counters and bytes moved."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": nbytes, "copies": 3}), flush=True)


def copy_bandwidth(torch, nbytes=1 << 30, reps=5):
    """Achievable HBM bandwidth on this GPU: a device-to-device copy of `nbytes` (read + write),
    timed with events on the copy's stream, median of `reps`."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    del src, dst
    return 2 * nbytes / statistics.median(ts) / 1e9


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def timed_median(fn, reps=3):
    """(median seconds, last result) of `reps` runs of fn."""
    ts, out = [], None
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        ts.append(time.perf_counter() - t0)
    return statistics.median(ts), out


def c5_cpu_subset(wl, count=20):
    """A fixed stratified subset of c5: problems ranked by cells x ordinates, the median problem of
    each of `count` equal strata of the ranking."""
    cost = np.array([f.cells * wl.n_ord[k] for k, f in enumerate(wl.fields)])
    order = np.argsort(cost, kind="stable")
    return [int(order[(2 * s + 1) * len(order) // (2 * count)]) for s in range(count)]


def oracle_rate(O, jobs, reps=3):
    """Median-of-`reps` updates/s of the oracle over `jobs` [(Problem, dirs, w, W, max_iter)], each
    run for exactly max_iter source iterations (no early stop)."""
    updates = sum(p.cells * len(w) * it for p, d, w, W, it in jobs)

    def run():
        for p, d, w, W, it in jobs:
            O.source_iterate(p, d, w, W, tol=-1.0, max_iter=it)

    dt, _ = timed_median(run, reps)
    return updates / dt, updates, dt


def cpu_baseline(workload, wl, gpu_updates_per_step):
    """The FP64 oracle as it stands (never tuned for this), on this host: median of 3 runs with all
    its OpenMP threads and with one thread, on a bounded sample of the workload (every ordinate
    set bit-identical to the GPU's)."""
    import oracle as O
    jobs = []
    if workload == "c5":
        sub = c5_cpu_subset(wl)
        for k in sub:
            f = wl.fields[k]
            nz, nt = O.stratified_spec(wl.n_ord[k])
            d, w = O.generate(O.ORD_STRATIFIED, nz, nt, seed=wl.problem_seed(k))
            jobs.append((O.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q), d, w, None, 1))
        what = (f"one source iteration of each of {len(sub)} c5 problems, a fixed stratified subset (the median "
                f"problem of each twentieth of the ranking by cells x ordinates)")
    else:
        f = wl.fields[0]
        n = wl.n_ord[0]
        if wl.ord_kind == "stratified":
            nz, nt = O.stratified_spec(n)
            d, w = O.generate(O.ORD_STRATIFIED, nz, nt, seed=wl.seed)
        else:
            d, w = O.generate(O.ORD_IID_SPHERE, n, seed=wl.seed)
        W = O.build_W(d, w, O.SCAT_HG, wl.g, fold=1) if wl.scattering == "hg" else None
        p = O.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
        iters = 1 if W is not None else 2
        samples = min(wl.samples, 4)
        for s in range(samples):
            if wl.samples > 1:
                nz, nt = O.stratified_spec(n)
                d, w = O.generate(O.ORD_STRATIFIED, nz, nt, seed=wl.seed, sample=s)
            jobs.append((p, d, w, W, iters))
        what = f"{iters} source iteration(s) of {samples} sample(s) of {workload}"
    threads = O.num_threads()
    rate, updates, dt = oracle_rate(O, jobs)
    O.set_num_threads(1)
    try:
        rate1, _, dt1 = oracle_rate(O, jobs)
    finally:
        O.set_num_threads(threads)
    return {"value": rate, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{what}: {updates:.3g} updates, median of 3 runs {dt:.2f} s (all cores), {dt1:.2f} s (1 core)",
            "single_core": {"value": rate1, "cores": 1},
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "runs": 3, "statistic": "median",
            "extrapolated_step_s": gpu_updates_per_step / rate,
            "extrapolation": "seconds the oracle would take for one GPU step's updates at the measured rate "
                             "(its cost per update does not depend on the iteration)"}


def time_to_error(R, torch):
    """bench_tte.py's protocol on the 64 x 64 isotropic problem, reduced to its summary."""
    import bench_tte as T
    s = T.measure(T.options(problem="iso64", quiet=True), R, torch)
    rom = {n: {"median_s": v["median_seconds"], "t": v["t"]} for n, v in s["rom"].items()}
    return {"problem": "iso64: 64x64, sigma_t 1, sigma_s 0.5, q = 1 on the central 0.1 square, vacuum",
            "error": "l2 (rms over cells) against FP64 DOM, 80400 Gaussian ordinates",
            "eps": s["eps_l2"], "eps_from": "FP64 DOM, uniform quadrature N = 6 (144 ordinates)",
            "T_DOM_fp64_s": s["T_DOM_fp64"], "T_DOM_fp32_s": s["T_DOM_fp32"], "T_ROM_s": s["T_ROM"],
            "rom_fp32_by_ordinates": rom, "seed_blocks": 5,
            "rom_over_dom_fp64": (s["T_ROM"] / s["T_DOM_fp64"]) if s["T_ROM"] and s["T_DOM_fp64"] else None,
            "replaces": "the M^2 vs t N^2 cost comparison of Sec. 4.2"}


def roofline(kind, scattering, fp64, upd_per_launch, avg_s, traffic, copy_gbs):
    if scattering == "iso" or scattering == "linear":
        achieved = FLOPS_PER_UPDATE * upd_per_launch / avg_s / 1e12
        peak = FP64_VECTOR_PEAK_TFLOPS if fp64 else FP32_VECTOR_PEAK_TFLOPS
        r = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak}
        if not fp64:
            r["frac_of_unpacked_fp32"] = achieved / FP32_UNPACKED_TFLOPS
        alg = BYTES_PER_ISO_UPDATE * upd_per_launch * (2 if fp64 else 1)
    else:
        achieved = BYTES_PER_ANG_UPDATE * upd_per_launch / avg_s / 1e9
        r = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": achieved / HBM_PEAK_GBS, "frac_of_copy": achieved / copy_gbs}
        alg = BYTES_PER_ANG_UPDATE * upd_per_launch
    r.update({"traffic": traffic, "kernel": kind, "avg_launch_us": avg_s * 1e6, "updates_per_launch": upd_per_launch,
              "updates_per_s_in_kernel": upd_per_launch / avg_s, "flops_per_update": FLOPS_PER_UPDATE,
              "algorithmic_bytes_per_launch": alg, "copy_gbs": copy_gbs})
    if traffic is not None:
        r["traffic_unit"] = "bytes per launch"
        r["hbm_gbs"] = traffic / avg_s / 1e9
        r["hbm_frac_of_peak"] = r["hbm_gbs"] / HBM_PEAK_GBS
        r["hbm_frac_of_copy"] = r["hbm_gbs"] / copy_gbs
        r["traffic_over_algorithmic"] = traffic / alg
    return r


def main():
    a = parse()
    if a.calibrate_copy:
        calibrate_copy(a.calibrate_copy)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2407_12527_amd import rom as R
    torch.cuda.set_device(0)

    wl = RI.WORKLOADS[a.workload]()
    fp64 = wl.precision == "fp64"
    opts = solve_opts(a, R, wl)
    shape = [0, 0, 0, 0, 0]

    if a.workload == "c5":
        hs = []
        for k, f in enumerate(wl.fields):
            h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
            m = wl.n_ord[k] // 4
            nz = max(d for d in range(1, int(m ** 0.5) + 1) if m % d == 0)
            d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, nz, m // nz, seed=wl.problem_seed(k))
            h.set_ordinates(d, w)
            hs.append(h)

        def step():
            _, stats, rc = R.solve_batch(hs, opts, download=False)  # fluxes stay in HBM
            if rc != 0:
                raise RuntimeError(f"batch did not converge (status {rc})")
            shape[:] = [stats[0].tile_x, stats[0].tile_y, stats[0].band, stats[0].lanes, stats[0].sweep]
            return sum(s.updates for s in stats), stats[0].sweep_ms, stats[0].sweeps, max(s.iters for s in stats)

        config = {"workload": DESCR["c5"], "problems": len(hs), "cells": sum(f.cells for f in wl.fields)}
    else:
        f = wl.fields[0]
        h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
        n = wl.n_ord[0]
        if wl.ord_kind == "stratified":
            m = n // 4
            nz = max(d for d in range(1, int(m ** 0.5) + 1) if m % d == 0)
            spec = (R.ROM_ORD_STRATIFIED, nz, m // nz)
        else:
            spec = (R.ROM_ORD_IID_SPHERE, n, 0)
        if wl.scattering == "hg":
            h.set_scattering(R.ROM_SCAT_HG, wl.g)
        ens = wl.samples > 1
        dirs, w = R.generate_ordinates(spec[0], spec[1], spec[2], seed=wl.seed, sample=0)

        def step():
            if ens:
                _, _, st, rc = h.ensemble(wl.samples, wl.seed, spec[0], spec[1], spec[2], opts, download=False)
                if rc != 0:
                    raise RuntimeError(f"ensemble did not converge (status {rc})")
                shape[:] = [st.tile_x, st.tile_y, st.band, st.lanes, st.sweep]
                return st.updates, st.sweep_ms, st.sweeps, st.max_iters
            h.set_ordinates(dirs, w)                     # ordinate ingestion
            _, st, rc = h.source_iterate(opts, download=False)
            if rc != 0:
                raise RuntimeError(f"solve did not converge (status {rc})")
            shape[:] = [st.tile_x, st.tile_y, st.band, st.lanes, st.sweep]
            return st.updates, st.sweep_ms, st.sweeps, st.iters

        config = {"workload": DESCR[a.workload], "cells": f.cells, "ordinates": n, "samples": wl.samples}

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot_upd, tot_sweep_ms, tot_sweeps, iters = 0, 0.0, 0, 0
    for _ in range(a.steps):
        u, sm, ns, it = step()
        tot_upd += u
        tot_sweep_ms += sm
        tot_sweeps += ns
        iters = it
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    config.update({"si_iterations": iters, **sweep_shape(shape), "shape_pinned": not a.autotune})
    copy_gbs = copy_bandwidth(torch)
    roof = None
    if tot_sweeps > 0:
        avg_s = tot_sweep_ms / tot_sweeps / 1e3
        upd_per_launch = tot_upd / tot_sweeps  # every running system sweeps once per launch
        kernel = "diag_kernel" if shape[4] == 2 else "sweep_kernel"
        roof = roofline(kernel, wl.scattering, fp64, upd_per_launch, avg_s, measured_traffic(a.workload, config),
                        copy_gbs)
    out = {
        "metric": "cell·ordinate sweep updates/s",
        "value": tot_upd / dt,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if fp64 else "f32",
        "data": "synthetic",
        "config": config,
        "roofline": roof,
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(a.workload, wl, tot_upd / a.steps)
    if not a.no_tte:
        out["tte"] = time_to_error(R, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
