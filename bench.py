"""Benchmark: cell-ordinate sweep updates/s of ROM source iteration on one MI355X.

One step = one pass of the whole hot path over the workload's synthetic input: ordinate
ingestion (rom_set_ordinates), source iteration to convergence (sweeps + partial-flux combine +
FP64 residual, replayed from a captured HIP graph) and the result left resident in HBM.  The
default workload is c2 (256 x 256 checkerboard, 256 stratified random ordinates, FP32 sweeps,
tolerance 1e-6).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c3|c4|c1] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import rom_inputs as RI  # noqa: E402

# Algorithmic work of one upwind cell-ordinate update: w*S (1 mul), + a*x and + b*y (2 fma = 4
# flops), sigma_t + a + b (1 add), the division (1), and the scalar-flux accumulation (1 add).
FLOPS_PER_UPDATE = 8
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X datasheet, FP32 vector
FP64_VECTOR_PEAK_TFLOPS = 78.6
BF16_MFMA_PEAK_TFLOPS = 2500.0
HBM_PEAK_GBS = 8000.0
BYTES_PER_ANG_UPDATE = 6         # FP32 source read + BF16 angular flux written, per update

# HBM bytes per sweep launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (scaled by a 256 MiB copy:
# 1 FETCH_SIZE KiB = 2 KiB read, 1 WRITE_SIZE KiB = 1 KiB written), for the kernel shape the
# autotuner picks on each workload.  Reported only while the kernel sources hash to what was
# profiled and the run used that shape; otherwise `traffic` is null.
KERNEL_SOURCES = {
    "row-lane": ["rom_common.h", "rom_device.h", "rom_diag.h", "rom_diag_f32.hip", "rom_diag_f64.hip"],
    "strip": ["rom_common.h", "rom_device.h", "rom_sweep.h", "rom_sweep_f32_16x16.hip", "rom_sweep_f32_16x8.hip",
              "rom_sweep_f32_8x4.hip", "rom_sweep_f32_8x8.hip", "rom_sweep_f64.hip"],
}
MEASURED_TRAFFIC = {  # workload: [(kernel family, shape as in config, source hash, bytes per launch), ...]
    "c2": [("row-lane", {"rows_per_block": 16, "ordinates_per_lane": 1, "waves_per_group": 4}, "e1f013e8ca59fc4f", 25516675),
           ("row-lane", {"rows_per_block": 64, "ordinates_per_lane": 2, "waves_per_group": 4}, "e1f013e8ca59fc4f", 38900795),
           ("row-lane", {"rows_per_block": 64, "ordinates_per_lane": 2, "waves_per_group": 2}, "e1f013e8ca59fc4f", 40638020)],
    "c1": [("row-lane", {"rows_per_block": 64, "ordinates_per_lane": 1, "waves_per_group": 2}, "e1f013e8ca59fc4f", 1810208),
           ("row-lane", {"rows_per_block": 64, "ordinates_per_lane": 1, "waves_per_group": 1}, "e1f013e8ca59fc4f", 1825374)],
    "c3": [("strip", {"sweep_tile": "16x16", "band": 4}, "18d77716fe5ec93c", 938536546)],
    "c4": [("strip", {"sweep_tile": "8x4", "band": 4}, "18d77716fe5ec93c", 446640762)],
    "c5": [("strip", {"sweep_tile": "16x16", "band": 4}, "18d77716fe5ec93c", 2737417550)],
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
    "c3": "c3: 512x512, ensemble of 64 samples x 128 stratified random ordinates, FP32, tol 1e-6",
    "c4": "c4: 256x256, HG g=0.8, 1024 stratified random ordinates, FP32 sweeps + BF16 MFMA contraction, tol 1e-6",
    "c5": "c5: 200 independent problems, sides in {64..1024}, n = 4m with m in 4..128, random 8x8 block maps, FP32, "
          "tol 1e-6, one persistent sweep launch per iteration",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2", choices=sorted(DESCR))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--tile", default="0x0", help="sweep chunk x strip size, e.g. 8x4 (0x0: automatic)")
    ap.add_argument("--band", type=int, default=0,
                    help="strips (strip sweep) or row blocks (row-lane sweep) per workgroup (0: automatic)")
    ap.add_argument("--sweep", default="auto", choices=["auto", "strip", "diag"],
                    help="sweep kernel (auto: the autotuner's choice)")
    ap.add_argument("--diag-rows", type=int, default=0, help="row-lane sweep: rows per lane block (16, 64)")
    ap.add_argument("--diag-k", type=int, default=0, help="row-lane sweep: ordinates per lane (1, 2, 4)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a device-to-device copy of BYTES (reference for HBM byte counters)")
    return ap.parse_args()


def kernel_opts(a, R):
    kind = {"auto": R.ROM_SWEEP_AUTO, "strip": R.ROM_SWEEP_STRIP, "diag": R.ROM_SWEEP_DIAG}[a.sweep]
    return {"sweep": kind, "diag_rows": a.diag_rows, "diag_k": a.diag_k}


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


def cpu_baseline(workload, seconds):
    """The FP64 oracle as it stands, on this host's cores, over whole solves of the same workload
    (repeated until about `seconds` of work); result in updates/s."""
    import oracle as O
    wl = RI.WORKLOADS[workload]()
    f = wl.fields[0]
    prob = O.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    n = wl.n_ord[0]
    if wl.ord_kind == "stratified":
        nz, nt = O.stratified_spec(n)
        dirs, w = O.generate(O.ORD_STRATIFIED, nz, nt, seed=wl.seed)
    else:
        dirs, w = O.generate(O.ORD_IID_SPHERE, n, seed=wl.seed)
    W = None
    if wl.scattering == "hg":
        W = O.build_W(dirs, w, O.SCAT_HG, wl.g, fold=1)
    updates, reps = 0, 0
    t0 = time.perf_counter()
    while True:
        max_iter = wl.max_iter if W is None else 2  # anisotropic: a bounded sample of iterations
        r = O.source_iterate(prob, dirs, w, W, tol=wl.tol if W is None else -1.0, max_iter=max_iter)
        updates += r["iters"] * f.cells * n
        reps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    what = f"{reps} full solve(s) of {workload}" if W is None else f"{reps} x 2 SI iterations of {workload}"
    return {"value": updates / dt, "unit": "updates/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{what}, {updates:.3g} updates in {dt:.1f} s"}


def bench_batch(a, wl, R, torch):
    """c5: all problems in one rom_solve_batch per step."""
    hs = []
    for k, f in enumerate(wl.fields):
        h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
        m = wl.n_ord[k] // 4
        nz = max(d for d in range(1, int(m ** 0.5) + 1) if m % d == 0)
        d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, nz, m // nz, seed=wl.problem_seed(k))
        h.set_ordinates(d, w)
        hs.append(h)
    tile = tuple(int(v) for v in a.tile.lower().split("x"))
    opts = R.si_opts(tol=wl.tol, max_iter=wl.max_iter, tile=tile, band=a.band, **kernel_opts(a, R))
    for _ in range(a.warmup):
        R.solve_batch(hs, opts, download=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    upd, sweep_ms, sweeps, iters, shape = 0, 0.0, 0, 0, [0, 0, 0, 0, 0]
    for _ in range(a.steps):
        _, stats, rc = R.solve_batch(hs, opts, download=False)  # fluxes stay in HBM
        if rc != 0:
            raise RuntimeError(f"batch did not converge (status {rc})")
        upd += sum(s.updates for s in stats)
        sweep_ms += stats[0].sweep_ms
        sweeps += stats[0].sweeps
        iters = max(s.iters for s in stats)
        shape = [stats[0].tile_x, stats[0].tile_y, stats[0].band, stats[0].lanes, stats[0].sweep]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # Every problem sweeps once per iteration until it converges, so the work of all sweep
    # launches is exactly the reported updates; achieved = flops / summed sweep time.
    avg_s = sweep_ms / max(sweeps, 1) / 1e3
    achieved = FLOPS_PER_UPDATE * upd / (sweep_ms / 1e3) / 1e12
    out = {"metric": "cell·ordinate sweep updates/s", "value": upd / dt, "unit": "updates/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": dt / a.steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": DESCR["c5"], "problems": len(hs), "cells": sum(f.cells for f in wl.fields),
                      "si_iterations": iters, **sweep_shape(shape)},
           "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": None, "kernel": "sweep_kernel",
                        "avg_launch_us": avg_s * 1e6, "updates_per_launch": upd / max(sweeps, 1)}}
    out["roofline"]["traffic"] = measured_traffic("c5", out["config"])
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline_batch(wl, a.cpu_seconds)
    print(json.dumps(out), flush=True)


def cpu_baseline_batch(wl, seconds):
    """The oracle over the batch's problems in order, whole solves, until about `seconds`."""
    import oracle as O
    updates, done = 0, 0
    t0 = time.perf_counter()
    for k, f in enumerate(wl.fields):
        prob = O.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
        nz, nt = O.stratified_spec(wl.n_ord[k])
        dirs, w = O.generate(O.ORD_STRATIFIED, nz, nt, seed=wl.problem_seed(k))
        r = O.source_iterate(prob, dirs, w, None, tol=wl.tol, max_iter=wl.max_iter)
        updates += r["iters"] * f.cells * len(w)
        done += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": updates / dt, "unit": "updates/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"first {done} of {len(wl.fields)} problems of c5 solved, {updates:.3g} updates in {dt:.1f} s"}


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
    if a.workload == "c5":
        return bench_batch(a, wl, R, torch)
    f = wl.fields[0]
    h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    n = wl.n_ord[0]
    fp64 = wl.precision == "fp64"
    prec = R.ROM_PREC_FP64 if fp64 else R.ROM_PREC_FP32
    tile = tuple(int(v) for v in a.tile.lower().split("x"))
    opts = R.si_opts(tol=wl.tol, max_iter=wl.max_iter, precision=prec, tile=tile, band=a.band, **kernel_opts(a, R))
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
            shape[:] = [st.tile_x, st.tile_y, st.band, st.lanes, st.sweep]
            return st.updates, st.sweep_ms, st.sweeps, st.max_iters
        h.set_ordinates(dirs, w)                     # ordinate ingestion
        _, st, rc = h.source_iterate(opts, download=False)
        if rc != 0:
            raise RuntimeError(f"solve did not converge (status {rc})")
        shape[:] = [st.tile_x, st.tile_y, st.band, st.lanes, st.sweep]
        return st.updates, st.sweep_ms, st.sweeps, st.iters

    shape = [0, 0, 0, 0, 0]

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

    value = tot_upd / dt
    roof = None
    if tot_sweeps > 0:
        avg_s = tot_sweep_ms / tot_sweeps / 1e3
        upd_per_sweep = f.cells * n * wl.samples
        kernel = "diag_kernel" if shape[4] == 2 else "sweep_kernel"
        if wl.scattering == "iso":
            achieved = FLOPS_PER_UPDATE * upd_per_sweep / avg_s / 1e12
            peak = FP64_VECTOR_PEAK_TFLOPS if fp64 else FP32_VECTOR_PEAK_TFLOPS
            roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak}
        else:
            # the sweep of a dense-kernel problem streams the per-ordinate source in and the
            # angular flux out: S (4 B) + psi (BF16, 2 B) per update
            achieved = BYTES_PER_ANG_UPDATE * upd_per_sweep / avg_s / 1e9
            roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS}
        roof.update({"traffic": None, "kernel": kernel, "avg_launch_us": avg_s * 1e6,
                     "updates_per_launch": upd_per_sweep})
    out = {
        "metric": "cell·ordinate sweep updates/s",
        "value": value,
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
        "config": {"workload": DESCR[a.workload], "cells": f.cells, "ordinates": n, "samples": wl.samples,
                   "si_iterations": iters, **sweep_shape(shape)},
        "roofline": roof,
    }
    if roof is not None:
        roof["traffic"] = measured_traffic(a.workload, out["config"])
        if roof["traffic"] is not None:
            roof["traffic_unit"] = "bytes per launch"
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(a.workload, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
