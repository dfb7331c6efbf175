"""Time to a fixed error: batched ROM ensembles against plain DOM on one GPU.

The paper compares DOM and ROM by cost model: M^2 for DOM with M ordinates and t*N^2 for t ROM
samples of N ordinates (Sec. 4.2, comparison of complexity, Fig. on cost versus error).  This
script replaces that model with wall-clock time on the device, for the same three ingredients:

  * reference phi_ref: FP64 DOM with the Gaussian quadrature of Appendix A (2N(N+1) ordinates;
    N = 200 gives the paper's 80 400), same grid, same upwind scheme, source iteration to 1e-10;
  * error: the l2 norm over cell centres of Sec. 2.2 (root mean square of phi - phi_ref), plus
    the max-norm e_inf of Sec. 4.2;
  * target eps: the error of FP64 DOM with the uniform quadrature of Appendix A at N = 6
    (144 ordinates, the DOM point the paper sets against ROM in Sec. 4.2).

DOM arm: uniform quadrature, N = 2..22, FP64 (and FP32 as context).  T_DOM(eps) is the shortest
solve whose error is at most eps.  ROM arm: stratified symmetric ordinates (Sec. 3.1) with
n = 16, 36, 64 per sample, ensembles of t = 1, 2, 4, ... samples in FP32 (BF16 contraction for
an anisotropic kernel); T_ROM(eps) is the time of the first ensemble whose mean reaches eps,
the median over five disjoint master seeds.  Every timed call is warm (its plan built and tuned
by an untimed call before) and includes the solve and the download of the result; a ROM call
also generates and ingests every sample's ordinates (and kernel matrix), while a DOM quadrature
is fixed and ingested once, untimed.  The median of three calls is reported.  A ROM seed whose
ensemble meets a diverging sample (possible for an unnormalized, strongly peaked kernel on a
random set) is reported as such and never reaches eps.

Problems (vacuum, unit square):
  iso64   -- 64 x 64,  sigma_t = 1, sigma_s = 0.5, isotropic, q = 1 on [0.45, 0.55)^2
  iso512  -- 512 x 512, sigma_t = 1, sigma_s = 0.5, isotropic, q = 1 on [0.49, 0.51)^2
  aniso64 -- 64 x 64,  sigma_t = 1, sigma_s = 0.8, Henyey-Greenstein g = 0.8 folded over the
             polar sign and row-normalized (every arm, the reference included), q = 1 on
             [0.45, 0.55)^2; the raw kernel makes some small random samples diverge
  aniso64raw -- the same with the raw (unnormalized) kernel
  aniso256 -- aniso64 on 256 x 256 cells, q = 1 on [0.45, 0.55)^2
  lin64   -- iso64 with the paper's linear kernel 1 + g cos(xi), g = 0.9 (eq. (2.1)), raw

Usage: python bench_tte.py --problem iso64 [--out FILE]; one JSON line per measurement on
stdout (flushed as it is taken), then a summary line.
"""
from __future__ import annotations

import argparse
import json
import math
import statistics
import sys
import time

import numpy as np

import rom_inputs as RI

PROBLEMS = {
    "iso64": dict(nx=64, sigma_s=0.5, lo=0.45, hi=0.55, scat="iso", g=0.0, ref_n=200),
    "iso512": dict(nx=512, sigma_s=0.5, lo=0.49, hi=0.51, scat="iso", g=0.0, ref_n=200),
    "aniso64": dict(nx=64, sigma_s=0.8, lo=0.45, hi=0.55, scat="hg", g=0.8, ref_n=80, norm=True),
    "aniso64raw": dict(nx=64, sigma_s=0.8, lo=0.45, hi=0.55, scat="hg", g=0.8, ref_n=80),
    "aniso256": dict(nx=256, sigma_s=0.8, lo=0.45, hi=0.55, scat="hg", g=0.8, ref_n=80, norm=True),
    "lin64": dict(nx=64, sigma_s=0.5, lo=0.45, hi=0.55, scat="linear", g=0.9, ref_n=200),
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--problem", default="iso64", choices=sorted(PROBLEMS))
    ap.add_argument("--ref-n", type=int, default=0, help="Gaussian N of the reference (0: problem default)")
    ap.add_argument("--dom-n", default="2-22", help="uniform quadrature N range of the DOM arm")
    ap.add_argument("--rom-n", default="16,36,64", help="ordinates per ROM sample")
    ap.add_argument("--t-max", type=int, default=4096)
    ap.add_argument("--seeds", type=int, default=5, help="disjoint master seeds of the ROM arm")
    ap.add_argument("--repeats", type=int, default=3)
    ap.add_argument("--tol", type=float, default=1e-6, help="source-iteration tolerance of both arms")
    ap.add_argument("--out", default="", help="also append every JSON line to this file")
    a = ap.parse_args()
    a.quiet = False
    return a


def l2_err(phi, ref):
    return float(np.sqrt(np.mean((phi - ref) ** 2)))


def inf_err(phi, ref):
    return float(np.max(np.abs(phi - ref)))


class Runner:
    def __init__(self, a, R, torch):
        self.a, self.R, self.torch = a, R, torch
        p = PROBLEMS[a.problem]
        self.p = p
        f = RI.uniform_fields(p["nx"], p["nx"], 1.0, p["sigma_s"], p["lo"], p["hi"])
        self.f = f
        self.h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
        if p["scat"] != "iso":
            kind = R.ROM_SCAT_HG if p["scat"] == "hg" else R.ROM_SCAT_LINEAR
            self.h.set_scattering(kind | (R.ROM_SCAT_NORMALIZE if p.get("norm") else 0), p["g"])
        self.outf = open(a.out, "a") if a.out else None

    def emit(self, rec):
        rec = {"problem": self.a.problem, **rec}
        line = json.dumps(rec)
        if not getattr(self.a, "quiet", False):
            print(line, flush=True)
        if self.outf:
            self.outf.write(line + "\n")
            self.outf.flush()

    def opts(self, fp64, tol, max_iter=20000):
        R = self.R
        return R.si_opts(tol=tol, max_iter=max_iter, precision=R.ROM_PREC_FP64 if fp64 else R.ROM_PREC_FP32)

    def timed(self, fn):
        """Warm-up call, then the median wall time of `repeats` calls (each synchronous)."""
        out = fn()
        ts = []
        for _ in range(self.a.repeats):
            self.torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            ts.append(time.perf_counter() - t0)
        return out, statistics.median(ts)

    def dom(self, kind, N, fp64, tol, timed=True):
        R = self.R
        dirs, w = R.generate_ordinates(kind, N)
        o = self.opts(fp64, tol)
        self.h.set_ordinates(dirs, w)  # a fixed quadrature: ingested once, outside the timing

        def run():
            phi, st, rc = self.h.source_iterate(o)
            if rc != 0:
                raise RuntimeError(f"DOM solve N={N} did not converge (status {rc})")
            return phi, st

        if timed:
            (phi, st), dt = self.timed(run)
        else:
            t0 = time.perf_counter()
            phi, st = run()
            dt = time.perf_counter() - t0
        return phi, st, dt, len(w)

    def rom(self, nq, t, seed, tol):
        """Ensemble of t samples; None when a sample's iteration diverges (a kernel matrix whose
        weighted row sums exceed sigma_t / sigma_s for that ordinate set)."""
        R = self.R
        o = self.opts(False, tol)

        def run():
            mean, _, st, rc = self.h.ensemble(t, seed, R.ROM_ORD_STRATIFIED, nq, nq, o)
            if rc != 0:
                raise RuntimeError(f"ROM ensemble n={4 * nq * nq} t={t} did not converge (status {rc})")
            return mean, st

        try:
            (mean, st), dt = self.timed(run)
        except R.RomError as e:
            if e.status != R.ROM_E_DIVERGED:
                raise
            return None, None, None
        return mean, st, dt


def main():
    a = parse()
    import torch
    from paper_2407_12527_amd import rom as R
    torch.cuda.set_device(0)
    measure(a, R, torch)


def options(**kw):
    """The command-line defaults as an argparse namespace, overridden by `kw` (for callers that
    import this module, such as bench.py)."""
    ns = argparse.Namespace(problem="iso64", ref_n=0, dom_n="2-22", rom_n="16,36,64", t_max=4096, seeds=5,
                            repeats=3, tol=1e-6, out="", quiet=False)
    for k, v in kw.items():
        setattr(ns, k, v)
    return ns


def measure(a, R, torch):
    """Run the whole protocol for a.problem; emits one JSON line per measurement (unless
    a.quiet) and returns the summary record."""
    run = Runner(a, R, torch)
    p = run.p
    ref_n = a.ref_n or p["ref_n"]
    t_start = time.perf_counter()

    # reference and a coarser Gaussian solve that bounds its own error
    phi_ref, st, dt, nref = run.dom(R.ROM_ORD_GAUSS2D, ref_n, True, 1e-10, timed=False)
    run.emit({"arm": "reference", "quadrature": "gauss", "N": ref_n, "ordinates": nref, "iters": st.iters,
              "seconds": dt})
    half = max(2, ref_n // 2)
    phi_half, st, dt, nh = run.dom(R.ROM_ORD_GAUSS2D, half, True, 1e-10, timed=False)
    ref_check = l2_err(phi_half, phi_ref)
    run.emit({"arm": "reference_check", "quadrature": "gauss", "N": half, "ordinates": nh, "l2": ref_check,
              "rel_l2": ref_check / float(np.sqrt(np.mean(phi_ref ** 2)))})

    # DOM arm
    lo, hi = (int(v) for v in a.dom_n.split("-"))
    dom_rows = []
    for fp64 in (True, False):
        for N in range(lo, hi + 1):
            phi, st, dt, n = run.dom(R.ROM_ORD_UNIFORM2D, N, fp64, a.tol)
            rec = {"arm": "dom", "precision": "fp64" if fp64 else "fp32", "N": N, "ordinates": n,
                   "iters": st.iters, "seconds": dt, "device_ms": st.device_ms, "l2": l2_err(phi, phi_ref),
                   "einf": inf_err(phi, phi_ref)}
            dom_rows.append(rec)
            run.emit(rec)
    eps_row = next(r for r in dom_rows if r["precision"] == "fp64" and r["N"] == 6)
    eps = eps_row["l2"]

    def t_dom(prec):
        ok = [r["seconds"] for r in dom_rows if r["precision"] == prec and r["l2"] <= eps]
        return min(ok) if ok else None

    # ROM arm
    rom_summary = {}
    diverged = []
    for n in (int(v) for v in a.rom_n.split(",")):
        nq = int(round(math.sqrt(n / 4)))
        if 4 * nq * nq != n:
            raise SystemExit(f"n = {n} is not 4 N^2")
        per_seed = []
        for sb in range(a.seeds):
            seed = 1000 + sb
            reached = None
            t = 1
            while t <= a.t_max:
                mean, st, dt = run.rom(nq, t, seed, a.tol)
                if mean is None:
                    # the diverging sample stays in every larger ensemble of this seed
                    run.emit({"arm": "rom", "ordinates": n, "seed": seed, "t": t, "diverged": True})
                    diverged.append((seed, t))
                    break
                e = l2_err(mean, phi_ref)
                rec = {"arm": "rom", "ordinates": n, "seed": seed, "t": t, "seconds": dt,
                       "device_ms": st.device_ms, "max_iters": st.max_iters, "l2": e, "einf": inf_err(mean, phi_ref)}
                run.emit(rec)
                if e <= eps:
                    reached = (t, dt)
                    break
                t *= 2
            per_seed.append(reached)
        hit = [r for r in per_seed if r is not None]
        rom_summary[n] = {
            "reached": len(hit), "seeds": a.seeds,
            "median_seconds": statistics.median(r[1] for r in hit) if len(hit) == a.seeds else None,
            "t": [r[0] if r else None for r in per_seed],
            "seconds": [r[1] if r else None for r in per_seed],
        }

    best_rom = [v["median_seconds"] for v in rom_summary.values() if v["median_seconds"] is not None]
    summary = {"arm": "summary", "eps_l2": eps, "eps_einf": eps_row["einf"], "tol": a.tol,
               "reference": {"gauss_N": ref_n, "ordinates": nref, "check_gauss_N": half, "check_l2": ref_check},
               "T_DOM_fp64": t_dom("fp64"), "T_DOM_fp32": t_dom("fp32"),
               "T_ROM": min(best_rom) if best_rom else None,
               "rom": {str(k): v for k, v in rom_summary.items()},
               "diverged": diverged, "wall_seconds": time.perf_counter() - t_start}
    run.emit(summary)
    return summary


if __name__ == "__main__":
    sys.exit(main())
