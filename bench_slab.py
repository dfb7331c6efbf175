"""ROM convergence in slab geometry (Sec. 4.1, Example 4.1, Table 2).

Example 4.1 on [0, 1] with nx = 50 cells (unknowns at the 51 grid points), the three inflow
cases, FP64.  Reference: DOM with 2560 Gauss-Legendre ordinates, source iteration to 1e-13.  For
n = 2, 4, 8, 16 ROM ordinates (Delta mu = 2/n = 1, 1/2, 1/4, 1/8), t samples (20 480 by default)
are solved in one launch each and every sample's flux is kept, giving

  * the error E = mean over samples of ||phi^xi - phi_ref||_2 (rms over the 51 points, Sec. 4.1);
  * the bias B = ||mean of phi^xi - phi_ref||_2 and its Monte Carlo noise;
  * the Monte Carlo error of an average of t' samples (rms over disjoint blocks) and its slope;

and the orders of E and B in Delta mu (least squares over the four n), which Table 2 prints as
1.37 / 1.32 / 1.04 (E) and 2.57 / 2.92 / 2.37 (B) for cases 1 / 2 / 3.  The paper's own spatial
scheme ([ShiA]) is not given in its text; this solver uses diamond difference at the grid points
for the reference and the samples alike.

Usage: python bench_slab.py [--t 20480] [--out FILE]; one JSON line per (case, n), then a summary.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

import rom_inputs as RI


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--t", type=int, default=20480)
    ap.add_argument("--nx", type=int, default=50)
    ap.add_argument("--ref-n", type=int, default=2560)
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--out", default="")
    return ap.parse_args()


def l2(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2)))


def slope(x, y):
    return float(np.polyfit(np.log(np.asarray(x)), np.log(np.asarray(y)), 1)[0])


def main():
    a = parse()
    import torch
    from paper_2407_12527_amd import rom as R
    torch.cuda.set_device(0)
    outf = open(a.out, "a") if a.out else None

    def emit(rec):
        line = json.dumps(rec)
        print(line, flush=True)
        if outf:
            outf.write(line + "\n")
            outf.flush()

    o_ref = R.si_opts(tol=1e-13, max_iter=20000, precision=R.ROM_PREC_FP64)
    o = R.si_opts(tol=1e-12, max_iter=20000, precision=R.ROM_PREC_FP64)
    summary = {"arm": "summary", "t": a.t, "cases": {}}
    t0 = time.perf_counter()
    for case in (1, 2, 3):
        f = RI.slab_example41(a.nx, case)
        s = R.Slab(f.nx, f.sigma_t, f.sigma_s, f.q)
        mu, w = R.slab_ordinates(R.ROM_SLAB_GAUSS, a.ref_n)
        ts = time.perf_counter()
        ref, it, _, rc = s.solve(mu, w, f.inflow(mu), o_ref)
        if rc != 0:
            raise RuntimeError(f"reference did not converge (status {rc})")
        ref = ref[0]
        emit({"arm": "reference", "case": case, "ordinates": a.ref_n, "iters": int(it[0]),
              "seconds": time.perf_counter() - ts})
        rows = []
        for n in (2, 4, 8, 16):
            ts = time.perf_counter()
            sets = [R.slab_ordinates(R.ROM_SLAB_RANDOM, n, a.seed, k) for k in range(a.t)]
            mus = np.array([m for m, _ in sets])
            ws = np.array([ww for _, ww in sets])
            phis, iters, st, rc = s.solve(mus, ws, f.inflow(mus), o)
            if rc != 0:
                raise RuntimeError(f"case {case} n={n}: status {rc}")
            errs = np.sqrt(np.mean((phis - ref[None, :]) ** 2, axis=1))
            mean = phis.mean(axis=0)
            mc, tp = [], 1
            while tp <= a.t // 2:
                nb = a.t // tp
                bm = phis[: nb * tp].reshape(nb, tp, -1).mean(axis=1)
                mc.append((tp, float(np.sqrt(np.mean(np.mean((bm - mean[None, :]) ** 2, axis=1))))))
                tp *= 2
            fit = [(m, e) for m, e in mc if m <= a.t // 64]
            rec = {"arm": "rom", "case": case, "n": n, "delta_mu": 2.0 / n, "t": a.t,
                   "E": float(errs.mean()), "E_std_err": float(errs.std() / math.sqrt(a.t)),
                   "B": l2(mean, ref), "B_noise": float(np.sqrt(np.mean(phis.var(axis=0, ddof=1)) / a.t)),
                   "mc_slope": slope([m for m, _ in fit], [e for _, e in fit]), "max_iters": int(iters.max()),
                   "device_ms": st.device_ms, "seconds": time.perf_counter() - ts}
            rows.append(rec)
            emit(rec)
        dm = [r["delta_mu"] for r in rows]
        summary["cases"][case] = {"E": {r["n"]: r["E"] for r in rows}, "B": {r["n"]: r["B"] for r in rows},
                                  "B_noise": {r["n"]: r["B_noise"] for r in rows},
                                  "order_E": slope(dm, [r["E"] for r in rows]),
                                  "order_B": slope(dm, [r["B"] for r in rows]),
                                  "mc_slope": [r["mc_slope"] for r in rows]}
    summary["seconds"] = time.perf_counter() - t0
    emit(summary)


if __name__ == "__main__":
    sys.exit(main())
