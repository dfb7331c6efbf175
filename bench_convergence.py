"""Convergence of ROM in X-Y geometry at the paper's scale (Sec. 4.2, Table 3, Figs. on the MC error
and on the error and bias orders).

Setup of Example 2.1 (100 x 100 cells, sigma_t = 1, sigma_s = 0.5, q = 2 on [0.4, 0.6]^2, vacuum),
diamond difference, FP64.  Reference: DOM with the Appendix A Gaussian quadrature, N = 200 (80 400
ordinates), source iteration to 1e-12.  For the isotropic kernel (g = 0) and the linear kernel
1 + g cos(xi) with g = 0.9 (eq. (2.1)), and for N = 1..4 (n = 4 N^2 stratified symmetric
ordinates per sample, Delta S = pi / (4 N^2)), t samples (10 240 by default) are solved and
each sample's flux is kept long enough to form

  * the error E = mean over samples of ||phi^xi - phi_ref||_2 (Sec. 4.1, l2 norm of Sec. 2.2);
  * the bias B = ||mean of phi^xi - phi_ref||_2;
  * the Monte Carlo error e_MC(t') = ||average of t' samples - average of all t|| (Sec. 4.1),
    estimated as the rms over the disjoint blocks of t' samples, for t' = 1, 2, 4, ...; its
    slope against t' (fitted for t' <= t/64) should be -1/2, and against (1/t' - 1/t)^(1/2),
    which accounts for the shared samples, exactly 1;

and the orders of E and B in Delta S (least squares over N = 1..4), which the paper reports as
0.74 and about 1.4.

Usage: python bench_convergence.py [--t 10240] [--out FILE]; one JSON line per (kernel, N), then
a summary line.
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
    ap.add_argument("--t", type=int, default=10240, help="samples per (kernel, N)")
    ap.add_argument("--chunk", type=int, default=1024, help="samples fetched per call")
    ap.add_argument("--ref-n", type=int, default=200, help="Gaussian N of the reference")
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--nmax", type=int, default=4)
    ap.add_argument("--kernels", default="0,0.9", help="linear-kernel g values (0: isotropic)")
    ap.add_argument("--out", default="")
    return ap.parse_args()


def l2(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2)))


def slope(x, y):
    """Least-squares slope of log y against log x."""
    lx, ly = np.log(np.asarray(x)), np.log(np.asarray(y))
    return float(np.polyfit(lx, ly, 1)[0])


def main():
    a = parse()
    import torch
    from paper_2407_12527_amd import rom as R
    torch.cuda.set_device(0)
    f = RI.example21()
    outf = open(a.out, "a") if a.out else None

    def emit(rec):
        line = json.dumps(rec)
        print(line, flush=True)
        if outf:
            outf.write(line + "\n")
            outf.flush()

    o_ref = R.si_opts(tol=1e-12, max_iter=5000, precision=R.ROM_PREC_FP64, scheme=R.ROM_SCHEME_DD)
    o = R.si_opts(tol=1e-10, max_iter=5000, precision=R.ROM_PREC_FP64, scheme=R.ROM_SCHEME_DD)
    summary = {"arm": "summary", "t": a.t, "kernels": {}}
    t0 = time.perf_counter()
    for g in (float(v) for v in a.kernels.split(",")):
        h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
        if g != 0.0:
            h.set_scattering(R.ROM_SCAT_LINEAR, g)
        d, w = R.generate_ordinates(R.ROM_ORD_GAUSS2D, a.ref_n)
        h.set_ordinates(d, w)
        ts = time.perf_counter()
        ref, st, rc = h.source_iterate(o_ref)
        if rc != 0:
            raise RuntimeError(f"reference did not converge (status {rc})")
        emit({"arm": "reference", "g": g, "ordinates": len(w), "iters": st.iters, "seconds": time.perf_counter() - ts})
        rows = []
        for N in range(1, a.nmax + 1):
            n = 4 * N * N
            ts = time.perf_counter()
            allphi = np.empty((a.t, f.cells))
            done, iters = 0, 0
            while done < a.t:
                b = min(a.chunk, a.t - done)
                phis, est, rc = h.ensemble_samples(b, a.seed, R.ROM_ORD_STRATIFIED, N, N, first=done, opts=o)
                if rc != 0:
                    raise RuntimeError(f"N={N} samples {done}..{done + b} did not converge (status {rc})")
                iters = max(iters, est.max_iters)
                allphi[done:done + b] = phis
                done += b
            errs = np.sqrt(np.mean((allphi - ref[None, :]) ** 2, axis=1))
            mean = allphi.mean(axis=0)
            E = float(errs.mean())
            B = l2(mean, ref)
            # statistical noise in B: the rms over cells of the standard error of the mean
            B_noise = float(np.sqrt(np.mean(allphi.var(axis=0, ddof=1)) / a.t))
            # MC error of an average of t' samples: rms over the disjoint blocks of t' samples of
            # ||block mean - mean of all t||; its expectation is s (1/t' - 1/t)^(1/2)
            mc = []
            tp = 1
            while tp <= a.t // 2:
                nb = a.t // tp
                bm = allphi[: nb * tp].reshape(nb, tp, f.cells).mean(axis=1)
                mc.append((tp, float(np.sqrt(np.mean(np.mean((bm - mean[None, :]) ** 2, axis=1))))))
                tp *= 2
            fit = [(m, e) for m, e in mc if m <= a.t // 64]
            rec = {"arm": "rom", "g": g, "N": N, "ordinates": n, "delta_s": math.pi / (4 * N * N), "t": a.t,
                   "E": E, "E_std_err": float(errs.std() / math.sqrt(a.t)), "B": B, "B_noise": B_noise,
                   "mc_slope": slope([m for m, _ in fit], [e for _, e in fit]),
                   "mc_slope_corrected": slope([math.sqrt(1 / m - 1 / a.t) for m, _ in mc], [e for _, e in mc]),
                   "mc": mc, "max_iters": iters, "seconds": time.perf_counter() - ts}
            rows.append(rec)
            emit(rec)
        ds = [r["delta_s"] for r in rows]
        summary["kernels"][str(g)] = {
            "E": {r["N"]: r["E"] for r in rows}, "B": {r["N"]: r["B"] for r in rows},
            "order_E": slope(ds, [r["E"] for r in rows]), "order_B": slope(ds, [r["B"] for r in rows]),
            "mc_slope": [r["mc_slope"] for r in rows], "mc_slope_corrected": [r["mc_slope_corrected"] for r in rows],
            "B_noise": {r["N"]: r["B_noise"] for r in rows}}
    summary["seconds"] = time.perf_counter() - t0
    emit(summary)


if __name__ == "__main__":
    sys.exit(main())
