"""Writes table1_uniform_g09_N20.npy: the FP64 oracle's reference density for Example 2.1 with the
linear kernel g = 0.9 (folded over +-zeta), diamond difference on 100 x 100 cells and the
Appendix A uniform quadrature of order N = 20 (1600 ordinates), source iteration to 1e-12.

Only the oracle is called.  Run from the repository root:  python tests/golden/make_table1_reference.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import rom_inputs as RI  # noqa: E402


def main():
    f = RI.example21()
    prob = O.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    dirs, w = O.generate(O.ORD_UNIFORM2D, 20)
    W = O.build_W(dirs, w, O.SCAT_LINEAR, 0.9, fold=1)
    res = O.source_iterate(prob, dirs, w, W, scheme=O.SCHEME_DD, tol=1e-12, max_iter=500)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "table1_uniform_g09_N20.npy")
    np.save(out, res["phi"])
    print("iters", res["iters"], "r", res["r"], "->", out)


if __name__ == "__main__":
    main()
