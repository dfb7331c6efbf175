"""The reference of the time-to-error study, pinned to the oracle.

The study's reference is FP64 DOM with the Appendix A Gaussian quadrature at N = 200 (80 400
ordinates, the paper's reference in Sec. 4.2) on the 64 x 64 isotropic problem.  The GPU FP64
path is checked against the FP64 oracle on the same bit-identical ordinate set for three fixed
source iterations (1e-11 normwise), and the two arms' quadratures are checked to be the ones the
oracle generates."""
import numpy as np
import pytest

import rom_inputs as RI

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_12527_amd import rom
    rom.lib()
    return rom


def test_gauss200_reference_three_iterations(R, orc):
    f = RI.uniform_fields(64, 64, 1.0, 0.5, 0.45, 0.55)
    d, w = R.generate_ordinates(R.ROM_ORD_GAUSS2D, 200)
    do, wo = orc.generate(orc.ORD_GAUSS2D, 200)
    assert len(w) == 80400
    assert np.array_equal(d, do) and np.array_equal(w, wo)
    h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    h.set_ordinates(d, w)
    phi, st, rc = h.source_iterate(R.si_opts(tol=-1.0, max_iter=3, precision=R.ROM_PREC_FP64))
    assert rc == R.ROM_NOT_CONVERGED and st.iters == 3
    ref = orc.source_iterate(orc.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q), d, w, None, tol=0.0, max_iter=3)
    assert np.linalg.norm(phi - ref["phi"]) / np.linalg.norm(ref["phi"]) < 1e-11


@pytest.mark.parametrize("N", [2, 6, 22])
def test_dom_arm_uniform_sets(R, orc, N):
    d, w = R.generate_ordinates(R.ROM_ORD_UNIFORM2D, N)
    do, wo = orc.generate(orc.ORD_UNIFORM2D, N)
    assert np.array_equal(d, do) and np.array_equal(w, wo)
