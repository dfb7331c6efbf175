"""GPU parity of per-sample ensemble output (rom_ensemble_samples): every returned flux against the
FP64 oracle on the same sample of the same ensemble (Sec. 4.1), sample offsets, agreement with
the ensemble moments, and the diamond-difference linear-kernel setting of the convergence study
(Sec. 4.2)."""
import numpy as np
import pytest

import parity
from parity import nrm

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


@pytest.mark.parametrize("first", [0, 5, 1000])
def test_samples_match_oracle(R, orc, first):
    f = RI.uniform_fields(30, 26, 1.0, 0.6, 0.4, 0.6)
    h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    p = orc.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    phis, st, rc = h.ensemble_samples(4, 9, R.ROM_ORD_STRATIFIED, 2, 3, first=first,
                                      opts=R.si_opts(tol=1e-11, precision=R.ROM_PREC_FP64))
    assert rc == 0 and phis.shape == (4, f.cells) and st.samples == 4
    for k in range(4):
        d, w = orc.generate(orc.ORD_STRATIFIED, 2, 3, seed=9, sample=first + k)
        ref = orc.source_iterate(p, d, w, None, tol=1e-13)["phi"]
        parity.check(phis[k], ref, 1e-9, what=str(k))


@pytest.mark.parametrize("prec,scheme", [("fp32", "step"), ("fp64", "dd"), ("fp32", "dd")])
def test_samples_with_boundary_inflow(R, orc, prec, scheme):
    """Isotropic inflow on two faces of a ragged grid with non-square cells: every sample of the
    ensemble sweeps its own ordinates from the same face values (16-lane groups, four samples per
    wavefront, one partly filled)."""
    rng = np.random.default_rng(44)
    nx, ny = 33, 21
    st = rng.uniform(0.5, 2.0, nx * ny)
    ss = st * rng.uniform(0.0, 0.8, nx * ny)
    q = rng.uniform(0.0, 1.0, nx * ny)
    inflow = {"left": rng.uniform(0, 1, ny), "top": rng.uniform(0, 1, nx)}
    box = (0.0, 1.2, 0.0, 0.9)
    h = R.Handle(nx, ny, st, ss, q, box=box, inflow=inflow)
    p = orc.Problem(nx, ny, st, ss, q, box=box, inflow=inflow)
    fp64 = prec == "fp64"
    sch = R.ROM_SCHEME_DD if scheme == "dd" else R.ROM_SCHEME_STEP
    o = R.si_opts(tol=-1.0, max_iter=6, precision=R.ROM_PREC_FP64 if fp64 else R.ROM_PREC_FP32, scheme=sch)
    phis, st_, rc = h.ensemble_samples(5, 21, R.ROM_ORD_STRATIFIED, 2, 2, opts=o)
    assert rc == R.ROM_NOT_CONVERGED and phis.shape == (5, nx * ny)
    for k in range(5):
        d, w = orc.generate(orc.ORD_STRATIFIED, 2, 2, seed=21, sample=k)
        osch = orc.SCHEME_DD if scheme == "dd" else orc.SCHEME_STEP
        ref = orc.source_iterate(p, d, w, None, tol=0.0, max_iter=6, scheme=osch)["phi"]
        parity.check(phis[k], ref, (1e-12 if fp64 else 1e-5), what=str(k))


def test_samples_agree_with_moments_and_pieces(R):
    f = RI.checkerboard_fields(40, 40)
    h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    o = R.si_opts(tol=1e-11, precision=R.ROM_PREC_FP64)
    whole, _, _ = h.ensemble_samples(12, 3, R.ROM_ORD_STRATIFIED, 2, 2, opts=o)
    a, _, _ = h.ensemble_samples(5, 3, R.ROM_ORD_STRATIFIED, 2, 2, first=0, opts=o)
    b, _, _ = h.ensemble_samples(7, 3, R.ROM_ORD_STRATIFIED, 2, 2, first=5, opts=o)
    np.testing.assert_allclose(np.vstack([a, b]), whole, rtol=1e-12, atol=1e-15)
    mean, var, _, _ = h.ensemble(12, 3, R.ROM_ORD_STRATIFIED, 2, 2, o)
    np.testing.assert_allclose(whole.mean(axis=0), mean, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(whole.var(axis=0, ddof=1), var, rtol=1e-9, atol=1e-15)


def test_samples_dd_linear_kernel(R, orc):
    """The convergence-study configuration: Example 2.1 physics on a smaller grid, diamond
    difference, linear kernel g = 0.9."""
    f = RI.uniform_fields(36, 36, 1.0, 0.5, 0.4, 0.6, q_val=2.0)
    h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    h.set_scattering(R.ROM_SCAT_LINEAR, 0.9)
    p = orc.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    o = R.si_opts(tol=1e-11, precision=R.ROM_PREC_FP64, scheme=R.ROM_SCHEME_DD)
    phis, _, rc = h.ensemble_samples(3, 2024, R.ROM_ORD_STRATIFIED, 3, 3, first=17, opts=o)
    assert rc == 0
    for k in range(3):
        d, w = orc.generate(orc.ORD_STRATIFIED, 3, 3, seed=2024, sample=17 + k)
        W = orc.build_W(d, w, orc.SCAT_LINEAR, 0.9, fold=1)
        ref = orc.source_iterate(p, d, w, W, scheme=orc.SCHEME_DD, tol=1e-13)["phi"]
        parity.check(phis[k], ref, 1e-9, what=str(k))


def test_samples_argument_errors(R):
    h = R.Handle(8, 8, np.ones(64), np.full(64, 0.5), np.ones(64))
    with pytest.raises(R.RomError):
        h.ensemble_samples(2, 0, R.ROM_ORD_STRATIFIED, 1, 1, first=-1)
    with pytest.raises(R.RomError):
        h.ensemble_samples(2, 0, R.ROM_ORD_STRATIFIED, 0, 1)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_ensemble_moments_across_batches(R, prec):
    """More samples than one launch takes (1024): the ensemble runs as 1024 + 76 samples and the
    batches' FP64 moments are merged by the pairwise update; mean and variance against two-pass
    moments of all 1100 per-sample fluxes (the same fluxes, taken by the per-sample call)."""
    f = RI.uniform_fields(12, 10, 1.0, 0.5, 0.3, 0.7)
    h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    o = R.si_opts(tol=1e-10 if prec == "fp64" else 1e-6,
                  precision=R.ROM_PREC_FP64 if prec == "fp64" else R.ROM_PREC_FP32)
    t = 1100
    phis, st1, rc1 = h.ensemble_samples(t, 5, R.ROM_ORD_STRATIFIED, 2, 2, opts=o)
    mean, var, st2, rc2 = h.ensemble(t, 5, R.ROM_ORD_STRATIFIED, 2, 2, o)
    assert rc1 == 0 and rc2 == 0 and st1.samples == t and st2.samples == t
    m = phis.mean(axis=0)
    v = ((phis - m) ** 2).sum(axis=0) / (t - 1)
    np.testing.assert_allclose(mean, m, rtol=1e-13, atol=0)
    np.testing.assert_allclose(var, v, rtol=1e-9, atol=1e-300)
