"""GPU parity of the linear-kernel moment contraction and of the normalized kernels.

The folded linear kernel 1 + g (c c' + s s') of eq. (2.1) is contracted inside the sweep through
three moments of the previous iterate (no angular flux, no GEMM); the oracle applies the same
kernel as a dense W (eq. (3.4)) to stored angular fluxes, so agreement checks the rank-3
factorization, the moment weights and the per-system g.  Normalized kernels (the remark of
Sec. 3.1) are checked on i.i.d. sets, where the row sums differ from 1.  Bars as elsewhere: FP64
fixed iterations 1e-11 normwise, FP32 converged 1e-5, BF16 contraction 2e-3."""
import zlib

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


def rand_problem(rng, nx, ny, ratio=0.8):
    st = rng.uniform(0.5, 3.0, nx * ny)
    ss = st * rng.uniform(0.0, ratio, nx * ny)
    q = rng.uniform(0.0, 2.0, nx * ny)
    return st, ss, q


def ordinate_set(R, kind, seed):
    if kind == "strat":
        return R.generate_ordinates(R.ROM_ORD_STRATIFIED, 2, 3, seed=seed)
    if kind == "iid":
        return R.generate_ordinates(R.ROM_ORD_IID_SPHERE, 21, seed=seed)
    return R.generate_ordinates(R.ROM_ORD_GAUSS2D, 4)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("scheme", ["step", "dd"])
@pytest.mark.parametrize("ords", ["strat", "iid", "gauss"])
@pytest.mark.parametrize("g", [0.9, -0.6])
def test_linear_kernel_fixed_iterations(R, orc, prec, scheme, ords, g):
    rng = np.random.default_rng(zlib.crc32(repr((prec, scheme, ords, g)).encode()))
    nx, ny = 37, 29   # ragged against every tile shape
    st, ss, q = rand_problem(rng, nx, ny)
    inflow = {"left": rng.uniform(0, 1, ny), "top": rng.uniform(0, 1, nx)}
    h = R.Handle(nx, ny, st, ss, q, inflow=inflow)
    d, w = ordinate_set(R, ords, 3)
    h.set_ordinates(d, w)
    h.set_scattering(R.ROM_SCAT_LINEAR, g)
    fp64 = prec == "fp64"
    sch = R.ROM_SCHEME_DD if scheme == "dd" else R.ROM_SCHEME_STEP
    o = R.si_opts(tol=-1.0, max_iter=6, precision=R.ROM_PREC_FP64 if fp64 else R.ROM_PREC_FP32, scheme=sch)
    phi, st_, rc = h.source_iterate(o)
    assert rc == R.ROM_NOT_CONVERGED and st_.iters == 6
    W = orc.build_W(d, w, orc.SCAT_LINEAR, g, fold=1)
    p = orc.Problem(nx, ny, st, ss, q, inflow=inflow)
    ref = orc.source_iterate(p, d, w, W, scheme=orc.SCHEME_DD if scheme == "dd" else orc.SCHEME_STEP, tol=0.0,
                             max_iter=6)
    parity.check(phi, ref["phi"], (1e-11 if fp64 else 1e-5))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_linear_kernel_converged(R, orc, prec):
    f = RI.uniform_fields(64, 48, 1.0, 0.7, 0.4, 0.6)
    h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 4, 8, seed=1)
    h.set_ordinates(d, w)
    h.set_scattering(R.ROM_SCAT_LINEAR, 0.9)
    fp64 = prec == "fp64"
    phi, st, rc = h.source_iterate(R.si_opts(tol=1e-9 if fp64 else 1e-6,
                                             precision=R.ROM_PREC_FP64 if fp64 else R.ROM_PREC_FP32))
    assert rc == R.ROM_OK
    W = orc.build_W(d, w, orc.SCAT_LINEAR, 0.9, fold=1)
    ref = orc.source_iterate(orc.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q), d, w, W, tol=1e-12)
    parity.check(phi, ref["phi"], (1e-8 if fp64 else 1e-5))
    assert st.sweep == R.ROM_SWEEP_STRIP  # the row-lane kernel takes isotropic sources only


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", ["linear", "hg"])
def test_normalized_kernels_iid(R, orc, prec, kind):
    rng = np.random.default_rng(7)
    nx, ny = 26, 33
    st, ss, q = rand_problem(rng, nx, ny, 0.9)
    h = R.Handle(nx, ny, st, ss, q)
    d, w = R.generate_ordinates(R.ROM_ORD_IID_SPHERE, 24, seed=11)
    h.set_ordinates(d, w)
    sk, ok, g = (R.ROM_SCAT_LINEAR, orc.SCAT_LINEAR, 0.9) if kind == "linear" else (R.ROM_SCAT_HG, orc.SCAT_HG, 0.8)
    h.set_scattering(sk | R.ROM_SCAT_NORMALIZE, g)
    fp64 = prec == "fp64"
    phi, _, rc = h.source_iterate(R.si_opts(tol=-1.0, max_iter=5, precision=R.ROM_PREC_FP64 if fp64 else R.ROM_PREC_FP32))
    Wn = orc.build_W(d, w, ok | orc.SCAT_NORMALIZE, g, fold=1)
    ref = orc.source_iterate(orc.Problem(nx, ny, st, ss, q), d, w, Wn, tol=0.0, max_iter=5)
    bar = 1e-11 if fp64 else (1e-5 if kind == "linear" else 2e-3)
    parity.check(phi, ref["phi"], bar)
    # the raw kernel gives another answer on this set
    W = orc.build_W(d, w, ok, g, fold=1)
    raw = orc.source_iterate(orc.Problem(nx, ny, st, ss, q), d, w, W, tol=0.0, max_iter=5)
    assert nrm(raw["phi"], ref["phi"]) > 1e-3


def test_normalized_hg_converges_where_raw_diverges(R, orc):
    """A small random set on which sigma_s rho(W) > sigma_t for raw HG g = 0.8: the raw iteration
    is reported as diverged, the normalized one converges to the oracle's fixed point."""
    f = RI.uniform_fields(24, 24, 1.0, 0.8, 0.4, 0.6)
    d, w = R.generate_ordinates(R.ROM_ORD_IID_SPHERE, 16, seed=0)
    Wraw = orc.build_W(d, w, orc.SCAT_HG, 0.8, fold=1)
    assert 0.8 * max(abs(np.linalg.eigvals(Wraw))) > 1.0
    h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    h.set_ordinates(d, w)
    h.set_scattering(R.ROM_SCAT_HG | R.ROM_SCAT_NORMALIZE, 0.8)
    phi, st, rc = h.source_iterate(R.si_opts(tol=1e-10, precision=R.ROM_PREC_FP64))
    assert rc == R.ROM_OK
    Wn = orc.build_W(d, w, orc.SCAT_HG | orc.SCAT_NORMALIZE, 0.8, fold=1)
    ref = orc.source_iterate(orc.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q), d, w, Wn, tol=1e-13)
    parity.check(phi, ref["phi"], 1e-9)


def test_linear_ensemble_samples_on_lanes(R, orc):
    f = RI.uniform_fields(40, 40, 1.0, 0.6, 0.45, 0.55)
    h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    h.set_scattering(R.ROM_SCAT_LINEAR, 0.9)
    mean, var, st, rc = h.ensemble(9, 5, R.ROM_ORD_STRATIFIED, 2, 2, R.si_opts(tol=1e-10, precision=R.ROM_PREC_FP64))
    assert rc == 0
    ref = orc.ensemble(orc.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q), orc.ORD_STRATIFIED, 2, 2, 5, 9,
                       scat_kind=orc.SCAT_LINEAR, g=0.9, tol=1e-10)
    parity.check(mean, ref["mean"], 1e-8)
    parity.check(var, ref["var"], 1e-6)


def test_linear_batch_per_system_g(R, orc):
    rng = np.random.default_rng(3)
    hs, refs = [], []
    for k, (nx, ny, g) in enumerate(((20, 30, 0.9), (33, 17, -0.4), (20, 30, 0.3))):
        st, ss, q = rand_problem(rng, nx, ny)
        h = R.Handle(nx, ny, st, ss, q)
        d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 2, 2 + k, seed=k)
        h.set_ordinates(d, w)
        h.set_scattering(R.ROM_SCAT_LINEAR, g)
        hs.append(h)
        W = orc.build_W(d, w, orc.SCAT_LINEAR, g, fold=1)
        refs.append(orc.source_iterate(orc.Problem(nx, ny, st, ss, q), d, w, W, tol=0.0, max_iter=7)["phi"])
    outs, _, rc = R.solve_batch(hs, R.si_opts(tol=-1.0, max_iter=7, precision=R.ROM_PREC_FP64))
    for k in range(3):
        parity.check(outs[k], refs[k], 1e-11, what=str(k))
    # a mixed batch (linear with isotropic) is refused
    iso = R.Handle(8, 8, np.ones(64), np.full(64, 0.5), np.ones(64))
    iso.set_ordinates(*R.generate_ordinates(R.ROM_ORD_STRATIFIED, 1, 1))
    with pytest.raises(R.RomError):
        R.solve_batch([hs[0], iso], R.si_opts(tol=1e-6))


def test_linear_refresh_g_and_normalization(R, orc):
    """The cached plan follows a new g (tables rewritten in place) and a switch to the normalized
    kernel (plan rebuilt), with new ordinates in between."""
    rng = np.random.default_rng(5)
    nx, ny = 30, 22
    st, ss, q = rand_problem(rng, nx, ny)
    h = R.Handle(nx, ny, st, ss, q)
    p = orc.Problem(nx, ny, st, ss, q)
    o = R.si_opts(tol=-1.0, max_iter=5, precision=R.ROM_PREC_FP64)
    steps = [(0.9, False, 0), (0.4, False, 0), (0.4, False, 1), (0.4, True, 1), (0.9, True, 2), (0.9, False, 2)]
    for g, norm, sample in steps:
        d, w = R.generate_ordinates(R.ROM_ORD_IID_SPHERE, 20, seed=sample)
        h.set_ordinates(d, w)
        h.set_scattering(R.ROM_SCAT_LINEAR | (R.ROM_SCAT_NORMALIZE if norm else 0), g)
        phi, _, _ = h.source_iterate(o)
        W = orc.build_W(d, w, orc.SCAT_LINEAR | (orc.SCAT_NORMALIZE if norm else 0), g, fold=1)
        ref = orc.source_iterate(p, d, w, W, tol=0.0, max_iter=5)["phi"]
        parity.check(phi, ref, 1e-11, what=str((g, norm, sample)))


def test_linear_g_zero_matches_isotropic(R):
    """g = 0 reduces the linear kernel to isotropic scattering: the moment sweep and the plain
    isotropic sweep agree (FP64)."""
    f = RI.checkerboard_fields(35, 35)
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 3, 3, seed=2)
    h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    h.set_ordinates(d, w)
    o = R.si_opts(tol=-1.0, max_iter=8, precision=R.ROM_PREC_FP64, sweep=R.ROM_SWEEP_STRIP)
    iso, _, _ = h.source_iterate(o)
    h.set_scattering(R.ROM_SCAT_LINEAR, 0.0)
    lin, _, _ = h.source_iterate(o)
    parity.check(lin, iso, 1e-14)
