"""GPU parity: librom's HIP path (through the C ABI) against the FP64 CPU oracle on the same
seeded inputs and bit-identical ordinate sets.

Every comparison is element-wise (tests/parity.py): the normwise figure
||phi_gpu - phi_oracle||_2 / ||phi_oracle||_2, the max-norm figure max|dphi| / max|phi_oracle|
(both at the bar), and the relative error of every cell whose flux is at least 1e-3 of the
maximum (at ten times the bar).  Bars:
  * FP32 sweeps: 1e-5 (a single sweep 1e-6..2e-6);  FP64 path: 1e-11 at a fixed iteration count,
    1e-9 when both sides stop on the same tolerance;
  * BF16 contraction (anisotropic FP32 path): 2e-3;
  * FP32 ensemble variance: 1e-5 (per cell 1e-4).
Tolerance-stopped solves are compared at the GPU's iteration count.  Cells in deep shadow (below
1e-3 of the maximum: behind thick absorbers the flux spans many decades) are held by the max-norm
figure only.
"""
import ctypes as C
import math

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


def rand_problem(rng, nx, ny, ratio=0.9):
    st = rng.uniform(0.5, 3.0, nx * ny)
    ss = st * rng.uniform(0.0, ratio, nx * ny)
    q = rng.uniform(0.0, 2.0, nx * ny)
    return st, ss, q


def both(R, orc, nx, ny, st, ss, q, box=(0.0, 1.0, 0.0, 1.0), inflow=None):
    h = R.Handle(nx, ny, st, ss, q, box=box, inflow=inflow)
    p = orc.Problem(nx, ny, st, ss, q, box=box, inflow=inflow)
    return h, p


# ------------------------------------------------------------------------------------ single sweep
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("tile", [(8, 4), (16, 16), (8, 8), (16, 8)])
@pytest.mark.parametrize("spec", [(2, 4), (8, 8), (1, 3)])
def test_sweep_isotropic_source(R, orc, prec, tile, spec):
    """One sweep psi = L^{-1} S (shared source) on a ragged 37 x 29 grid with non-square cells,
    varying cross sections and isotropic inflow on two faces.  (FP64 sweeps take 8 x 4 and 8 x 8
    tiles only; other shapes are refused with ROM_E_ARG.)"""
    rng = np.random.default_rng(11)
    nx, ny = 37, 29
    st, ss, q = rand_problem(rng, nx, ny)
    inflow = {"left": rng.uniform(0, 1, ny), "top": rng.uniform(0, 1, nx)}
    h, p = both(R, orc, nx, ny, st, ss, q, box=(0.0, 1.3, 0.0, 0.7), inflow=inflow)
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, *spec, seed=5, sample=2)
    h.set_ordinates(d, w)
    S = rng.uniform(0.0, 3.0, nx * ny)
    o = R.si_opts(precision=R.ROM_PREC_FP64 if prec == "fp64" else R.ROM_PREC_FP32, tile=tile)
    if prec == "fp64" and tile[0] != 8:
        with pytest.raises(R.RomError) as ei:
            h.sweep(S, o, want_psi=True)
        assert ei.value.status == R.ROM_E_ARG
        return
    phi, psi = h.sweep(S, o, want_psi=True)
    psi_ref = orc.sweep(p, d, S)
    phi_ref = orc.scalar_flux(w, psi_ref)
    tol = 1e-12 if prec == "fp64" else 1e-6
    parity.check(phi, phi_ref, tol)
    parity.check(psi, psi_ref, (1e-12 if prec == "fp64" else 2e-6))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_sweep_per_ordinate_source_and_angular_inflow(R, orc, prec):
    rng = np.random.default_rng(12)
    nx, ny = 23, 41
    st, ss, q = rand_problem(rng, nx, ny)
    h, p = both(R, orc, nx, ny, st, ss, q)
    d, w = R.generate_ordinates(R.ROM_ORD_IID_SPHERE, 19, seed=3)
    h.set_ordinates(d, w)
    n = len(w)
    ang = {"right": rng.uniform(0, 2, (n, ny)), "bottom": rng.uniform(0, 2, (n, nx))}
    for face, v in (("right", R.ROM_FACE_RIGHT), ("bottom", R.ROM_FACE_BOTTOM)):
        h.set_inflow_angular(v, ang[face])
    p.inflow_angular = {k: np.ascontiguousarray(v) for k, v in ang.items()}
    S = rng.uniform(0.0, 1.0, (n, nx * ny))
    o = R.si_opts(precision=R.ROM_PREC_FP64 if prec == "fp64" else R.ROM_PREC_FP32)
    phi, psi = h.sweep(S, o, want_psi=True)
    psi_ref = orc.sweep(p, d, S)
    tol = 1e-12 if prec == "fp64" else 2e-6
    parity.check(psi, psi_ref, tol)
    parity.check(phi, orc.scalar_flux(w, psi_ref), tol)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_sweep_diamond_difference(R, orc, prec):
    rng = np.random.default_rng(13)
    nx, ny = 30, 18
    st, ss, q = rand_problem(rng, nx, ny)
    h, p = both(R, orc, nx, ny, st, ss, q, inflow={"bottom": rng.uniform(0, 1, nx)})
    d, w = R.generate_ordinates(R.ROM_ORD_UNIFORM2D, 3)
    h.set_ordinates(d, w)
    S = rng.uniform(0.0, 1.0, nx * ny)
    o = R.si_opts(precision=R.ROM_PREC_FP64 if prec == "fp64" else R.ROM_PREC_FP32, scheme=R.ROM_SCHEME_DD)
    phi = h.sweep(S, o)
    ref = orc.scalar_flux(w, orc.sweep(p, d, S, scheme=orc.SCHEME_DD))
    parity.check(phi, ref, (1e-12 if prec == "fp64" else 1e-5))


@pytest.mark.parametrize("shape", [(1, 1), (1, 17), (23, 1), (5, 3)])
def test_sweep_degenerate_grids(R, orc, shape):
    nx, ny = shape
    rng = np.random.default_rng(14)
    st, ss, q = rand_problem(rng, nx, ny)
    h, p = both(R, orc, nx, ny, st, ss, q, inflow={"left": np.ones(ny), "bottom": np.ones(nx)})
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 2, 2, seed=1)
    h.set_ordinates(d, w)
    S = rng.uniform(0, 1, nx * ny)
    phi = h.sweep(S, R.si_opts(precision=R.ROM_PREC_FP64))
    parity.check(phi, orc.scalar_flux(w, orc.sweep(p, d, S)), 1e-13)


@pytest.mark.parametrize("kernel", ["strip", "row-lane"])
@pytest.mark.parametrize("shape", [(1500, 2), (2, 1500), (700, 41)])
def test_sweep_elongated_grids(R, orc, kernel, shape):
    """Long strips and tall stacks: hundreds of chunks per strip, or hundreds of strips (8 x 4
    tiles in bands of 2, so most strip boundaries go through global memory) and of 16-row blocks,
    with inflow on all four faces; FP64, so the result is the oracle's to rounding."""
    nx, ny = shape
    rng = np.random.default_rng(nx + 7 * ny)
    st, ss, q = rand_problem(rng, nx, ny)
    inflow = {"left": rng.uniform(0, 1, ny), "right": rng.uniform(0, 1, ny), "bottom": rng.uniform(0, 1, nx),
              "top": rng.uniform(0, 1, nx)}
    h, p = both(R, orc, nx, ny, st, ss, q, box=(0.0, 2.0, 0.0, 1.0), inflow=inflow)
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 2, 3, seed=3)
    h.set_ordinates(d, w)
    S = rng.uniform(0, 1, nx * ny)
    if kernel == "strip":
        o = R.si_opts(precision=R.ROM_PREC_FP64, sweep=R.ROM_SWEEP_STRIP, tile=(8, 4), band=2)
    else:
        o = R.si_opts(precision=R.ROM_PREC_FP64, sweep=R.ROM_SWEEP_DIAG, diag_rows=16, diag_k=1, band=4)
    phi = h.sweep(S, o)
    parity.check(phi, orc.scalar_flux(w, orc.sweep(p, d, S)), 1e-12)


def test_single_ordinate(R, orc):
    nx, ny = 9, 7
    st, ss, q = np.ones(63), np.full(63, 0.3), np.ones(63)
    h, p = both(R, orc, nx, ny, st, ss, q)
    d = np.array([[0.6, -0.48, math.sqrt(1 - 0.36 - 0.2304)]])
    w = np.array([1.0])
    h.set_ordinates(d, w)
    phi, st_, rc = h.source_iterate(R.si_opts(precision=R.ROM_PREC_FP64, tol=1e-12))
    ref = orc.source_iterate(p, d, w, None, tol=1e-12)
    assert rc == 0 and st_.iters == ref["iters"]
    parity.check(phi, ref["phi"], 1e-13)


# ------------------------------------------------------------------------------------ source iteration
def test_si_c1_fp64(R, orc):
    """Workload c1 (64 x 64, 32 i.i.d. sphere ordinates, FP64, tol 1e-8): at a fixed iteration
    count and converged."""
    wl = RI.c1()
    f = wl.fields[0]
    h, p = both(R, orc, f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    d, w = R.generate_ordinates(R.ROM_ORD_IID_SPHERE, 32, seed=0)
    h.set_ordinates(d, w)
    phi, st, rc = h.source_iterate(R.si_opts(tol=-1.0, max_iter=6, precision=R.ROM_PREC_FP64))
    ref = orc.source_iterate(p, d, w, None, tol=0.0, max_iter=6)
    assert rc == R.ROM_NOT_CONVERGED and st.iters == 6
    parity.check(phi, ref["phi"], 1e-11)
    phi, st, rc = h.source_iterate(R.si_opts(tol=1e-8, precision=R.ROM_PREC_FP64))
    ref = orc.source_iterate(p, d, w, None, tol=1e-8)
    assert rc == 0 and st.iters == ref["iters"]
    parity.check(phi, ref["phi"], 1e-9)
    assert st.updates == ref["iters"] * 4096 * 32


def test_si_c2_full_size(R, orc):
    """Workload c2 at full size (256 x 256 checkerboard, 256 stratified ordinates, FP32)."""
    wl = RI.c2()
    f = wl.fields[0]
    h, p = both(R, orc, f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 8, 8, seed=0)
    h.set_ordinates(d, w)
    phi, st, rc = h.source_iterate(R.si_opts(tol=1e-6))
    assert rc == 0
    parity.si_check(orc, p, d, w, None, phi, st.iters, 1e-6, 1e-5, what="c2")
    # the checkerboard and the stratified set are mirror symmetric
    P = phi.reshape(256, 256)
    assert nrm(P[:, ::-1], P) < 1e-6 and nrm(P[::-1, :], P) < 1e-6
    # determinism: a second solve is bitwise identical
    phi2, _, _ = h.source_iterate(R.si_opts(tol=1e-6))
    assert np.array_equal(phi, phi2)


@pytest.mark.parametrize("tile", [(8, 4), (16, 16)])
def test_si_fp32_fixed_iterations(R, orc, tile):
    rng = np.random.default_rng(21)
    nx, ny = 70, 45
    st, ss, q = rand_problem(rng, nx, ny, 0.95)
    h, p = both(R, orc, nx, ny, st, ss, q, inflow={"right": rng.uniform(0, 1, ny)})
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 4, 8, seed=9)
    h.set_ordinates(d, w)
    phi, stt, rc = h.source_iterate(R.si_opts(tol=-1.0, max_iter=9, tile=tile))
    ref = orc.source_iterate(p, d, w, None, tol=0.0, max_iter=9)
    assert rc == R.ROM_NOT_CONVERGED and stt.iters == 9
    parity.check(phi, ref["phi"], 1e-5)


def test_si_zero_source_and_not_converged(R, orc):
    h = R.Handle(8, 8, np.ones(64), np.full(64, 0.5), np.zeros(64))
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 1, 2)
    h.set_ordinates(d, w)
    phi, st, rc = h.source_iterate(R.si_opts(tol=1e-8))
    assert rc == 0 and st.iters == 1 and np.all(phi == 0)
    h2 = R.Handle(8, 8, np.ones(64), np.full(64, 0.9), np.ones(64))
    h2.set_ordinates(d, w)
    phi, st, rc = h2.source_iterate(R.si_opts(tol=1e-12, max_iter=3))
    assert rc == R.ROM_NOT_CONVERGED and st.iters == 3 and st.final_r > 1e-12


def test_phi_device(R, orc):
    import torch
    wl = RI.c1()
    f = wl.fields[0]
    h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    d, w = R.generate_ordinates(R.ROM_ORD_IID_SPHERE, 32, seed=0)
    h.set_ordinates(d, w)
    phi, st, rc = h.source_iterate(R.si_opts(tol=1e-6))
    t = h.phi_device_tensor()
    assert t.dtype == torch.float32
    np.testing.assert_array_equal(t.cpu().numpy().astype(np.float64), phi)


# ------------------------------------------------------------------------------------ anisotropic
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_si_anisotropic_hg(R, orc, prec):
    """HG g = 0.8 (folded), sigma_s/sigma_t = 0.8: BF16 MFMA contraction (FP32 path) or FP64."""
    nx = ny = 40
    f = RI.uniform_fields(nx, ny, 1.0, 0.8, 0.45, 0.55)
    h, p = both(R, orc, nx, ny, f.sigma_t, f.sigma_s, f.q)
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 4, 8, seed=0)
    h.set_ordinates(d, w)
    h.set_scattering(R.ROM_SCAT_HG, 0.8)
    W = orc.build_W(d, w, orc.SCAT_HG, 0.8, fold=1)
    o = R.si_opts(tol=1e-7, precision=R.ROM_PREC_FP64 if prec == "fp64" else R.ROM_PREC_FP32)
    phi, st, rc = h.source_iterate(o)
    assert rc == 0
    parity.si_check(orc, p, d, w, W, phi, st.iters, 1e-7, 1e-9 if prec == "fp64" else 2e-3)


@pytest.mark.parametrize("shape", [(23, 17, 16, 4), (37, 29, 64, 1)])
def test_si_anisotropic_large_contraction_ragged(R, orc, shape):
    """320 ordinates (80 per quadrant) on the row-lane dense path pad to 384 kernel columns: the
    256 x 256 contraction tiles end in a half tile of 128 columns, and the cell count (391, 1073)
    leaves a ragged last row tile.  Three fixed iterations against the oracle at the BF16 bar."""
    nx, ny, rows, k = shape
    rng = np.random.default_rng(nx * ny)
    st, ss, q = rand_problem(rng, nx, ny, 0.8)
    h, p = both(R, orc, nx, ny, st, ss, q, inflow={"left": rng.uniform(0, 1, ny)})
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 8, 10, seed=4)
    assert d.shape[0] == 320
    h.set_ordinates(d, w)
    h.set_scattering(R.ROM_SCAT_HG, 0.6)
    W = orc.build_W(d, w, orc.SCAT_HG, 0.6, fold=1)
    o = R.si_opts(tol=-1.0, max_iter=3, precision=R.ROM_PREC_FP32, sweep=R.ROM_SWEEP_DIAG, diag_rows=rows,
                  diag_k=k, band=4)
    phi, stt, rc = h.source_iterate(o)
    assert rc == R.ROM_NOT_CONVERGED and stt.iters == 3
    ref = orc.source_iterate(p, d, w, W, tol=0.0, max_iter=3)
    parity.check(phi, ref["phi"], 2e-3)


def test_si_anisotropic_dense_fixed_iterations_fp64(R, orc):
    """A non-symmetric caller kernel with unequal weights (Gaussian set): pins the orientation of
    the contraction on the GPU at a fixed iteration count."""
    rng = np.random.default_rng(31)
    nx, ny = 20, 14
    st, ss, q = rand_problem(rng, nx, ny, 0.6)
    h, p = both(R, orc, nx, ny, st, ss, q)
    d, w = R.generate_ordinates(R.ROM_ORD_GAUSS2D, 4)
    h.set_ordinates(d, w)
    P = rng.uniform(0.2, 1.5, (len(w), len(w)))
    h.set_scattering(R.ROM_SCAT_DENSE, 0.0, P)
    W = orc.build_W(d, w, orc.SCAT_DENSE, P=P)
    phi, st_, rc = h.source_iterate(R.si_opts(tol=-1.0, max_iter=5, precision=R.ROM_PREC_FP64))
    ref = orc.source_iterate(p, d, w, W, tol=0.0, max_iter=5)
    parity.check(phi, ref["phi"], 1e-12)


# ------------------------------------------------------------------------------------ ensemble / batch
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_ensemble_mean_var(R, orc, prec):
    """Samples packed two per wavefront (32 ordinates per quadrant): mean and variance against
    the oracle's two-pass FP64 moments over the same bit-identical sample sets."""
    nx, ny = 96, 80
    f = RI.uniform_fields(nx, ny, 1.0, 0.5, 0.45, 0.55)
    h, p = both(R, orc, nx, ny, f.sigma_t, f.sigma_s, f.q)
    t = 6
    o = R.si_opts(tol=1e-7, precision=R.ROM_PREC_FP64 if prec == "fp64" else R.ROM_PREC_FP32)
    mean, var, st, rc = h.ensemble(t, 7, R.ROM_ORD_STRATIFIED, 4, 8, o)
    ref = orc.ensemble(p, orc.ORD_STRATIFIED, 4, 8, 7, t, tol=1e-7)
    assert rc == 0 and st.samples == t
    parity.check(mean, ref["mean"], (1e-10 if prec == "fp64" else 1e-5))
    # the variance is formed in FP64 from FP32 per-sample fluxes whose relative error is ~1e-6;
    # their spread phi_s - mean is a few per cent of phi here, so the variance carries about
    # 2e-6 / 0.03 ~ 1e-4 relative error at most and ~1e-6 normwise (measured 4e-7): the FP32 bar
    parity.check(var, ref["var"], 1e-8 if prec == "fp64" else 1e-5, cell_tol=1e-7 if prec == "fp64" else 1e-4)
    assert st.min_iters == int(ref["iters"].min()) or prec == "fp32"


def test_batch_uneven_problems(R, orc):
    wl = RI.c5(count=5, sides=(16, 24, 40), m_range=(4, 20))
    hs, cases = [], []
    for k, f in enumerate(wl.fields):
        h, p = both(R, orc, f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
        nz, nt = orc.stratified_spec(wl.n_ord[k])
        d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, nz, nt, seed=wl.problem_seed(k))
        h.set_ordinates(d, w)
        hs.append(h)
        cases.append((p, d, w))
    outs, stats, rc = R.solve_batch(hs, R.si_opts(tol=1e-6))
    assert rc == 0
    for k, (o_, (p, d, w)) in enumerate(zip(outs, cases)):
        parity.si_check(orc, p, d, w, None, o_, stats[k].iters, 1e-6, 1e-5, what=str(k))


def test_batch_without_download_then_with(R, orc):
    """A batch solve that leaves the fluxes on the device reports the same iteration counts as
    one that downloads them, and the following downloading solve (plan reused, first sources set
    again by the one-launch initialization) still matches the oracle."""
    wl = RI.c5(count=4, sides=(16, 32), m_range=(4, 12))
    hs, cases = [], []
    for k, f in enumerate(wl.fields):
        h, p = both(R, orc, f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
        nz, nt = orc.stratified_spec(wl.n_ord[k])
        d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, nz, nt, seed=wl.problem_seed(k))
        h.set_ordinates(d, w)
        hs.append(h)
        cases.append((p, d, w))
    o = R.si_opts(tol=1e-6)
    outs0, st0, rc0 = R.solve_batch(hs, o, download=False)
    assert rc0 == 0 and outs0 == [None] * len(hs)
    outs1, st1, rc1 = R.solve_batch(hs, o)
    assert rc1 == 0
    for a, b, o_, (p, d, w) in zip(st0, st1, outs1, cases):
        assert a.iters == b.iters
        parity.si_check(orc, p, d, w, None, o_, b.iters, 1e-6, 1e-5)


def test_si_near_critical_many_replays(R, orc):
    """sigma_s / sigma_t = 0.99 on an optically thick square (20 mean free paths a side): source
    iteration needs about 420 iterations, so the captured graph is replayed many times (8
    iterations per replay on the first solve, the previous count split into replays of at most 64
    on the next).  FP64 iteration count and flux against the oracle; the repeated solve is
    bitwise identical."""
    f = RI.uniform_fields(24, 24, 1.0, 0.99, 0.4, 0.6)
    h, p = both(R, orc, f.nx, f.ny, f.sigma_t, f.sigma_s, f.q, box=(0.0, 20.0, 0.0, 20.0))
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 2, 2, seed=4)
    h.set_ordinates(d, w)
    o = R.si_opts(tol=1e-8, max_iter=5000, precision=R.ROM_PREC_FP64)
    phi, st, rc = h.source_iterate(o)
    ref = orc.source_iterate(p, d, w, None, tol=1e-8, max_iter=5000)
    assert rc == 0 and st.iters > 300 and abs(st.iters - ref["iters"]) <= 1
    parity.check(phi, ref["phi"], (1e-10 if st.iters == ref["iters"] else 1e-7))
    phi2, st2, rc2 = h.source_iterate(o)
    assert rc2 == 0 and st2.iters == st.iters and np.array_equal(phi, phi2)
