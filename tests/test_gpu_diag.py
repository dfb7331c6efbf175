"""GPU parity of the row-lane ("diagonal") sweep kernel against the FP64 oracle.

Covers the lane shapes (16- and 64-row blocks, 1, 2 or 4 ordinates per lane, FP32 and FP64),
grids that are ragged against the 16/64-row blocks and the 8-step unroll, degenerate grids,
inflow on every face, wavefront counts that force several rounds through the workgroup (the
row buffer that carries a block's top row from the last wavefront to the first), quadrants with
fewer ordinates than a task holds, source iteration, batches, ensembles and refreshed plans.
Bars as in the other parity tests, element-wise (normwise, max-norm and per cell above 1e-3 of the
maximum; tests/parity.py): FP32 1e-5 for phi (2e-6 for single sweeps), FP64 1e-12
(single sweeps) and 1e-11 (fixed iteration counts)."""
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


def diag_opts(R, prec, rows, k, band=0, **kw):
    return R.si_opts(precision=R.ROM_PREC_FP64 if prec == "fp64" else R.ROM_PREC_FP32, sweep=R.ROM_SWEEP_DIAG,
                     diag_rows=rows, diag_k=k, band=band, **kw)


SHAPES = [(16, 1), (16, 2), (16, 4), (64, 1), (64, 2), (64, 4)]


# FP64 row-lane sweeps take 1 or 2 ordinates per lane (4 is refused: test_refuses_unsupported)
@pytest.mark.parametrize("prec,rows,k", [("fp32", r, k) for r, k in SHAPES] +
                         [("fp64", r, k) for r, k in SHAPES if k <= 2])
def test_single_sweep_shapes(R, orc, prec, rows, k):
    rng = np.random.default_rng(101)
    nx, ny = 37, 83
    st, ss, q = rand_problem(rng, nx, ny)
    inflow = {"left": rng.uniform(0, 1, ny), "right": rng.uniform(0, 1, ny), "bottom": rng.uniform(0, 1, nx),
              "top": rng.uniform(0, 1, nx)}
    h = R.Handle(nx, ny, st, ss, q, box=(0.0, 1.3, 0.0, 0.7), inflow=inflow)
    p = orc.Problem(nx, ny, st, ss, q, box=(0.0, 1.3, 0.0, 0.7), inflow=inflow)
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 2, 3, seed=5, sample=1)
    h.set_ordinates(d, w)
    S = rng.uniform(0.0, 3.0, nx * ny)
    phi = h.sweep(S, diag_opts(R, prec, rows, k))
    ref = orc.scalar_flux(w, orc.sweep(p, d, S))
    parity.check(phi, ref, (1e-12 if prec == "fp64" else 2e-6))


@pytest.mark.parametrize("shape", [(1, 1), (1, 17), (23, 1), (5, 3), (8, 16), (9, 65), (130, 7)])
@pytest.mark.parametrize("rows", [16, 64])
def test_single_sweep_degenerate_and_ragged(R, orc, shape, rows):
    rng = np.random.default_rng(102)
    nx, ny = shape
    st, ss, q = rand_problem(rng, nx, ny)
    inflow = {"left": rng.uniform(0, 1, ny), "top": rng.uniform(0, 1, nx)}
    h = R.Handle(nx, ny, st, ss, q, inflow=inflow)
    p = orc.Problem(nx, ny, st, ss, q, inflow=inflow)
    d, w = R.generate_ordinates(R.ROM_ORD_IID_SPHERE, 11, seed=7)
    h.set_ordinates(d, w)
    S = rng.uniform(0.0, 1.0, nx * ny)
    phi = h.sweep(S, diag_opts(R, "fp64", rows, 1))
    ref = orc.scalar_flux(w, orc.sweep(p, d, S))
    parity.check(phi, ref, 1e-12)


@pytest.mark.parametrize("band", [1, 2, 3, 16])
@pytest.mark.parametrize("rows", [16, 64])
def test_single_sweep_rounds(R, orc, band, rows):
    """More row blocks than wavefronts: blocks go round the workgroup several times (the last
    wavefront hands its top row to the first through the LDS row buffer)."""
    rng = np.random.default_rng(103)
    nx, ny = 45, 300
    st, ss, q = rand_problem(rng, nx, ny)
    inflow = {"right": rng.uniform(0, 1, ny), "bottom": rng.uniform(0, 1, nx)}
    h = R.Handle(nx, ny, st, ss, q, inflow=inflow)
    p = orc.Problem(nx, ny, st, ss, q, inflow=inflow)
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 2, 2, seed=9)
    h.set_ordinates(d, w)
    S = rng.uniform(0.0, 1.0, nx * ny)
    phi = h.sweep(S, diag_opts(R, "fp32", rows, 2, band=band))
    ref = orc.scalar_flux(w, orc.sweep(p, d, S))
    parity.check(phi, ref, 2e-6)


def test_single_sweep_angular_inflow(R, orc):
    rng = np.random.default_rng(104)
    nx, ny = 23, 41
    st, ss, q = rand_problem(rng, nx, ny)
    h = R.Handle(nx, ny, st, ss, q)
    d, w = R.generate_ordinates(R.ROM_ORD_IID_SPHERE, 19, seed=3)
    h.set_ordinates(d, w)
    n = len(w)
    ang = {"right": rng.uniform(0, 2, (n, ny)), "bottom": rng.uniform(0, 2, (n, nx))}
    h.set_inflow_angular(R.ROM_FACE_RIGHT, ang["right"])
    h.set_inflow_angular(R.ROM_FACE_BOTTOM, ang["bottom"])
    p = orc.Problem(nx, ny, st, ss, q, inflow_angular={k: np.ascontiguousarray(v) for k, v in ang.items()})
    S = rng.uniform(0.0, 1.0, nx * ny)
    phi = h.sweep(S, diag_opts(R, "fp64", 16, 2))
    parity.check(phi, orc.scalar_flux(w, orc.sweep(p, d, S)), 1e-12)


def test_refuses_unsupported(R):
    h = R.Handle(8, 8, np.ones(64), np.full(64, 0.5), np.ones(64))
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 1, 2)
    h.set_ordinates(d, w)
    with pytest.raises(R.RomError) as ei:
        h.sweep(np.ones(64), diag_opts(R, "fp32", 16, 1), want_psi=True)
    assert ei.value.status == R.ROM_E_UNSUPPORTED
    with pytest.raises(R.RomError) as ei:
        h.source_iterate(diag_opts(R, "fp32", 16, 1, scheme=R.ROM_SCHEME_DD))
    assert ei.value.status == R.ROM_E_UNSUPPORTED
    with pytest.raises(R.RomError) as ei:
        h.source_iterate(diag_opts(R, "fp64", 16, 4))
    assert ei.value.status == R.ROM_E_ARG


# ------------------------------------------------------------------------------------ source iteration
@pytest.mark.parametrize("rows,k", [(16, 1), (16, 4), (64, 2)])
def test_si_c2_full_size(R, orc, rows, k):
    """Workload c2 (256 x 256 checkerboard, 256 stratified ordinates, FP32, tol 1e-6)."""
    f = RI.c2().fields[0]
    h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    p = orc.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 8, 8, seed=0)
    h.set_ordinates(d, w)
    phi, st, rc = h.source_iterate(diag_opts(R, "fp32", rows, k, tol=1e-6))
    ref = orc.source_iterate(p, d, w, None, tol=1e-6)
    assert rc == 0 and abs(st.iters - ref["iters"]) <= 1 and st.sweep == R.ROM_SWEEP_DIAG
    parity.check(phi, ref["phi"], 1e-5)
    P = phi.reshape(256, 256)
    assert nrm(P[:, ::-1], P) < 1e-6 and nrm(P[::-1, :], P) < 1e-6
    phi2, _, _ = h.source_iterate(diag_opts(R, "fp32", rows, k, tol=1e-6))
    assert np.array_equal(phi, phi2)


def test_si_c1_fp64_fixed_iterations(R, orc):
    wl = RI.c1()
    f = wl.fields[0]
    h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    p = orc.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    d, w = R.generate_ordinates(R.ROM_ORD_IID_SPHERE, 32, seed=0)
    h.set_ordinates(d, w)
    phi, st, rc = h.source_iterate(diag_opts(R, "fp64", 16, 1, tol=-1.0, max_iter=6))
    ref = orc.source_iterate(p, d, w, None, tol=0.0, max_iter=6)
    assert st.iters == 6
    parity.check(phi, ref["phi"], 1e-11)
    phi, st, rc = h.source_iterate(diag_opts(R, "fp64", 16, 1, tol=1e-8))
    ref = orc.source_iterate(p, d, w, None, tol=1e-8)
    assert rc == 0 and st.iters == ref["iters"]
    parity.check(phi, ref["phi"], 1e-9)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("m", [25, 17])
def test_si_many_slots_ragged(R, orc, prec, m):
    """One ordinate per task (64 rows x 1 ordinate per lane): a system of 4 m = 100 or 68 partial
    slots, more than 64 and not a multiple of the combine's 8 waves, so the 8-wave combine takes
    its ragged tail; fixed iterations against the oracle."""
    nx, ny = 40, 36
    f = RI.uniform_fields(nx, ny, 1.0, 0.7, 0.4, 0.6)
    h = R.Handle(nx, ny, f.sigma_t, f.sigma_s, f.q)
    p = orc.Problem(nx, ny, f.sigma_t, f.sigma_s, f.q)
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 1, m, seed=3)
    assert len(w) == 4 * m
    h.set_ordinates(d, w)
    phi, st, rc = h.source_iterate(diag_opts(R, prec, 64, 1, tol=-1.0, max_iter=5))
    ref = orc.source_iterate(p, d, w, None, tol=0.0, max_iter=5)
    assert st.iters == 5 and st.sweep == R.ROM_SWEEP_DIAG
    parity.check(phi, ref["phi"], (1e-12 if prec == "fp64" else 1e-5))


def test_batch_uneven_and_refresh(R, orc):
    wl = RI.c5(count=6, sides=(16, 40, 100, 300), m_range=(4, 40), master_seed=5)
    hs, probs, sets = [], [], []
    for k, f in enumerate(wl.fields):
        hs.append(R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q))
        probs.append(orc.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q))
        nz, nt = orc.stratified_spec(wl.n_ord[k])
        sets.append(R.generate_ordinates(R.ROM_ORD_STRATIFIED, nz, nt, seed=wl.problem_seed(k)))
        hs[-1].set_ordinates(*sets[-1])
    o = diag_opts(R, "fp32", 16, 2, tol=1e-6)
    for rep in range(2):
        outs, stats, rc = R.solve_batch(hs, o)
        assert rc == 0
        for k in range(len(hs)):
            ref = orc.source_iterate(probs[k], sets[k][0], sets[k][1], None, tol=1e-6)["phi"]
            parity.check(outs[k], ref, 1e-5, what=str((rep, k)))
        nz, nt = orc.stratified_spec(wl.n_ord[1])
        sets[1] = R.generate_ordinates(R.ROM_ORD_STRATIFIED, nz, nt, seed=wl.problem_seed(1), sample=3)
        hs[1].set_ordinates(*sets[1])


def test_ensemble(R, orc):
    nx, ny = 96, 80
    f = RI.uniform_fields(nx, ny, 1.0, 0.5, 0.45, 0.55)
    h = R.Handle(nx, ny, f.sigma_t, f.sigma_s, f.q)
    p = orc.Problem(nx, ny, f.sigma_t, f.sigma_s, f.q)
    for seed in (7, 8):
        mean, var, st, rc = h.ensemble(6, seed, R.ROM_ORD_STRATIFIED, 4, 8, diag_opts(R, "fp32", 64, 1, tol=1e-7))
        ref = orc.ensemble(p, orc.ORD_STRATIFIED, 4, 8, seed, 6, tol=1e-7)
        assert rc == 0 and st.sweep == R.ROM_SWEEP_DIAG
        parity.check(mean, ref["mean"], 1e-5)
        parity.check(var, ref["var"], 1e-5, cell_tol=1e-4)  # FP32 bar, as for the strip kernel


def test_autotune_picks_a_valid_kernel(R, orc):
    """Automatic choice (strip or row-lane) on c2: the result meets the bar whichever wins."""
    f = RI.c2().fields[0]
    h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    p = orc.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 8, 8, seed=0)
    h.set_ordinates(d, w)
    phi, st, rc = h.source_iterate(R.si_opts(tol=1e-6))
    assert rc == 0 and st.sweep in (R.ROM_SWEEP_STRIP, R.ROM_SWEEP_DIAG)
    ref = orc.source_iterate(p, d, w, None, tol=1e-6)
    parity.check(phi, ref["phi"], 1e-5)


# ------------------------------------------------------------------------------------ dense kernels
# The row-lane sweep with per-ordinate sources: it reads the contraction's S[cell][npad] and writes
# the weighted angular flux as BF16 for the next contraction.  Bar: the BF16 contraction's 2e-3.
@pytest.mark.parametrize("rows,k", SHAPES)
def test_dense_kernel_shapes_fixed_iterations(R, orc, rows, k):
    """HG g = 0.8 (folded) on a grid ragged against the row blocks, isotropic inflow on every face,
    quadrants with fewer ordinates than a task holds; four iterations on both sides."""
    rng = np.random.default_rng(303)
    nx, ny = 45, 70
    st, ss, q = rand_problem(rng, nx, ny, 0.8)
    inflow = {"left": rng.uniform(0, 1, ny), "right": rng.uniform(0, 1, ny), "bottom": rng.uniform(0, 1, nx),
              "top": rng.uniform(0, 1, nx)}
    h = R.Handle(nx, ny, st, ss, q, box=(0.0, 1.3, 0.0, 0.7), inflow=inflow)
    p = orc.Problem(nx, ny, st, ss, q, box=(0.0, 1.3, 0.0, 0.7), inflow=inflow)
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 3, 5, seed=8, sample=2)  # 15 per quadrant
    h.set_ordinates(d, w)
    h.set_scattering(R.ROM_SCAT_HG, 0.8)
    phi, st_, rc = h.source_iterate(diag_opts(R, "fp32", rows, k, tol=-1.0, max_iter=4))
    assert rc == R.ROM_NOT_CONVERGED and st_.iters == 4 and st_.sweep == R.ROM_SWEEP_DIAG
    W = orc.build_W(d, w, orc.SCAT_HG, 0.8, fold=1)
    ref = orc.source_iterate(p, d, w, W, tol=-1.0, max_iter=4)
    parity.check(phi, ref["phi"], 2e-3, what=f"rows {rows} k {k}")


def test_dense_kernel_c4_path(R, orc):
    """The c4 ordinate set (1024 stratified ordinates, HG g = 0.8) on 128 x 128 cells with the
    row-lane sweep (16 rows x 4 ordinates per lane): three iterations against the oracle, and to
    convergence against the strip sweep's solve."""
    g = RI.uniform_fields(128, 128, 1.0, 0.8, 0.45, 0.55)
    h = R.Handle(g.nx, g.ny, g.sigma_t, g.sigma_s, g.q)
    h.set_scattering(R.ROM_SCAT_HG, 0.8)
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 16, 16, seed=0)
    h.set_ordinates(d, w)
    phi, st_, rc = h.source_iterate(diag_opts(R, "fp32", 16, 4, tol=-1.0, max_iter=3))
    assert rc == R.ROM_NOT_CONVERGED and st_.iters == 3
    p = orc.Problem(g.nx, g.ny, g.sigma_t, g.sigma_s, g.q)
    W = orc.build_W(d, w, orc.SCAT_HG, 0.8, fold=1)
    ref = orc.source_iterate(p, d, w, W, tol=-1.0, max_iter=3)
    parity.check(phi, ref["phi"], 2e-3, what="c4 path, row-lane")
    conv, st_c, rc = h.source_iterate(diag_opts(R, "fp32", 16, 4, tol=1e-6))
    strip, st_s, rc2 = h.source_iterate(R.si_opts(tol=1e-6, tile=(8, 4), band=4, sweep=R.ROM_SWEEP_STRIP))
    assert rc == 0 and rc2 == 0 and abs(st_c.iters - st_s.iters) <= 1
    parity.check(conv, strip, 2e-3, what="row-lane vs strip, converged")


def test_dense_caller_kernel_and_reuse(R, orc):
    """A non-symmetric caller kernel with unequal weights (pins the orientation of the contraction
    through the row-lane layout), then new ordinate values for the cached plan (refresh: lane
    table, inflow and kernel matrix rewritten in place)."""
    rng = np.random.default_rng(31)
    nx, ny = 33, 20
    st, ss, q = rand_problem(rng, nx, ny, 0.6)
    h = R.Handle(nx, ny, st, ss, q)
    p = orc.Problem(nx, ny, st, ss, q)
    d, w = R.generate_ordinates(R.ROM_ORD_GAUSS2D, 4)
    h.set_ordinates(d, w)
    P = rng.uniform(0.2, 1.5, (len(w), len(w)))
    h.set_scattering(R.ROM_SCAT_DENSE, 0.0, P)
    o = diag_opts(R, "fp32", 16, 2, tol=-1.0, max_iter=5)
    phi, _, _ = h.source_iterate(o)
    W = orc.build_W(d, w, orc.SCAT_DENSE, P=P)
    parity.check(phi, orc.source_iterate(p, d, w, W, tol=-1.0, max_iter=5)["phi"], 2e-3, what="dense P")
    h.set_scattering(R.ROM_SCAT_HG, 0.6)
    for sample in (0, 1):
        d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 3, 3, seed=4, sample=sample)
        h.set_ordinates(d, w)
        phi, st_, _ = h.source_iterate(o)
        assert st_.sweep == R.ROM_SWEEP_DIAG
        W = orc.build_W(d, w, orc.SCAT_HG, 0.6, fold=1)
        parity.check(phi, orc.source_iterate(p, d, w, W, tol=-1.0, max_iter=5)["phi"], 2e-3, what=f"sample {sample}")


def test_dense_kernel_ensemble(R, orc):
    """An ensemble of HG samples (normalized kernel) on the row-lane sweep: each sample's flux
    against the oracle at the GPU's iteration count."""
    f = RI.uniform_fields(40, 36, 1.0, 0.8, 0.45, 0.55)
    h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    p = orc.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    h.set_scattering(R.ROM_SCAT_HG | R.ROM_SCAT_NORMALIZE, 0.8)
    o = diag_opts(R, "fp32", 16, 1, tol=1e-6)
    phis, st_, rc = h.ensemble_samples(6, 3, R.ROM_ORD_STRATIFIED, 2, 2, opts=o)
    assert rc == 0 and st_.sweep == R.ROM_SWEEP_DIAG
    for k in range(6):
        d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 2, 2, seed=3, sample=k)
        W = orc.build_W(d, w, orc.SCAT_HG | orc.SCAT_NORMALIZE, 0.8, fold=1)
        ref = orc.source_iterate(p, d, w, W, tol=1e-6)
        # each sample stops on its own; a stop one iteration apart moves phi by at most tol * max phi
        assert st_.min_iters - 1 <= ref["iters"] <= st_.max_iters + 1
        parity.check(phis[k], ref["phi"], 2e-3, what=f"sample {k}")
