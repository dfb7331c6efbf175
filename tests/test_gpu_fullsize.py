"""Parity at the full workload sizes, in the launch configuration the bench times (strip sweep,
the autotuner's tile and band), on outputs the FP64 oracle can compute within seconds plus
properties that hold at any size:

* c3 (512 x 512, 64 samples of 128 stratified ordinates): two samples' fluxes against the oracle;
  the FP64 mean and variance of the ensemble call against two-pass moments of all 64 per-sample
  fluxes; mirror symmetry of the mean;
* c4 (256 x 256, 1024 ordinates, HG g = 0.8, BF16 contraction): the full solve converges and is
  mirror symmetric; the same 1024-ordinate set, contraction and tile on a 20 x 20 grid (ragged
  8-wide chunks) against the oracle;
* c5 (200 uneven problems in one persistent launch): the three problems with the fewest updates
  against the oracle, every problem converged.
"""
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


def nrm(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def mirror_err(phi, n):
    P = np.asarray(phi).reshape(n, n)
    return max(nrm(P[:, ::-1], P), nrm(P[::-1, :], P))


def test_c3_full_size(R, orc):
    wl = RI.c3()
    f = wl.fields[0]
    h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    o = R.si_opts(tol=wl.tol, max_iter=wl.max_iter, tile=(16, 16), band=4, sweep=R.ROM_SWEEP_STRIP)
    phis, st, rc = h.ensemble_samples(wl.samples, wl.seed, R.ROM_ORD_STRATIFIED, 4, 8, opts=o)
    assert rc == 0 and phis.shape == (64, f.nx * f.ny)
    mean, var, est, rc = h.ensemble(wl.samples, wl.seed, R.ROM_ORD_STRATIFIED, 4, 8, o)
    assert rc == 0
    m = phis.mean(axis=0)
    v = ((phis - m) ** 2).sum(axis=0) / (wl.samples - 1)
    assert np.max(np.abs(mean - m)) <= 1e-12 * np.max(np.abs(m))
    assert np.max(np.abs(var - v)) <= 1e-10 * np.max(np.abs(v))
    assert mirror_err(mean, f.nx) < 1e-5
    p = orc.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    for k in (0, 37):
        d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 4, 8, seed=wl.seed, sample=k)
        ref = orc.source_iterate(p, d, w, None, tol=wl.tol)
        assert nrm(phis[k], ref["phi"]) < 1e-5, k


def test_c4_full_size(R, orc):
    wl = RI.c4()
    f = wl.fields[0]
    h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    h.set_scattering(R.ROM_SCAT_HG, wl.g)
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 16, 16, seed=wl.seed)
    assert len(w) == 1024
    h.set_ordinates(d, w)
    o = R.si_opts(tol=wl.tol, max_iter=wl.max_iter, tile=(8, 4), band=4, sweep=R.ROM_SWEEP_STRIP)
    phi, st, rc = h.source_iterate(o)
    assert rc == 0 and st.final_r <= wl.tol
    assert mirror_err(phi, f.nx) < 1e-4  # BF16 angular flux in the contraction
    # the same ordinate set, kernel, precision and launch shape on a grid the oracle solves quickly
    g = RI.uniform_fields(20, 20, 1.0, 0.8, 0.45, 0.55)
    hs = R.Handle(g.nx, g.ny, g.sigma_t, g.sigma_s, g.q)
    hs.set_scattering(R.ROM_SCAT_HG, wl.g)
    hs.set_ordinates(d, w)
    phi_s, st_s, rc = hs.source_iterate(o)
    assert rc == 0
    p = orc.Problem(g.nx, g.ny, g.sigma_t, g.sigma_s, g.q)
    W = orc.build_W(d, w, orc.SCAT_HG, wl.g, fold=1)
    ref = orc.source_iterate(p, d, w, W, tol=wl.tol)
    assert nrm(phi_s, ref["phi"]) < 2e-3


def test_c5_full_size(R, orc):
    wl = RI.c5()
    hs, sets = [], []
    for k, f in enumerate(wl.fields):
        h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
        nz, nt = orc.stratified_spec(wl.n_ord[k])
        d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, nz, nt, seed=wl.problem_seed(k))
        h.set_ordinates(d, w)
        hs.append(h)
        sets.append((d, w))
    o = R.si_opts(tol=wl.tol, max_iter=wl.max_iter, tile=(16, 16), band=4, sweep=R.ROM_SWEEP_STRIP)
    outs, stats, rc = R.solve_batch(hs, o)
    assert rc == 0 and all(s.status == 0 for s in stats)
    cost = [f.nx * f.ny * wl.n_ord[k] for k, f in enumerate(wl.fields)]
    for k in np.argsort(cost)[:3]:
        f = wl.fields[k]
        p = orc.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
        ref = orc.source_iterate(p, sets[k][0], sets[k][1], None, tol=wl.tol)
        assert abs(stats[k].iters - ref["iters"]) <= 1, k
        assert nrm(outs[k], ref["phi"]) < 1e-5, k
