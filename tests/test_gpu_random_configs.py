"""Seeded random configurations against the FP64 oracle: grid sizes from 1 to 70 cells a side,
non-square boxes, random cross sections and sources, inflow on a random subset of faces, random
stratified or i.i.d. ordinate sets, step or diamond difference, FP32 or FP64, isotropic, linear
or Henyey-Greenstein scattering (optionally normalized), and an explicit sweep kernel, tile and
band drawn among the supported ones (or the autotuner's choice).  Each case runs four source
iterations from phi = 0 and compares the flux with the oracle's four iterations."""
import numpy as np
import pytest

import parity
from parity import nrm

pytestmark = pytest.mark.gpu

CASES = 64


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_12527_amd import rom
    rom.lib()
    return rom


def draw(R, orc, seed):
    """One configuration; everything the library and the oracle need, and the tolerance."""
    rng = np.random.default_rng(9000 + seed)
    nx, ny = int(rng.integers(1, 71)), int(rng.integers(1, 71))
    box = (0.0, float(rng.uniform(0.3, 3.0)), 0.0, float(rng.uniform(0.3, 3.0)))
    cells = nx * ny
    st = rng.uniform(0.2, 3.0, cells)
    ss = st * rng.uniform(0.0, 0.9, cells)
    q = rng.uniform(0.0, 1.0, cells) * (rng.uniform(0, 1, cells) > 0.3)
    inflow = {}
    for face, n in (("left", ny), ("right", ny), ("bottom", nx), ("top", nx)):
        if rng.uniform() < 0.5:
            inflow[face] = rng.uniform(0.0, 1.0, n)
    if rng.uniform() < 0.5:
        d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, int(rng.integers(1, 4)), int(rng.integers(1, 6)),
                                    seed=int(rng.integers(0, 1 << 30)))
    else:
        d, w = R.generate_ordinates(R.ROM_ORD_IID_SPHERE, int(rng.integers(4, 41)), seed=int(rng.integers(0, 1 << 30)))
    fp64 = bool(rng.uniform() < 0.5)
    dd = bool(rng.uniform() < 0.3)
    u = rng.uniform()
    scat = "iso" if u < 0.6 else ("linear" if u < 0.8 else "hg")
    g = float(rng.uniform(-0.9, 0.9)) if scat == "linear" else 0.8
    norm = scat != "iso" and bool(rng.uniform() < 0.5)
    # kernel shape: the row-lane sweep takes isotropic step-scheme problems only
    kw = {}
    k = rng.uniform()
    if scat == "iso" and not dd and k < 0.4:
        kw = dict(sweep=R.ROM_SWEEP_DIAG, diag_rows=int(rng.choice([16, 64])),
                  diag_k=int(rng.choice([1, 2] if fp64 else [1, 2, 4])), band=int(rng.choice([1, 2, 4])))
    elif k < 0.85:
        tiles = [(8, 4), (8, 8)] if fp64 else [(8, 4), (8, 8), (16, 8), (16, 16)]
        kw = dict(sweep=R.ROM_SWEEP_STRIP, tile=tiles[int(rng.integers(0, len(tiles)))],
                  band=int(rng.choice([1, 2, 4, 8])))
    tol = 1e-11 if fp64 else (2e-3 if scat == "hg" else 1e-5)
    return dict(nx=nx, ny=ny, box=box, st=st, ss=ss, q=q, inflow=inflow or None, d=d, w=w, fp64=fp64, dd=dd,
                scat=scat, g=g, norm=norm, kw=kw, tol=tol)


@pytest.mark.parametrize("seed", range(CASES))
def test_random_configuration(R, orc, seed):
    c = draw(R, orc, seed)
    h = R.Handle(c["nx"], c["ny"], c["st"], c["ss"], c["q"], box=c["box"], inflow=c["inflow"])
    p = orc.Problem(c["nx"], c["ny"], c["st"], c["ss"], c["q"], box=c["box"], inflow=c["inflow"])
    W = None
    if c["scat"] != "iso":
        rk = R.ROM_SCAT_LINEAR if c["scat"] == "linear" else R.ROM_SCAT_HG
        ok = orc.SCAT_LINEAR if c["scat"] == "linear" else orc.SCAT_HG
        h.set_scattering(rk | (R.ROM_SCAT_NORMALIZE if c["norm"] else 0), c["g"])
        W = orc.build_W(c["d"], c["w"], ok | (orc.SCAT_NORMALIZE if c["norm"] else 0), c["g"], fold=1)
    h.set_ordinates(c["d"], c["w"])
    kw = dict(c["kw"])
    while True:
        o = R.si_opts(tol=-1.0, max_iter=4, precision=R.ROM_PREC_FP64 if c["fp64"] else R.ROM_PREC_FP32,
                      scheme=R.ROM_SCHEME_DD if c["dd"] else R.ROM_SCHEME_STEP, **kw)
        try:
            phi, st, rc = h.source_iterate(o)
            break
        except R.RomError as e:
            # an explicit band whose LDS rings do not fit the tile and source kind is refused
            # before any device work; halve it
            assert e.status == R.ROM_E_ARG and "band too large" in str(e) and kw.get("band", 0) > 1, e
            kw["band"] //= 2
    assert rc == R.ROM_NOT_CONVERGED and st.iters == 4
    ref = orc.source_iterate(p, c["d"], c["w"], W, scheme=orc.SCHEME_DD if c["dd"] else orc.SCHEME_STEP,
                             tol=0.0, max_iter=4)["phi"]
    summary = {k: c[k] for k in ("nx", "ny", "fp64", "dd", "scat", "norm", "kw")}
    parity.check(phi, ref, c["tol"], what=str((summary, len(c["w"]))))


@pytest.mark.parametrize("seed", range(24))
def test_random_ensemble(R, orc, seed):
    """Ensembles: random grid, stratified spec, sample count (several samples share a wavefront
    when a quadrant holds 16 or 32 ordinates), scheme, precision and scattering kind; each
    sample's flux after four iterations against the oracle on the same bit-identical set."""
    rng = np.random.default_rng(7000 + seed)
    nx, ny = int(rng.integers(3, 41)), int(rng.integers(3, 41))
    cells = nx * ny
    st = rng.uniform(0.3, 2.5, cells)
    ss = st * rng.uniform(0.0, 0.85, cells)
    q = rng.uniform(0.0, 1.0, cells)
    inflow = {"bottom": rng.uniform(0, 1, nx)} if rng.uniform() < 0.5 else None
    nz, nt = int(rng.integers(1, 4)), int(rng.integers(1, 5))
    t = int(rng.integers(1, 13))
    seed_o = int(rng.integers(0, 1 << 30))
    fp64 = bool(rng.uniform() < 0.5)
    dd = bool(rng.uniform() < 0.3)
    scat = ["iso", "linear", "hg"][int(rng.integers(0, 3))]
    h = R.Handle(nx, ny, st, ss, q, inflow=inflow)
    p = orc.Problem(nx, ny, st, ss, q, inflow=inflow)
    ok = None
    if scat != "iso":
        rk, ok = (R.ROM_SCAT_LINEAR, orc.SCAT_LINEAR) if scat == "linear" else (R.ROM_SCAT_HG, orc.SCAT_HG)
        h.set_scattering(rk | R.ROM_SCAT_NORMALIZE, 0.7)
    o = R.si_opts(tol=-1.0, max_iter=4, precision=R.ROM_PREC_FP64 if fp64 else R.ROM_PREC_FP32,
                  scheme=R.ROM_SCHEME_DD if dd else R.ROM_SCHEME_STEP)
    phis, st_, rc = h.ensemble_samples(t, seed_o, R.ROM_ORD_STRATIFIED, nz, nt, opts=o)
    assert rc == R.ROM_NOT_CONVERGED and phis.shape == (t, cells)
    tol = 1e-11 if fp64 else (2e-3 if scat == "hg" else 1e-5)
    for k in range(t):
        d, w = orc.generate(orc.ORD_STRATIFIED, nz, nt, seed=seed_o, sample=k)
        W = None if ok is None else orc.build_W(d, w, ok | orc.SCAT_NORMALIZE, 0.7, fold=1)
        ref = orc.source_iterate(p, d, w, W, scheme=orc.SCHEME_DD if dd else orc.SCHEME_STEP, tol=0.0,
                                 max_iter=4)["phi"]
        parity.check(phis[k], ref, tol, what=str((k, nx, ny, nz, nt, t, fp64, dd, scat)))


@pytest.mark.parametrize("seed", range(16))
def test_random_batch(R, orc, seed):
    """Batches of 2 to 6 uneven problems in one persistent launch per iteration (random sizes,
    ordinate sets and counts, isotropic scattering); four iterations of each against the oracle."""
    rng = np.random.default_rng(8000 + seed)
    k = int(rng.integers(2, 7))
    fp64 = bool(rng.uniform() < 0.5)
    hs, refs = [], []
    for i in range(k):
        nx, ny = int(rng.integers(2, 49)), int(rng.integers(2, 49))
        cells = nx * ny
        st = rng.uniform(0.3, 2.5, cells)
        ss = st * rng.uniform(0.0, 0.85, cells)
        q = rng.uniform(0.0, 1.0, cells)
        if rng.uniform() < 0.5:
            d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, int(rng.integers(1, 4)), int(rng.integers(1, 6)),
                                        seed=int(rng.integers(0, 1 << 30)))
        else:
            d, w = R.generate_ordinates(R.ROM_ORD_IID_SPHERE, int(rng.integers(4, 33)), seed=int(rng.integers(0, 1 << 30)))
        h = R.Handle(nx, ny, st, ss, q)
        h.set_ordinates(d, w)
        hs.append(h)
        refs.append(orc.source_iterate(orc.Problem(nx, ny, st, ss, q), d, w, None, tol=0.0, max_iter=4)["phi"])
    o = R.si_opts(tol=-1.0, max_iter=4, precision=R.ROM_PREC_FP64 if fp64 else R.ROM_PREC_FP32)
    outs, stats, rc = R.solve_batch(hs, o)
    assert rc == R.ROM_NOT_CONVERGED
    for i in range(k):
        assert stats[i].iters == 4
        parity.check(outs[i], refs[i], (1e-11 if fp64 else 1e-5), what=str((i, k, fp64)))


@pytest.mark.parametrize("seed", range(16))
def test_random_slab(R, orc, seed):
    """Slab geometry: random grid (1 to 200 cells), fields, interval, ROM sets or Gauss / midpoint
    quadratures of random even size, a ragged number of systems per launch, random inflow values;
    five iterations in FP64 (max-norm 1e-12) or FP32 (normwise 1e-5) against the oracle."""
    rng = np.random.default_rng(6000 + seed)
    nx = int(rng.integers(1, 201))
    x0 = float(rng.uniform(-1.0, 1.0))
    x1 = x0 + float(rng.uniform(0.2, 4.0))
    st = rng.uniform(0.3, 3.0, nx + 1)
    ss = st * rng.uniform(0.0, 0.9, nx + 1)
    q = rng.uniform(0.0, 1.0, nx + 1)
    s = R.Slab(nx, st, ss, q, x0=x0, x1=x1)
    n = 2 * int(rng.integers(1, 21))
    kind = int(rng.integers(0, 3))
    t = int(rng.integers(1, 71)) if kind == R.ROM_SLAB_RANDOM else 1
    sets = [R.slab_ordinates(kind, n, 17, k) for k in range(t)]
    mu = np.array([m for m, _ in sets])
    w = np.array([x for _, x in sets])
    inflow = rng.uniform(0.0, 2.0, (t, n))
    fp64 = bool(rng.uniform() < 0.5)
    phis, iters, st_, rc = s.solve(mu, w, inflow, R.si_opts(tol=-1.0, max_iter=5,
                                                          precision=R.ROM_PREC_FP64 if fp64 else R.ROM_PREC_FP32))
    assert rc == R.ROM_NOT_CONVERGED and np.all(iters == 5)
    for k in range(t):
        ref = orc.slab_source_iterate(nx, x0, x1, st, ss, q, mu[k], w[k], inflow[k], tol=0.0, max_iter=5)["phi"]
        if fp64:
            assert np.max(np.abs(phis[k] - ref)) <= 1e-12 * np.max(np.abs(ref)), (k, nx, n, kind, t)
        else:
            parity.check(phis[k], ref, 1e-5, what=str((k, nx, n, kind, t)))
