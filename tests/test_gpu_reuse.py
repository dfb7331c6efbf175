"""GPU parity of cached plans: a handle re-solved after new ordinates, new angular inflow or a new
kernel parameter (tables rewritten in place, captured graph kept), after a change of quadrant
counts (plan rebuilt), and repeated batches and ensembles.  Every solve is checked against the
FP64 oracle on the same bit-identical ordinate set, to the same bars as the other parity tests
(FP64 fixed iterations 1e-11 normwise, FP32 1e-5, BF16 contraction 2e-3)."""
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


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_new_ordinates_same_and_changed_layout(R, orc, prec):
    rng = np.random.default_rng(41)
    nx, ny = 45, 38
    st, ss, q = rand_problem(rng, nx, ny)
    inflow = {"left": rng.uniform(0, 1, ny), "bottom": rng.uniform(0, 1, nx)}
    h = R.Handle(nx, ny, st, ss, q, inflow=inflow)
    p = orc.Problem(nx, ny, st, ss, q, inflow=inflow)
    fp64 = prec == "fp64"
    o = R.si_opts(tol=-1.0, max_iter=7, precision=R.ROM_PREC_FP64 if fp64 else R.ROM_PREC_FP32)
    bar = 1e-11 if fp64 else 1e-5
    sets = [R.generate_ordinates(R.ROM_ORD_STRATIFIED, 2, 4, seed=3, sample=s) for s in range(3)]
    sets.append(R.generate_ordinates(R.ROM_ORD_IID_SPHERE, 32, seed=4))     # other quadrant counts
    sets.append(R.generate_ordinates(R.ROM_ORD_STRATIFIED, 2, 4, seed=3, sample=5))
    for d, w in sets:
        h.set_ordinates(d, w)
        phi, stt, rc = h.source_iterate(o)
        ref = orc.source_iterate(p, d, w, None, tol=0.0, max_iter=7)
        assert rc == R.ROM_NOT_CONVERGED and stt.iters == 7
        parity.check(phi, ref["phi"], bar)


def test_new_angular_inflow_values(R, orc):
    rng = np.random.default_rng(42)
    nx, ny = 30, 26
    st, ss, q = rand_problem(rng, nx, ny, 0.7)
    h = R.Handle(nx, ny, st, ss, q)
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 2, 2, seed=1)
    h.set_ordinates(d, w)
    n = len(w)
    o = R.si_opts(tol=-1.0, max_iter=5, precision=R.ROM_PREC_FP64)
    for rep in range(2):
        ang = rng.uniform(0, 2, (n, ny))
        h.set_inflow_angular(R.ROM_FACE_RIGHT, ang)
        p = orc.Problem(nx, ny, st, ss, q, inflow_angular={"right": np.ascontiguousarray(ang)})
        phi, _, _ = h.source_iterate(o)
        ref = orc.source_iterate(p, d, w, None, tol=0.0, max_iter=5)
        parity.check(phi, ref["phi"], 1e-11, what=str(rep))
    # back to vacuum: the plan's inflow presence changes, so it is rebuilt
    h.set_inflow_angular(R.ROM_FACE_RIGHT, None)
    phi, _, _ = h.source_iterate(o)
    ref = orc.source_iterate(orc.Problem(nx, ny, st, ss, q), d, w, None, tol=0.0, max_iter=5)
    parity.check(phi, ref["phi"], 1e-11)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_anisotropic_new_ordinates_and_g(R, orc, prec):
    nx = ny = 24
    f = RI.uniform_fields(nx, ny, 1.0, 0.8, 0.4, 0.6)
    h = R.Handle(nx, ny, f.sigma_t, f.sigma_s, f.q)
    p = orc.Problem(nx, ny, f.sigma_t, f.sigma_s, f.q)
    fp64 = prec == "fp64"
    o = R.si_opts(tol=-1.0, max_iter=6, precision=R.ROM_PREC_FP64 if fp64 else R.ROM_PREC_FP32)
    for sample, g in ((0, 0.8), (1, 0.8), (1, 0.5)):
        d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 4, 4, seed=2, sample=sample)
        h.set_ordinates(d, w)
        h.set_scattering(R.ROM_SCAT_HG, g)
        W = orc.build_W(d, w, orc.SCAT_HG, g, fold=1)
        phi, _, _ = h.source_iterate(o)
        ref = orc.source_iterate(p, d, w, W, tol=0.0, max_iter=6)
        parity.check(phi, ref["phi"], (1e-11 if fp64 else 2e-3), what=str((sample, g)))


def test_batch_repeat_and_changed_member(R, orc):
    wl = RI.c5(count=4, sides=(16, 32, 40), m_range=(4, 12), master_seed=3)
    hs, probs, sets = [], [], []
    for k, f in enumerate(wl.fields):
        hs.append(R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q))
        probs.append(orc.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q))
        nz, nt = orc.stratified_spec(wl.n_ord[k])
        d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, nz, nt, seed=wl.problem_seed(k))
        hs[-1].set_ordinates(d, w)
        sets.append((d, w))
    o = R.si_opts(tol=1e-6)
    out1, _, rc1 = R.solve_batch(hs, o)
    out2, _, rc2 = R.solve_batch(hs, o)
    assert rc1 == 0 and rc2 == 0
    for a, b in zip(out1, out2):
        assert np.array_equal(a, b)
    nz, nt = orc.stratified_spec(wl.n_ord[2])
    sets[2] = R.generate_ordinates(R.ROM_ORD_STRATIFIED, nz, nt, seed=wl.problem_seed(2), sample=1)
    hs[2].set_ordinates(*sets[2])
    out3, _, rc3 = R.solve_batch(hs, o)
    assert rc3 == 0
    for k in range(len(hs)):
        ref = orc.source_iterate(probs[k], sets[k][0], sets[k][1], None, tol=1e-6)["phi"]
        parity.check(out3[k], ref, 1e-5, what=str(k))
    # the same handles in another order form another batch
    out4, _, rc4 = R.solve_batch(hs[::-1], o)
    assert rc4 == 0
    for a, b in zip(out4[::-1], out3):
        parity.check(a, b, 1e-6)


def test_ensemble_twice_other_seed(R, orc):
    nx, ny = 48, 40
    f = RI.uniform_fields(nx, ny, 1.0, 0.5, 0.4, 0.6)
    h = R.Handle(nx, ny, f.sigma_t, f.sigma_s, f.q)
    p = orc.Problem(nx, ny, f.sigma_t, f.sigma_s, f.q)
    o = R.si_opts(tol=1e-7, precision=R.ROM_PREC_FP64)
    for seed in (7, 8):
        mean, var, st, rc = h.ensemble(5, seed, R.ROM_ORD_STRATIFIED, 2, 4, o)
        ref = orc.ensemble(p, orc.ORD_STRATIFIED, 2, 4, seed, 5, tol=1e-7)
        assert rc == 0
        parity.check(mean, ref["mean"], 1e-10, what=str(seed))
        parity.check(var, ref["var"], 1e-8, what=str(seed))


def test_autotuned_shape_reported(R):
    wl = RI.c1()
    f = wl.fields[0]
    h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 2, 4, seed=0)
    h.set_ordinates(d, w)
    _, st, rc = h.source_iterate(R.si_opts(tol=1e-6))
    assert rc == 0
    if st.sweep == R.ROM_SWEEP_STRIP:
        assert (st.tile_x, st.tile_y) in ((8, 4), (8, 8), (16, 8), (16, 16))
        assert 1 <= st.band <= 8 and st.lanes in (16, 32, 64)
    else:
        assert st.sweep == R.ROM_SWEEP_DIAG
        assert st.tile_y in (16, 64) and st.tile_x in (1, 2, 4) and 1 <= st.band <= 16


def test_distinct_handles_from_several_threads(R, orc):
    """Distinct handles may be used from different threads: four host threads each build, autotune
    and solve three problems of their own shapes at the same time (every first solve of a shape
    captures a graph while the other threads allocate, copy and free), and every result matches
    the oracle."""
    import threading
    rng = np.random.default_rng(77)
    nthreads, per = 4, 3
    probs = []
    for k in range(nthreads * per):
        nx, ny = 20 + 4 * (k % 5), 16 + 2 * (k % 3)
        st = rng.uniform(0.5, 2.0, nx * ny)
        ss = st * rng.uniform(0.0, 0.7, nx * ny)
        q = rng.uniform(0.0, 1.0, nx * ny)
        d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 1 + k % 2, 2 + k % 3, seed=k)
        probs.append((nx, ny, st, ss, q, d, w))
    out = [None] * len(probs)
    errs = []

    def work(i):
        try:
            for k in range(i * per, (i + 1) * per):
                nx, ny, st, ss, q, d, w = probs[k]
                h = R.Handle(nx, ny, st, ss, q)
                h.set_ordinates(d, w)
                out[k] = h.source_iterate(R.si_opts(tol=1e-6))[0]
                h.close()
        except Exception as e:  # reported after the join
            errs.append(e)

    refs = [orc.source_iterate(orc.Problem(nx, ny, st, ss, q), d, w, None, tol=1e-6)["phi"]
            for (nx, ny, st, ss, q, d, w) in probs]
    for rnd in range(3):  # the threads' calls interleave differently each round
        out[:] = [None] * len(probs)
        ts = [threading.Thread(target=work, args=(i,)) for i in range(nthreads)]
        for t in ts:
            t.start()
        for t in ts:
            t.join(timeout=120)
        assert not errs, (rnd, errs)
        for k in range(len(probs)):
            parity.check(out[k], refs[k], 1e-5, what=str((rnd, k)))


def test_solve_on_a_caller_stream(R, orc):
    """A handle bound to a caller's HIP stream (a torch stream at default priority) runs its plan
    there: the result is bitwise that of the default-stream solve of a twin handle, the device
    result is readable after the stream's work, and the ensemble path works on it too."""
    import torch
    rng = np.random.default_rng(8)
    nx, ny = 40, 28
    st, ss, q = rand_problem(rng, nx, ny, 0.8)
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 2, 4, seed=6)
    a = R.Handle(nx, ny, st, ss, q)
    a.set_ordinates(d, w)
    phi_a, _, rc = a.source_iterate(R.si_opts(tol=1e-6))
    assert rc == 0
    b = R.Handle(nx, ny, st, ss, q)
    s = torch.cuda.Stream()
    b.use_torch_stream(s)
    b.set_ordinates(d, w)
    with torch.cuda.stream(s):
        phi_b, _, rc = b.source_iterate(R.si_opts(tol=1e-6))
        dev = b.phi_device_tensor()
    s.synchronize()
    assert rc == 0 and np.array_equal(phi_a, phi_b)
    np.testing.assert_array_equal(dev.cpu().numpy().astype(np.float64), phi_b)
    mean_a, _, _, rc_a = a.ensemble(6, 2, R.ROM_ORD_STRATIFIED, 2, 2, R.si_opts(tol=1e-6))
    mean_b, _, _, rc_b = b.ensemble(6, 2, R.ROM_ORD_STRATIFIED, 2, 2, R.si_opts(tol=1e-6))
    assert rc_a == 0 and rc_b == 0 and np.array_equal(mean_a, mean_b)
    ref = orc.source_iterate(orc.Problem(nx, ny, st, ss, q), d, w, None, tol=1e-6)["phi"]
    parity.check(phi_b, ref, 1e-5)
