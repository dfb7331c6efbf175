"""Pins of the FP64 oracle against facts that do not come from the oracle itself: printed values
of the paper, published generator outputs, closed forms, a brute-force direct solve, exact
conservation identities, symmetry and library routines.  CPU only.

Each test names the mistake class it is there to catch.
"""
import math
import os

import numpy as np
import pytest

import rom_inputs as RI

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _prob(orc, nx, ny, st, ss, q, box=(0.0, 1.0, 0.0, 1.0), inflow=None, inflow_angular=None):
    return orc.Problem(nx, ny, st, ss, q, box=box, inflow=inflow, inflow_angular=inflow_angular)


def _rand_fields(rng, nx, ny, ratio_max=0.9):
    st = rng.uniform(0.5, 3.0, nx * ny)
    ss = st * rng.uniform(0.0, ratio_max, nx * ny)
    q = rng.uniform(0.0, 2.0, nx * ny)
    return st, ss, q


# ------------------------------------------------------------------------------------ generator
def test_splitmix64_published_outputs(orc):
    """SplitMix64 as published (Steele et al. 2014): first outputs for seed 1234567."""
    lines = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64.txt")) if l.strip() and l[0] != "#"]
    seed = int(lines[0][1])
    want = [int(l[0]) for l in lines[1:]]
    got = [int(v) for v in orc.splitmix64_stream(seed, len(want))]
    assert got == want


def test_u01_and_sample_streams(orc):
    """u = (x >> 11) 2^-53 lies in [0, 1); sample s's stream seed is master output s+1."""
    xs = orc.splitmix64_stream(7, 4)
    for x in xs:
        u = orc.u01(int(x))
        assert 0.0 <= u < 1.0
        assert u == (int(x) >> 11) * 2.0 ** -53
    assert orc.u01(0) == 0.0
    assert orc.u01(2**64 - 1) == 1.0 - 2.0 ** -53
    master = orc.splitmix64_stream(42, 3)
    assert [orc.sample_seed(42, s) for s in range(3)] == [int(v) for v in master]


# ------------------------------------------------------------------------------------ quadratures
@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 40, 400])
def test_gauss_legendre_matches_numpy(orc, n):
    x, w = orc.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(np.sort(x), np.sort(xr), atol=2e-15, rtol=0)
    # numpy's weights lose ~1e-9 relative near the ends for large n (eigenvalue method)
    np.testing.assert_allclose(w[np.argsort(x)], wr[np.argsort(xr)], atol=0, rtol=1e-12 if n <= 40 else 2e-9)
    assert abs(w.sum() - 2.0) < 1e-14


@pytest.mark.parametrize("kind,N,count", [("uniform2d", 20, 1600), ("gauss2d", 20, 840), ("gauss2d", 200, 80400),
                                          ("uniform2d", 3, 36), ("gauss2d", 5, 60)])
def test_quadrature_counts_weights_symmetry(orc, kind, N, count):
    """Ordinate counts 4N^2 / 2N(N+1) (Sec. 2, Table 1; Sec. 4.2), weights sum to 1, directions are
    unit vectors, quadrants are exact mirror images (eq. (3.5))."""
    k = orc.ORD_UNIFORM2D if kind == "uniform2d" else orc.ORD_GAUSS2D
    dirs, w = orc.generate(k, N)
    assert dirs.shape == (count, 3)
    assert abs(w.sum() - 1.0) < 1e-12
    np.testing.assert_allclose((dirs ** 2).sum(1), 1.0, atol=1e-14)
    m = count // 4
    q1 = dirs[:m]
    assert np.all(q1[:, 0] > 0) and np.all(q1[:, 1] > 0) and np.all(q1[:, 2] > 0)
    assert np.array_equal(dirs[m:2 * m], q1 * [-1, 1, 1])
    assert np.array_equal(dirs[2 * m:3 * m], q1 * [-1, -1, 1])
    assert np.array_equal(dirs[3 * m:], q1 * [1, -1, 1])
    assert np.array_equal(w[:m], w[m:2 * m]) and np.array_equal(w[:m], w[3 * m:])


def test_uniform2d_nodes_closed_form(orc):
    """eq. (A.5): zeta_i = (2N-2i+1)/(2N), theta_j = (2j-1)pi/(4N), l = (i-1)N + j."""
    N = 4
    dirs, w = orc.generate(orc.ORD_UNIFORM2D, N)
    for i in range(1, N + 1):
        for j in range(1, N + 1):
            l = (i - 1) * N + (j - 1)
            z = (2 * N - 2 * i + 1) / (2 * N)
            th = (2 * j - 1) * math.pi / (4 * N)
            assert abs(dirs[l, 2] - z) < 1e-15
            assert abs(math.atan2(dirs[l, 1], dirs[l, 0]) - th) < 1e-14
            assert w[l] == 1.0 / (4 * N * N)


def test_gauss2d_levels(orc):
    """Appendix A Gaussian set: level i (counting from the pole) has i azimuths (2j-1)pi/(4i) at the
    i-th largest positive root of L_2N; its weights sum per quadrant to the Gauss weight / 4."""
    N = 6
    dirs, w = orc.generate(orc.ORD_GAUSS2D, N)
    xr, wr = np.polynomial.legendre.leggauss(2 * N)
    pos = np.argsort(-xr)[:N]
    l = 0
    for i in range(1, N + 1):
        z, gw = xr[pos[i - 1]], wr[pos[i - 1]]
        for j in range(1, i + 1):
            assert abs(dirs[l, 2] - z) < 1e-14
            assert abs(math.atan2(dirs[l, 1], dirs[l, 0]) - (2 * j - 1) * math.pi / (4 * i)) < 1e-13
            assert abs(w[l] - gw / (4 * i)) < 1e-14
            l += 1


def test_zeta_bands(orc):
    assert [orc.zeta_bands(m) for m in (1, 4, 8, 9, 16, 32, 64, 256, 7, 12, 128)] == [1, 2, 2, 3, 4, 4, 8, 16, 1, 3, 8]


@pytest.mark.parametrize("nz,nt,sample", [(8, 8, 0), (4, 8, 5), (1, 7, 2), (16, 16, 0)])
def test_stratified_draws_in_cells(orc, nz, nt, sample):
    """Sec. 3.1 steps 1-2 and Sec. 4.2: one draw in every (zeta, theta) cell, index l = i*nt + j,
    mirrored quadrants (eq. (3.5)), weights 1/n (eq. (3.4))."""
    dirs, w = orc.generate(orc.ORD_STRATIFIED, nz, nt, seed=3, sample=sample)
    m = nz * nt
    assert dirs.shape == (4 * m, 3)
    np.testing.assert_array_equal(w, np.full(4 * m, 1.0 / (4 * m)))
    for i in range(nz):
        for j in range(nt):
            c, s, z = dirs[i * nt + j]
            assert 1.0 - (i + 1) / nz <= z <= 1.0 - i / nz
            th = math.atan2(s, c)
            assert j * (math.pi / 2) / nt - 1e-15 <= th <= (j + 1) * (math.pi / 2) / nt + 1e-15
            assert abs(c * c + s * s + z * z - 1.0) < 1e-14
    q1 = dirs[:m]
    assert np.array_equal(dirs[m:2 * m], q1 * [-1, 1, 1])
    assert np.array_equal(dirs[2 * m:3 * m], q1 * [-1, -1, 1])
    assert np.array_equal(dirs[3 * m:], q1 * [1, -1, 1])


def test_stratified_exact_draw_formula(orc):
    """The first cell's point is built from the first two uniforms of the sample's stream."""
    nz, nt, seed, s = 4, 8, 11, 3
    dirs, _ = orc.generate(orc.ORD_STRATIFIED, nz, nt, seed=seed, sample=s)
    xs = orc.splitmix64_stream(orc.sample_seed(seed, s), 2)
    uz, ut = orc.u01(int(xs[0])), orc.u01(int(xs[1]))
    z = 1.0 - (0 + uz) / nz
    th = (0 + ut) * (0.5 * math.pi) / nt
    rho = math.sqrt((1.0 - z) * (1.0 + z))
    assert dirs[0, 2] == z
    assert dirs[0, 0] == rho * math.cos(th) and dirs[0, 1] == rho * math.sin(th)


def test_stratified_within_cell_positions_uniform(orc):
    """Within-cell coordinates over many samples are U(0,1) (Kolmogorov-Smirnov)."""
    from scipy import stats
    nz, nt = 2, 4
    fz, ft = [], []
    for s in range(400):
        d, _ = orc.generate(orc.ORD_STRATIFIED, nz, nt, seed=0, sample=s)
        for i in range(nz):
            for j in range(nt):
                c, sn, z = d[i * nt + j]
                fz.append((1.0 - z) * nz - i)
                ft.append(math.atan2(sn, c) / (math.pi / 2) * nt - j)
    assert stats.kstest(fz, "uniform").pvalue > 1e-3
    assert stats.kstest(ft, "uniform").pvalue > 1e-3


def test_iid_sphere_statistics(orc):
    """i.i.d. uniform directions on the sphere: zeta ~ U(-1,1), azimuth ~ U(0, 2 pi)."""
    from scipy import stats
    d, w = orc.generate(orc.ORD_IID_SPHERE, 4000, seed=0, sample=0)
    assert abs(w.sum() - 1.0) < 1e-12
    np.testing.assert_allclose((d ** 2).sum(1), 1.0, atol=1e-14)
    assert stats.kstest((d[:, 2] + 1) / 2, "uniform").pvalue > 1e-3
    az = (np.arctan2(d[:, 1], d[:, 0]) % (2 * np.pi)) / (2 * np.pi)
    assert stats.kstest(az, "uniform").pvalue > 1e-3


# ------------------------------------------------------------------------------------ kernels
def test_linear_kernel_fold_is_planar_cosine(orc):
    """Folding 1 + g mu over +-zeta' leaves 1 + g(cc' + ss') (eq. (2.1))."""
    d, w = orc.generate(orc.ORD_STRATIFIED, 2, 3, seed=1)
    W = orc.build_W(d, w, orc.SCAT_LINEAR, 0.9, fold=1)
    P = 1.0 + 0.9 * (d[:, 0:1] * d[:, 0] + d[:, 1:2] * d[:, 1])
    np.testing.assert_allclose(W, w[:, None] * P, rtol=1e-15, atol=1e-16)
    Wr = orc.build_W(d, w, orc.SCAT_LINEAR, 0.9, fold=0)
    np.testing.assert_allclose(Wr, w[:, None] * (P + 0.9 * d[:, 2:3] * d[:, 2]), rtol=1e-15, atol=1e-16)


def test_hg_normalized_and_iso_W(orc):
    """HG averages to 1 over the sphere (the normalization of P required after eq. (1.2));
    ISO gives W[l', l] = w_l'; DENSE copies P scaled by the source weights."""
    from scipy import integrate
    g = 0.8
    val, _ = integrate.quad(lambda mu: (1 - g * g) / (1 + g * g - 2 * g * mu) ** 1.5, -1, 1, limit=200)
    assert abs(0.5 * val - 1.0) < 1e-10
    d, w = orc.generate(orc.ORD_GAUSS2D, 3)
    W = orc.build_W(d, w, orc.SCAT_ISO)
    np.testing.assert_array_equal(W, np.repeat(w[:, None], len(w), 1))
    P = np.random.default_rng(0).uniform(0, 1, (len(w), len(w)))
    np.testing.assert_allclose(orc.build_W(d, w, orc.SCAT_DENSE, P=P), w[:, None] * P, rtol=1e-15)
    # HG with the fold is a symmetric kernel: W / w_l' is symmetric
    Wh = orc.build_W(d, w, orc.SCAT_HG, 0.8, fold=1)
    Ph = Wh / w[:, None]
    np.testing.assert_allclose(Ph, Ph.T, rtol=1e-14)


def test_hg_fold_column_sums_near_one(orc):
    """With the fold, sum_l' w_l' P_l'l over a fine stratified set approaches the sphere average 1."""
    d, w = orc.generate(orc.ORD_STRATIFIED, 16, 16, seed=0)
    W = orc.build_W(d, w, orc.SCAT_HG, 0.8, fold=1)
    cs = W.sum(0)
    assert 0.85 < cs.min() and cs.max() < 1.1
    Wr = orc.build_W(d, w, orc.SCAT_HG, 0.8, fold=0)
    assert Wr.sum(0).max() > 1.3  # the unfolded upper-hemisphere kernel over-counts forward peaks


def test_linear_kernel_is_rank_three(orc):
    """The folded linear kernel on any set is w_l' (1 + g(c c' + s s')): W = w (1 1^T + g c c^T +
    g s s^T), rank 3, so the contraction sum_l' W[l', l] psi_l' equals
    phi + g (c_l Jx + s_l Jy) with phi, Jx, Jy the w-, w c- and w s-moments of psi (eq. (2.1),
    eq. (3.4)).  Checked against numpy's matrix rank and a random psi."""
    d, w = orc.generate(orc.ORD_IID_SPHERE, 40, seed=5)
    g = 0.9
    W = orc.build_W(d, w, orc.SCAT_LINEAR, g, fold=1)
    assert np.linalg.matrix_rank(W, tol=1e-10) == 3
    psi = np.random.default_rng(1).uniform(0, 1, len(w))
    phi, jx, jy = w @ psi, (w * d[:, 0]) @ psi, (w * d[:, 1]) @ psi
    np.testing.assert_allclose(W.T @ psi, phi + g * (d[:, 0] * jx + d[:, 1] * jy), rtol=1e-14)


@pytest.mark.parametrize("kind,g", [("hg", 0.8), ("hg", 0.95), ("linear", 0.9)])
def test_normalized_kernel_spectral_radius(orc, kind, g):
    """Normalizing each row of P to a unit weighted sum (remark of Sec. 3.1) makes W^T a
    contraction in the w-weighted l1 norm, so rho(W) <= 1 for every nonnegative kernel; the raw
    HG kernel on a small random set exceeds 1 (the source of divergent samples).  A column
    rescaling instead of a row rescaling fails the weighted-sum identity checked here."""
    k = orc.SCAT_HG if kind == "hg" else orc.SCAT_LINEAR
    worst_raw = 0.0
    for seed in range(6):
        d, w = orc.generate(orc.ORD_IID_SPHERE, 16, seed=seed)
        Wn = orc.build_W(d, w, k | orc.SCAT_NORMALIZE, g, fold=1)
        assert np.all(Wn >= 0.0)
        rho = max(abs(np.linalg.eigvals(Wn)))
        assert rho <= 1.0 + 1e-12
        # sum over outgoing l of w_l P~_l'l = 1, i.e. sum_l w_l W~[l', l] = w_l'
        np.testing.assert_allclose(Wn @ w, w, rtol=1e-13)
        worst_raw = max(worst_raw, max(abs(np.linalg.eigvals(orc.build_W(d, w, k, g, fold=1)))))
    if kind == "hg":
        assert worst_raw > 1.5


def test_normalization_is_identity_where_rows_already_sum_to_one(orc):
    """ISO rows sum to sum w = 1, and the folded linear kernel's rows sum to
    1 + g (c' sum w c + s' sum w s) = 1 on mirror-symmetric sets (eq. (3.5)): normalizing changes
    nothing there.  On an i.i.d. set the linear rows differ from 1 and the change is visible."""
    for kind, p1, p2 in ((orc.ORD_STRATIFIED, 2, 3), (orc.ORD_UNIFORM2D, 4, 0), (orc.ORD_GAUSS2D, 5, 0)):
        d, w = orc.generate(kind, p1, p2, seed=2)
        for sk, g in ((orc.SCAT_ISO, 0.0), (orc.SCAT_LINEAR, 0.9)):
            np.testing.assert_allclose(orc.build_W(d, w, sk | orc.SCAT_NORMALIZE, g), orc.build_W(d, w, sk, g),
                                       rtol=1e-13, atol=1e-16)
    d, w = orc.generate(orc.ORD_IID_SPHERE, 12, seed=2)
    diff = orc.build_W(d, w, orc.SCAT_LINEAR | orc.SCAT_NORMALIZE, 0.9) - orc.build_W(d, w, orc.SCAT_LINEAR, 0.9)
    assert np.max(np.abs(diff)) > 1e-3


def test_normalized_kernel_conserves_particles(orc):
    """C-4 summed over ordinates with weights w: with normalized rows the scattering gain
    integrates to exactly sigma_s phi^{k-1} per cell (sum_l w_l W~[l', l] = w_l'), so
    sum_l w_l [|c| dy sum(psi_out - psi_in)_x + |s| dx sum(psi_out - psi_in)_y]
    + sum sigma_t phi^k dA = sum (sigma_s phi^{k-1} + q) dA at every iterate.  The raw HG kernel
    on the same i.i.d. set breaks it, which shows the identity has teeth."""
    rng = np.random.default_rng(11)
    nx, ny = 7, 5
    box = (0.0, 1.0, 0.0, 1.3)
    dx, dy = 1.0 / nx, 1.3 / ny
    st, ss, q = _rand_fields(rng, nx, ny, 0.5)
    inflow = {"left": rng.uniform(0, 1, ny), "bottom": rng.uniform(0, 1, nx), "right": rng.uniform(0, 1, ny),
              "top": rng.uniform(0, 1, nx)}
    prob = _prob(orc, nx, ny, st, ss, q, box=box, inflow=inflow)
    dirs, w = orc.generate(orc.ORD_IID_SPHERE, 10, seed=9)

    def imbalance(W, k):
        prev = orc.source_iterate(prob, dirs, w, W, tol=0.0, max_iter=k - 1)["phi"] if k > 1 else np.zeros(nx * ny)
        cur = orc.source_iterate(prob, dirs, w, W, tol=0.0, max_iter=k, want_psi=True)
        lhs = np.sum(st * cur["phi"]) * dx * dy
        for l in range(len(w)):
            c, s = dirs[l, 0], dirs[l, 1]
            P = cur["psi"][l].reshape(ny, nx)
            xin, xout = (inflow["left"], P[:, -1]) if c >= 0 else (inflow["right"], P[:, 0])
            yin, yout = (inflow["bottom"], P[-1, :]) if s >= 0 else (inflow["top"], P[0, :])
            lhs += w[l] * (abs(c) * dy * np.sum(xout - xin) + abs(s) * dx * np.sum(yout - yin))
        rhs = np.sum(ss * prev + q) * dx * dy
        return abs(lhs - rhs) / abs(rhs)

    Wn = orc.build_W(dirs, w, orc.SCAT_HG | orc.SCAT_NORMALIZE, 0.8, fold=1)
    for k in (1, 2, 4):
        assert imbalance(Wn, k) <= 1e-12
    assert imbalance(orc.build_W(dirs, w, orc.SCAT_HG, 0.8, fold=1), 3) > 1e-3


def test_infinite_medium_normalized_kernel(orc):
    """C-2 with a normalized HG kernel on an i.i.d. set: the constant fixed point
    v = (sigma_t I - sigma_s W~^T)^{-1} q 1 is reproduced, and the iteration converges although
    the raw kernel's sigma_s rho(W) exceeds sigma_t on this set."""
    nx, ny = 5, 4
    st, ss, qv = 1.0, 0.8, 1.0
    dirs, w = orc.generate(orc.ORD_IID_SPHERE, 16, seed=0)
    n = len(w)
    W = orc.build_W(dirs, w, orc.SCAT_HG | orc.SCAT_NORMALIZE, 0.8, fold=1)
    assert ss * max(abs(np.linalg.eigvals(orc.build_W(dirs, w, orc.SCAT_HG, 0.8, fold=1)))) > st
    v = np.linalg.solve(st * np.eye(n) - ss * W.T, np.full(n, qv))
    ang = {k: np.repeat(v[:, None], ny if k in ("left", "right") else nx, 1) for k in ("left", "right", "bottom", "top")}
    prob = _prob(orc, nx, ny, np.full(nx * ny, st), np.full(nx * ny, ss), np.full(nx * ny, qv), inflow_angular=ang)
    res = orc.source_iterate(prob, dirs, w, W, tol=1e-15, max_iter=3000, want_psi=True)
    assert res["status"] == 0
    np.testing.assert_allclose(res["psi"], np.repeat(v[:, None], nx * ny, 1), rtol=1e-11)


# ------------------------------------------------------------------------------------ sweeps
def _lattice_path(nx, ny, alpha, beta, L, B):
    """Closed form of psi_ij = alpha psi_{i-1,j} + beta psi_{i,j-1} with psi_{-1,j} = L_j,
    psi_{i,-1} = B_i: a sum over monotone lattice paths from the inflow faces."""
    out = np.zeros((ny, nx))
    for j in range(ny):
        for i in range(nx):
            v = 0.0
            for jp in range(j + 1):
                v += math.comb(i + j - jp, i) * alpha ** (i + 1) * beta ** (j - jp) * L[jp]
            for ip in range(i + 1):
                v += math.comb(j + i - ip, j) * beta ** (j + 1) * alpha ** (i - ip) * B[ip]
            out[j, i] = v
    return out


@pytest.mark.parametrize("quad", [(1, 1), (-1, 1), (-1, -1), (1, -1)])
def test_pure_absorber_lattice_paths(orc, quad):
    """C-1: sigma_s = 0, q = 0, one ordinate, inflow on its two upstream faces.  The upwind sweep is
    the discrete propagator whose solution is a lattice-path sum; every quadrant, non-square cells."""
    nx, ny = 7, 5
    box = (0.0, 1.4, 0.0, 0.5)
    dx, dy = 1.4 / nx, 0.5 / ny
    st = 1.3
    rng = np.random.default_rng(1)
    Lv, Bv = rng.uniform(0.5, 2.0, ny), rng.uniform(0.5, 2.0, nx)
    c0, s0 = 0.6, 0.48
    c, s = quad[0] * c0, quad[1] * s0
    dirs = np.array([[c, s, math.sqrt(1 - c0 * c0 - s0 * s0)]])
    faces = {}
    faces["left" if c > 0 else "right"] = Lv
    faces["bottom" if s > 0 else "top"] = Bv
    # the decoy faces carry values that must be ignored
    faces.setdefault("left", np.full(ny, 99.0))
    faces.setdefault("right", np.full(ny, 99.0))
    faces.setdefault("bottom", np.full(nx, 99.0))
    faces.setdefault("top", np.full(nx, 99.0))
    prob = _prob(orc, nx, ny, np.full(nx * ny, st), np.zeros(nx * ny), np.zeros(nx * ny), box=box, inflow=faces)
    psi = orc.sweep(prob, dirs, np.zeros(nx * ny))[0].reshape(ny, nx)
    a, b = c0 / dx, s0 / dy
    # the closed form runs in sweep coordinates: face arrays are re-indexed along the sweep
    Ls = Lv if s > 0 else Lv[::-1]
    Bs = Bv if c > 0 else Bv[::-1]
    ref = _lattice_path(nx, ny, a / (st + a + b), b / (st + a + b), Ls, Bs)
    # map back from sweep coordinates to storage coordinates
    if c < 0:
        ref = ref[:, ::-1]
    if s < 0:
        ref = ref[::-1, :]
    np.testing.assert_allclose(psi, ref, rtol=1e-13)


def test_pure_absorber_ray_limit_first_order(orc):
    """C-1 ray limit: along s = 0 the sweep tends to exp(-sigma_t x / c) at first order in dx."""
    st, c = 2.0, 0.8
    errs = []
    for nx in (32, 64, 128, 256):
        prob = _prob(orc, nx, 1, np.full(nx, st), np.zeros(nx), np.zeros(nx), inflow={"left": np.ones(1)})
        psi = orc.sweep(prob, np.array([[c, 0.0, math.sqrt(1 - c * c)]]), np.zeros(nx))[0]
        errs.append(abs(psi[-1] - math.exp(-st * 1.0 / c)))
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(3)]
    assert all(0.9 < r < 1.1 for r in rates), rates


def _brute_force(orc, prob, dirs, W):
    """Assemble the whole upwind DOM system (eq. (3.1) with the first-order upwind cell balance)
    as one dense matrix over (ordinate, cell) and solve it directly."""
    nx, ny = prob.nx, prob.ny
    x0, x1, y0, y1 = prob.box
    dx, dy = (x1 - x0) / nx, (y1 - y0) / ny
    n = dirs.shape[0]
    cells = nx * ny
    A = np.zeros((n * cells, n * cells))
    rhs = np.zeros(n * cells)
    fin = prob.inflow
    fang = prob.inflow_angular

    def face(name, l, k):
        if name in fang:
            return fang[name].reshape(n, -1)[l, k]
        return fin[name][k] if name in fin else 0.0

    for l in range(n):
        c, s = dirs[l, 0], dirs[l, 1]
        a, b = abs(c) / dx, abs(s) / dy
        for j in range(ny):
            for i in range(nx):
                r = l * cells + j * nx + i
                cell = j * nx + i
                A[r, r] += prob.sigma_t[cell] + a + b
                iu = i - 1 if c >= 0 else i + 1
                ju = j - 1 if s >= 0 else j + 1
                if 0 <= iu < nx:
                    A[r, l * cells + j * nx + iu] -= a
                else:
                    rhs[r] += a * face("left" if c >= 0 else "right", l, j)
                if 0 <= ju < ny:
                    A[r, l * cells + ju * nx + i] -= b
                else:
                    rhs[r] += b * face("bottom" if s >= 0 else "top", l, i)
                rhs[r] += prob.q[cell]
                for lp in range(n):
                    A[r, lp * cells + cell] -= prob.sigma_s[cell] * W[lp, l]
    psi = np.linalg.solve(A, rhs).reshape(n, cells)
    return psi


@pytest.mark.parametrize("scat", ["iso", "hg", "dense"])
def test_brute_force_direct_solve(orc, scat):
    """C-3: source iteration to 1e-15 equals the direct solve of the assembled system, with varying
    cross sections, non-square cells, isotropic and angular inflow, and a non-symmetric W."""
    rng = np.random.default_rng(5)
    nx, ny = 5, 4
    st, ss, q = _rand_fields(rng, nx, ny, 0.8)
    dirs, w = orc.generate(orc.ORD_STRATIFIED, 1, 2, seed=9, sample=1)
    n = len(w)
    w = rng.uniform(0.5, 1.5, n)
    w /= w.sum()  # unequal weights make W non-symmetric
    if scat == "iso":
        W = orc.build_W(dirs, w, orc.SCAT_ISO)
    elif scat == "hg":
        W = orc.build_W(dirs, w, orc.SCAT_HG, 0.6, fold=1)
    else:
        W = orc.build_W(dirs, w, orc.SCAT_DENSE, P=rng.uniform(0.2, 1.4, (n, n)))
    inflow = {"left": rng.uniform(0, 1, ny), "top": rng.uniform(0, 1, nx)}
    ang = {"bottom": rng.uniform(0, 1, (n, nx)), "right": rng.uniform(0, 1, (n, ny))}
    prob = _prob(orc, nx, ny, st, ss, q, box=(0.0, 1.0, 0.0, 0.6), inflow=inflow, inflow_angular=ang)
    ref_psi = _brute_force(orc, prob, dirs, W)
    res = orc.source_iterate(prob, dirs, w, W, tol=1e-15, max_iter=2000, want_psi=True)
    np.testing.assert_allclose(res["psi"], ref_psi, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(res["phi"], (w[:, None] * ref_psi).sum(0), rtol=1e-11)
    if scat == "iso":
        iso = orc.source_iterate(prob, dirs, w, None, tol=1e-15, max_iter=2000)
        np.testing.assert_allclose(iso["phi"], res["phi"], rtol=1e-12)


def test_infinite_medium_isotropic(orc):
    """C-2: uniform medium with isotropic inflow q/(sigma_t - sigma_s) on every face: the discrete
    solution is exactly that constant for every ordinate."""
    nx, ny = 12, 9
    st, ss, qv = 1.5, 1.2, 0.7
    psi_inf = qv / (st - ss)
    faces = {k: np.full(nx if k in ("bottom", "top") else ny, psi_inf) for k in ("left", "right", "bottom", "top")}
    prob = _prob(orc, nx, ny, np.full(nx * ny, st), np.full(nx * ny, ss), np.full(nx * ny, qv), inflow=faces)
    dirs, w = orc.generate(orc.ORD_STRATIFIED, 2, 4, seed=0)
    res = orc.source_iterate(prob, dirs, w, None, tol=1e-15, max_iter=1000, want_psi=True)
    np.testing.assert_allclose(res["psi"], psi_inf, rtol=1e-13)
    # the iterate contracts at no more than sigma_s/sigma_t per step (max-norm bound)
    assert res["iters"] <= math.ceil(math.log(1e-15 * (1 - ss / st)) / math.log(ss / st)) + 3


def test_infinite_medium_anisotropic_gauss(orc):
    """C-2, anisotropic: with unequal Gaussian weights and HG scattering the constant solution is
    v = (sigma_t I - sigma_s W^T)^{-1} q 1, so the orientation of W is pinned."""
    nx, ny = 6, 6
    st, ss, qv = 2.0, 1.6, 1.0
    dirs, w = orc.generate(orc.ORD_GAUSS2D, 3)
    n = len(w)
    W = orc.build_W(dirs, w, orc.SCAT_HG, 0.7, fold=1)
    v = np.linalg.solve(st * np.eye(n) - ss * W.T, np.full(n, qv))
    ang = {"left": np.repeat(v[:, None], ny, 1), "right": np.repeat(v[:, None], ny, 1),
           "bottom": np.repeat(v[:, None], nx, 1), "top": np.repeat(v[:, None], nx, 1)}
    prob = _prob(orc, nx, ny, np.full(nx * ny, st), np.full(nx * ny, ss), np.full(nx * ny, qv), inflow_angular=ang)
    res = orc.source_iterate(prob, dirs, w, W, tol=1e-15, max_iter=2000, want_psi=True)
    np.testing.assert_allclose(res["psi"], np.repeat(v[:, None], nx * ny, 1), rtol=1e-12)
    # the transposed contraction is a different fixed point
    v_wrong = np.linalg.solve(st * np.eye(n) - ss * W, np.full(n, qv))
    assert np.max(np.abs(v_wrong - v)) > 1e-3


@pytest.mark.parametrize("aniso", [False, True])
def test_particle_balance_every_iteration(orc, aniso):
    """C-4: the upwind balance telescopes exactly at every iterate k (lagged source), per ordinate:
    |c| dy sum_j (psi_out - psi_in)_x + |s| dx sum_i (psi_out - psi_in)_y + sum sigma_t psi dA
    = sum S dA, with S from psi^{k-1}.  Non-square cells catch an a/b swap."""
    rng = np.random.default_rng(2)
    nx, ny = 9, 6
    box = (0.0, 1.0, 0.0, 1.7)
    dx, dy = 1.0 / nx, 1.7 / ny
    st, ss, q = _rand_fields(rng, nx, ny)
    inflow = {"left": rng.uniform(0, 1, ny), "bottom": rng.uniform(0, 1, nx), "right": rng.uniform(0, 1, ny),
              "top": rng.uniform(0, 1, nx)}
    prob = _prob(orc, nx, ny, st, ss, q, box=box, inflow=inflow)
    dirs, w = orc.generate(orc.ORD_STRATIFIED, 2, 2, seed=4)
    n = len(w)
    W = orc.build_W(dirs, w, orc.SCAT_HG, 0.5, fold=1) if aniso else None
    for k in (1, 2, 5):
        prev = np.zeros((n, nx * ny)) if k == 1 else \
            orc.source_iterate(prob, dirs, w, W, tol=0.0, max_iter=k - 1, want_psi=True)["psi"]
        cur = orc.source_iterate(prob, dirs, w, W, tol=0.0, max_iter=k, want_psi=True)["psi"]
        Wm = W if aniso else np.repeat(w[:, None], n, 1)
        S = ss[None, :] * (Wm.T @ prev) + q[None, :]
        for l in range(n):
            c, s = dirs[l, 0], dirs[l, 1]
            P = cur[l].reshape(ny, nx)
            if c >= 0:
                xin, xout = inflow["left"], P[:, -1]
            else:
                xin, xout = inflow["right"], P[:, 0]
            if s >= 0:
                yin, yout = inflow["bottom"], P[-1, :]
            else:
                yin, yout = inflow["top"], P[0, :]
            lhs = abs(c) * dy * np.sum(xout - xin) + abs(s) * dx * np.sum(yout - yin) + np.sum(st * cur[l]) * dx * dy
            rhs = np.sum(S[l]) * dx * dy
            assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(rhs))


def test_quadrant_symmetry(orc):
    """C-5: a problem symmetric under x -> 1-x and y -> 1-y with a mirror-symmetric ordinate set has
    a mirror-symmetric density (up to summation order)."""
    f = RI.checkerboard_fields(42, 42)
    prob = _prob(orc, 42, 42, f.sigma_t, f.sigma_s, f.q)
    dirs, w = orc.generate(orc.ORD_STRATIFIED, 2, 3, seed=8)
    phi = orc.source_iterate(prob, dirs, w, None, tol=1e-13)["phi"].reshape(42, 42)
    np.testing.assert_allclose(phi, phi[:, ::-1], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(phi, phi[::-1, :], rtol=1e-12, atol=1e-15)
    d2, w2 = orc.generate(orc.ORD_UNIFORM2D, 3)  # also symmetric under x <-> y
    phi2 = orc.source_iterate(prob, d2, w2, None, tol=1e-13)["phi"].reshape(42, 42)
    np.testing.assert_allclose(phi2, phi2.T, rtol=1e-12, atol=1e-15)


def test_neumann_first_iterate(orc):
    """C-6: the first iterate from phi^0 = 0 is L^{-1} q, the first term of eq. (3.10)."""
    rng = np.random.default_rng(3)
    nx, ny = 10, 7
    st, ss, q = _rand_fields(rng, nx, ny)
    prob = _prob(orc, nx, ny, st, ss, q, inflow={"top": rng.uniform(0, 1, nx)})
    dirs, w = orc.generate(orc.ORD_STRATIFIED, 2, 2, seed=1)
    one = orc.source_iterate(prob, dirs, w, None, tol=0.0, max_iter=1, want_psi=True)
    psi = orc.sweep(prob, dirs, q)
    np.testing.assert_array_equal(one["psi"], psi)
    two = orc.source_iterate(prob, dirs, w, None, tol=0.0, max_iter=2, want_psi=True)
    psi2 = orc.sweep(prob, dirs, ss * (w[:, None] * psi).sum(0) + q)
    np.testing.assert_allclose(two["psi"], psi2, rtol=1e-15)


def test_positivity(orc):
    """C-7: non-negative data keep psi and phi non-negative (remark after eq. (3.4))."""
    rng = np.random.default_rng(4)
    nx, ny = 16, 11
    st, ss, q = _rand_fields(rng, nx, ny, 0.95)
    q[rng.uniform(size=q.size) < 0.7] = 0.0
    prob = _prob(orc, nx, ny, st, ss, q)
    dirs, w = orc.generate(orc.ORD_IID_SPHERE, 13, seed=0)
    W = orc.build_W(dirs, w, orc.SCAT_HG, 0.8, fold=1)
    res = orc.source_iterate(prob, dirs, w, W, tol=1e-10, want_psi=True)
    assert np.all(res["psi"] >= 0) and np.all(res["phi"] >= 0) and res["phi"].max() > 0


def test_vacuum_zero_source_converges_immediately(orc):
    prob = _prob(orc, 4, 4, np.ones(16), np.full(16, 0.5), np.zeros(16))
    dirs, w = orc.generate(orc.ORD_STRATIFIED, 1, 1)
    res = orc.source_iterate(prob, dirs, w, None, tol=1e-8)
    assert res["iters"] == 1 and res["status"] == 0 and np.all(res["phi"] == 0)


def test_not_converged_status(orc):
    f = RI.uniform_fields(8, 8, 1.0, 0.9, 0.4, 0.6)
    prob = _prob(orc, 8, 8, f.sigma_t, f.sigma_s, f.q)
    dirs, w = orc.generate(orc.ORD_STRATIFIED, 1, 2)
    res = orc.source_iterate(prob, dirs, w, None, tol=1e-14, max_iter=3, want_hist=True)
    assert res["status"] == 1 and res["iters"] == 3 and len(res["hist"]) == 3 and res["r"] > 1e-14


# ------------------------------------------------------------------------------------ ensemble
def test_ensemble_mean_var_match_numpy(orc):
    """Sec. 4.1 average over samples: the oracle's mean and variance equal numpy's of the per-sample
    solutions, each of which equals an independent single solve with that sample's ordinates."""
    f = RI.uniform_fields(12, 10, 1.0, 0.5, 0.3, 0.7)
    prob = _prob(orc, 12, 10, f.sigma_t, f.sigma_s, f.q)
    res = orc.ensemble(prob, orc.ORD_STRATIFIED, 1, 2, 17, 6, tol=1e-10, want_phis=True)
    np.testing.assert_allclose(res["mean"], res["phis"].mean(0), rtol=1e-14)
    np.testing.assert_allclose(res["var"], res["phis"].var(0, ddof=1), rtol=1e-10, atol=1e-20)
    d, w = orc.generate(orc.ORD_STRATIFIED, 1, 2, seed=17, sample=4)
    single = orc.source_iterate(prob, d, w, None, tol=1e-10)
    np.testing.assert_array_equal(single["phi"], res["phis"][4])
    assert len(set(np.round(res["phis"][:, 5], 12))) == 6  # samples differ


# ------------------------------------------------------------------------------------ paper numbers
def _table1():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1.txt")) if l.strip() and l[0] != "#"]
    return [(r[0], float(r[1]), int(r[2]), float(r[3])) for r in rows]


def _l2(a, b):
    return math.sqrt(np.mean((a - b) ** 2))  # eq. (2.2)


def _round4(v):
    return float("%.3E" % v)


def test_paper_table1_uniform_isotropic(orc):
    """Table 1, uniform quadrature, g = 0: all four printed errors reproduced to every printed digit
    (diamond difference, Example 2.1, reference N = 20)."""
    f = RI.example21()
    prob = _prob(orc, f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    ref_d, ref_w = orc.generate(orc.ORD_UNIFORM2D, 20)
    ref = orc.source_iterate(prob, ref_d, ref_w, None, scheme=orc.SCHEME_DD, tol=1e-12)["phi"]
    for quad, g, N, err in _table1():
        if quad != "uniform" or g != 0.0:
            continue
        d, w = orc.generate(orc.ORD_UNIFORM2D, N)
        phi = orc.source_iterate(prob, d, w, None, scheme=orc.SCHEME_DD, tol=1e-12)["phi"]
        assert _round4(_l2(phi, ref)) == err, (N, _l2(phi, ref), err)


def test_paper_table1_uniform_linear_kernel_fold(orc):
    """Table 1, uniform quadrature, g = 0.9: the +-zeta fold of the linear kernel reproduces the
    printed errors at N = 5, 4, 3 to every digit (the unfolded kernel, with its own N = 20
    reference, gives 4.674E-03 / 6.023E-03 / 9.280E-03 instead).  The printed
    N = 2 entry (2.075E-02) contradicts the row's own stated order 0.73, which the folded value
    1.632E-02 does satisfy, so it is read as a misprint and only the order is checked there."""
    ref_path = os.path.join(GOLDEN, "table1_uniform_g09_N20.npy")
    ref = np.load(ref_path)
    f = RI.example21()
    prob = _prob(orc, f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    errs = {}
    for quad, g, N, err in _table1():
        if quad != "uniform" or g != 0.9:
            continue
        d, w = orc.generate(orc.ORD_UNIFORM2D, N)
        W = orc.build_W(d, w, orc.SCAT_LINEAR, 0.9, fold=1)
        phi = orc.source_iterate(prob, d, w, W, scheme=orc.SCHEME_DD, tol=1e-12)["phi"]
        errs[N] = _l2(phi, ref)
        if N >= 3:
            assert _round4(errs[N]) == err, (N, errs[N], err)
    order = math.log(errs[2] / errs[5]) / math.log((4 * 25) / (4 * 4))
    assert round(order, 2) == 0.72 or round(order, 2) == 0.73


def test_paper_table1_gauss_close(orc):
    """Table 1, 2D Gaussian quadrature, g = 0: with the Appendix A construction as read here the
    errors agree with the printed ones to within 4 % but not to every digit (the text leaves some
    detail of the authors' construction open), and the convergence order is the printed 0.82 to
    within 0.06."""
    f = RI.example21()
    prob = _prob(orc, f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    ref_d, ref_w = orc.generate(orc.ORD_GAUSS2D, 20)
    ref = orc.source_iterate(prob, ref_d, ref_w, None, scheme=orc.SCHEME_DD, tol=1e-12)["phi"]
    errs = {}
    for quad, g, N, err in _table1():
        if quad != "gauss" or g != 0.0:
            continue
        d, w = orc.generate(orc.ORD_GAUSS2D, N)
        errs[N] = _l2(orc.source_iterate(prob, d, w, None, scheme=orc.SCHEME_DD, tol=1e-12)["phi"], ref)
        assert abs(errs[N] - err) < 0.04 * err, (N, errs[N], err)
    order = math.log(errs[2] / errs[5]) / math.log(60 / 12)
    assert abs(order - 0.82) < 0.06
