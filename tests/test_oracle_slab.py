"""Pins of the slab-geometry oracle (Sec. 4.1, Example 4.1) against facts that do not come from it:
the published SplitMix64 stream, closed forms of the discrete pure absorber, the exact constant
solution of an infinite medium, a dense direct solve of the whole discrete system, mirror
symmetry and the second-order spatial convergence of the scheme.  CPU only."""
import math

import numpy as np
import pytest

import rom_inputs as RI


def example41(nx, case):
    f = RI.slab_example41(nx, case)
    return f.sigma_t, f.sigma_s, f.q, f.inflow


_M64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def _finalize(z):
    """SplitMix64's output function, from its published definition (Steele, Lea, Flood 2014)."""
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def test_rom_sampler_cells_mirror_and_stream(orc):
    """Sec. 4.1: n equal cells of [-1, 1]; one uniform draw per cell of [-1, 0] (the stream of the
    sample, cells in order), mirrored: mu_l = -mu_{n+1-l}; weights 2/n, here normalized to 1/n.
    The stream is recomputed here in plain Python: sample s starts from output s + 1 of the master
    generator, and u = (x >> 11) 2^-53."""
    for n in (2, 4, 8, 16):
        for sample in (0, 3):
            mu, w = orc.slab_rom_ordinates(n, seed=11, sample=sample)
            width = 2.0 / n
            st = _finalize((11 + (sample + 1) * _GAMMA) & _M64)
            for l in range(n // 2):
                st = (st + _GAMMA) & _M64
                u = (_finalize(st) >> 11) * 2.0 ** -53
                assert mu[l] == -1.0 + l * width + u * width
                assert -1.0 + l * width <= mu[l] < -1.0 + (l + 1) * width
            np.testing.assert_array_equal(mu[n // 2:], -mu[: n // 2][::-1])
            np.testing.assert_array_equal(w, np.full(n, 1.0 / n))


def test_quadratures(orc):
    mu, w = orc.slab_quadrature(orc.SLAB_GAUSS, 12)
    x, gw = np.polynomial.legendre.leggauss(12)
    np.testing.assert_allclose(np.sort(mu), x, atol=1e-14)
    np.testing.assert_allclose(w[np.argsort(mu)], gw / 2, rtol=1e-13)
    mu, w = orc.slab_quadrature(orc.SLAB_UNIFORM, 6)
    np.testing.assert_allclose(mu, [-5 / 6, -1 / 2, -1 / 6, 1 / 6, 1 / 2, 5 / 6], atol=1e-15)
    assert abs(w.sum() - 1) < 1e-15


@pytest.mark.parametrize("mu0", [0.7, -0.35, 0.05])
def test_pure_absorber_closed_form(orc, mu0):
    """No scattering, no source, constant sigma: diamond difference gives the geometric sequence
    psi_k = psi_in rho^k, rho = (|mu|/dx - sigma/2) / (|mu|/dx + sigma/2), from the entry face
    (which oscillates in sign when |mu|/dx < sigma/2)."""
    nx, sig = 25, 3.0
    dx = 1.0 / nx
    psi = orc.slab_sweep(nx, 0.0, 1.0, np.full(nx + 1, sig), [mu0], [2.0], np.zeros(nx + 1))[0]
    a = abs(mu0) / dx
    rho = (a - sig / 2) / (a + sig / 2)
    k = np.arange(nx + 1) if mu0 > 0 else np.arange(nx + 1)[::-1]
    np.testing.assert_allclose(psi, 2.0 * rho ** k, rtol=1e-13, atol=1e-300)


def test_pure_absorber_second_order(orc):
    """The exit value converges to exp(-sigma / mu) at second order (Richardson ratio 4)."""
    sig, mu0 = 2.0, 0.4
    errs = []
    for nx in (20, 40, 80, 160):
        psi = orc.slab_sweep(nx, 0.0, 1.0, np.full(nx + 1, sig), [mu0], [1.0], np.zeros(nx + 1))[0]
        errs.append(abs(psi[-1] - math.exp(-sig / mu0)))
    ratios = [errs[k] / errs[k + 1] for k in range(3)]
    assert all(3.8 < r < 4.2 for r in ratios), ratios


def test_infinite_medium(orc):
    """Constant fields with inflow q/(sigma_t - sigma_s) from both sides: the discrete solution is
    that constant at every grid point, for any ordinate set."""
    nx = 17
    st, ss, qv = 2.0, 1.5, 0.7
    v = qv / (st - ss)
    mu, w = orc.slab_rom_ordinates(8, seed=5, sample=1)
    r = orc.slab_source_iterate(nx, 0.0, 1.0, np.full(nx + 1, st), np.full(nx + 1, ss), np.full(nx + 1, qv),
                                mu, w, np.full(8, v), tol=1e-15, max_iter=2000)
    np.testing.assert_allclose(r["phi"], v, rtol=1e-13)


@pytest.mark.parametrize("case", [1, 2, 3])
def test_direct_solve_of_the_discrete_system(orc, case):
    """The whole discrete slab system (inflow rows, one diamond-difference row per ordinate and
    cell, phi = sum w psi inside the scattering term) assembled densely and solved by numpy
    equals the converged source iteration."""
    nx = 7
    st, ss, q, inflow = example41(nx, case)
    mu, w = orc.slab_rom_ordinates(6, seed=2, sample=4)
    n, nn = len(mu), nx + 1
    dx = 1.0 / nx
    A = np.zeros((n * nn, n * nn))
    b = np.zeros(n * nn)
    idx = lambda l, i: l * nn + i  # noqa: E731
    row = 0
    for l in range(n):
        entry = 0 if mu[l] > 0 else nx
        A[row, idx(l, entry)] = 1.0
        b[row] = inflow(mu[l])
        row += 1
        for i in range(nx):
            sc = 0.5 * (st[i] + st[i + 1])
            i_in, i_out = (i, i + 1) if mu[l] > 0 else (i + 1, i)
            A[row, idx(l, i_out)] += abs(mu[l]) / dx + 0.5 * sc
            A[row, idx(l, i_in)] += -abs(mu[l]) / dx + 0.5 * sc
            for node in (i, i + 1):   # -(1/2) sigma_s phi at both ends of the cell
                for lp in range(n):
                    A[row, idx(lp, node)] -= 0.5 * ss[node] * w[lp]
            b[row] = 0.5 * (q[i] + q[i + 1])
            row += 1
    psi = np.linalg.solve(A, b).reshape(n, nn)
    phi_direct = w @ psi
    r = orc.slab_source_iterate(nx, 0.0, 1.0, st, ss, q, mu, w, inflow(mu), tol=1e-15, max_iter=5000)
    np.testing.assert_allclose(r["phi"], phi_direct, rtol=1e-12)


def test_mirror_symmetry(orc):
    """Fields symmetric about x = 1/2, the same inflow function of |mu| on both faces and a
    mirror-symmetric set give phi(x) = phi(1 - x)."""
    nx = 40
    x = np.linspace(0.0, 1.0, nx + 1)
    st = 1 + 6 * (x - 0.5) ** 2
    ss = 0.6 * st
    q = 1 + np.cos(2 * np.pi * x)
    mu, w = orc.slab_rom_ordinates(10, seed=3, sample=0)
    inf = 1 + np.abs(mu)
    phi = orc.slab_source_iterate(nx, 0.0, 1.0, st, ss, q, mu, w, inf, tol=1e-15, max_iter=5000)["phi"]
    np.testing.assert_allclose(phi, phi[::-1], rtol=1e-13)


def test_example41_second_order_in_space(orc):
    """Example 4.1, case 1, fixed Gauss quadrature: phi at x = 0.5 converges at second order in dx
    (Richardson ratio near 4)."""
    mu, w = orc.slab_quadrature(orc.SLAB_GAUSS, 16)
    vals = []
    for nx in (50, 100, 200, 400):
        st, ss, q, inflow = example41(nx, 1)
        phi = orc.slab_source_iterate(nx, 0.0, 1.0, st, ss, q, mu, w, inflow(mu), tol=1e-14, max_iter=5000)["phi"]
        vals.append(phi[nx // 2])
    d = [abs(vals[k] - vals[k + 1]) for k in range(3)]
    assert 3.6 < d[0] / d[1] < 4.4 and 3.6 < d[1] / d[2] < 4.4, d
