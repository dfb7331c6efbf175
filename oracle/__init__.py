"""FP64 CPU oracle for ROM/DOM source iteration (test infrastructure, not product code).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package.  It wraps ``rom_oracle.c`` (plain C, double precision) through ctypes and
shares nothing with the GPU library: no code, no header, no tables.

Paper: Li, Tang, Yang, "Random ordinate method for mitigating the ray effect in radiative
transport equation simulations", arXiv:2407.12527.  Each wrapped function names the passage it
follows in ``rom_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rom_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SCHEME_STEP, SCHEME_DD = 0, 1
SCAT_ISO, SCAT_LINEAR, SCAT_HG, SCAT_DENSE = 0, 1, 2, 3
SCAT_NORMALIZE = 0x10  # flag OR-ed into a kernel kind: rows of P rescaled to unit weighted sum
ORD_STRATIFIED, ORD_IID_SPHERE, ORD_UNIFORM2D, ORD_GAUSS2D = 0, 1, 2, 3
OK, NOT_CONVERGED = 0, 1


def build(force: bool = True) -> str:
    """Compile rom_oracle.c with gcc (-O2, OpenMP, no FMA contraction) into liboracle.so."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-builtin", "-fPIC", "-shared",
           "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("x0", C.c_double), ("x1", C.c_double),
                ("y0", C.c_double), ("y1", C.c_double)]


class Inflow(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in
                ("left", "right", "bottom", "top", "aleft", "aright", "abottom", "atop")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.orc_splitmix64_next.argtypes = [C.POINTER(C.c_uint64)]
        L.orc_splitmix64_next.restype = C.c_uint64
        L.orc_u01.argtypes = [C.c_uint64]
        L.orc_u01.restype = C.c_double
        L.orc_sample_seed.argtypes = [C.c_uint64, C.c_int64]
        L.orc_sample_seed.restype = C.c_uint64
        L.orc_zeta_bands.argtypes = [C.c_int]
        L.orc_ordinate_count.argtypes = [C.c_int, C.c_int, C.c_int]
        L.orc_generate.argtypes = [C.c_int, C.c_int, C.c_int, C.c_uint64, C.c_int64, P, P]
        L.orc_gauss_legendre.argtypes = [C.c_int, P, P]
        L.orc_build_W.argtypes = [C.c_int, P, P, C.c_int, C.c_double, C.c_int, P, P]
        L.orc_sweep.argtypes = [C.POINTER(Grid), P, C.c_int, P, P, C.c_int, C.POINTER(Inflow), C.c_int, P]
        L.orc_source_iterate.argtypes = [C.POINTER(Grid), P, P, P, C.POINTER(Inflow), C.c_int, P, P, P,
                                         C.c_int, C.c_double, C.c_int, P, P, C.POINTER(C.c_int),
                                         C.POINTER(C.c_double), P]
        L.orc_ensemble.argtypes = [C.POINTER(Grid), P, P, P, C.POINTER(Inflow), C.c_int, C.c_int, C.c_int,
                                   C.c_uint64, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, C.c_double,
                                   C.c_int, P, P, P, P]
        L.orc_slab_ordinates_rom.argtypes = [C.c_int, C.c_uint64, C.c_int64, P, P]
        L.orc_slab_quadrature.argtypes = [C.c_int, C.c_int, P, P]
        L.orc_slab_sweep.argtypes = [C.c_int, C.c_double, C.c_double, P, C.c_int, P, P, P, P]
        L.orc_slab_source_iterate.argtypes = [C.c_int, C.c_double, C.c_double, P, P, P, C.c_int, P, P, P,
                                              C.c_double, C.c_int, P, C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


# ------------------------------------------------------------------ random numbers, ordinates
def splitmix64_stream(seed: int, count: int) -> np.ndarray:
    st = C.c_uint64(seed)
    out = np.empty(count, dtype=np.uint64)
    for k in range(count):
        out[k] = lib().orc_splitmix64_next(C.byref(st))
    return out


def u01(x: int) -> float:
    return lib().orc_u01(C.c_uint64(x))


def sample_seed(seed: int, sample: int) -> int:
    return lib().orc_sample_seed(seed, sample)


def zeta_bands(m: int) -> int:
    return lib().orc_zeta_bands(m)


def ordinate_count(kind: int, p1: int, p2: int = 0) -> int:
    return lib().orc_ordinate_count(kind, p1, p2)


def generate(kind: int, p1: int, p2: int = 0, seed: int = 0, sample: int = 0):
    """Ordinate set (dirs [n,3] = (c, s, zeta), weights [n]).  STRATIFIED: p1 x p2 zeta x theta
    cells per quadrant (Sec. 3.1, Sec. 4.2); IID_SPHERE: p1 iid directions; UNIFORM2D / GAUSS2D:
    the Appendix A quadratures of order p1."""
    n = ordinate_count(kind, p1, p2)
    if n <= 0:
        raise ValueError("bad ordinate spec")
    dirs = np.empty((n, 3))
    w = np.empty(n)
    rc = lib().orc_generate(kind, p1, p2, seed, sample, _p(dirs), _p(w))
    if rc != 0:
        raise ValueError(f"orc_generate failed ({rc})")
    return dirs, w


def stratified_spec(n: int):
    """(nz, nt) for n = 4m random ordinates: nz = largest divisor of m not above sqrt(m)."""
    if n % 4:
        raise ValueError("stratified sets need n = 4m")
    m = n // 4
    nz = zeta_bands(m)
    return nz, m // nz


def gauss_legendre(n: int):
    x = np.empty(n)
    w = np.empty(n)
    lib().orc_gauss_legendre(n, _p(x), _p(w))
    return x, w


def build_W(dirs, w, kind=SCAT_ISO, g=0.0, fold=1, P=None) -> np.ndarray:
    """W[l', l] = w_l' P(u_l', u_l) (eq. (3.4)); with kind | SCAT_NORMALIZE each row l' of P is
    divided by r_l' = sum_l w_l P(u_l', u_l) (the remark of Sec. 3.1 on mass conservation)."""
    dirs = _f64(dirs)
    w = _f64(w)
    n = w.shape[0]
    W = np.empty((n, n))
    P = _f64(P)
    rc = lib().orc_build_W(n, _p(dirs), _p(w), kind, g, fold, _p(P), _p(W))
    if rc != 0:
        raise ValueError("orc_build_W failed")
    return W


# ------------------------------------------------------------------ problem description
class Problem:
    """Grid, cell fields and inflow of eq. (1.1)-(1.2) on a uniform nx x ny cell-centred grid.
    Cell (i, j) is stored at j*nx + i."""

    def __init__(self, nx, ny, sigma_t, sigma_s, q, box=(0.0, 1.0, 0.0, 1.0), inflow=None,
                 inflow_angular=None):
        self.nx, self.ny = int(nx), int(ny)
        cells = self.nx * self.ny
        self.sigma_t = _f64(sigma_t).reshape(cells)
        self.sigma_s = _f64(sigma_s).reshape(cells)
        self.q = _f64(q).reshape(cells)
        self.box = tuple(float(v) for v in box)
        self.inflow = {k: _f64(v) for k, v in (inflow or {}).items() if v is not None}
        self.inflow_angular = {k: _f64(v) for k, v in (inflow_angular or {}).items() if v is not None}

    @property
    def cells(self):
        return self.nx * self.ny

    def _grid(self):
        x0, x1, y0, y1 = self.box
        return Grid(self.nx, self.ny, x0, x1, y0, y1)

    def _inflow(self):
        f = Inflow()
        for k in ("left", "right", "bottom", "top"):
            setattr(f, k, _p(self.inflow.get(k)))
            setattr(f, "a" + k, _p(self.inflow_angular.get(k)))
        return f


def sweep(prob: Problem, dirs, src, scheme=SCHEME_STEP) -> np.ndarray:
    """psi [n, cells] = L^{-1} src for every ordinate; src is [cells] (shared) or [n, cells]."""
    dirs = _f64(dirs)
    n = dirs.shape[0]
    src = _f64(src)
    per = 1 if src.ndim == 2 else 0
    psi = np.empty((n, prob.cells))
    g = prob._grid()
    f = prob._inflow()
    rc = lib().orc_sweep(C.byref(g), _p(prob.sigma_t), n, _p(dirs), _p(src), per, C.byref(f), scheme, _p(psi))
    if rc != 0:
        raise ValueError("orc_sweep failed")
    return psi


def scalar_flux(w, psi) -> np.ndarray:
    return (np.asarray(w)[:, None] * psi).sum(axis=0)


def source_iterate(prob: Problem, dirs, w, W=None, scheme=SCHEME_STEP, tol=1e-8, max_iter=1000,
                   want_psi=False, want_hist=False):
    """Source iteration from phi^0 = 0 (Sec. 3.2, eq. (3.10)); returns a dict with phi, iters,
    r (final relative change), status and optionally psi and the residual history."""
    dirs = _f64(dirs)
    w = _f64(w)
    W = _f64(W)
    n = w.shape[0]
    phi = np.empty(prob.cells)
    psi = np.empty((n, prob.cells)) if want_psi else None
    hist = np.zeros(max_iter) if want_hist else None
    it = C.c_int(0)
    r = C.c_double(0.0)
    g = prob._grid()
    f = prob._inflow()
    rc = lib().orc_source_iterate(C.byref(g), _p(prob.sigma_t), _p(prob.sigma_s), _p(prob.q), C.byref(f), n,
                                  _p(dirs), _p(w), _p(W), scheme, tol, max_iter, _p(phi), _p(psi),
                                  C.byref(it), C.byref(r), _p(hist))
    if rc < 0:
        raise ValueError(f"orc_source_iterate failed ({rc})")
    out = {"phi": phi, "iters": it.value, "r": r.value, "status": rc}
    if want_psi:
        out["psi"] = psi
    if want_hist:
        out["hist"] = hist[: it.value]
    return out


def ensemble(prob: Problem, ord_kind, p1, p2, seed, t, scat_kind=SCAT_ISO, g=0.0, fold=1,
             scheme=SCHEME_STEP, tol=1e-6, max_iter=1000, want_phis=False):
    """t independent samples, mean and unbiased variance (Sec. 4.1, eq. (4.6))."""
    mean = np.empty(prob.cells)
    var = np.empty(prob.cells)
    phis = np.empty((t, prob.cells)) if want_phis else None
    iters = np.zeros(t, dtype=np.int32)
    gr = prob._grid()
    f = prob._inflow()
    rc = lib().orc_ensemble(C.byref(gr), _p(prob.sigma_t), _p(prob.sigma_s), _p(prob.q), C.byref(f), ord_kind,
                            p1, p2, seed, t, scat_kind, g, fold, scheme, tol, max_iter, _p(mean), _p(var),
                            _p(phis), _p(iters))
    if rc < 0:
        raise ValueError(f"orc_ensemble failed ({rc})")
    out = {"mean": mean, "var": var, "iters": iters, "status": rc}
    if want_phis:
        out["phis"] = phis
    return out


# ------------------------------------------------------------------ slab geometry (Sec. 4.1)
SLAB_GAUSS, SLAB_UNIFORM = 0, 1


def slab_rom_ordinates(n: int, seed: int = 0, sample: int = 0):
    """ROM slab ordinates (Sec. 4.1): one uniform draw in each of the n/2 cells of [-1, 0],
    mirrored into [0, 1]; weights 1/n (sum 1)."""
    mu = np.empty(n)
    w = np.empty(n)
    if lib().orc_slab_ordinates_rom(n, seed, sample, _p(mu), _p(w)) != 0:
        raise ValueError("orc_slab_ordinates_rom failed")
    return mu, w


def slab_quadrature(kind: int, n: int):
    """DOM slab quadrature: SLAB_GAUSS (Gauss-Legendre) or SLAB_UNIFORM (midpoints); weights sum 1."""
    mu = np.empty(n)
    w = np.empty(n)
    if lib().orc_slab_quadrature(kind, n, _p(mu), _p(w)) != 0:
        raise ValueError("orc_slab_quadrature failed")
    return mu, w


def slab_sweep(nx, x0, x1, sigma_t, mu, inflow, S):
    """psi [n, nx+1] for node sources S [nx+1] (diamond difference at the grid points)."""
    mu = _f64(mu)
    psi = np.empty((mu.size, nx + 1))
    rc = lib().orc_slab_sweep(nx, x0, x1, _p(_f64(sigma_t)), mu.size, _p(mu), _p(_f64(inflow)), _p(_f64(S)), _p(psi))
    if rc != 0:
        raise ValueError(f"orc_slab_sweep failed ({rc})")
    return psi


def slab_source_iterate(nx, x0, x1, sigma_t, sigma_s, q, mu, w, inflow, tol=1e-10, max_iter=10000):
    """Slab source iteration from phi^0 = 0; fields at the nx + 1 grid points."""
    mu = _f64(mu)
    phi = np.empty(nx + 1)
    it = C.c_int(0)
    r = C.c_double(0.0)
    rc = lib().orc_slab_source_iterate(nx, x0, x1, _p(_f64(sigma_t)), _p(_f64(sigma_s)), _p(_f64(q)), mu.size,
                                       _p(mu), _p(_f64(w)), _p(_f64(inflow)), tol, max_iter, _p(phi),
                                       C.byref(it), C.byref(r))
    if rc < 0:
        raise ValueError(f"orc_slab_source_iterate failed ({rc})")
    return {"phi": phi, "iters": it.value, "r": r.value, "status": rc}
