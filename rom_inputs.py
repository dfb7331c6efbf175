"""Seeded synthetic inputs for the ROM source-iteration workloads.

This module only builds problem data: grids, piecewise-constant cross-section maps, sources and
master seeds.  It holds none of the method's arithmetic (no ordinates, no sweeps, no iteration),
so that both the FP64 oracle and the GPU library can be fed from it without sharing any code
with each other.

Cell (i, j) of an nx x ny grid on [x0,x1] x [y0,y1] is stored at j*nx + i; piecewise-constant
data is sampled at cell centres with half-open [lo, hi) membership.

Workloads (all vacuum inflow, unit square):
  * ``c1`` -- 64 x 64, sigma_t = 1, sigma_s = 0.5, isotropic, q = 1 on the central 0.1 square,
    32 i.i.d. sphere ordinates (seed 0), FP64, tolerance 1e-8, one sample.
  * ``c2`` -- 256 x 256, 7 x 7 checkerboard of blocks: even blocks scatter (sigma_t = 1,
    sigma_s = 0.9), odd blocks absorb (sigma_t = 10, sigma_s = 0); q = 1 in the centre block;
    256 stratified random ordinates (8 x 8 per quadrant, seed 0), FP32, tolerance 1e-6.
  * ``c3`` -- 512 x 512, sigma_t = 1, sigma_s = 0.5, q = 1 on the central 0.02 square, an
    ensemble of 64 samples x 128 stratified random ordinates (4 x 8 per quadrant), FP32,
    tolerance 1e-6.
  * ``c4`` -- 256 x 256, Henyey-Greenstein g = 0.8, sigma_t = 1, sigma_s = 0.8, q = 1 on the
    central 0.1 square, 1024 stratified random ordinates (16 x 16 per quadrant), FP32 sweeps
    with a BF16 contraction, tolerance 1e-6.
  * ``c5`` -- 200 independent problems: grid sides drawn from {64,...,1024}, n = 4m with
    m ~ U{4..128}, sigma_t log-uniform in [0.1, 10] and sigma_s/sigma_t ~ U[0, 0.95] on a random
    8 x 8 block map, q = 1 on the central 0.1 square, FP32, tolerance 1e-6.
The example of Sec. 2 of the paper (``example21``) is 100 x 100, sigma_t = 1, sigma_s = 0.5,
q = 2 on [0.4, 0.6]^2.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Fields:
    """Cell data of one problem (float64 arrays of length nx*ny, row-major in y)."""
    nx: int
    ny: int
    sigma_t: np.ndarray
    sigma_s: np.ndarray
    q: np.ndarray
    box: tuple = (0.0, 1.0, 0.0, 1.0)
    inflow: dict = field(default_factory=dict)  # face -> [ny] or [nx] isotropic values

    @property
    def cells(self) -> int:
        return self.nx * self.ny


@dataclass
class Workload:
    """One configuration: problem fields plus the ordinate recipe and the solver settings."""
    name: str
    fields: list            # list[Fields], one per independent problem
    ord_kind: str           # "stratified" | "iid_sphere" | "uniform2d" | "gauss2d"
    n_ord: list             # ordinates per problem
    samples: int            # ROM samples per problem
    seed: int
    tol: float
    precision: str          # "fp64" | "fp32"
    scattering: str = "iso"  # "iso" | "hg" | "linear"
    g: float = 0.0
    max_iter: int = 2000
    seeds: list = None      # per-problem master seeds (defaults to [seed]*len(fields))

    def problem_seed(self, k: int) -> int:
        return self.seeds[k] if self.seeds is not None else self.seed


def cell_centres(n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    d = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * d


def box_indicator(nx: int, ny: int, lo: float, hi: float, box=(0.0, 1.0, 0.0, 1.0)) -> np.ndarray:
    """1 on cells whose centre lies in [lo, hi) x [lo, hi), else 0 (flattened, j*nx + i)."""
    xc = cell_centres(nx, box[0], box[1])
    yc = cell_centres(ny, box[2], box[3])
    inx = (xc >= lo) & (xc < hi)
    iny = (yc >= lo) & (yc < hi)
    return (iny[:, None] & inx[None, :]).astype(np.float64).reshape(-1)


def uniform_fields(nx, ny, sigma_t, sigma_s, q_lo, q_hi, q_val=1.0) -> Fields:
    cells = nx * ny
    return Fields(nx, ny, np.full(cells, float(sigma_t)), np.full(cells, float(sigma_s)),
                  q_val * box_indicator(nx, ny, q_lo, q_hi))


def checkerboard_fields(nx, ny, blocks=7) -> Fields:
    """blocks x blocks checkerboard: block (I, J) = (floor(blocks*x), floor(blocks*y)) of the cell
    centre; I+J even scatters (sigma_t 1, sigma_s 0.9), odd absorbs (sigma_t 10, sigma_s 0);
    q = 1 in the centre block."""
    xc = cell_centres(nx)
    yc = cell_centres(ny)
    bi = np.floor(blocks * xc).astype(int)
    bj = np.floor(blocks * yc).astype(int)
    I = np.broadcast_to(bi[None, :], (ny, nx))
    J = np.broadcast_to(bj[:, None], (ny, nx))
    even = ((I + J) % 2) == 0
    st = np.where(even, 1.0, 10.0).reshape(-1)
    ss = np.where(even, 0.9, 0.0).reshape(-1)
    mid = blocks // 2
    q = ((I == mid) & (J == mid)).astype(np.float64).reshape(-1)
    return Fields(nx, ny, st, ss, q)


def block_map_fields(nx, ny, rng: np.random.Generator, blocks=8) -> Fields:
    """Random blocks x blocks map: sigma_t log-uniform in [0.1, 10], sigma_s/sigma_t ~ U[0, 0.95];
    q = 1 on the central 0.1 square."""
    log_st = rng.uniform(np.log(0.1), np.log(10.0), size=(blocks, blocks))
    ratio = rng.uniform(0.0, 0.95, size=(blocks, blocks))
    st_b = np.exp(log_st)
    ss_b = st_b * ratio
    bi = np.minimum((cell_centres(nx) * blocks).astype(int), blocks - 1)
    bj = np.minimum((cell_centres(ny) * blocks).astype(int), blocks - 1)
    st = st_b[bj[:, None], bi[None, :]].reshape(-1)
    ss = ss_b[bj[:, None], bi[None, :]].reshape(-1)
    q = box_indicator(nx, ny, 0.45, 0.55)
    return Fields(nx, ny, st, ss, q)


def c1() -> Workload:
    return Workload("c1", [uniform_fields(64, 64, 1.0, 0.5, 0.45, 0.55)], "iid_sphere", [32], 1, 0, 1e-8,
                    "fp64")


def c2(n=256) -> Workload:
    return Workload("c2", [checkerboard_fields(n, n)], "stratified", [256], 1, 0, 1e-6, "fp32")


def c3(n=512, samples=64) -> Workload:
    return Workload("c3", [uniform_fields(n, n, 1.0, 0.5, 0.49, 0.51)], "stratified", [128], samples, 0, 1e-6,
                    "fp32")


def c4(n=256, n_ord=1024) -> Workload:
    return Workload("c4", [uniform_fields(n, n, 1.0, 0.8, 0.45, 0.55)], "stratified", [n_ord], 1, 0, 1e-6,
                    "fp32", scattering="hg", g=0.8)


C5_SIDES = (64, 128, 256, 512, 1024)


def c5(count=200, master_seed=0, sides=C5_SIDES, m_range=(4, 128)) -> Workload:
    rng = np.random.default_rng(master_seed)
    fields, n_ord, seeds = [], [], []
    for _ in range(count):
        nx = int(rng.choice(sides))
        ny = int(rng.choice(sides))
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        fields.append(block_map_fields(nx, ny, rng))
        n_ord.append(4 * m)
        seeds.append(int(rng.integers(0, 2**63 - 1)))
    return Workload("c5", fields, "stratified", n_ord, 1, master_seed, 1e-6, "fp32", seeds=seeds)


def example21(n=100) -> Fields:
    """Example 2.1: 100 x 100 cells on the unit square, sigma_t 1, sigma_s 0.5, q = 2 on
    [0.4, 0.6]^2, vacuum inflow."""
    return uniform_fields(n, n, 1.0, 0.5, 0.4, 0.6, q_val=2.0)


@dataclass
class SlabFields:
    """Slab problem on [x0, x1] with nx cells; fields at the nx + 1 grid points x_i = x0 + i dx,
    and the boundary inflow as a function of mu (left face for mu > 0, right face for mu < 0)."""
    nx: int
    sigma_t: np.ndarray
    sigma_s: np.ndarray
    q: np.ndarray
    inflow: object
    x0: float = 0.0
    x1: float = 1.0


def slab_example41(nx=50, case=1) -> SlabFields:
    """Example 4.1 (Sec. 4.1): sigma_t = 10x^2 + 1, sigma_s = 5x^2 + 0.5, q = 1 + x on [0, 1], with
    the inflow of case 1 (smooth), 2 (continuous, not differentiable) or 3 (discontinuous)."""
    x = np.linspace(0.0, 1.0, nx + 1)

    def inflow(mu):
        mu = np.asarray(mu, dtype=float)
        if case == 1:
            return np.where(mu > 0, 3 * mu, -5 * mu)
        if case not in (2, 3):
            raise ValueError("case must be 1, 2 or 3")
        left = np.where(mu > 1 / 3, (4 / 3 if case == 2 else 3) - mu, 3 * mu)
        right = np.where(mu < -1 / 3, (2 if case == 2 else 4) + mu, -5 * mu)
        return np.where(mu > 0, left, right)

    return SlabFields(nx, 10 * x * x + 1, 5 * x * x + 0.5, 1 + x, inflow)


WORKLOADS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5}
