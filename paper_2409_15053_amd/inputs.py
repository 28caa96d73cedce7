"""Seeded synthetic inputs shared by the GPU path's tests and the oracle's tests.

This module builds matrices and random blocks only.  It holds none of the
filtered Lanczos arithmetic (no filter, no recurrence, no orthogonalisation),
so the oracle and the HIP path can both consume its output without sharing
any of the method.

Matrices are returned as ``Csr`` triples in the layout the C-ABI expects:
zero-based ``rowptr`` int32[n+1], ``colind`` int32[nnz] with columns sorted
inside each row, ``val`` float64[nnz], full symmetric storage (both
triangles), as the paper stores its Hamiltonians on the GPU (Section 3.2.1).

Workloads (stand-ins for the PARSEC Hamiltonians of Table 1, which are not
available here; see the input recipe in the design notes):

* ``laplacian_2d``: 5-point finite-difference Laplacian, Dirichlet, h = 1.
* ``laplacian_3d``: 7-point Laplacian plus an optional diagonal potential.
* ``laplacian_3d_13pt``: 4th-order 13-point Laplacian plus optional potential.
* ``gaussian_wells``: sum of negative Gaussian wells on the grid
  (a real-space Hamiltonian-shaped potential, Section 1's Kohn-Sham setting).
* ``random_sym``: small random sparse symmetric matrices for edge cases.
"""
from __future__ import annotations

import dataclasses

import numpy as np

BASE_SEED = 240915053


@dataclasses.dataclass
class Csr:
    n: int
    rowptr: np.ndarray  # int32[n+1]
    colind: np.ndarray  # int32[nnz]
    val: np.ndarray     # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.colind.shape[0])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.colind, self.rowptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        d[rows, self.colind] = self.val
        return d


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _stencil_csr(shape, offsets, coeffs, diag) -> Csr:
    """CSR of a constant-coefficient stencil on a Dirichlet grid.

    ``offsets`` are integer displacement tuples (one per stencil point other
    than the centre) with matching ``coeffs``; ``diag`` is the per-row
    diagonal (float64[n]).  Columns come out sorted because the stencil points
    are visited in increasing linear offset.
    """
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    n = int(np.prod(shape))
    strides = [int(np.prod(shape[d + 1:])) for d in range(dim)]
    pts = [((0,) * dim, None)] + list(zip(offsets, coeffs))
    lin = [sum(o[d] * strides[d] for d in range(dim)) for o, _ in pts]
    order = np.argsort(lin, kind="stable")
    idx = np.indices(shape).reshape(dim, n)
    cols = np.empty((n, len(pts)), dtype=np.int64)
    vals = np.empty((n, len(pts)), dtype=np.float64)
    mask = np.empty((n, len(pts)), dtype=bool)
    rows = np.arange(n, dtype=np.int64)
    for slot, p in enumerate(order):
        off, cf = pts[p]
        ok = np.ones(n, dtype=bool)
        for d in range(dim):
            q = idx[d] + off[d]
            ok &= (q >= 0) & (q < shape[d])
        cols[:, slot] = rows + lin[p]
        vals[:, slot] = diag if cf is None else cf
        mask[:, slot] = ok
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    colind = cols[mask].astype(np.int32)
    val = vals[mask].astype(np.float64)
    return Csr(n, rowptr.astype(np.int32), colind, val)


def laplacian_2d(N: int) -> Csr:
    """5-point Laplacian on an N x N Dirichlet grid (diagonal 4, neighbours -1)."""
    offs = [(-1, 0), (1, 0), (0, -1), (0, 1)]
    return _stencil_csr((N, N), offs, [-1.0] * 4, np.full(N * N, 4.0))


def laplacian_3d(N: int, potential: np.ndarray | None = None) -> Csr:
    """7-point Laplacian on an N^3 Dirichlet grid plus a diagonal potential."""
    offs = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    diag = np.full(N ** 3, 6.0)
    if potential is not None:
        diag = diag + np.asarray(potential, dtype=np.float64).reshape(-1)
    return _stencil_csr((N, N, N), offs, [-1.0] * 6, diag)


# 4th-order central second difference, negated: (1/12, -4/3, 5/2, -4/3, 1/12)
FOURTH_ORDER_1D = {0: 2.5, 1: -4.0 / 3.0, 2: 1.0 / 12.0}


def laplacian_3d_13pt(N: int, potential: np.ndarray | None = None) -> Csr:
    """4th-order 13-point Laplacian on an N^3 Dirichlet grid plus a potential.

    Per axis the negated 4th-order stencil gives 5/2 on the diagonal, -4/3 at
    distance 1 and +1/12 at distance 2, so the 3D diagonal is 7.5.
    """
    offs, cfs = [], []
    for d in range(3):
        for dist in (1, 2):
            for sgn in (-1, 1):
                o = [0, 0, 0]
                o[d] = sgn * dist
                offs.append(tuple(o))
                cfs.append(FOURTH_ORDER_1D[dist])
    diag = np.full(N ** 3, 3 * FOURTH_ORDER_1D[0])
    if potential is not None:
        diag = diag + np.asarray(potential, dtype=np.float64).reshape(-1)
    return _stencil_csr((N, N, N), offs, cfs, diag)


def uniform_potential(N: int, seed: int, dim: int = 3) -> np.ndarray:
    """V_i ~ U[0,1) per grid point (PCG64)."""
    return rng(seed).random(N ** dim)


def separable_potential(N: int, seed: int) -> tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    """V(x,y,z) = vx(x) + vy(y) + vz(z), each 1D factor ~ U[0,1).

    Returns the 3D field (flattened, z fastest) and the three 1D factors.
    """
    g = rng(seed)
    vx, vy, vz = g.random(N), g.random(N), g.random(N)
    field = vx[:, None, None] + vy[None, :, None] + vz[None, None, :]
    return field.reshape(-1), vx, vy, vz


def gaussian_wells(N: int, seed: int, count: int = 16) -> np.ndarray:
    """V(r) = -sum_w d_w exp(-|r - c_w|^2 / (2 s_w^2)) on an N^3 grid.

    Centres c_w ~ U[0, N-1]^3, depths d_w ~ U[1,5], widths s_w ~ U[2,6], all in
    grid units.
    """
    g = rng(seed)
    centres = g.uniform(0.0, N - 1.0, size=(count, 3))
    depths = g.uniform(1.0, 5.0, size=count)
    widths = g.uniform(2.0, 6.0, size=count)
    ax = np.arange(N, dtype=np.float64)
    V = np.zeros((N, N, N))
    for (cx, cy, cz), d, s in zip(centres, depths, widths):
        gx = np.exp(-((ax - cx) ** 2) / (2 * s * s))
        gy = np.exp(-((ax - cy) ** 2) / (2 * s * s))
        gz = np.exp(-((ax - cz) ** 2) / (2 * s * s))
        V -= d * gx[:, None, None] * gy[None, :, None] * gz[None, None, :]
    return V.reshape(-1)


def random_sym(n: int, density: float, seed: int, diag_shift: float = 0.0) -> Csr:
    """Random sparse symmetric matrix with N(0,1) entries and a full diagonal."""
    g = rng(seed)
    m = max(1, int(density * n * n / 2))
    i = g.integers(0, n, size=m)
    j = g.integers(0, n, size=m)
    v = g.standard_normal(m)
    d = np.zeros((n, n))
    np.add.at(d, (i, j), v)
    d = d + d.T
    d[np.arange(n), np.arange(n)] += g.standard_normal(n) + diag_shift
    return dense_to_csr(d)


def dense_to_csr(d: np.ndarray) -> Csr:
    n = d.shape[0]
    mask = d != 0.0
    mask[np.arange(n), np.arange(n)] = True
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    rows, cols = np.nonzero(mask)
    return Csr(n, rowptr.astype(np.int32), cols.astype(np.int32), d[rows, cols].astype(np.float64))


def diagonal_csr(diag: np.ndarray) -> Csr:
    n = diag.shape[0]
    return Csr(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
               np.asarray(diag, dtype=np.float64).copy())


def random_block(n: int, r: int, seed: int) -> np.ndarray:
    """n x r row-major block of N(0,1) entries (PCG64)."""
    return rng(seed).standard_normal((n, r))


# ---------------------------------------------------------------- workloads

def workload_c1() -> dict:
    """2D 5-point Laplacian, 40 x 40 grid, interval [0.5, 1.0], degree 50, r = 1."""
    return dict(name="lap2d_40", A=laplacian_2d(40), alpha=0.5, beta=1.0, degree=50,
                block=1, seed=BASE_SEED)


def workload_c2(N: int = 100) -> dict:
    """3D 7-point Laplacian on N^3 plus U[0,1) potential, r = 8, FP64."""
    V = uniform_potential(N, BASE_SEED + 2)
    return dict(name=f"lap3d7_{N}_U01", A=laplacian_3d(N, V), block=8, seed=BASE_SEED + 2)


def workload_c3(N: int = 120) -> dict:
    """3D 13-point 4th-order Laplacian on N^3 plus 16 Gaussian wells, r = 16."""
    V = gaussian_wells(N, BASE_SEED + 3)
    return dict(name=f"lap3d13_{N}_wells16", A=laplacian_3d_13pt(N, V), block=16,
                seed=BASE_SEED + 3)


def lap1d_eigenvalues(N: int) -> np.ndarray:
    """Eigenvalues 4 sin^2(j pi / (2(N+1))) of the 1D Dirichlet second difference
    (used only to place synthetic intervals, not as a reference)."""
    j = np.arange(1, N + 1)
    return 4.0 * np.sin(j * np.pi / (2 * (N + 1))) ** 2


def batch_family(count: int = 64, seed: int = BASE_SEED + 4, gmin: int = 20, gmax: int = 60,
                 tmin: int = 10, tmax: int = 60) -> list:
    """Independent problems for the batched form: 3D 7-point Laplacian on a
    g^3 grid plus a U[0,1) potential, g = round(exp(U[ln gmin, ln gmax]))
    (n log-uniform), and a low-end interval [0, beta] meant to hold about t
    eigenvalues, t ~ U{tmin..tmax}: beta is the t-th smallest eigenvalue of
    the potential-free Laplacian plus the potential's mean 0.5, plus a
    seeded offset of at most one local level spacing."""
    g = rng(seed)
    out = []
    for i in range(count):
        N = int(round(float(np.exp(g.uniform(np.log(gmin), np.log(gmax))))))
        t = int(g.integers(tmin, tmax + 1))
        pseed = int(g.integers(0, 2 ** 31))
        jitter = float(g.uniform(0.0, 1.0))
        mu = lap1d_eigenvalues(N)
        k = min(N, 12)
        lap = np.sort((mu[:k, None, None] + mu[None, :k, None] + mu[None, None, :k]).ravel())
        base = lap[t - 1] + 0.5
        spacing = lap[t] - lap[t - 1] if lap[t] > lap[t - 1] else 1e-3
        out.append(dict(name=f"lap3d7_{N}_U01_s{pseed}", N=N, potential_seed=pseed, alpha=0.0,
                        beta=float(base + jitter * spacing), target=t))
    return out


def build_batch_matrix(spec: dict) -> Csr:
    return laplacian_3d(spec["N"], uniform_potential(spec["N"], spec["potential_seed"]))


def serve_family(count: int = 512, seed: int = BASE_SEED + 5, gmin: int = 30, gmax: int = 100,
                 tmin: int = 10, tmax: int = 200, wells: int = 16, degree: int = 60) -> list:
    """Requests for the serving form: 4th-order 13-point Laplacian on a g^3
    grid plus 16 Gaussian wells (as the 120^3 Hamiltonian), g =
    round(exp(U[ln gmin, ln gmax])), a target count t ~ U{tmin..tmax} of
    eigenvalues at the low end of the spectrum, and a fixed filter degree.
    The interval is placed from t by build_serve_problem."""
    g = rng(seed)
    out = []
    for i in range(count):
        N = int(round(float(np.exp(g.uniform(np.log(gmin), np.log(gmax))))))
        pseed = int(g.integers(0, 2 ** 31))
        t = int(g.integers(tmin, tmax + 1))
        out.append(dict(name=f"lap3d13_{N}_wells{wells}_s{pseed}", N=N, potential_seed=pseed, wells=wells,
                        target=t, degree=degree))
    return out


def weyl_count(V: np.ndarray, E: float) -> float:
    """Semiclassical (Weyl) number of eigenvalues below E of -Laplacian + V
    on a unit grid: sum over grid points of (E - V_i)_+^{3/2} / (6 pi^2)."""
    return float(np.sum(np.clip(E - V, 0.0, None) ** 1.5) / (6.0 * np.pi ** 2))


def gershgorin_lower(A: Csr) -> float:
    """min_i (a_ii - sum_{j != i} |a_ij|) of a CSR matrix."""
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    on = rows == A.colind
    diag = np.zeros(A.n)
    rad = np.zeros(A.n)
    np.add.at(diag, rows[on], A.val[on])
    np.add.at(rad, rows[~on], np.abs(A.val[~on]))
    return float(np.min(diag - rad))


def build_serve_problem(spec: dict):
    """(A, alpha, beta) of one serving request: alpha one unit below the
    matrix's Gershgorin lower bound, beta where the Weyl estimate of the
    number of eigenvalues below it equals the request's target count (found
    by bisection; the estimate tracks the true count of these matrices to a
    few percent)."""
    V = gaussian_wells(spec["N"], spec["potential_seed"], spec["wells"])
    A = laplacian_3d_13pt(spec["N"], V)
    lo = gershgorin_lower(A)
    a, b = float(np.min(V)), float(np.min(V)) + 20.0
    for _ in range(100):
        mid = 0.5 * (a + b)
        if weyl_count(V, mid) < spec["target"]:
            a = mid
        else:
            b = mid
    return A, lo - 1.0, 0.5 * (a + b)


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    return np.cumsum(rng(seed).exponential(1.0 / rate, size=count))
