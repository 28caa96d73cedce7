"""FP64 CPU oracle for the filtered Lanczos procedure (FLP).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
``cpu_baseline`` leg may import this module.  It shares no code with the GPU
library (neither imports the other); both consume the seeded inputs built by
``paper_2409_15053_amd.inputs``, which holds none of the method.

Each function is written from the paper (Aurentz, Kalantzis, Saad, "Cucheb: a
GPU implementation of the filtered Lanczos procedure") and cites the passage
it follows.  Everything is FP64.  The sparse products run in ``oracle_core.c``
(plain loops); the small dense eigenproblems use LAPACK through NumPy/SciPy.

Readings taken where the paper is silent (each is listed in the design
notes as well):

* eps of the degree rule (eq. optimaldegree) = 0.31227: the one value that
  reproduces all five automatic degrees of Table 2 from the bounds of
  Table 1, with the exact weighted norm of the indicator.
* spectrum bounds: k0 = 40 unfiltered Lanczos steps, Ritz residual
  widening, a margin of 1e-3 of the width, clamped to Gershgorin.
* convergence check every s = 30 block steps; candidates are Ritz values
  of p(A) at or above half the filter's smaller endpoint value; stop when
  every candidate's residual bound is below tol_p * max|theta| and the
  candidate count did not change since the previous check.
* eigenvalues are recovered by Rayleigh-Ritz with A on the span of the
  converged candidate Ritz vectors (reduces to eq. rayleigh when the filter
  values are distinct); membership in [alpha, beta] is decided there.
* relative residual = ||Ax - lambda x|| / ||A|| with
  ||A|| = max(|lambda_min|, |lambda_max|).
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import time

import numpy as np
import scipy.linalg

from . import build_oracle

DEGREE_EPS = 0.31227
DEGREE_MAX = 2000
CHECK_EVERY = 30
BOUNDS_STEPS = 40

_lib = None


def _core():
    global _lib
    if _lib is None:
        path = build_oracle.build()
        lib = ctypes.CDLL(path)
        i32, f64, p = ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
        lib.oracle_csr_spmm.argtypes = [i32, p, p, p, i32, p, p]
        lib.oracle_csr_spmm.restype = None
        lib.oracle_cheb_forward.argtypes = [i32, p, p, p, i32, f64, f64, i32, p, p, p, p]
        lib.oracle_cheb_forward.restype = None
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_core().oracle_num_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check_csr(A):
    assert A.rowptr.dtype == np.int32 and A.colind.dtype == np.int32
    assert A.val.dtype == np.float64
    assert A.rowptr.flags.c_contiguous and A.colind.flags.c_contiguous and A.val.flags.c_contiguous


# ------------------------------------------------------------ sparse products

def spmm(A, X: np.ndarray) -> np.ndarray:
    """Y = A X for a CSR matrix and an n x r block (Section 3.2.1: CSR SpMV)."""
    _check_csr(A)
    X = np.ascontiguousarray(X, dtype=np.float64)
    vec = X.ndim == 1
    X2 = X.reshape(A.n, -1)
    r = X2.shape[1]
    Y = np.empty((A.n, r))
    _core().oracle_csr_spmm(A.n, _ptr(A.rowptr), _ptr(A.colind), _ptr(A.val), r, _ptr(X2), _ptr(Y))
    return Y.reshape(-1) if vec else Y


# ------------------------------------------------------------ filter (Section 2.2)

def affine_map(lmin: float, lmax: float) -> tuple[float, float]:
    """c and e of eq. (transf): A := (A - cI)/e maps [lmin, lmax] onto [-1, 1]."""
    return 0.5 * (lmin + lmax), 0.5 * (lmax - lmin)


def cheb_coeffs(alpha: float, beta: float, m: int) -> np.ndarray:
    """Chebyshev coefficients b_0..b_m of the indicator of [alpha, beta] in [-1,1].

    The closed form of Section 2.2 (Jackson):
    b_0 = (acos(alpha) - acos(beta)) / pi,
    b_i = 2 (sin(i acos(alpha)) - sin(i acos(beta))) / (i pi), i > 0.
    """
    a, b = math.acos(alpha), math.acos(beta)
    out = np.empty(m + 1)
    out[0] = (a - b) / math.pi
    for i in range(1, m + 1):
        out[i] = 2.0 * (math.sin(i * a) - math.sin(i * b)) / (i * math.pi)
    return out


def cheb_eval(coeffs: np.ndarray, z):
    """p(z) = sum_i b_i T_i(z) by the recurrence T_{i+1} = 2 z T_i - T_{i-1}
    (eq. def:cheb1), T_0 = 1, T_1 = z."""
    z = np.asarray(z, dtype=np.float64)
    t_prev = np.ones_like(z)
    y = coeffs[0] * t_prev
    if len(coeffs) == 1:
        return y
    t_cur = z.copy()
    y = y + coeffs[1] * t_cur
    for i in range(2, len(coeffs)):
        t_next = 2.0 * z * t_cur - t_prev
        y = y + coeffs[i] * t_next
        t_prev, t_cur = t_cur, t_next
    return y


def indicator_norm_sq(alpha: float, beta: float) -> float:
    """||phi||^2 in L^2_mu: integral of 1/sqrt(1-z^2) over [alpha, beta]
    = acos(alpha) - acos(beta) (= pi b_0)."""
    return math.acos(alpha) - math.acos(beta)


def truncation_error_sq(alpha: float, beta: float, m: int) -> float:
    """||p_m - phi||^2 in L^2_mu.

    p_m is the orthogonal projection of phi onto degree <= m (Section 2.2's
    orthogonality relation), so by Parseval
    ||p_m - phi||^2 = ||phi||^2 - pi b_0^2 - (pi/2) sum_{i=1..m} b_i^2.
    """
    b = cheb_coeffs(alpha, beta, m)
    return indicator_norm_sq(alpha, beta) - math.pi * b[0] ** 2 - 0.5 * math.pi * float(np.sum(b[1:] ** 2))


def filter_degree(alpha: float, beta: float, eps: float = DEGREE_EPS, m_max: int = DEGREE_MAX) -> int:
    """Smallest m > 0 with ||p_m - phi|| < eps ||phi|| (eq. optimaldegree).

    alpha, beta are already mapped into [-1, 1].
    """
    phi2 = indicator_norm_sq(alpha, beta)
    a, b = math.acos(alpha), math.acos(beta)
    err2 = phi2 - math.pi * ((a - b) / math.pi) ** 2
    for m in range(1, m_max + 1):
        bm = 2.0 * (math.sin(m * a) - math.sin(m * b)) / (m * math.pi)
        err2 -= 0.5 * math.pi * bm * bm
        if math.sqrt(max(err2, 0.0)) < eps * math.sqrt(phi2):
            return m
    return m_max


def filter_apply(A, lmin: float, lmax: float, coeffs: np.ndarray, V: np.ndarray) -> np.ndarray:
    """W = p(Ahat) V, Ahat = (A - cI)/e (eq. transf), by the forward recurrence.

    The paper applies p(A) with Clenshaw (Section 2.2); the oracle uses the
    forward three-term recurrence on purpose so the two sides do not share
    an algorithm.  ``V`` is an n x r block (or a vector).
    """
    _check_csr(A)
    c, e = affine_map(lmin, lmax)
    V = np.ascontiguousarray(V, dtype=np.float64)
    vec = V.ndim == 1
    V2 = V.reshape(A.n, -1)
    r = V2.shape[1]
    W = np.empty_like(V2)
    work = np.empty(3 * A.n * r)
    b = np.ascontiguousarray(coeffs, dtype=np.float64)
    _core().oracle_cheb_forward(A.n, _ptr(A.rowptr), _ptr(A.colind), _ptr(A.val), r, c, e,
                                len(b) - 1, _ptr(b), _ptr(V2), _ptr(W), _ptr(work))
    return W.reshape(-1) if vec else W


# ------------------------------------------------------------ spectrum bounds

def gershgorin(A) -> tuple[float, float]:
    """Gershgorin enclosure [min_i a_ii - R_i, max_i a_ii + R_i]."""
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    diag = np.zeros(A.n)
    rad = np.zeros(A.n)
    on = rows == A.colind
    np.add.at(diag, rows[on], A.val[on])
    np.add.at(rad, rows[~on], np.abs(A.val[~on]))
    return float(np.min(diag - rad)), float(np.max(diag + rad))


def lanczos_tridiag(A, q0: np.ndarray, k: int):
    """k steps of single-vector Lanczos with A and full reorthogonalisation.

    Returns (alphas, betas, beta_k): T is tridiagonal with diagonal alphas and
    off-diagonal betas[:-1]; beta_k is the norm of the final residual.
    """
    n = A.n
    k = min(k, n)
    Q = np.zeros((n, k + 1), order="F")
    Q[:, 0] = q0 / np.linalg.norm(q0)
    al = np.zeros(k)
    be = np.zeros(k)
    for j in range(k):
        w = spmm(A, Q[:, j])
        # full reorthogonalisation, two passes of classical Gram-Schmidt
        h = Q[:, : j + 1].T @ w
        w -= Q[:, : j + 1] @ h
        h2 = Q[:, : j + 1].T @ w
        w -= Q[:, : j + 1] @ h2
        al[j] = h[j] + h2[j]
        be[j] = np.linalg.norm(w)
        if be[j] == 0.0 or j == k - 1:
            return al[: j + 1], be[: j + 1], be[j]
        Q[:, j + 1] = w / be[j]
    return al, be, be[-1]


def spectrum_bounds(A, start: np.ndarray, k0: int = BOUNDS_STEPS) -> tuple[float, float]:
    """Estimate [lambda_min, lambda_max] by a few Lanczos steps (Section 2.2).

    lambda_min = theta_1 - rho_1 - delta, lambda_max = theta_k + rho_k + delta,
    with rho_i = |beta_k w_i(k)| the Ritz residual bound and
    delta = 1e-3 (theta_k - theta_1); then clamped to the Gershgorin enclosure.
    """
    al, be, bk = lanczos_tridiag(A, start, k0)
    k = len(al)
    if k == 1:
        theta, W = np.array([al[0]]), np.ones((1, 1))
    else:
        theta, W = scipy.linalg.eigh_tridiagonal(al, be[: k - 1])
    rho = np.abs(bk * W[-1, :])
    delta = 1e-3 * (theta[-1] - theta[0])
    lo = theta[0] - rho[0] - delta
    hi = theta[-1] + rho[-1] + delta
    g_lo, g_hi = gershgorin(A)
    return max(lo, g_lo), min(hi, g_hi)


# ------------------------------------------------------------ block Lanczos (Section 2.3)

def orthonormal_start(start: np.ndarray) -> np.ndarray:
    """Orthonormal start block from an n x r block: Q of its QR with a
    non-negative diagonal of R."""
    Q, R = np.linalg.qr(start)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s


@dataclasses.dataclass
class OracleResult:
    evals: np.ndarray
    evecs: np.ndarray
    resid: np.ndarray
    lmin: float
    lmax: float
    degree: int
    iters: int
    mv: int
    basis_cols: int
    times: dict
    converged: bool
    repairs: int = 0  # basis columns the block QR replaced (rank-deficient blocks)


def _block_qr(W: np.ndarray, Qb: np.ndarray, g: np.random.Generator):
    """W = Q_{j+1} S_j with S_j upper triangular, diag >= 0 (eq. lanczos).

    Returns (Q_{j+1}, S_j, number of replaced columns).  When the
    Householder QR leaves a diagonal entry at or below 1e-10 times the
    block's norm, the block is numerically rank deficient: it is then
    factorised again one column at a time (Gram-Schmidt, each projection
    taken twice), and a column whose remainder after projection on the
    columns before it is at or below that threshold is replaced by a random
    vector orthogonalised against the basis and those columns, with zero
    diagonal in S_j.  The columns after it are projected on the replacement
    too, so W = Q_{j+1} S_j keeps holding up to the dropped remainders
    (each at most the threshold) and Q_{j+1} stays orthonormal and
    orthogonal to the basis: the block keeps its width r (the reading of
    the paper's block Lanczos with a fixed block size).
    """
    nrm = np.linalg.norm(W)
    thr = 1e-10 * max(nrm, 1e-300)
    Qn, S = np.linalg.qr(W)
    sgn = np.sign(np.diag(S))
    sgn[sgn == 0] = 1.0
    Qn = Qn * sgn
    S = sgn[:, None] * S
    if np.all(np.abs(np.diag(S)) > thr):
        return Qn, S, 0
    n, r = W.shape
    Qn = np.zeros((n, r))
    S = np.zeros((r, r))
    replaced = 0
    for j in range(r):
        w = W[:, j].copy()
        for _ in range(2):
            h = Qn[:, :j].T @ w
            w -= Qn[:, :j] @ h
            S[:j, j] += h
        d = np.linalg.norm(w)
        if d > thr:
            Qn[:, j] = w / d
            S[j, j] = d
            continue
        # dependent column: a random direction orthogonal to everything so far
        v = g.standard_normal(n)
        others = np.concatenate([Qb, Qn[:, :j]], axis=1)
        for _ in range(2):
            v -= others @ (others.T @ v)
        Qn[:, j] = v / np.linalg.norm(v)
        S[j, j] = 0.0
        replaced += 1
    return Qn, S, replaced


def assemble_T(D: list, S: list) -> np.ndarray:
    """Block tridiagonal T_k with D_i on the diagonal and S_i / S_i^T beside it
    (eq. lanczos)."""
    k = len(D)
    r = D[0].shape[0]
    T = np.zeros((k * r, k * r))
    for i in range(k):
        T[i * r:(i + 1) * r, i * r:(i + 1) * r] = D[i]
        if i + 1 < k:
            T[(i + 1) * r:(i + 2) * r, i * r:(i + 1) * r] = S[i]
            T[i * r:(i + 1) * r, (i + 1) * r:(i + 2) * r] = S[i].T
    return T


def lanczos_step(A, lmin, lmax, coeffs, Qk: np.ndarray, r: int, g: np.random.Generator,
                 tally: dict | None = None):
    """One block step of FLP (Section 2.3, eq. lanczos; Section 3.2.2).

    Qk (n x k) holds the basis so far; its last r columns are Q_j.
    W = p(A) Q_j; full reorthogonalisation of W against every column of Qk
    (classical Gram-Schmidt, two passes); D_j = symmetric part of the
    Q_j^T p(A) Q_j block of the projection; W = Q_{j+1} S_j.
    Returns (D_j, S_j, Q_{j+1}, seconds in the filter, seconds in ORTH);
    ``tally["repairs"]`` (when given) counts the columns the block QR
    replaced.
    """
    t1 = time.perf_counter()
    W = filter_apply(A, lmin, lmax, coeffs, Qk[:, -r:])
    t_mv = time.perf_counter() - t1
    t1 = time.perf_counter()
    H1 = Qk.T @ W
    W = W - Qk @ H1
    H2 = Qk.T @ W
    W = W - Qk @ H2
    Hj = (H1 + H2)[-r:, :]
    Dj = 0.5 * (Hj + Hj.T)
    Qn, Sj, replaced = _block_qr(W, Qk, g)
    if tally is not None:
        tally["repairs"] = tally.get("repairs", 0) + replaced
    return Dj, Sj, Qn, t_mv, time.perf_counter() - t1


class _Basis:
    """Lanczos basis kept as one column-major array (columns contiguous) that
    grows by doubling, so Qk = basis[:, :k] is a view."""

    def __init__(self, n: int, first: np.ndarray):
        self.n = n
        self.buf = np.empty((n, max(256, first.shape[1])), order="F")
        self.k = 0
        self.append(first)

    def append(self, block: np.ndarray):
        r = block.shape[1]
        if self.k + r > self.buf.shape[1]:
            nb = np.empty((self.n, 2 * self.buf.shape[1] + r), order="F")
            nb[:, :self.k] = self.buf[:, :self.k]
            self.buf = nb
        self.buf[:, self.k:self.k + r] = block
        self.k += r

    def view(self) -> np.ndarray:
        return self.buf[:, :self.k]


def flp_solve(A, alpha: float, beta: float, block: int = 1, degree: int = 0,
              start: np.ndarray | None = None, seed: int = 0, tol: float = 1e-9,
              check_every: int = CHECK_EVERY, max_basis: int = 0,
              bounds: tuple[float, float] | None = None,
              bounds_start: np.ndarray | None = None, k0: int = BOUNDS_STEPS) -> OracleResult:
    """Every eigenpair of symmetric A in [alpha, beta] by FLP (Sections 2-3).

    Steps: spectrum bounds (Section 2.2) -> affine map (eq. transf) ->
    Chebyshev coefficients and degree (Section 2.2, eq. optimaldegree) ->
    block Lanczos on p(A) with full reorthogonalisation (Section 2.3,
    eq. lanczos; Section 3.2.2) -> periodic convergence check on the Ritz
    values of T_k (Section 3.2.2) -> Rayleigh-Ritz with A (eq. rayleigh,
    eq. proj).
    """
    t0 = time.perf_counter()
    times = {}
    n = A.n
    g = np.random.Generator(np.random.PCG64(seed))
    if bounds is None:
        if bounds_start is None:
            bounds_start = g.standard_normal(n)
        lmin, lmax = spectrum_bounds(A, bounds_start, k0)
    else:
        lmin, lmax = bounds
    times["pre"] = time.perf_counter() - t0

    # interval validity (Section 3.2.2): clamp to the spectrum, reject if empty
    lo, hi = max(alpha, lmin), min(beta, lmax)
    if not (lo <= hi):
        raise ValueError("interval does not meet the spectrum")
    c, e = affine_map(lmin, lmax)
    a1 = min(max((lo - c) / e, -1.0), 1.0)
    b1 = min(max((hi - c) / e, -1.0), 1.0)
    m = degree if degree > 0 else filter_degree(a1, b1)
    coeffs = cheb_coeffs(a1, b1, m)
    tau = 0.5 * min(float(cheb_eval(coeffs, a1)), float(cheb_eval(coeffs, b1)))
    tol_p = 1e-10

    r = block
    if start is None:
        start = g.standard_normal((n, r))
    if max_basis <= 0:
        max_basis = n
    max_steps = max(1, min(max_basis, n) // r)

    basis = _Basis(n, orthonormal_start(np.asarray(start, dtype=np.float64).reshape(n, r)))
    D, S = [], []
    t_mv = t_orth = 0.0
    prev_count = -1
    converged = False
    steps = 0
    sel = None
    tally = {"repairs": 0}
    while steps < max_steps:
        Dj, Sj, Qn, dt_mv, dt_orth = lanczos_step(A, lmin, lmax, coeffs, basis.view(), r, g, tally)
        D.append(Dj)
        S.append(Sj)
        t_mv += dt_mv
        t_orth += dt_orth
        steps += 1
        last = steps == max_steps or (steps + 1) * r > n
        if steps % check_every == 0 or last:
            T = assemble_T(D, S)
            theta, Wt = scipy.linalg.eigh(T)
            rho = np.linalg.norm(S[-1] @ Wt[-r:, :], axis=0)
            cand = np.nonzero(theta >= tau)[0]
            big = max(float(np.max(np.abs(theta))), 1e-300)
            ok = bool(np.all(rho[cand] <= tol_p * big))
            if (ok and len(cand) == prev_count) or last:
                converged = ok and len(cand) == prev_count
                sel = (cand, Wt)
                break
            prev_count = len(cand)
        basis.append(Qn)
    times["mv"] = t_mv
    times["orth"] = t_orth

    t1 = time.perf_counter()
    cand, Wt = sel
    Qb = basis.view()
    anorm = max(abs(lmin), abs(lmax))
    if len(cand) == 0:
        evals = np.zeros(0)
        X = np.zeros((n, 0))
        res = np.zeros(0)
    else:
        Y = Qb @ Wt[:, cand]
        Y, _ = np.linalg.qr(Y)
        AY = spmm(A, Y)
        G = Y.T @ AY
        lam, Z = scipy.linalg.eigh(0.5 * (G + G.T))
        keep = (lam >= alpha) & (lam <= beta)
        X = Y @ Z[:, keep]
        AX = AY @ Z[:, keep]
        evals = lam[keep]
        res = np.linalg.norm(AX - X * evals, axis=0) / anorm
    times["rr"] = time.perf_counter() - t1
    times["total"] = time.perf_counter() - t0
    return OracleResult(evals=evals, evecs=X, resid=res, lmin=lmin, lmax=lmax, degree=m,
                        iters=steps, mv=r * m * steps, basis_cols=Qb.shape[1], times=times,
                        converged=converged, repairs=tally["repairs"])


# ------------------------------------------------------------ definition for tiny n

def dense_eigs_in_interval(A, alpha: float, beta: float):
    """The result by its definition (program summary; Section 2.2): every
    eigenpair of A with alpha <= lambda <= beta, from a dense symmetric
    eigensolve.  Feasible for n up to a few thousand."""
    d = A.to_dense() if hasattr(A, "to_dense") else np.asarray(A)
    lam, V = np.linalg.eigh(d)
    keep = (lam >= alpha) & (lam <= beta)
    return lam[keep], V[:, keep]
