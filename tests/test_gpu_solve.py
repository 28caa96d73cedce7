"""End-to-end parity of flp_solve (GPU, through the C ABI) against the
oracle and against closed forms.

Contract (stated for every result): the eigenvalue count in [alpha, beta]
is exact, eigenvalues agree within 1e-10 relative, and every residual
||A x - lambda x|| / ||A|| is at most 1e-9.  Eigenvectors are compared by
principal angles inside each cluster (eigenvalues closer than 1e-8 ||A||),
||sin Theta|| <= 1e-7.
"""
import math

import numpy as np
import pytest

from oracle import flp_oracle as O
from paper_2409_15053_amd import flp
from paper_2409_15053_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a visible MI355X"
    flp.load()
    return t


def lap1d(N):
    j = np.arange(1, N + 1)
    return 4 * np.sin(j * np.pi / (2 * (N + 1))) ** 2


def check_against(res, want_vals, want_vecs=None, anorm=None):
    got = np.sort(res["evals"])
    assert res["count"] == len(want_vals), (res["count"], len(want_vals))
    if len(want_vals) == 0:
        return
    rel = np.abs(got - want_vals) / np.maximum(np.abs(want_vals), 1e-300)
    assert np.max(rel) <= 1e-10, np.max(rel)
    assert np.max(res["resid"]) <= 1e-9, np.max(res["resid"])
    X = res["evecs"].cpu().numpy()
    assert np.max(np.abs(X.T @ X - np.eye(X.shape[1]))) < 1e-10
    if want_vecs is not None:
        # principal angles per cluster
        gap = 1e-8 * anorm
        i = 0
        while i < len(want_vals):
            j = i + 1
            while j < len(want_vals) and want_vals[j] - want_vals[j - 1] < gap:
                j += 1
            Ug = X[:, i:j]
            Uw = want_vecs[:, i:j]
            s = np.linalg.svd(Uw.T @ Ug, compute_uv=False)
            sin_max = math.sqrt(max(0.0, 1.0 - float(np.min(s)) ** 2))
            assert sin_max <= 1e-7, (i, j, sin_max)
            i = j


def test_c1_laplacian_2d(torch):
    """2D 5-point Laplacian on 40 x 40, [0.5, 1.0], degree 50, r = 1: the 69
    eigenvalues 4 sin^2(j pi/82) + 4 sin^2(k pi/82) (33 of them double)."""
    w = I.workload_c1()
    A = w["A"]
    mu = lap1d(40)
    exact = np.sort((mu[:, None] + mu[None, :]).ravel())
    exact = exact[(exact >= 0.5) & (exact <= 1.0)]
    dA = flp.DeviceCsr.from_host(A)
    res = flp.flp_solve(dA, 0.5, 1.0, block=1, degree=50, seed=w["seed"])
    assert res["converged"]
    lam, V = O.dense_eigs_in_interval(A, 0.5, 1.0)
    check_against(res, exact, V, anorm=8.0)
    # iters: the block steps behind the result, a multiple of the check
    # cadence; mv also counts the few steps taken while the deciding check
    # ran, all of them full filter applications of degree 50
    assert res["stats"]["iters"] % 30 == 0
    assert res["stats"]["mv"] % 50 == 0 and res["stats"]["mv"] >= 1 * 50 * res["stats"]["iters"]
    # the oracle on the same problem finds the same set
    ores = O.flp_solve(A, 0.5, 1.0, block=1, degree=50, seed=w["seed"])
    assert len(ores.evals) == res["count"]
    assert np.max(np.abs(np.sort(ores.evals) - np.sort(res["evals"])) / exact) <= 1e-10


@pytest.mark.parametrize("block", [1, 2, 3, 4])
def test_random_sparse_interior(torch, block):
    A = I.random_sym(600, 0.015, seed=40 + block)
    lam_all = np.linalg.eigvalsh(A.to_dense())
    i0, i1 = 250, 289
    alpha = 0.5 * (lam_all[i0 - 1] + lam_all[i0])
    beta = 0.5 * (lam_all[i1] + lam_all[i1 + 1])
    dA = flp.DeviceCsr.from_host(A)
    res = flp.flp_solve(dA, alpha, beta, block=block, seed=3)
    want, V = O.dense_eigs_in_interval(A, alpha, beta)
    check_against(res, want, V, anorm=np.max(np.abs(lam_all)))


@pytest.mark.parametrize("kind,N,block", [("7pt", 16, 8), ("13pt", 13, 16), ("7pt", 20, 4)])
def test_kronecker_separable_3d(torch, kind, N, block):
    field, vx, vy, vz = I.separable_potential(N, seed=17 + N)
    if kind == "7pt":
        A = I.laplacian_3d(N, field)
        st = {0: 2.0, 1: -1.0}
    else:
        A = I.laplacian_3d_13pt(N, field)
        st = {0: I.FOURTH_ORDER_1D[0], 1: I.FOURTH_ORDER_1D[1], 2: I.FOURTH_ORDER_1D[2]}

    def one_d(v):
        T = np.zeros((N, N))
        for d, cf in st.items():
            idx = np.arange(N - d)
            T[idx, idx + d] = cf
            T[idx + d, idx] = cf
        np.fill_diagonal(T, st[0] + v)
        return np.linalg.eigvalsh(T)

    a, b, c = one_d(vx), one_d(vy), one_d(vz)
    spec = np.sort((a[:, None, None] + b[None, :, None] + c[None, None, :]).ravel())
    i0, i1 = 5, 84
    alpha = 0.5 * (spec[i0 - 1] + spec[i0])
    beta = 0.5 * (spec[i1] + spec[i1 + 1])
    dA = flp.DeviceCsr.from_host(A)
    res = flp.flp_solve(dA, alpha, beta, block=block, seed=N)
    check_against(res, spec[i0:i1 + 1])


def test_hamiltonian_wells_dense(torch):
    N = 15
    A = I.laplacian_3d_13pt(N, I.gaussian_wells(N, I.BASE_SEED + 3))
    lam_all = np.linalg.eigvalsh(A.to_dense())
    i0, i1 = 10, 69
    alpha = 0.5 * (lam_all[i0 - 1] + lam_all[i0])
    beta = 0.5 * (lam_all[i1] + lam_all[i1 + 1])
    dA = flp.DeviceCsr.from_host(A)
    res = flp.flp_solve(dA, alpha, beta, block=16, seed=1)
    want, V = O.dense_eigs_in_interval(A, alpha, beta)
    check_against(res, want, V, anorm=np.max(np.abs(lam_all)))


def test_uniform_potential_lowest_block8(torch):
    N = 16
    A = I.laplacian_3d(N, I.uniform_potential(N, I.BASE_SEED + 2))
    lam_all = np.linalg.eigvalsh(A.to_dense())
    i1 = 49
    alpha = lam_all[0] - 1.0
    beta = 0.5 * (lam_all[i1] + lam_all[i1 + 1])
    dA = flp.DeviceCsr.from_host(A)
    res = flp.flp_solve(dA, alpha, beta, block=8, seed=2)
    want, V = O.dense_eigs_in_interval(A, alpha, beta)
    check_against(res, want, V, anorm=np.max(np.abs(lam_all)))


def test_empty_interval_in_gap(torch):
    A = I.diagonal_csr(np.array([0.0, 1.0, 2.0, 3.0, 4.0] * 20))
    dA = flp.DeviceCsr.from_host(A)
    res = flp.flp_solve(dA, 1.2, 1.8, block=1, seed=1)
    assert res["count"] == 0


def test_interval_outside_spectrum_errors(torch):
    A = I.laplacian_2d(10)
    dA = flp.DeviceCsr.from_host(A)
    with pytest.raises(flp.FlpError) as ei:
        flp.flp_solve(dA, 100.0, 200.0, block=1)
    assert ei.value.code == flp.FLP_E_INTERVAL


def test_multiplicity_with_blocks(torch):
    """A diagonal matrix with a 5-fold eigenvalue inside the interval; block
    Lanczos (Section 2.3) recovers every copy through breakdown repair."""
    d = np.concatenate([np.linspace(-3, -1, 150), np.full(5, 0.5), np.linspace(1, 4, 150)])
    A = I.diagonal_csr(d)
    dA = flp.DeviceCsr.from_host(A)
    res = flp.flp_solve(dA, 0.0, 0.9, block=2, seed=4)
    assert res["count"] == 5
    assert np.max(np.abs(res["evals"] - 0.5)) < 1e-12
    assert np.max(res["resid"]) <= 1e-9


def test_start_block_given(torch):
    A = I.laplacian_2d(30)
    mu = lap1d(30)
    exact = np.sort((mu[:, None] + mu[None, :]).ravel())
    exact = exact[(exact >= 1.0) & (exact <= 1.6)]
    dA = flp.DeviceCsr.from_host(A)
    start = I.random_block(A.n, 4, seed=9)
    res = flp.flp_solve(dA, 1.0, 1.6, block=4, start=start)
    check_against(res, exact)


@pytest.mark.parametrize("case", ["wells13", "uniform7"])
def test_fp32_filter_with_fp64_polish(torch, case):
    """FP32 filter recurrence, FP64 Lanczos/Rayleigh-Ritz and FP64 polish
    sweeps: same contract as the FP64 path (exact count, 1e-10 relative
    eigenvalues, residuals <= 1e-9)."""
    if case == "wells13":
        N = 15
        A = I.laplacian_3d_13pt(N, I.gaussian_wells(N, I.BASE_SEED + 3))
        block, i0, i1 = 16, 10, 69
    else:
        N = 16
        A = I.laplacian_3d(N, I.uniform_potential(N, I.BASE_SEED + 2))
        block, i0, i1 = 8, 0, 49
    lam_all = np.linalg.eigvalsh(A.to_dense())
    alpha = lam_all[0] - 1.0 if i0 == 0 else 0.5 * (lam_all[i0 - 1] + lam_all[i0])
    beta = 0.5 * (lam_all[i1] + lam_all[i1 + 1])
    dA = flp.DeviceCsr.from_host(A, with_fp32=True)
    res = flp.flp_solve(dA, alpha, beta, block=block, seed=5, prec=flp.FLP_PREC_FP32_FILTER)
    want, V = O.dense_eigs_in_interval(A, alpha, beta)
    check_against(res, want, V, anorm=np.max(np.abs(lam_all)))
    assert res["stats"]["polish_sweeps"] >= 1


def test_fp32_and_fp64_agree(torch):
    N = 14
    A = I.laplacian_3d(N, I.uniform_potential(N, 77))
    lam_all = np.linalg.eigvalsh(A.to_dense())
    alpha = 0.5 * (lam_all[29] + lam_all[30])
    beta = 0.5 * (lam_all[79] + lam_all[80])
    dA = flp.DeviceCsr.from_host(A)
    r64 = flp.flp_solve(dA, alpha, beta, block=8, seed=1)
    r32 = flp.flp_solve(dA, alpha, beta, block=8, seed=1, prec=flp.FLP_PREC_FP32_FILTER)
    assert r64["count"] == r32["count"] == 50
    assert np.max(np.abs(r64["evals"] - r32["evals"]) / np.abs(r64["evals"])) <= 1e-10
    assert max(np.max(r64["resid"]), np.max(r32["resid"])) <= 1e-9


def test_full_size_lap3d7_100_against_oracle_reference(torch):
    """The benchmark's solve at full size (n = 1e6, block 8, degree 100):
    the 104 eigenvalues the oracle found in [0, beta] (tests/golden, made by
    the oracle only), exact count, 1e-10 relative, residuals <= 1e-9."""
    import json
    import os
    from .conftest import GOLDEN
    with open(os.path.join(GOLDEN, "c2_lap3d7_100_U01.json")) as f:
        ref = json.load(f)
    w = I.workload_c2(100)
    dA = flp.DeviceCsr.from_host(w["A"])
    for prec in (flp.FLP_PREC_FP64, flp.FLP_PREC_FP32_FILTER):
        res = flp.flp_solve(dA, ref["alpha"], ref["beta"], block=8, degree=100, seed=7, prec=prec,
                            want_vectors=False)
        want = np.asarray(ref["evals"])
        assert res["count"] == ref["count"] == len(want)
        assert np.max(np.abs(np.sort(res["evals"]) - want) / want) <= 1e-10
        assert np.max(res["resid"]) <= 1e-9


def test_symmetry_check(torch):
    """The opt-in O(nnz) check: symmetric inputs pass; a perturbed value or a
    missing transpose entry is FLP_E_NOTSYM, also through flp_solve."""
    A = I.laplacian_3d(8, I.uniform_potential(8, 3))
    assert flp.flp_check_symmetric(flp.DeviceCsr.from_host(A))
    B = I.Csr(A.n, A.rowptr.copy(), A.colind.copy(), A.val.copy())
    p = int(B.rowptr[10]) + 1                       # an off-diagonal entry of row 10
    B.val[p] += 1e-6
    dB = flp.DeviceCsr.from_host(B)
    assert not flp.flp_check_symmetric(dB)
    assert flp.flp_check_symmetric(dB, tol=1e-5)      # within a relative 1e-5
    with pytest.raises(flp.FlpError) as e:
        flp.flp_solve(dB, 1.0, 2.0, block=2, sym_tol=0.0)
    assert e.value.code == flp.FLP_E_NOTSYM
    r = flp.flp_solve(flp.DeviceCsr.from_host(A), 1.0, 1.5, block=2, sym_tol=0.0, want_vectors=False)
    assert r["count"] > 0
    # a stored a_ij whose a_ji is missing
    dense = A.to_dense()
    dense[3, 200] = -0.5                             # no (200, 3) partner
    C = I.dense_to_csr(dense)
    assert not flp.flp_check_symmetric(flp.DeviceCsr.from_host(C))


def test_custom_allocator(torch):
    """flp_set_allocator: every device allocation of a solve and of a batch
    goes through the caller's functions (torch's caching allocator here),
    every one comes back, and the results are those of hipMalloc memory."""
    w = I.workload_c1()
    A = w["A"]
    dA = flp.DeviceCsr.from_host(A)
    ref = flp.flp_solve(dA, 0.5, 1.0, block=2, degree=50, seed=3)
    bref, _ = flp.flp_solve_batch([dA, dA], [0.5, 1.0], [1.0, 1.5], block=2, degree=50, seeds=[3, 4])
    counts = {"alloc": 0, "free": 0}
    alloc0, free0 = flp.torch_allocator()

    def alloc(n):
        counts["alloc"] += 1
        return alloc0(n)

    def free(p):
        counts["free"] += 1
        free0(p)

    flp.flp_release_workspace()
    flp.flp_set_allocator(alloc, free)
    try:
        got = flp.flp_solve(dA, 0.5, 1.0, block=2, degree=50, seed=3)
        bres, _ = flp.flp_solve_batch([dA, dA], [0.5, 1.0], [1.0, 1.5], block=2, degree=50, seeds=[3, 4])
        flp.flp_release_workspace()
    finally:
        flp.flp_set_allocator()
    torch.cuda.synchronize()
    assert counts["alloc"] > 0
    assert counts["free"] == counts["alloc"]
    assert got["count"] == ref["count"]
    assert np.array_equal(got["evals"], ref["evals"])
    for a, b in zip(bres, bref):                     # the batch against itself on hipMalloc memory
        assert a["count"] == b["count"] and np.array_equal(a["evals"], b["evals"])
    # and the batch agrees with the single solve to the parity tolerance
    assert np.max(np.abs(bres[0]["evals"] - ref["evals"]) / np.abs(ref["evals"])) <= 1e-12


def test_full_size_kronecker_13pt_120(torch):
    """The c3 shape at full size (13-point stencil on 120^3, n = 1.728e6,
    block 16) with a separable potential, so the spectrum is every sum of the
    three 1D operators' eigenvalues (dense eigh of 120 x 120): about 300
    eigenvalues above the lowest 20, both filter precisions, exact count,
    1e-10 relative, residuals <= 1e-9."""
    N = 120
    field, vx, vy, vz = I.separable_potential(N, seed=1203)
    A = I.laplacian_3d_13pt(N, field)
    st = {0: I.FOURTH_ORDER_1D[0], 1: I.FOURTH_ORDER_1D[1], 2: I.FOURTH_ORDER_1D[2]}

    def one_d(v):
        T = np.zeros((N, N))
        for d, cf in st.items():
            idx = np.arange(N - d)
            T[idx, idx + d] = cf
            T[idx + d, idx] = cf
        np.fill_diagonal(T, st[0] + v)
        return np.linalg.eigvalsh(T)

    a, b, c = one_d(vx), one_d(vy), one_d(vz)
    lo = np.sort((a[:, None, None] + b[None, :, None] + c[None, None, :]).ravel())[:2000]
    # endpoints in the widest gaps near eigenvalues 20 and 320
    g0 = 15 + int(np.argmax(np.diff(lo[15:26])))
    g1 = 315 + int(np.argmax(np.diff(lo[315:326])))
    alpha = 0.5 * (lo[g0] + lo[g0 + 1])
    beta = 0.5 * (lo[g1] + lo[g1 + 1])
    want = lo[g0 + 1:g1 + 1]
    dA = flp.DeviceCsr.from_host(A, with_fp32=True)
    for prec in (flp.FLP_PREC_FP64, flp.FLP_PREC_FP32_FILTER):
        res = flp.flp_solve(dA, alpha, beta, block=16, degree=100, seed=11, prec=prec, want_vectors=False)
        assert res["count"] == len(want), (prec, res["count"], len(want))
        assert np.max(np.abs(np.sort(res["evals"]) - want) / np.abs(want)) <= 1e-10
        assert np.max(res["resid"]) <= 1e-9
