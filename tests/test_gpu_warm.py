"""Warm start for a sequence of related problems (flp_opts.warm): the
eigenvectors of one matrix start the solve of the next, slightly changed
one, as in a self-consistent-field loop (Section 1).  Every result must
meet the single-solve contract against the dense definition (exact count,
eigenvalues within 1e-10 relative, residuals <= 1e-9), whether the warm
start certified it or fell back to the cold solve."""
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


N = 14


def scf_matrix(delta, seed=3):
    """7-point Laplacian N^3 + U[0,1) potential + delta * U[-1,1) change."""
    base = I.uniform_potential(N, 9100)
    change = 2.0 * I.rng(seed).random(N ** 3) - 1.0
    return I.laplacian_3d(N, base + delta * change)


def interval():
    lam = np.linalg.eigvalsh(scf_matrix(0.0).to_dense())
    return lam[0] - 0.5, 0.5 * (lam[39] + lam[40])


def check(res, A, alpha, beta):
    want, _ = O.dense_eigs_in_interval(A, alpha, beta)
    assert res["count"] == len(want)
    assert np.max(np.abs(np.sort(res["evals"]) - want) / np.abs(want)) <= 1e-10
    assert np.max(res["resid"]) <= 1e-9


@pytest.mark.parametrize("prec", [flp.FLP_PREC_FP64, flp.FLP_PREC_FP32_FILTER])
def test_scf_sequence_warm_started(torch, prec):
    """delta = 0 (cold), then 1e-3, 1e-2, 5e-2 changes of the potential, each
    solve warm-started from the previous result's eigenvectors."""
    alpha, beta = interval()
    A0 = scf_matrix(0.0)
    d0 = flp.DeviceCsr.from_host(A0, with_fp32=True)
    prev = flp.flp_solve(d0, alpha, beta, block=4, seed=1, prec=prec)
    check(prev, A0, alpha, beta)
    assert prev["stats"]["warm_status"] == 0
    for delta in (1e-3, 1e-2, 5e-2):
        A = scf_matrix(delta)
        dA = flp.DeviceCsr.from_host(A, with_fp32=True)
        res = flp.flp_solve(dA, alpha, beta, block=4, seed=2, prec=prec, warm=prev["evecs"])
        print(f"delta={delta}: warm_status={res['stats']['warm_status']} sweeps={res['stats']['warm_sweeps']} "
              f"count={res['count']}", flush=True)
        check(res, A, alpha, beta)
        if delta <= 1e-2:
            assert res["stats"]["warm_status"] == 1  # certified by the warm start itself
        assert res["stats"]["warm_status"] in (1, 2)
        prev = res


def test_warm_start_from_unrelated_vectors(torch):
    """A warm block that spans the wrong space (random vectors, too few of
    them): the result is still exact (certified or by the fallback)."""
    alpha, beta = interval()
    A = scf_matrix(1e-2)
    dA = flp.DeviceCsr.from_host(A)
    junk = torch.randn((A.n, 10), dtype=torch.float64, device="cuda:0")
    res = flp.flp_solve(dA, alpha, beta, block=4, seed=5, warm=junk)
    check(res, A, alpha, beta)
    assert res["stats"]["warm_status"] in (1, 2)


def test_warm_start_identical_matrix_is_quick(torch):
    """Warm-starting the same matrix from its own eigenvectors certifies the
    result by the warm start itself (the pairs inside are exact from the
    first Rayleigh-Ritz; the sweeps settle the random guards past the
    filter's transition band) and reproduces the cold eigenvalues."""
    alpha, beta = interval()
    A = scf_matrix(0.0)
    dA = flp.DeviceCsr.from_host(A)
    cold = flp.flp_solve(dA, alpha, beta, block=4, seed=1)
    res = flp.flp_solve(dA, alpha, beta, block=4, seed=3, warm=cold["evecs"])
    check(res, A, alpha, beta)
    assert res["stats"]["warm_status"] == 1 and 2 <= res["stats"]["warm_sweeps"] <= 16
    assert np.max(np.abs(res["evals"] - cold["evals"]) / np.abs(cold["evals"])) <= 1e-12


def test_warm_start_argument_errors(torch):
    A = scf_matrix(0.0)
    dA = flp.DeviceCsr.from_host(A)
    lib = flp.load()
    import ctypes
    o = flp.default_opts()
    o.block = 4
    o.warm_count = 3  # a count without a block
    res = ctypes.POINTER(flp.FlpResultC)()
    assert lib.flp_solve(ctypes.byref(dA.c), 0.1, 0.5, ctypes.byref(o), ctypes.byref(res)) == flp.FLP_E_ARG
    # the batched form takes no warm start
    junk = torch.randn((A.n, 4), dtype=torch.float64, device="cuda:0")
    o.warm = junk.data_ptr()
    arr = (ctypes.POINTER(flp.FlpCsrC) * 1)(ctypes.pointer(dA.c))
    al, be = np.array([0.1]), np.array([0.5])
    one = (ctypes.POINTER(flp.FlpResultC) * 1)()
    codes = np.zeros(1, dtype=np.int32)
    rc = lib.flp_solve_batch(1, ctypes.cast(arr, ctypes.c_void_p), al.ctypes.data_as(ctypes.c_void_p),
                             be.ctypes.data_as(ctypes.c_void_p), ctypes.cast(ctypes.pointer(o), ctypes.c_void_p), 0,
                             ctypes.cast(one, ctypes.c_void_p), codes.ctypes.data_as(ctypes.c_void_p), None)
    assert rc == flp.FLP_E_ARG or int(codes[0]) == flp.FLP_E_ARG
    if one[0]:
        lib.flp_result_free(one[0])
