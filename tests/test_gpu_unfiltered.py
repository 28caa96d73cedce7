"""Unfiltered block Lanczos (p(Ahat) = Ahat), the variant that Section 4.1
sets beside the filtered procedure after Table 3: the same result contract
(exact count, eigenvalues within 1e-10 relative, residuals <= 1e-9) against
dense eigh and the Kronecker-sum spectrum, and the basis it needs compared
with the filtered solve's on the same problem."""
import ctypes

import numpy as np
import pytest

from paper_2409_15053_amd import flp
from paper_2409_15053_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a visible MI355X"
    flp.load()
    return t


def contract(res, want):
    assert res["converged"]
    assert res["count"] == len(want), (res["count"], len(want))
    got = np.sort(res["evals"])
    assert np.max(np.abs(got - want) / np.abs(want)) <= 1e-10
    assert np.max(res["resid"]) <= 1e-9
    X = res["evecs"].cpu().numpy()
    assert np.max(np.abs(X.T @ X - np.eye(X.shape[1]))) < 1e-10


def window(lam, i0, cnt):
    alpha = lam[0] - 0.5 if i0 == 0 else 0.5 * (lam[i0 - 1] + lam[i0])
    beta = 0.5 * (lam[i0 + cnt - 1] + lam[i0 + cnt])
    return alpha, beta, lam[i0:i0 + cnt]


def test_unfiltered_c1_laplacian_2d(torch):
    """The 40 x 40 Laplacian on [0.5, 1.0]: 69 eigenvalues, 33 of them double
    (closed form); a block of 4 resolves the multiplicity."""
    N = 40
    A = I.laplacian_2d(N)
    j = np.arange(1, N + 1)
    mu = 4 * np.sin(j * np.pi / (2 * (N + 1))) ** 2
    lam = np.sort((mu[:, None] + mu[None, :]).ravel())
    want = lam[(lam >= 0.5) & (lam <= 1.0)]
    assert len(want) == 69
    res = flp.flp_solve(flp.DeviceCsr.from_host(A), 0.5, 1.0, block=4, seed=3, unfiltered=True)
    contract(res, want)
    assert res["degree"] == 1


@pytest.mark.parametrize("i0,cnt,block", [(0, 40, 8), (150, 30, 8), (60, 25, 4)])
def test_unfiltered_windows_dense(torch, i0, cnt, block):
    N = 14
    A = I.laplacian_3d(N, I.uniform_potential(N, seed=7))
    lam = np.linalg.eigvalsh(A.to_dense())
    alpha, beta, want = window(lam, i0, cnt)
    res = flp.flp_solve(flp.DeviceCsr.from_host(A), alpha, beta, block=block, seed=11, unfiltered=True)
    contract(res, want)
    st = res["stats"]
    assert st["mv"] >= block * st["iters"]


def test_unfiltered_kronecker_40(torch):
    """64000 unknowns with a separable potential: the exact spectrum is the
    Kronecker sum of three 1D spectra; the lowest 30 eigenvalues above the
    bottom five."""
    N = 40
    field, vx, vy, vz = I.separable_potential(N, seed=23)
    A = I.laplacian_3d(N, field)

    def one_d(v):
        T = np.diag(2.0 + v) - np.eye(N, k=1) - np.eye(N, k=-1)
        return np.linalg.eigvalsh(T)

    a, b, c = one_d(vx), one_d(vy), one_d(vz)
    spec = np.sort((a[:, None, None] + b[None, :, None] + c[None, None, :]).ravel())
    alpha, beta, want = window(spec, 5, 30)
    res = flp.flp_solve(flp.DeviceCsr.from_host(A), alpha, beta, block=8, seed=5, unfiltered=True)
    contract(res, want)


def test_unfiltered_needs_a_larger_basis(torch):
    """The memory point of Section 4.1: for an interior window the
    unfiltered basis is several times the filtered one (which trades it for
    filter products)."""
    N = 16
    A = I.laplacian_3d(N, I.uniform_potential(N, seed=9))
    lam = np.linalg.eigvalsh(A.to_dense())
    alpha, beta, want = window(lam, 400, 30)
    dA = flp.DeviceCsr.from_host(A)
    plain = flp.flp_solve(dA, alpha, beta, block=8, seed=2, unfiltered=True, want_vectors=False)
    filt = flp.flp_solve(dA, alpha, beta, block=8, seed=2, want_vectors=False)
    for res in (plain, filt):
        assert res["count"] == len(want) and np.max(res["resid"]) <= 1e-9
    assert plain["stats"]["basis_cols"] > 2 * filt["stats"]["basis_cols"]
    assert plain["stats"]["mv"] < filt["stats"]["mv"]


def test_unfiltered_rejected_outside_flp_solve(torch):
    A = I.laplacian_3d(10)
    dA = flp.DeviceCsr.from_host(A, with_fp32=True)
    with pytest.raises(flp.FlpError):
        flp.flp_solve(dA, 0.5, 0.9, block=4, unfiltered=True, prec=flp.FLP_PREC_FP32_FILTER)
    lib = flp.load()
    o = flp.default_opts()
    o.block = 4
    o.unfiltered = 1
    opts = (flp.FlpOptsC * 1)()
    opts[0] = o
    arr = (ctypes.POINTER(flp.FlpCsrC) * 1)(ctypes.pointer(dA.c))
    al = np.array([0.5])
    be = np.array([0.9])
    res = (ctypes.POINTER(flp.FlpResultC) * 1)()
    codes = np.zeros(1, dtype=np.int32)
    bst = flp.FlpBatchStatsC()
    rc = lib.flp_solve_batch(1, ctypes.cast(arr, ctypes.c_void_p), flp._np_ptr(al), flp._np_ptr(be),
                             ctypes.cast(opts, ctypes.c_void_p), 0, ctypes.cast(res, ctypes.c_void_p),
                             flp._np_ptr(codes), ctypes.byref(bst))
    assert rc == flp.FLP_E_ARG
    one = ctypes.POINTER(flp.FlpResultC)()
    rc = lib.flp_solve_sliced(ctypes.byref(dA.c), 0.5, 0.9, 2, ctypes.byref(o), ctypes.byref(one))
    assert rc == flp.FLP_E_ARG


def test_whole_spectrum(torch):
    """An interval around the whole spectrum: the ideal filter is the
    constant 1, so the filtered solve refuses it; unfiltered Lanczos returns
    every eigenpair once the basis spans the space (n a multiple of r)."""
    A = I.random_sym(200, 0.05, seed=3, diag_shift=10.0)  # eigenvalues away from 0
    lam = np.linalg.eigvalsh(A.to_dense())
    dA = flp.DeviceCsr.from_host(A)
    with pytest.raises(flp.FlpError) as e:
        flp.flp_solve(dA, lam[0] - 1.0, lam[-1] + 1.0, block=4)
    assert e.value.code == flp.FLP_E_ARG
    res = flp.flp_solve(dA, lam[0] - 1.0, lam[-1] + 1.0, block=4, seed=1, unfiltered=True)
    contract(res, lam)
