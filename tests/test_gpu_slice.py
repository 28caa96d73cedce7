"""Spectrum slicing on one GPU (flp_solve_sliced, through the C ABI): the
merged result of several slices solved as one batch must be the result of
the whole interval — exact count against dense eigh, eigenvalues within
1e-10 relative, residuals <= 1e-9, eigenvectors by principal angles per
cluster (||sin Theta|| <= 1e-7) — and must equal the unsliced solve's
eigenvalues."""
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


def principal_sin(X, Y):
    """Largest sine of the principal angles between span(X) and span(Y)."""
    qx, _ = np.linalg.qr(X)
    qy, _ = np.linalg.qr(Y)
    s = np.linalg.svd(qx.T @ qy, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - np.min(s) ** 2)))


def check(res, A, alpha, beta, anorm):
    lam, V = O.dense_eigs_in_interval(A, alpha, beta)
    assert res["count"] == len(lam), (res["count"], len(lam))
    got = res["evals"]
    assert np.all(np.diff(got) >= 0)  # ascending
    assert np.max(np.abs(got - lam) / np.abs(lam)) <= 1e-10
    assert np.max(res["resid"]) <= 1e-9
    X = res["evecs"].cpu().numpy()
    assert np.max(np.abs(X.T @ X - np.eye(res["count"]))) <= 1e-8
    # eigenvectors, cluster by cluster
    i = 0
    while i < len(lam):
        j = i + 1
        while j < len(lam) and lam[j] - lam[j - 1] < 1e-8 * anorm:
            j += 1
        assert principal_sin(X[:, i:j], V[:, i:j]) <= 1e-7
        i = j


@pytest.mark.parametrize("nslices", [1, 2, 3, 5])
@pytest.mark.parametrize("prec", [flp.FLP_PREC_FP64, flp.FLP_PREC_FP32_FILTER])
def test_sliced_equals_whole_interval(torch, nslices, prec):
    A = I.laplacian_3d(14, I.uniform_potential(14, 77))  # n = 2744
    lam_all = np.linalg.eigvalsh(A.to_dense())
    alpha = lam_all[0] - 0.3
    beta = 0.5 * (lam_all[139] + lam_all[140])  # 140 eigenvalues
    dA = flp.DeviceCsr.from_host(A, with_fp32=True)
    res = flp.flp_solve_sliced(dA, alpha, beta, nslices, block=8, seed=5, prec=prec)
    assert res["converged"]
    check(res, A, alpha, beta, anorm=max(abs(lam_all[0]), abs(lam_all[-1])))
    whole = flp.flp_solve(dA, alpha, beta, block=8, seed=5, prec=prec, want_vectors=False)
    assert whole["count"] == res["count"]
    assert np.max(np.abs(np.sort(whole["evals"]) - res["evals"]) / np.abs(res["evals"])) <= 1e-10


def test_sliced_interior_interval_with_multiplicities(torch):
    """2D Laplacian (doubly degenerate eigenvalues) on an interior interval."""
    A = I.laplacian_2d(30)
    lam_all = np.linalg.eigvalsh(A.to_dense())
    alpha, beta = 1.001, 1.9  # interior, away from eigenvalues
    assert np.min(np.abs(lam_all - alpha)) > 1e-4 and np.min(np.abs(lam_all - beta)) > 1e-4
    dA = flp.DeviceCsr.from_host(A)
    res = flp.flp_solve_sliced(dA, alpha, beta, 4, block=4, seed=9)
    check(res, A, alpha, beta, anorm=8.0)


def test_sliced_argument_errors(torch):
    A = I.laplacian_2d(10)
    dA = flp.DeviceCsr.from_host(A)
    for ns in (0, 257):
        with pytest.raises(flp.FlpError) as e:
            flp.flp_solve_sliced(dA, 0.5, 1.0, ns, block=2)
        assert e.value.code == flp.FLP_E_ARG
    with pytest.raises(flp.FlpError) as e:
        flp.flp_solve_sliced(dA, 20.0, 30.0, 2, block=2)
    assert e.value.code == flp.FLP_E_INTERVAL
