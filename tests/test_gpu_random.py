"""Randomised parity of flp_solve and flp_solve_batch against the dense
definition (LAPACK eigh of the same matrix): 7- and 13-point stencils with a
uniform or Gaussian-well potential on 10^3..18^3 grids, interior windows of
10..150 eigenvalues with endpoints at gap midpoints, block sizes 4, 8 and 16,
both filter precisions.  Contract: exact count, eigenvalues within 1e-10
relative, residuals <= 1e-9."""
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


def random_case(rng, nmin=12, nmax=19, cmin=20, cmax=150):
    N = int(rng.integers(nmin, nmax))
    seed = int(rng.integers(1, 10**6))
    V = I.uniform_potential(N, seed) if rng.random() < 0.5 else I.gaussian_wells(N, seed)
    A = I.laplacian_3d(N, V) if rng.random() < 0.5 else I.laplacian_3d_13pt(N, V)
    lam = np.linalg.eigvalsh(A.to_dense())
    cnt = int(rng.integers(cmin, cmax))
    i0 = int(rng.integers(0, min(len(lam) - cnt - 2, 400)))
    alpha = lam[0] - 0.5 if i0 == 0 else 0.5 * (lam[i0 - 1] + lam[i0])
    beta = 0.5 * (lam[i0 + cnt - 1] + lam[i0 + cnt])
    return A, alpha, beta, lam[(lam >= alpha) & (lam <= beta)]


def meets_contract(res, want):
    assert res["count"] == len(want)
    got = np.sort(res["evals"])
    assert np.max(np.abs(got - want) / np.abs(want)) <= 1e-10
    assert np.max(res["resid"]) <= 1e-9


@pytest.mark.parametrize("seed", range(6))
def test_random_single_solves(torch, seed):
    rng = np.random.default_rng(1000 + seed)
    A, alpha, beta, want = random_case(rng)
    r = int(rng.choice([4, 8, 16]))
    dA = flp.DeviceCsr.from_host(A, with_fp32=True)
    for prec in (flp.FLP_PREC_FP64, flp.FLP_PREC_FP32_FILTER):
        res = flp.flp_solve(dA, alpha, beta, block=r, seed=int(rng.integers(0, 10**6)), prec=prec,
                            want_vectors=False)
        assert res["converged"]
        meets_contract(res, want)


@pytest.mark.parametrize("seed", range(2))
def test_random_batches(torch, seed):
    rng = np.random.default_rng(2000 + seed)
    r = int(rng.choice([4, 8, 16]))
    prec = flp.FLP_PREC_FP32_FILTER if seed == 0 else flp.FLP_PREC_FP64
    cases = [random_case(rng, 10, 18, 10, 120) for _ in range(8)]
    dAs = [flp.DeviceCsr.from_host(c[0], with_fp32=True) for c in cases]
    res, _ = flp.flp_solve_batch(dAs, [c[1] for c in cases], [c[2] for c in cases], block=r,
                                 seeds=[int(x) for x in rng.integers(0, 10**6, len(cases))], prec=prec,
                                 want_vectors=False)
    for c, rr in zip(cases, res):
        meets_contract(rr, c[3])
