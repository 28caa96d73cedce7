"""Full-size solves against the oracle's references (tests/golden, written
by tests/golden/make_references.py, which calls only oracle/): the 120^3
Hamiltonian with 16 Gaussian wells (an interior window of 311 eigenvalues),
the 64 problems of the batched workload and the first 32 requests of the
serving stream.  Every solve must find the oracle's count, every eigenvalue
within 1e-10 relative, with residuals <= 1e-9 (Section 4, Table 2), in both
filter precisions."""
import json
import os

import numpy as np
import pytest

from paper_2409_15053_amd import flp
from paper_2409_15053_amd import inputs as I

from .conftest import GOLDEN

pytestmark = pytest.mark.gpu

PRECS = [flp.FLP_PREC_FP64, flp.FLP_PREC_FP32_FILTER]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a visible MI355X"
    flp.load()
    return t


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def check(res, want, what):
    assert res["converged"], what
    want = np.asarray(want)
    assert res["count"] == len(want), (what, res["count"], len(want))
    if len(want):
        got = np.sort(np.asarray(res["evals"]))
        assert np.max(np.abs(got - want) / np.abs(want)) <= 1e-10, what
        assert np.max(res["resid"]) <= 1e-9, what


@pytest.mark.parametrize("prec", PRECS)
def test_c3_wells_against_oracle_reference(torch, prec):
    """n = 1.728e6, 22.2e6 nonzeros, block 16, degree 100, the oracle's
    interval (endpoints at gap midpoints near the Weyl levels of 20 and 320
    eigenvalues): the 311 eigenvalues of the oracle's solve."""
    ref = golden("c3_lap3d13_120_wells16.json")
    w = I.workload_c3(120)
    A = w["A"]
    assert (A.n, A.nnz) == (ref["n"], ref["nnz"])
    dA = flp.DeviceCsr.from_host(A, "cuda:0", with_fp32=True)
    res = flp.flp_solve(dA, ref["alpha"], ref["beta"], block=16, degree=ref["degree"], seed=3, prec=prec,
                        want_vectors=False)
    check(res, ref["evals"], "c3")


@pytest.mark.parametrize("prec", PRECS)
def test_c4_batch64_against_oracle_reference(torch, prec):
    """The batched form on its 64 problems (3D 7-point + U[0,1) on 20^3 to
    60^3 grids, 10 to 60 eigenvalues each), block 8, one flp_solve_batch
    call: every problem's count and eigenvalues are the oracle's."""
    ref = golden("c4_batch64.json")
    fam = I.batch_family(64)
    assert [f["name"] for f in fam] == [p["name"] for p in ref["problems"]]
    dAs = [flp.DeviceCsr.from_host(I.build_batch_matrix(f), "cuda:0", with_fp32=True) for f in fam]
    res, _ = flp.flp_solve_batch(dAs, [p["alpha"] for p in ref["problems"]], [p["beta"] for p in ref["problems"]],
                                 block=8, seeds=[11 + i for i in range(len(dAs))], prec=prec, want_vectors=False)
    for r, p in zip(res, ref["problems"]):
        check(r, p["evals"], p["name"])


@pytest.mark.parametrize("prec", PRECS)
def test_c5_serve32_against_oracle_reference(torch, prec):
    """The first 32 requests of the serving stream (13-point + 16 wells on
    30^3 to 100^3 grids, up to 200 eigenvalues each, degree 60), all
    submitted at once to one server (block 16): every result's count and
    eigenvalues are the oracle's."""
    ref = golden("c5_serve32.json")
    fam = I.serve_family(32)
    assert [f["name"] for f in fam] == [p["name"] for p in ref["problems"]]
    sv = flp.Server(block=16, prec=prec, max_active=64, max_basis=2048)
    try:
        dAs, tickets = [], []
        for i, (f, p) in enumerate(zip(fam, ref["problems"])):
            A, _, _ = I.build_serve_problem(f)
            assert (A.n, A.nnz) == (p["n"], p["nnz"])
            dAs.append(flp.DeviceCsr.from_host(A, "cuda:0", with_fp32=True))
            tickets.append(sv.submit(dAs[-1], p["alpha"], p["beta"], seed=21 + i, degree=f["degree"]))
        res = [sv.wait(t) for t in tickets]
    finally:
        sv.close()
    for r, p in zip(res, ref["problems"]):
        check(r, p["evals"], p["name"])
