"""Serving form (continuous batching): requests submitted while others run
are admitted into the active set, and each result is the same alone and
in the mix (same count; eigenvalues within 1e-10 relative; residuals
<= 1e-9 against the dense definition)."""
import time

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


def family(grids, seed0, counts):
    out = []
    for i, (N, cnt) in enumerate(zip(grids, counts)):
        A = I.laplacian_3d(N, I.uniform_potential(N, seed0 + i))
        lam = np.linalg.eigvalsh(A.to_dense())
        out.append((A, lam[0] - 0.5, 0.5 * (lam[cnt - 1] + lam[cnt])))
    return out


@pytest.mark.parametrize("prec", [flp.FLP_PREC_FP32_FILTER, flp.FLP_PREC_FP64])
def test_server_staggered_arrivals_match_alone(torch, prec):
    cases = family([8, 9, 10, 11, 12, 13, 9, 10], 4000, [10, 12, 14, 16, 18, 20, 22, 24])
    dAs = [flp.DeviceCsr.from_host(A, with_fp32=True) for A, *_ in cases]
    sv = flp.Server(block=8, prec=prec, max_active=4)
    tickets = []
    try:
        # first wave, then more requests while the first ones run
        for i in range(4):
            tickets.append(sv.submit(dAs[i], cases[i][1], cases[i][2], seed=100 + i))
        time.sleep(0.05)
        for i in range(4, 8):
            tickets.append(sv.submit(dAs[i], cases[i][1], cases[i][2], seed=100 + i))
        got = [sv.wait(t) for t in tickets]
        st = sv.stats()
    finally:
        sv.close()
    assert st["solves"] == 8 and st["block_steps"] > 0
    assert st["graph_captures"] >= 2  # the active set changed while running
    for i, (A, alpha, beta) in enumerate(cases):
        want, _ = O.dense_eigs_in_interval(A, alpha, beta)
        r = got[i]
        assert r["count"] == len(want)
        assert np.max(np.abs(np.sort(r["evals"]) - want) / np.abs(want)) <= 1e-10
        assert np.max(r["resid"]) <= 1e-9
        assert r["stats"]["t_total"] > 0  # latency recorded
        alone = flp.flp_solve(dAs[i], alpha, beta, block=8, seed=100 + i, prec=prec, max_basis=1024)
        assert alone["count"] == r["count"]
        assert np.max(np.abs(alone["evals"] - r["evals"]) / np.abs(r["evals"])) <= 1e-10


def test_server_poll_pending_and_errors(torch):
    A = I.laplacian_3d(10, I.uniform_potential(10, 1))
    lam = np.linalg.eigvalsh(A.to_dense())
    dA = flp.DeviceCsr.from_host(A)
    sv = flp.Server(block=4, prec=flp.FLP_PREC_FP64, max_active=2)
    try:
        t = sv.submit(dA, lam[0] - 0.1, 0.5 * (lam[11] + lam[12]), seed=1)
        r = None
        for _ in range(2000):
            r = sv.poll(t)
            if r is not None:
                break
            time.sleep(0.005)
        assert r is not None and r["count"] == 12
        bad = sv.submit(dA, 50.0, 60.0, seed=2)  # outside the spectrum
        with pytest.raises(flp.FlpError) as ei:
            sv.wait(bad)
        assert ei.value.code == flp.FLP_E_INTERVAL
        assert "does not meet" in flp.load().flp_last_error().decode()
    finally:
        sv.close()


def test_server_cancel(torch):
    """Cancelled requests report FLP_E_CANCELLED (a queued one at once, a
    running one at a block-step boundary); the others complete correctly and
    the server keeps serving."""
    cases = [I.laplacian_3d(N, I.uniform_potential(N, 50 + N)) for N in (10, 11, 12, 13, 14, 12)]
    sv = flp.Server(block=4, prec=flp.FLP_PREC_FP64, max_active=2, max_basis=600)
    try:
        dAs = [flp.DeviceCsr.from_host(A) for A in cases]
        tickets = []
        for i, A in enumerate(cases):
            lam = np.linalg.eigvalsh(A.to_dense())
            tickets.append((sv.submit(dAs[i], lam[0] - 0.5, 0.5 * (lam[29] + lam[30]), seed=i), A, lam))
        sv.cancel(tickets[5][0])                     # queued behind four others
        sv.cancel(tickets[0][0])                     # probably running
        cancelled = 0
        for t, A, lam in tickets:
            try:
                r = sv.wait(t)
            except flp.FlpError as e:
                assert e.code == flp.FLP_E_CANCELLED
                cancelled += 1
                continue
            want = lam[(lam >= lam[0] - 0.5) & (lam <= 0.5 * (lam[29] + lam[30]))]
            assert r["count"] == len(want) == 30
            assert np.max(np.abs(np.sort(r["evals"]) - want) / np.abs(want)) <= 1e-10
        assert cancelled >= 1
        # still serving after cancellations
        lam = np.linalg.eigvalsh(cases[1].to_dense())
        r = sv.wait(sv.submit(dAs[1], lam[0] - 0.5, 0.5 * (lam[19] + lam[20]), seed=9))
        assert r["count"] == 20
        with pytest.raises(flp.FlpError):
            sv.cancel(123456789)                     # unknown ticket
    finally:
        sv.close()


@pytest.mark.parametrize("prec", [flp.FLP_PREC_FP32_FILTER, flp.FLP_PREC_FP64])
def test_server_admission_by_memory_footprint(torch, prec):
    """A device-memory budget that holds the admission footprint of two
    requests at a time: six requests submitted together are admitted two
    at a time as earlier ones complete (the queue's head waits for memory),
    and every result is still exact against the dense definition and the
    same as the request solved alone.  With the default budget all six are
    admitted at once."""
    cases = family([12] * 6, 7100, [12, 16, 20, 24, 14, 18])  # equal sizes: equal footprints
    dAs = [flp.DeviceCsr.from_host(A, with_fp32=True) for A, *_ in cases]
    probe = flp.Server(block=8, prec=prec, max_active=8, max_basis=512)
    try:
        fps = [probe.footprint(dA) for dA in dAs]
    finally:
        probe.close()
    assert all(f > 0 for f in fps)
    # the footprint covers at least the basis of max_basis columns
    assert all(f >= min(512, A.n) * A.n * 8 for f, (A, *_ ) in zip(fps, cases))
    assert max(fps) == min(fps)
    budget = 2.5 * fps[0]  # room for two admissions, not three
    sv = flp.Server(block=8, prec=prec, max_active=8, max_basis=512, mem_budget=budget)
    try:
        tickets = [sv.submit(dAs[i], a, b, seed=60 + i) for i, (A, a, b) in enumerate(cases)]
        got = [sv.wait(t) for t in tickets]
        st = sv.stats()
    finally:
        sv.close()
    assert st["mem_budget"] == pytest.approx(budget, rel=1e-12)
    assert st["peak_active"] <= 2
    assert st["admission_waits"] >= 1
    assert st["peak_mem_reserved"] > 0
    for i, (A, alpha, beta) in enumerate(cases):
        want, _ = O.dense_eigs_in_interval(A, alpha, beta)
        r = got[i]
        assert r["count"] == len(want)
        assert np.max(np.abs(np.sort(r["evals"]) - want) / np.abs(want)) <= 1e-10
        assert np.max(r["resid"]) <= 1e-9
        alone = flp.flp_solve(dAs[i], alpha, beta, block=8, seed=60 + i, prec=prec, max_basis=512,
                              want_vectors=False)
        assert alone["count"] == r["count"]
        assert np.max(np.abs(alone["evals"] - r["evals"]) / np.abs(r["evals"])) <= 1e-10
    # the default budget (70 % of free device memory) admits all of them at once
    sv = flp.Server(block=8, prec=prec, max_active=8, max_basis=512)
    try:
        tickets = [sv.submit(dAs[i], a, b, seed=60 + i) for i, (A, a, b) in enumerate(cases)]
        got2 = [sv.wait(t) for t in tickets]
        st2 = sv.stats()
    finally:
        sv.close()
    assert st2["admission_waits"] == 0 and st2["peak_active"] >= 2
    for r, r2 in zip(got, got2):
        assert r["count"] == r2["count"]
