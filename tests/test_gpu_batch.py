"""Batched form (segmented filter launches over many solves, HIP graph
replay): every result meets the single-solve contract against the oracle's
dense definition, each solve gives the same result alone and inside the
mix, and graph replay reproduces eager launches exactly."""
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


def small_family(grids, seed0, counts):
    """3D 7-point Laplacian + U[0,1) potential on several grids, each with a
    low-end interval holding counts[i] eigenvalues (endpoints at gap
    midpoints of the dense spectrum)."""
    cases = []
    for i, (N, cnt) in enumerate(zip(grids, counts)):
        A = I.laplacian_3d(N, I.uniform_potential(N, seed0 + i))
        lam = np.linalg.eigvalsh(A.to_dense())
        alpha = lam[0] - 0.5
        beta = 0.5 * (lam[cnt - 1] + lam[cnt])
        cases.append((A, alpha, beta, lam))
    return cases


def check(res, A, alpha, beta, lam_all):
    want, _ = O.dense_eigs_in_interval(A, alpha, beta)
    assert res["count"] == len(want)
    got = np.sort(res["evals"])
    assert np.max(np.abs(got - want) / np.abs(want)) <= 1e-10
    assert np.max(res["resid"]) <= 1e-9


@pytest.mark.parametrize("prec", [flp.FLP_PREC_FP64, flp.FLP_PREC_FP32_FILTER])
def test_batch_against_dense(torch, prec):
    cases = small_family([8, 9, 10, 11, 12, 13], 500, [10, 14, 18, 22, 26, 30])
    dAs = [flp.DeviceCsr.from_host(A, with_fp32=(prec == flp.FLP_PREC_FP32_FILTER)) for A, *_ in cases]
    res, st = flp.flp_solve_batch(dAs, [c[1] for c in cases], [c[2] for c in cases], block=8,
                                  seeds=list(range(1, 7)), prec=prec)
    for r, (A, alpha, beta, lam) in zip(res, cases):
        check(r, A, alpha, beta, lam)
    assert st["block_steps"] >= 30 and st["graph_captures"] >= 1
    assert st["graph_replays"] == st["block_steps"]


def test_batch_mixed_degrees_aligned(torch):
    cases = small_family([9, 10, 11], 700, [12, 16, 20])
    dAs = [flp.DeviceCsr.from_host(A) for A, *_ in cases]
    res, st = flp.flp_solve_batch(dAs, [c[1] for c in cases], [c[2] for c in cases], block=4,
                                  degree=[12, 31, 47], seeds=[3, 4, 5])
    for r, (A, alpha, beta, lam), m in zip(res, cases, [12, 31, 47]):
        assert r["degree"] == m
        check(r, A, alpha, beta, lam)
    assert st["filter_launches"] == 47 * st["block_steps"] or st["graph_captures"] > 1


def test_each_solve_same_alone_and_in_mix(torch):
    """Mix invariance: the batched result of every problem equals the
    single-solve result (same seed and options) within 1e-12 relative, with
    identical counts."""
    cases = small_family([8, 10, 12, 14], 900, [10, 20, 25, 30])
    dAs = [flp.DeviceCsr.from_host(A) for A, *_ in cases]
    seeds = [11, 12, 13, 14]
    res, _ = flp.flp_solve_batch(dAs, [c[1] for c in cases], [c[2] for c in cases], block=8, seeds=seeds)
    for i, (A, alpha, beta, lam) in enumerate(cases):
        alone = flp.flp_solve(dAs[i], alpha, beta, block=8, seed=seeds[i])
        assert alone["count"] == res[i]["count"]
        assert np.max(np.abs(alone["evals"] - res[i]["evals"]) / np.abs(alone["evals"])) <= 1e-12
        check(res[i], A, alpha, beta, lam)


def test_graph_replay_matches_eager(torch):
    """Each block step's filter launches are replayed from a HIP graph; with
    eager host work and synchronisations between replays, every replay must
    reproduce the eager launches: the results agree bit for bit."""
    cases = small_family([9, 11, 13], 1200, [12, 18, 24])
    dAs = [flp.DeviceCsr.from_host(A) for A, *_ in cases]
    args = ([c[1] for c in cases], [c[2] for c in cases])
    rg, sg = flp.flp_solve_batch(dAs, *args, block=8, seeds=[1, 2, 3], use_graph=True)
    re_, se = flp.flp_solve_batch(dAs, *args, block=8, seeds=[1, 2, 3], use_graph=False)
    assert sg["graph_replays"] >= 30 and se["graph_replays"] == 0
    for a, b in zip(rg, re_):
        assert a["count"] == b["count"]
        assert np.array_equal(a["evals"], b["evals"])
        assert np.array_equal(a["resid"], b["resid"])


def test_tuned_segmented_shape_matches_default(torch):
    """The batched engine tunes the segmented launch's shape on the largest
    active matrix; the tuned and the default shapes give the same bits."""
    cases = small_family([9, 12, 14], 1300, [10, 16, 20])
    dAs = [flp.DeviceCsr.from_host(A, with_fp32=True) for A, *_ in cases]
    args = ([c[1] for c in cases], [c[2] for c in cases])
    for prec in (flp.FLP_PREC_FP64, flp.FLP_PREC_FP32_FILTER):
        try:
            flp.flp_set_autotune(False)
            r0, _ = flp.flp_solve_batch(dAs, *args, block=8, seeds=[4, 5, 6], prec=prec)
            flp.flp_set_autotune(True)
            # a non-default shape and tile-to-XCD mapping for every launch
            flp.flp_set_filter_shape(1, 8, 0, True, tile_chunk=3)
            r1, _ = flp.flp_solve_batch(dAs, *args, block=8, seeds=[4, 5, 6], prec=prec)
            flp.flp_set_filter_shape(0, 0, 0)
            r2, _ = flp.flp_solve_batch(dAs, *args, block=8, seeds=[4, 5, 6], prec=prec)
        finally:
            flp.flp_set_filter_shape(0, 0, 0)
            flp.flp_set_autotune(True)
        for a, b, c in zip(r0, r1, r2):
            assert a["count"] == b["count"] == c["count"]
            assert np.array_equal(a["evals"], b["evals"]) and np.array_equal(a["evals"], c["evals"])


def test_batch_dependent_blocks_repaired(torch):
    """Solves whose filtered blocks become numerically dependent (an
    eigenvalue of multiplicity above the block size, a matrix with few
    distinct eigenvalues) go through the host repair of the segmented block
    step (random replacement, Section 2.3); every solve of the batch, the
    repaired ones and a regular one, meets the contract."""
    d1 = np.concatenate([np.linspace(-3, -1, 150), np.full(5, 0.5), np.linspace(1, 4, 150)])
    d2 = np.concatenate([np.linspace(-3, -1, 100), np.repeat([0.25, 0.75], 6), np.linspace(1.5, 4, 100)])
    A3 = I.laplacian_3d(9, I.uniform_potential(9, 31))
    lam3 = np.linalg.eigvalsh(A3.to_dense())
    mats = [I.diagonal_csr(d1), I.diagonal_csr(d2), A3]
    alphas = [0.0, 0.0, lam3[0] - 0.5]
    betas = [0.9, 1.0, 0.5 * (lam3[11] + lam3[12])]
    dAs = [flp.DeviceCsr.from_host(A) for A in mats]
    res, _ = flp.flp_solve_batch(dAs, alphas, betas, block=4, seeds=[4, 5, 6])
    for i in range(2):  # the same solves alone (single-solve path) agree
        alone = flp.flp_solve(dAs[i], alphas[i], betas[i], block=4, seed=4 + i)
        assert alone["count"] == res[i]["count"]
    assert res[0]["count"] == 5
    assert np.max(np.abs(res[0]["evals"] - 0.5)) < 1e-12 and np.max(res[0]["resid"]) <= 1e-9
    assert res[1]["count"] == 12
    assert np.max(np.abs(np.sort(res[1]["evals"]) - np.repeat([0.25, 0.75], 6))) < 1e-12
    assert np.max(res[1]["resid"]) <= 1e-9
    check(res[2], A3, alphas[2], betas[2], lam3)
