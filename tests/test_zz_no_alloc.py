"""The allocation-free filter application (flp_filter_apply_noalloc) against
flp_filter_apply on the same inputs: both run the same Clenshaw steps with
the same per-element summation order, so the results must be bit-identical
(every launch configuration of the filter kernel gives the same bits).  Two
calls in a row share the device's scratch array, the second on a smaller
problem; then the limit and argument errors."""
import ctypes

import numpy as np
import pytest

from oracle import flp_oracle as O
from paper_2409_15053_amd import flp
from paper_2409_15053_amd import inputs as I

pytestmark = pytest.mark.gpu

MAX_ELEMS = 1 << 20


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a visible MI355X"
    flp.load()
    return t


def case(torch, A, r, m, seed):
    lmin, lmax = O.gershgorin(A)
    a = lmin + 0.05 * (lmax - lmin)
    b = lmin + 0.2 * (lmax - lmin)
    f = flp.flp_build_filter(a, b, m, lmin, lmax)
    V = torch.from_numpy(I.random_block(A.n, r, seed)).to("cuda:0")
    return f, V


@pytest.mark.parametrize("prec", [flp.FLP_PREC_FP64, flp.FLP_PREC_FP32_FILTER])
def test_noalloc_matches_filter_apply_twice(torch, prec):
    # first call: 46^3 13-point Hamiltonian (n = 97 336) at r = 8 (near the
    # limit in FP64); second: a smaller 7-point problem at r = 3
    cases = [(I.laplacian_3d_13pt(46, I.gaussian_wells(46, 11)), 8, 40, 5),
             (I.laplacian_3d(17, I.uniform_potential(17, 12)), 3, 25, 6)]
    for A, r, m, seed in cases:
        assert A.n * r <= MAX_ELEMS
        dA = flp.DeviceCsr.from_host(A, "cuda:0", with_fp32=True)
        f, V = case(torch, A, r, m, seed)
        Wref = torch.empty_like(V)
        flp.flp_filter_apply(f, dA, V, Wref, prec=prec, format=flp.FLP_FORMAT_CSR)
        W = torch.full_like(V, float("nan"))
        flp.flp_filter_apply_noalloc(f, dA, V, W, prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(W, Wref), (A.n, r, prec)


def test_noalloc_strided_blocks(torch):
    A = I.laplacian_3d(13, I.uniform_potential(13, 3))
    dA = flp.DeviceCsr.from_host(A, "cuda:0", with_fp32=True)
    f, V = case(torch, A, 4, 30, 9)
    Vs = torch.zeros((A.n, 7), dtype=torch.float64, device="cuda:0")
    Vs[:, 1:5] = V
    Ws = torch.full((A.n, 6), float("nan"), dtype=torch.float64, device="cuda:0")
    Wref = torch.empty_like(V)
    flp.flp_filter_apply(f, dA, V, Wref, format=flp.FLP_FORMAT_CSR)
    flp.flp_filter_apply_noalloc(f, dA, Vs[:, 1:5], Ws[:, 2:6])
    torch.cuda.synchronize()
    assert torch.equal(Ws[:, 2:6], Wref)
    assert torch.isnan(Ws[:, :2]).all()


def test_noalloc_limits_and_errors(torch):
    A = I.laplacian_3d(12)
    dA = flp.DeviceCsr.from_host(A, "cuda:0")  # no FP32 values
    f, V = case(torch, A, 2, 10, 1)
    W = torch.empty_like(V)
    with pytest.raises(flp.FlpError) as e:  # FP32 needs the caller's FP32 values
        flp.flp_filter_apply_noalloc(f, dA, V, W, prec=flp.FLP_PREC_FP32_FILTER)
    assert e.value.code == flp.FLP_E_ARG
    big = I.laplacian_3d(102)  # n * r = 1 061 208 * 1 > 2^20
    dB = flp.DeviceCsr.from_host(big, "cuda:0")
    Vb = torch.zeros((big.n, 1), dtype=torch.float64, device="cuda:0")
    with pytest.raises(flp.FlpError) as e:
        flp.flp_filter_apply_noalloc(f, dB, Vb, torch.empty_like(Vb))
    assert e.value.code == flp.FLP_E_NOMEM
    with pytest.raises(flp.FlpError):
        flp.flp_filter_apply_noalloc(f, dA, V, V)  # W overlaps V
