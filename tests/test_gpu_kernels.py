"""GPU parity of the individual hot-path calls against the CPU oracle.

Every call goes through the C ABI (libflp.so) and is compared element by
element with the oracle on the same seeded inputs.

Tolerances (derived from the arithmetic, stated per test):
* SpMM: each output sums at most k = max nnz/row products, so
  |err| <= k u sum_j |a_ij x_j| (u = 2^-53), for both sides together 2k u.
* filter (Clenshaw on the GPU vs the forward recurrence in the oracle):
  each of the m steps rounds an SpMM plus a three-term update, and the
  rounding errors of step k reach the result through the recurrence with
  a gain of at most m (Chebyshev polynomials of the second kind are
  bounded by their degree on [-1, 1]); hence
  |err| <= 2 m^2 (k + 4) u sum_i |b_i| max|V| for both sides together.
  FP32 filter: the same bound with u = 2^-24 and m in place of m^2 (the
  FP64 oracle's own error is negligible; the FP32 error is dominated by
  the rounding of V, A and each step, which the filter sums with gain
  sum_i |b_i|).
* Gram-Schmidt / QR: backward stable, 1e-12 relative.
"""
import numpy as np
import pytest

from oracle import flp_oracle as O
from paper_2409_15053_amd import flp
from paper_2409_15053_amd import inputs as I

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a visible MI355X"
    flp.load()
    return t


def dev(t, a):
    return t.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def max_row_nnz(A):
    return int(np.max(np.diff(A.rowptr)))


MATRICES = {
    "lap2d_13": lambda: I.laplacian_2d(13),
    "rand_97": lambda: I.random_sym(97, 0.08, seed=3),
    "lap3d7_9_U": lambda: I.laplacian_3d(9, I.uniform_potential(9, 4)),
    "lap3d13_8_wells": lambda: I.laplacian_3d_13pt(8, I.gaussian_wells(8, 5)),
    "diag_31": lambda: I.diagonal_csr(np.linspace(-2, 3, 31)),
}


@pytest.mark.parametrize("name", list(MATRICES))
@pytest.mark.parametrize("r", [1, 2, 3, 4, 5, 8, 16, 32])
def test_spmm_parity(torch, name, r):
    A = MATRICES[name]()
    X = I.random_block(A.n, r, seed=r)
    dA = flp.DeviceCsr.from_host(A)
    Y = torch.zeros((A.n, r), dtype=torch.float64, device="cuda:0")
    flp.flp_spmm(dA, dev(torch, X), Y)
    torch.cuda.synchronize()
    want = O.spmm(A, X)
    bound = 2 * max_row_nnz(A) * U64 * (np.abs(A.to_scipy()) @ np.abs(X))
    assert np.all(np.abs(Y.cpu().numpy() - want) <= bound + 1e-300)


def test_spmm_strided_block(torch):
    A = I.laplacian_3d(7)
    X = I.random_block(A.n, 20, seed=1)
    dA = flp.DeviceCsr.from_host(A)
    Xd = dev(torch, X)
    Y = torch.zeros((A.n, 20), dtype=torch.float64, device="cuda:0")
    flp.flp_spmm(dA, Xd[:, 4:12], Y[:, 2:10])
    torch.cuda.synchronize()
    got = Y.cpu().numpy()
    assert np.allclose(got[:, 2:10], O.spmm(A, X[:, 4:12]), rtol=0, atol=1e-12)
    assert np.all(got[:, :2] == 0) and np.all(got[:, 10:] == 0)


def filter_case(A, alpha, beta, m, r, seed):
    lmin, lmax = O.gershgorin(A)
    f = flp.flp_build_filter(alpha, beta, m, lmin, lmax)
    b = f.coeffs()
    V = I.random_block(A.n, r, seed=seed)
    return f, b, V, lmin, lmax


@pytest.mark.parametrize("name", list(MATRICES))
@pytest.mark.parametrize("m", [1, 2, 3, 4, 17, 60])
@pytest.mark.parametrize("r", [1, 3, 8, 16])
def test_filter_apply_fp64_parity(torch, name, m, r):
    A = MATRICES[name]()
    lmin, lmax = O.gershgorin(A)
    width = lmax - lmin
    alpha, beta = lmin + 0.3 * width, lmin + 0.45 * width
    f, b, V, lmin, lmax = filter_case(A, alpha, beta, m, r, seed=m * 7 + r)
    dA = flp.DeviceCsr.from_host(A)
    W = torch.empty((A.n, r), dtype=torch.float64, device="cuda:0")
    flp.flp_filter_apply(f, dA, dev(torch, V), W)
    torch.cuda.synchronize()
    want = O.filter_apply(A, lmin, lmax, b, V)
    k = max_row_nnz(A)
    tol = 2 * m * m * (k + 4) * U64 * np.sum(np.abs(b)) * np.max(np.abs(V))
    err = np.max(np.abs(W.cpu().numpy() - want))
    assert err <= tol, (err, tol)


@pytest.mark.parametrize("m", [1, 2, 5, 40])
@pytest.mark.parametrize("r", [1, 4, 8, 16])
def test_filter_apply_fp32_parity(torch, m, r):
    A = I.laplacian_3d(10, I.uniform_potential(10, 9))
    lmin, lmax = O.gershgorin(A)
    f, b, V, lmin, lmax = filter_case(A, 6.0, 7.5, m, r, seed=m + r)
    dA = flp.DeviceCsr.from_host(A)
    W = torch.empty((A.n, r), dtype=torch.float64, device="cuda:0")
    flp.flp_filter_apply(f, dA, dev(torch, V), W, prec=flp.FLP_PREC_FP32_FILTER)
    torch.cuda.synchronize()
    want = O.filter_apply(A, lmin, lmax, b, V)
    k = max_row_nnz(A)
    tol = 2 * m * (k + 4) * U32 * np.sum(np.abs(b)) * np.max(np.abs(V))
    err = np.max(np.abs(W.cpu().numpy() - want))
    assert err <= tol, (err, tol)


def test_filter_apply_ragged_large_grid(torch):
    """Several thousand tiles with a ragged tail (n not a multiple of any tile)."""
    A = I.laplacian_3d_13pt(37, I.gaussian_wells(37, 11))   # n = 50653
    lmin, lmax = O.gershgorin(A)
    f = flp.flp_build_filter(-2.0, -0.5, 30, lmin, lmax)
    b = f.coeffs()
    V = I.random_block(A.n, 16, seed=2)
    dA = flp.DeviceCsr.from_host(A)
    W = torch.empty((A.n, 16), dtype=torch.float64, device="cuda:0")
    flp.flp_filter_apply(f, dA, dev(torch, V), W)
    torch.cuda.synchronize()
    want = O.filter_apply(A, lmin, lmax, b, V)
    tol = 2 * 30 * 30 * (13 + 4) * U64 * np.sum(np.abs(b)) * np.max(np.abs(V))
    assert np.max(np.abs(W.cpu().numpy() - want)) <= tol


SHAPE_CASES = {
    # (r, prec): forced (lanes per row, columns per lane, group width, nontemporal streams, tile chunk,
    # LDS window); a negative tile chunk is the pencil walk over planes of that many rows (the 23^3
    # grid's 529); LDS window 2 is the sliding window, its halo and plane taken from the matrix
    # (plane 1058 here, halo 46 or 529 as the ring fits the LDS, row ranges shorter than a step)
    (8, flp.FLP_PREC_FP64): [(4, 2, 8, 0, 0, 0), (2, 4, 8, 1, 4, 0), (1, 8, 8, 0, 32, 0), (2, 2, 4, 1, 1, 0),
                             (1, 4, 4, 0, 7, 0), (1, 2, 2, 1, 0, 0), (4, 2, 8, 1, -529, 0), (2, 2, 4, 0, -1058, 0),
                             (4, 2, 8, 0, 0, 1), (2, 4, 8, 1, 4, 1), (1, 8, 8, 0, -529, 1), (2, 2, 4, 0, 0, 1),
                             (1, 2, 2, 1, 3, 1), (4, 2, 8, 0, 0, 2), (1, 8, 8, 1, 0, 2), (2, 2, 4, 0, 0, 2)],
    (16, flp.FLP_PREC_FP64): [(8, 2, 16, 1, 0, 0), (4, 4, 16, 0, 4, 0), (2, 8, 16, 1, 32, 0), (4, 2, 8, 0, 5, 0),
                              (2, 4, 8, 1, 0, 0), (1, 8, 8, 0, 1, 0), (4, 4, 16, 0, -529, 0),
                              (8, 2, 16, 1, -529, 0), (4, 4, 16, 1, -1058, 0), (4, 4, 16, 0, 0, 1),
                              (8, 2, 16, 1, -529, 1), (2, 8, 16, 0, 4, 1), (16, 2, 32, 0, 0, 1),
                              (4, 4, 16, 0, 0, 2), (8, 2, 16, 1, 0, 2), (2, 8, 16, 0, 0, 2), (4, 2, 8, 0, 0, 2)],
    (8, flp.FLP_PREC_FP32_FILTER): [(2, 4, 8, 1, 0, 0), (1, 8, 8, 0, 4, 0), (1, 4, 4, 1, 32, 0),
                                    (2, 4, 8, 0, -529, 0), (2, 4, 8, 0, 0, 1), (1, 8, 8, 1, 4, 1),
                                    (2, 4, 8, 0, 0, 2), (1, 8, 8, 1, 0, 2)],
    (16, flp.FLP_PREC_FP32_FILTER): [(4, 4, 16, 0, 0, 0), (2, 8, 16, 1, 4, 0), (2, 4, 8, 1, 3, 0),
                                     (1, 8, 8, 0, 32, 0), (4, 4, 16, 1, -529, 0), (4, 4, 16, 0, 0, 1),
                                     (2, 8, 16, 1, -529, 1), (1, 4, 4, 0, 0, 1), (4, 4, 16, 0, 0, 2),
                                     (2, 8, 16, 1, 0, 2), (1, 4, 4, 0, 0, 2)],
}


@pytest.mark.parametrize("r,prec", list(SHAPE_CASES))
def test_filter_launch_shapes_bit_identical(torch, r, prec):
    """Every launch configuration the autotuner may pick (rows per
    wavefront, columns per lane, column-group width, ordinary or nontemporal
    loads of the streamed operands, tile-to-XCD mapping, including chunk
    sizes that leave a ragged tail of tiles) sums each output element
    in the same order: all of them give the same bits, and that result is
    within the parity bound of the oracle."""
    A = I.laplacian_3d_13pt(23, I.gaussian_wells(23, 7))  # n = 12167: ragged last tile
    lmin, lmax = O.gershgorin(A)
    f, b, V, lmin, lmax = filter_case(A, -3.0, -1.0, 12, r, seed=r + prec)
    dA = flp.DeviceCsr.from_host(A)
    Vd = dev(torch, V)
    outs = []
    try:
        flp.flp_set_autotune(False)
        W0 = torch.empty((A.n, r), dtype=torch.float64, device="cuda:0")
        flp.flp_filter_apply(f, dA, Vd, W0, prec=prec)
        for lpr, vec, gw, nt, ch, win in SHAPE_CASES[(r, prec)]:
            for fmt in (flp.FLP_FORMAT_CSR, flp.FLP_FORMAT_SELL):
                flp.flp_set_filter_shape(lpr, vec, gw, bool(nt), tile_chunk=ch, lds_window=win)
                W = torch.empty((A.n, r), dtype=torch.float64, device="cuda:0")
                flp.flp_filter_apply(f, dA, Vd, W, prec=prec, format=fmt)
                outs.append(((lpr, vec, gw, nt, ch, win, fmt), W))
        flp.flp_set_filter_shape(0, 0, 0)
        flp.flp_set_autotune(True)
        info = flp.flp_tune_filter(dA, r, prec, format=flp.FLP_FORMAT_CSR)
        assert info["candidates"] >= 2 and info["us_per_step"] > 0
        assert r % info["group_width"] == 0
        assert info["lanes_per_row"] * info["cols_per_lane"] == info["group_width"]
        Wt = torch.empty((A.n, r), dtype=torch.float64, device="cuda:0")
        flp.flp_filter_apply(f, dA, Vd, Wt, prec=prec)
        outs.append(("tuned", Wt))
    finally:
        flp.flp_set_filter_shape(0, 0, 0)
        flp.flp_set_autotune(True)
    torch.cuda.synchronize()
    for cfg, W in outs:
        assert torch.equal(W, W0), cfg
    want = O.filter_apply(A, lmin, lmax, b, V)
    k = max_row_nnz(A)
    if prec == flp.FLP_PREC_FP64:
        tol = 2 * 12 * 12 * (k + 4) * U64 * np.sum(np.abs(b)) * np.max(np.abs(V))
    else:
        tol = 2 * 12 * (k + 4) * U32 * np.sum(np.abs(b)) * np.max(np.abs(V))
    assert np.max(np.abs(W0.cpu().numpy() - want)) <= tol


def principal(A, m):
    """The leading m x m block of a CSR matrix (symmetric when A is)."""
    keep = A.colind < m
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    sel = keep & (rows < m)
    cnt = np.bincount(rows[sel], minlength=m)
    rowptr = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int32)
    return I.Csr(m, rowptr, A.colind[sel].astype(np.int32), A.val[sel].copy())


@pytest.mark.parametrize("ragged", [False, True])
@pytest.mark.parametrize("prec", [flp.FLP_PREC_FP64, flp.FLP_PREC_FP32_FILTER])
def test_filter_sliding_window_long_ranges(torch, prec, ragged):
    """The sliding window over row ranges of several steps: on the 13-point
    64^3 grid (plane 4096 rows, in-plane reach 128 rows) each workgroup's
    range is a fraction of a plane and its LDS ring wraps several times.
    Ragged: the leading 61 planes and 1000 rows (a partial last plane and a
    last range shorter than the others).  Same bits as the plain launch on
    both storages, oracle parity in FP64."""
    A = I.laplacian_3d_13pt(64, I.gaussian_wells(64, 4))
    if ragged:
        A = principal(A, 61 * 4096 + 1000)
    r = 16
    f, b, V, lmin, lmax = filter_case(A, -3.0, -1.0, 6, r, seed=11)
    dA = flp.DeviceCsr.from_host(A)
    Vd = dev(torch, V)
    v16 = 2 if prec == flp.FLP_PREC_FP64 else 4
    outs = []
    try:
        flp.flp_set_autotune(False)
        flp.flp_set_filter_shape(r // v16, v16, r, False, tile_chunk=0, lds_window=0)
        W0 = torch.empty((A.n, r), dtype=torch.float64, device="cuda:0")
        flp.flp_filter_apply(f, dA, Vd, W0, prec=prec)
        for lpr in (r // v16, r // (2 * v16)):
            for fmt in (flp.FLP_FORMAT_CSR, flp.FLP_FORMAT_SELL):
                flp.flp_set_filter_shape(lpr, r // lpr, r, False, tile_chunk=0, lds_window=2)
                W = torch.empty((A.n, r), dtype=torch.float64, device="cuda:0")
                flp.flp_filter_apply(f, dA, Vd, W, prec=prec, format=fmt)
                outs.append(((lpr, fmt), W))
    finally:
        flp.flp_set_filter_shape(0, 0, 0)
        flp.flp_set_autotune(True)
    torch.cuda.synchronize()
    for cfg, W in outs:
        assert torch.equal(W, W0), cfg
    if prec == flp.FLP_PREC_FP64:
        want = O.filter_apply(A, lmin, lmax, b, V)
        tol = 2 * 6 * 6 * (max_row_nnz(A) + 4) * U64 * np.sum(np.abs(b)) * np.max(np.abs(V))
        assert np.max(np.abs(W0.cpu().numpy() - want)) <= tol


def test_filter_apply_errors(torch):
    A = I.laplacian_2d(5)
    dA = flp.DeviceCsr.from_host(A)
    f = flp.flp_build_filter(1.0, 2.0, 5, 0.0, 8.0)
    V = torch.zeros((A.n, 2), dtype=torch.float64, device="cuda:0")
    with pytest.raises(flp.FlpError):
        flp.flp_filter_apply(f, dA, V, V)  # aliasing
    W = torch.zeros((A.n, 40), dtype=torch.float64, device="cuda:0")
    with pytest.raises(flp.FlpError):
        flp.flp_filter_apply(f, dA, torch.zeros_like(W), W)  # r > 32
    # interleaved blocks of one buffer overlap even though they share no entry
    B = torch.zeros((A.n, 4), dtype=torch.float64, device="cuda:0")
    with pytest.raises(flp.FlpError):
        flp.flp_filter_apply(f, dA, B[:, 0:2], B[:, 2:4])
    with pytest.raises(flp.FlpError):
        flp.flp_filter_apply(f, dA, V, torch.zeros_like(V), format=7)  # unknown storage
    lib = flp.load()
    Wd = torch.zeros_like(V)
    # leading dimensions below r are refused at the boundary
    rc = lib.flp_filter_apply(f.h, flp.ctypes.byref(dA.c), V.data_ptr(), 1, Wd.data_ptr(), 2, 2,
                              flp.FLP_PREC_FP64, flp.FLP_FORMAT_CSR, None)
    assert rc == flp.FLP_E_ARG


@pytest.mark.parametrize("prec", [flp.FLP_PREC_FP64, flp.FLP_PREC_FP32_FILTER])
@pytest.mark.parametrize("r,ldv,ldw,v0,w0", [(3, 7, 5, 2, 1), (8, 20, 12, 4, 2), (16, 16, 24, 0, 8), (5, 5, 9, 0, 3)])
def test_filter_apply_strided_and_sliced_storage(torch, prec, r, ldv, ldw, v0, w0):
    """V and W as column ranges of wider blocks (leading dimensions ldv, ldw),
    the products on A in CSR and in its sliced ELL copy: the two storages
    give the same bits, the columns of W outside the range are untouched,
    and the result is within the parity bound of the oracle's forward
    recurrence."""
    A = I.laplacian_3d_13pt(19, I.gaussian_wells(19, 3))  # n = 6859: ragged last slice
    m = 25
    f, b, V, lmin, lmax = filter_case(A, -2.5, -0.5, m, r, seed=r * 11 + ldv)
    dA = flp.DeviceCsr.from_host(A)
    big = np.full((A.n, ldv), 7.0)
    big[:, v0:v0 + r] = V
    Vd = dev(torch, big)
    outs = {}
    for fmt in (flp.FLP_FORMAT_CSR, flp.FLP_FORMAT_SELL, flp.FLP_FORMAT_AUTO):
        Wb = torch.full((A.n, ldw), -3.0, dtype=torch.float64, device="cuda:0")
        flp.flp_filter_apply(f, dA, Vd[:, v0:v0 + r], Wb[:, w0:w0 + r], prec=prec, format=fmt)
        outs[fmt] = Wb
    torch.cuda.synchronize()
    base = outs[flp.FLP_FORMAT_CSR].cpu().numpy()
    for fmt, Wb in outs.items():
        got = Wb.cpu().numpy()
        assert np.array_equal(got, base), fmt
        assert np.all(got[:, :w0] == -3.0) and np.all(got[:, w0 + r:] == -3.0)
    assert np.all(Vd.cpu().numpy() == big)
    want = O.filter_apply(A, lmin, lmax, b, V)
    k = max_row_nnz(A)
    if prec == flp.FLP_PREC_FP64:
        tol = 2 * m * m * (k + 4) * U64 * np.sum(np.abs(b)) * np.max(np.abs(V))
    else:
        tol = 2 * m * (k + 4) * U32 * np.sum(np.abs(b)) * np.max(np.abs(V))
    err = np.max(np.abs(base[:, w0:w0 + r] - want))
    assert err <= tol, (err, tol)


@pytest.mark.parametrize("n,k,r", [(1000, 1, 1), (1000, 7, 3), (5003, 48, 8), (20011, 160, 16), (777, 16, 16),
                                   # bases of 256+ columns against 8 and 16 columns: the FMA projection
                                   (30011, 300, 8), (20011, 520, 16), (4099, 256, 8), (9001, 130, 8)])
def test_block_orth_parity(torch, n, k, r):
    g = np.random.Generator(np.random.PCG64(n + k))
    Q, _ = np.linalg.qr(g.standard_normal((n, k)))
    ldq = k + 5
    Qp = np.zeros((n, ldq))
    Qp[:, :k] = Q
    W = g.standard_normal((n, r))
    Qd = dev(torch, Qp)
    Wd = dev(torch, W)
    H = flp.flp_block_orth(Qd, k, Wd)
    # the definition: two passes of classical Gram-Schmidt
    H1 = Q.T @ W
    W1 = W - Q @ H1
    H2 = Q.T @ W1
    W2 = W1 - Q @ H2
    assert np.max(np.abs(H - (H1 + H2))) < 1e-12 * np.max(np.abs(W)) * np.sqrt(n)
    got = Wd.cpu().numpy()
    assert np.max(np.abs(got - W2)) < 1e-12 * np.max(np.abs(W))
    assert np.max(np.abs(Q.T @ got)) < 1e-13 * np.sqrt(n) * np.max(np.abs(W))


@pytest.mark.parametrize("n,r", [(100, 1), (1000, 3), (4099, 8), (30000, 16)])
def test_block_qr_parity(torch, n, r):
    g = np.random.Generator(np.random.PCG64(n * r))
    W = g.standard_normal((n, r)) @ np.triu(g.standard_normal((r, r)) + 3 * np.eye(r))
    Wd = dev(torch, W)
    S = flp.flp_block_qr(Wd)
    Qn = Wd.cpu().numpy()
    # unique QR with a positive diagonal (eq. lanczos: S upper triangular)
    Qr, R = np.linalg.qr(W)
    sg = np.sign(np.diag(R))
    R = sg[:, None] * R
    assert np.allclose(np.tril(S, -1), 0)
    assert np.all(np.diag(S) > 0)
    assert np.max(np.abs(S - R)) < 1e-11 * np.max(np.abs(R))
    assert np.max(np.abs(Qn.T @ Qn - np.eye(r))) < 1e-13
    assert np.max(np.abs(Qn @ S - W)) < 1e-12 * np.max(np.abs(W))


def test_block_qr_rank_deficient_is_reported(torch):
    g = np.random.Generator(np.random.PCG64(1))
    W = g.standard_normal((500, 4))
    W[:, 3] = W[:, 0] - 2 * W[:, 1]
    with pytest.raises(flp.FlpError):
        flp.flp_block_qr(dev(torch, W))


def lap1d(N):
    j = np.arange(1, N + 1)
    return 4 * np.sin(j * np.pi / (2 * (N + 1))) ** 2


@pytest.mark.parametrize("case", ["2d40", "3d20", "3d13pt16"])
def test_bounds_enclose_spectrum(torch, case):
    if case == "2d40":
        A, lo, hi = I.laplacian_2d(40), 2 * lap1d(40)[0], 2 * lap1d(40)[-1]
    elif case == "3d20":
        A, lo, hi = I.laplacian_3d(20), 3 * lap1d(20)[0], 3 * lap1d(20)[-1]
    else:
        A = I.laplacian_3d_13pt(16)
        w = np.linalg.eigvalsh(np.diag(np.full(16, 2.5)) + np.diag(np.full(15, -4 / 3), 1) +
                               np.diag(np.full(15, -4 / 3), -1) + np.diag(np.full(14, 1 / 12), 2) +
                               np.diag(np.full(14, 1 / 12), -2))
        lo, hi = 3 * w[0], 3 * w[-1]
    dA = flp.DeviceCsr.from_host(A)
    lmin, lmax = flp.flp_estimate_bounds(dA, 40, 7)
    glo, ghi = O.gershgorin(A)
    assert lmin <= lo and lmax >= hi
    assert glo <= lmin and lmax <= ghi


@pytest.mark.parametrize("prec", [flp.FLP_PREC_FP64, flp.FLP_PREC_FP32_FILTER])
def test_filter_apply_full_size_lap3d7_100(torch, prec):
    """Full-size filter parity at the benchmark's launch configuration:
    7-point Laplacian on 100^3 + U[0,1) potential (n = 1e6), block 8,
    degree 100, on the sliced ELL copy the solver reads by default (the
    tuned launches the benchmark times) and on CSR: identical bits, within
    the bound of the oracle."""
    w = I.workload_c2(100)
    A = w["A"]
    lmin, lmax = O.gershgorin(A)
    m = 100
    f = flp.flp_build_filter(0.0, 0.51, m, lmin, lmax)
    b = f.coeffs()
    V = I.random_block(A.n, 8, seed=123)
    dA = flp.DeviceCsr.from_host(A, with_fp32=(prec == flp.FLP_PREC_FP32_FILTER))
    Vd = dev(torch, V)
    outs = []
    for fmt in (flp.FLP_FORMAT_SELL, flp.FLP_FORMAT_CSR):
        W = torch.empty((A.n, 8), dtype=torch.float64, device="cuda:0")
        flp.flp_filter_apply(f, dA, Vd, W, prec=prec, format=fmt)
        outs.append(W)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])
    flp.flp_release_workspace()
    want = O.filter_apply(A, lmin, lmax, b, V)
    k = max_row_nnz(A)
    if prec == flp.FLP_PREC_FP64:
        tol = 2 * m * m * (k + 4) * U64 * np.sum(np.abs(b)) * np.max(np.abs(V))
    else:
        tol = 2 * m * (k + 4) * U32 * np.sum(np.abs(b)) * np.max(np.abs(V))
    err = np.max(np.abs(outs[0].cpu().numpy() - want))
    assert err <= tol, (err, tol)


@pytest.mark.parametrize("prec", [flp.FLP_PREC_FP64, flp.FLP_PREC_FP32_FILTER])
def test_filter_apply_full_size_lap3d13_120(torch, prec):
    """Full-size filter parity on the 13-point 120^3 Hamiltonian with 16
    Gaussian wells (n = 1.728e6, nnz = 2.2e7), block 16, on the sliced ELL
    copy and on CSR (identical bits), within the bound of the oracle."""
    w = I.workload_c3(120)
    A = w["A"]
    lmin, lmax = O.gershgorin(A)
    m = 30
    f = flp.flp_build_filter(-2.0, -1.0, m, lmin, lmax)
    b = f.coeffs()
    V = I.random_block(A.n, 16, seed=7)
    dA = flp.DeviceCsr.from_host(A)
    Vd = dev(torch, V)
    outs = []
    for fmt in (flp.FLP_FORMAT_SELL, flp.FLP_FORMAT_CSR):
        W = torch.empty((A.n, 16), dtype=torch.float64, device="cuda:0")
        flp.flp_filter_apply(f, dA, Vd, W, prec=prec, format=fmt)
        outs.append(W)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])
    flp.flp_release_workspace()
    want = O.filter_apply(A, lmin, lmax, b, V)
    if prec == flp.FLP_PREC_FP64:
        tol = 2 * m * m * (13 + 4) * U64 * np.sum(np.abs(b)) * np.max(np.abs(V))
    else:
        tol = 2 * m * (13 + 4) * U32 * np.sum(np.abs(b)) * np.max(np.abs(V))
    err = np.max(np.abs(outs[0].cpu().numpy() - want))
    assert err <= tol, (err, tol)
