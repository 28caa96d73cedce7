"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol declared in include/flp.h, validates arguments, and its host-side
arithmetic (filter coefficients, degree rule, banded eigensolver) matches
the oracle and LAPACK."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import flp_oracle as O
from paper_2409_15053_amd import flp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "flp.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(flp_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = flp.load()
    names = declared_symbols()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(flp.EXPORTS)


def test_struct_mirrors_match_the_header():
    """Every ctypes mirror in the binding has the size of its C struct (a
    short mirror would let the library write past it)."""
    lib = flp.load()
    sizes = (ctypes.c_int64 * 16)()
    n = lib.flp_abi_sizes(sizes, 16)
    mirrors = [flp.FlpCsrC, flp.FlpOptsC, flp.FlpStatsC, flp.FlpResultC, flp.FlpTuneInfoC, flp.FlpBatchStatsC,
               flp.FlpServerOptsC]
    assert n == len(mirrors)
    for m, s in zip(mirrors, sizes[:n]):
        assert ctypes.sizeof(m) == s, (m.__name__, ctypes.sizeof(m), s)


def test_version():
    assert flp.flp_version().startswith("flp-mi355x")


@pytest.mark.parametrize("alpha,beta,lmin,lmax,m", [
    (0.5, 1.0, 0.0, 8.0, 50), (-0.645, -0.0053, -1.21, 32.8, 0), (-1.0, -0.5, -1.0, 1.0, 80),
    (0.1, 0.3, -1.0, 1.0, 0), (-5.0, 0.2, -1.0, 1.0, 10)])
def test_filter_matches_oracle(alpha, beta, lmin, lmax, m):
    f = flp.flp_build_filter(alpha, beta, m, lmin, lmax)
    info = f.info()
    c, e = O.affine_map(lmin, lmax)
    a1 = min(max((max(alpha, lmin) - c) / e, -1), 1)
    b1 = min(max((min(beta, lmax) - c) / e, -1), 1)
    assert abs(info["alpha"] - a1) < 1e-15 and abs(info["beta"] - b1) < 1e-15
    want_m = m if m > 0 else O.filter_degree(a1, b1)
    assert f.degree == want_m
    b = O.cheb_coeffs(a1, b1, want_m)
    assert np.max(np.abs(f.coeffs() - b)) < 1e-14
    z = np.linspace(-1, 1, 41)
    assert np.max(np.abs(f.eval(z) - O.cheb_eval(b, z))) < 1e-12


def test_filter_table2_auto_degrees_through_abi():
    rows = [(-1.21, 32.8, -0.645, -0.0053, 49), (-1.23, 32.7, -0.650, -0.0096, 49),
            (-1.21, 49.8, -0.640, -0.0028, 61), (-1.20, 43.1, -0.660, -0.3300, 98),
            (-1.25, 1300.0, -0.640, 0.0, 308)]
    for lo, hi, a, b, m in rows:
        assert flp.flp_build_filter(a, b, 0, lo, hi).degree == m


@pytest.mark.parametrize("args,code", [
    ((1.0, 0.5, 10, -1.0, 1.0), flp.FLP_E_ARG),           # alpha >= beta
    ((float("nan"), 0.5, 10, -1.0, 1.0), flp.FLP_E_ARG),  # NaN
    ((0.0, 0.5, 10, 1.0, -1.0), flp.FLP_E_ARG),           # lmin >= lmax
    ((2.0, 3.0, 10, -1.0, 1.0), flp.FLP_E_INTERVAL),      # outside the spectrum
    ((0.0, 0.5, 200000, -1.0, 1.0), flp.FLP_E_ARG),       # degree too large
])
def test_filter_argument_errors(args, code):
    with pytest.raises(flp.FlpError) as ei:
        flp.flp_build_filter(*args)
    assert ei.value.code == code


def test_solve_rejects_bad_csr_without_gpu():
    lib = flp.load()
    A = flp.FlpCsrC(0, 0, None, None, None, None)
    res = ctypes.POINTER(flp.FlpResultC)()
    assert lib.flp_solve(ctypes.byref(A), 0.0, 1.0, None, ctypes.byref(res)) == flp.FLP_E_ARG
    assert b"n must be positive" in lib.flp_last_error()
    A = flp.FlpCsrC(10, 1 << 31, 1, 1, 1, None)
    assert lib.flp_solve(ctypes.byref(A), 0.0, 1.0, None, ctypes.byref(res)) == flp.FLP_E_ARG


# the eigenvector columns are built in tiles of 8, 16 or 32 (the widest
# that gives every thread one): N = 20 and 24 take 16-column tiles on one
# thread, 60 and up 32, and the larger ones several threads
@pytest.mark.parametrize("N,bw", [(1, 0), (2, 1), (7, 1), (20, 3), (24, 23), (60, 1), (60, 3), (97, 8), (120, 16),
                                  (80, 79), (257, 40), (300, 299), (420, 419)])
def test_host_banded_eigensolver_against_lapack(N, bw):
    g = np.random.Generator(np.random.PCG64(N * 100 + bw))
    M = g.standard_normal((N, N))
    M = M + M.T
    i, j = np.indices((N, N))
    M[np.abs(i - j) > bw] = 0.0
    ev, Z = flp.flp_host_sym_eig(M, bw)
    w = np.linalg.eigvalsh(M)
    scale = max(1.0, np.max(np.abs(w)))
    assert np.max(np.abs(ev - w)) < 1e-13 * scale * max(1, N) ** 0.5
    assert np.max(np.abs(M @ Z - Z * ev)) < 1e-12 * scale * max(1, N) ** 0.5
    assert np.max(np.abs(Z.T @ Z - np.eye(N))) < 1e-12 * max(1, N) ** 0.5


def test_host_dense_eigensolver_multiplicities():
    # the dense (Householder) path on a Rayleigh-Ritz-like matrix: exact
    # multiplicities, a 1e-13 cluster and a zero block
    g = np.random.Generator(np.random.PCG64(11))
    d = np.concatenate([np.full(40, 0.5), np.full(3, 2.0), [2.0 + 1e-13], g.uniform(-1, 3, 150), np.zeros(7)])
    N = d.size
    Qr, _ = np.linalg.qr(g.standard_normal((N, N)))
    M = (Qr * d) @ Qr.T
    M = 0.5 * (M + M.T)
    ev, Z = flp.flp_host_sym_eig(M)
    assert np.max(np.abs(ev - np.sort(d))) < 1e-13 * N
    assert np.max(np.abs(Z.T @ Z - np.eye(N))) < 1e-13 * N
    assert np.max(np.abs(M @ Z - Z * ev)) < 1e-13 * N


def test_host_eigensolver_degenerate_and_clustered():
    # block-tridiagonal with exact multiplicities and a tight cluster
    d = np.array([1.0, 1.0, 1.0, 2.0, 2.0 + 1e-13, 3.0, -1.0, -1.0])
    g = np.random.Generator(np.random.PCG64(5))
    Qr, _ = np.linalg.qr(g.standard_normal((8, 8)))
    M = (Qr * d) @ Qr.T
    M = 0.5 * (M + M.T)
    ev, Z = flp.flp_host_sym_eig(M)
    assert np.max(np.abs(ev - np.sort(d))) < 1e-14 * 8
    assert np.max(np.abs(Z.T @ Z - np.eye(8))) < 1e-13
    assert np.max(np.abs(M @ Z - Z * ev)) < 1e-13


@pytest.mark.parametrize("scale", [1e-200, 1e-120, 1e120, 1e200])
def test_host_eigensolver_far_scales(scale):
    # a tridiagonal and a banded matrix whose entries all lie near 1e-200
    # (or 1e200): the rotations' squares would underflow (overflow) unscaled
    g = np.random.Generator(np.random.PCG64(int(np.log10(scale)) + 400))
    for N, bw in [(60, 1), (90, 6)]:
        M = g.standard_normal((N, N))
        M = M + M.T
        i, j = np.indices((N, N))
        M[np.abs(i - j) > bw] = 0.0
        ev = flp.flp_host_sym_eig(M * scale, bw, vectors=False)
        w = np.linalg.eigvalsh(M)
        assert np.max(np.abs(ev / scale - w)) < 1e-13 * np.max(np.abs(w)) * N ** 0.5


def test_opts_defaults_and_new_codes():
    o = flp.default_opts()
    assert o.sym_tol < 0          # the symmetry check is opt-in
    assert o.block == 1 and o.check_every == 0 and abs(o.eps - 0.31227) < 1e-12
    assert o.unfiltered == 0 and o.polish_degree == 0 and o.format == flp.FLP_FORMAT_AUTO
    assert flp.FLP_E_CANCELLED == -8 and flp.FLP_E_NOTSYM == -3


@pytest.mark.parametrize("m", [1, 2, 3, 17, 100])
def test_filter_divided_difference(m):
    """The polish's divided difference g(z) = (p(z) - p(t)) / (z - t), from
    Chebyshev synthetic division, against its definition at sample points:
    (z - t) g(z) = p(z) - p(t) with g evaluated by numpy's Chebyshev series."""
    f = flp.flp_build_filter(-0.6, -0.2, m, -1.0, 1.0)
    b = f.coeffs()
    rng = np.random.default_rng(m)
    for t in [-0.999, -0.4, 0.0, 0.35, 0.999, rng.uniform(-1, 1)]:
        c = f.divided(t)
        assert len(c) == m
        z = np.concatenate([rng.uniform(-1, 1, 50), [-1.0, 1.0]])
        z = z[np.abs(z - t) > 1e-3]
        g = np.polynomial.chebyshev.chebval(z, c)
        lhs = (z - t) * g
        rhs = np.polynomial.chebyshev.chebval(z, b) - np.polynomial.chebyshev.chebval(t, b)
        assert np.max(np.abs(lhs - rhs)) <= 1e-12 * max(1.0, np.max(np.abs(b)) * m)
        # the limit at z = t is p'(t)
        dp = np.polynomial.chebyshev.chebval(t, np.polynomial.chebyshev.chebder(b))
        assert abs(np.polynomial.chebyshev.chebval(t, c) - dp) <= 1e-9 * max(1.0, abs(dp))


@pytest.mark.parametrize("prec", [flp.FLP_PREC_FP64, flp.FLP_PREC_FP32_FILTER])
@pytest.mark.parametrize("segmented", [False, True])
def test_filter_launch_shape_covers_every_column(prec, segmented):
    """Lane-to-column mapping of the filter kernels for every block width
    1..32: lane s of a row owns columns [s*vec, s*vec + vec), so the lanes
    of a row cover all r columns (lanes * vec >= r); with 16-byte-aligned
    widths the mapping is exact, otherwise one column per lane on the next
    power of two, whose lanes past column r - 1 leave the kernel (the
    guard `c0 >= r` of both kernels)."""
    v16 = 4 if prec == flp.FLP_PREC_FP32_FILTER else 2
    for r in range(1, 33):
        sh = flp.flp_filter_launch_shape(r, prec, segmented)
        lpr, vec = sh["lanes_per_row"], sh["cols_per_lane"]
        assert sh["group_width"] == r
        assert 64 % lpr == 0 and sh["rows_per_wave"] * lpr == 64
        assert lpr * vec >= r, (r, lpr, vec)
        owned = [c for s_ in range(lpr) for c in range(s_ * vec, s_ * vec + vec) if c < r]
        assert owned == list(range(r))  # each column exactly once
        if lpr * vec > r:
            assert vec == 1 and lpr == 1 << (r - 1).bit_length()
        if r % v16 == 0 and r // v16 in (1, 2, 4, 8, 16) and vec > 1:
            assert lpr * vec == r
    # the paper's block size 3 (Table 2) and other widths with no aligned shape
    for r in (3, 5, 6, 7, 9, 12, 15):
        sh = flp.flp_filter_launch_shape(r, prec, segmented)
        assert sh["lanes_per_row"] * sh["cols_per_lane"] >= r
    with pytest.raises(flp.FlpError):
        flp.flp_filter_launch_shape(0, prec, segmented)
    with pytest.raises(flp.FlpError):
        flp.flp_filter_launch_shape(33, prec, segmented)


@pytest.mark.parametrize("tiles", [0, 1, 7, 8, 9, 63, 64, 225, 1000, 27000, 27001, 15625, 15626])
@pytest.mark.parametrize("chunk,rpt", [(0, 64), (4, 64), (32, 32), (-14400, 64), (-10000, 64), (-10000, 32),
                                       (-28800, 64), (-512, 64), (-1024, 16), (-1 << 20, 64)])
def test_tile_order_is_a_permutation(tiles, chunk, rpt):
    """Every tile-to-XCD traversal of the filter kernels hands each row tile
    to exactly one workgroup (ragged plane counts, planes of fewer than 8
    tiles, planes longer than the launch, partial last planes)."""
    order = flp.flp_tile_order(tiles, chunk, rpt)
    assert np.array_equal(np.sort(order), np.arange(tiles))


def test_tile_order_pencil_walk():
    """The pencil walk over planes of 225 tiles (the 120^3 grid's planes of
    14 400 rows at 64 rows per tile): workgroup b runs on XCD b % 8, and the
    workgroups of XCD x, in dispatch order, take the x-th eighth of the
    walk that goes through pencil 0 (columns 0..27 of every plane) plane
    after plane, then pencil 1, ..., pencil 7 (columns 196..224), then the
    tiles past the last full plane."""
    for G in (27000, 27000 + 100):
        PT = 225
        Z = G // PT
        lo = [p * PT // 8 for p in range(9)]
        walk = [z * PT + c for p in range(8) for z in range(Z) for c in range(lo[p], lo[p + 1])]
        walk += list(range(Z * PT, G))
        order = flp.flp_tile_order(G, -14400, 64)
        start = 0
        for x in range(8):
            cnt = G // 8 + (1 if x < G % 8 else 0)
            assert np.array_equal(order[x::8], walk[start:start + cnt])
            start += cnt
    with pytest.raises(flp.FlpError):
        flp.flp_tile_order(10, 0, 0)
