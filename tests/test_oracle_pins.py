"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test names the mistake it is there to catch.  None of them re-types an
oracle formula: the checks are hand-derived fixtures (tests/golden), closed
forms, dense brute-force solves of Eq. (1) built a different way (tests/brute),
textbook routines (numpy pinv, scipy DCT) and invariants.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import brute
import oracle
from paper_2008_10273_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

SHAPES = [(2, 1), (1, 3), (3, 3), (4, 3), (3, 5), (6, 6), (7, 4), (8, 8), (5, 9)]


def _rng(seed):
    return np.random.default_rng(seed)


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([float(Fraction(t)) for t in line.split()])
    return rows


# ---------------------------------------------------------------- golden

def test_golden_green_path3():
    """Hand-derived pinv of the 3x1 operator: catches a wrong omega weight,
    a missing mirror image or a wrong fold of x + x' + 1 in the table."""
    rows = _read_golden("green_path3.txt")
    w, h = map(int, rows[0])
    G = np.array(rows[1:])
    np.testing.assert_allclose(oracle.green_matrix(w, h), G, atol=1e-13)


@pytest.mark.parametrize("name", ["decode_4x1.txt", "decode_2x2.txt", "decode_3x2.txt"])
def test_golden_decodes(name):
    """Hand-solved Eq. (1) cases (the 3x2 one is non-square: catches a
    transposed w/h), with c = A u at mask points and a = block mean."""
    rows = _read_golden(name)
    w, h = map(int, rows[0])
    pos = np.array(rows[1], dtype=np.uint16)
    r = np.array(rows[2])
    u = np.array(rows[3:3 + h])
    c_ref = np.array(rows[3 + h])
    a_ref = rows[4 + h][0]
    np.testing.assert_allclose(oracle.block_direct(w, h, pos, r), u, atol=1e-12)
    c, a, ug = oracle.block_green(w, h, pos, r)
    np.testing.assert_allclose(ug[0], u, atol=1e-12)
    np.testing.assert_allclose(c[0], c_ref, atol=1e-12)
    assert abs(a[0] - a_ref) < 1e-12


# ------------------------------------------------------ textbook routines

@pytest.mark.parametrize("w,h", SHAPES)
@pytest.mark.parametrize("s", [1, 2])
def test_green_matrix_is_pinv(w, h, s):
    """G from the Toeplitz-plus-Hankel table equals numpy's pseudo-inverse of
    A = (-L)^s: pins eigenvalues, weights, images and index order at once."""
    G = oracle.green_matrix(w, h, 0, float(s))
    np.testing.assert_allclose(G, np.linalg.pinv(brute.operator(w, h, s)), atol=1e-11)


@pytest.mark.parametrize("w,h", [(4, 3), (6, 6), (5, 9)])
def test_green_matrix_is_dct_diagonalised(w, h):
    """Eq. (4): G = C^T diag(lambda) C with scipy's orthonormal DCT-II, for
    the continuous-symbol operator too (op 1, which has no stencil form)."""
    for op in (0, 1):
        lam = oracle.eigenvalues(w, h, op, 1.0)
        C = np.kron(brute.dct_matrix(h), brute.dct_matrix(w))
        np.testing.assert_allclose(oracle.green_matrix(w, h, op, 1.0),
                                   C.T @ np.diag(lam.ravel()) @ C, atol=1e-11)


def test_eigenvalues_are_operator_spectrum():
    """The discrete eigenvalues are the spectrum of -L (catches using the
    continuous symbol by mistake, or swapped axes on a non-square block)."""
    w, h = 5, 3
    lam = oracle.eigenvalues(w, h, 0, 1.0).ravel()
    mu = np.sort(np.linalg.eigvalsh(brute.neg_laplacian(w, h)))
    got = np.sort(np.concatenate([[0.0], 1.0 / lam[1:]]))
    np.testing.assert_allclose(got, mu, atol=1e-12)


@pytest.mark.parametrize("w,h", [(8, 8), (5, 3), (16, 12), (32, 28)])
def test_continuous_symbol_is_the_refined_grid_limit(w, h):
    """Op 1 (Sec. 2.2: the eigenvalues alone define the operator) is the
    Laplacian of the continuous w x h rectangle with reflecting sides.  Its
    eigenvalue of mode (p, q) is the limit of m^2 times the 5-point
    operator's eigenvalue of that mode on the rectangle sampled m times finer
    (spacing 1/m).  That spectrum comes from numpy.linalg.eigvalsh of the
    1-D path Laplacians (the 2-D grid is their Cartesian product, so mode
    (p, q) is the sum of the p-th and q-th 1-D values; checked on a small
    grid below); the error falls as 1/m^2, and Richardson's step from m and
    2m cancels that term."""
    def scaled_1d(n, m):
        return m * m * np.sort(np.linalg.eigvalsh(brute.path_laplacian(n * m)))

    def grid_mu(m):
        ex, ey = scaled_1d(w, m), scaled_1d(h, m)
        return ey[:h, None] + ex[None, :w]

    m = 24
    extrap = (4.0 * grid_mu(2 * m) - grid_mu(m)) / 3.0
    lam = oracle.eigenvalues(w, h, 1, 1.0)
    assert lam[0, 0] == 0.0
    mu = np.where(lam > 0, 1.0 / np.where(lam > 0, lam, 1.0), 0.0)
    np.testing.assert_allclose(mu[lam > 0], extrap[lam > 0], rtol=2e-6)
    # s enters as lam = mu^-s for every mode (biharmonic and fractional)
    for s in (2.0, 0.5):
        np.testing.assert_allclose(oracle.eigenvalues(w, h, 1, s)[lam > 0], mu[lam > 0] ** -s, rtol=1e-12)


def test_grid_spectrum_is_the_sum_of_path_spectra():
    """The Cartesian-product structure the previous pin relies on: the 2-D
    5-point operator's spectrum is every sum of one eigenvalue of each 1-D
    path Laplacian."""
    w, h = 7, 5
    ex = np.linalg.eigvalsh(brute.path_laplacian(w))
    ey = np.linalg.eigvalsh(brute.path_laplacian(h))
    got = np.sort((ey[:, None] + ex[None, :]).ravel())
    np.testing.assert_allclose(got, np.sort(np.linalg.eigvalsh(brute.neg_laplacian(w, h))), atol=1e-12)


# --------------------------------------------------- brute-force Eq. (1)

@pytest.mark.parametrize("w,h", SHAPES)
@pytest.mark.parametrize("s", [1, 2])
def test_direct_matches_dense_eq1(w, h, s):
    """Banded solve of the plain definition vs one dense solve of Eq. (1)."""
    rng = _rng(w * 100 + h * 10 + s)
    N = w * h
    for K in sorted({1, 2, max(1, N // 4), max(1, N // 2), N - 1 if N > 1 else 1, N}):
        pos = np.sort(rng.choice(N, K, replace=False)).astype(np.uint16)
        r = rng.uniform(-64, 64, K)
        ref = brute.solve_eq1(w, h, pos, r, brute.operator(w, h, s))
        np.testing.assert_allclose(oracle.block_direct(w, h, pos, r, s), ref, atol=1e-9)


@pytest.mark.parametrize("w,h", SHAPES + [(16, 16), (16, 8), (16, 12)])
@pytest.mark.parametrize("s", [1.0, 2.0])
def test_green_route_matches_dense_eq1(w, h, s):
    """The Green's route (Eqs. 2-3) reaches the plain definition (Eq. 1)."""
    rng = _rng(7 * w + h)
    N = w * h
    A = brute.operator(w, h, int(s))
    for K in sorted({1, min(3, N), max(1, N // 10), max(1, N // 2), N - 1 if N > 1 else 1, N}):
        pos = np.sort(rng.choice(N, K, replace=False)).astype(np.uint16)
        r = rng.uniform(-64, 64, (2, K))
        c, a, u = oracle.block_green(w, h, pos, r, 0, s)
        for t in range(2):
            np.testing.assert_allclose(u[t], brute.solve_eq1(w, h, pos, r[t], A), atol=1e-9)


@pytest.mark.parametrize("w,h", [(4, 3), (8, 8), (16, 12)])
def test_eq4_dct_evaluation(w, h):
    """u from Eq. (4), IDCT(lambda * DCT(M c)) + a with scipy, equals the
    oracle's direct Green sum: pins the evaluation step."""
    rng = _rng(w + h)
    N = w * h
    K = max(2, N // 8)
    pos = np.sort(rng.choice(N, K, replace=False)).astype(np.uint16)
    r = rng.uniform(-64, 64, K)
    c, a, u = oracle.block_green(w, h, pos, r)
    lam = oracle.eigenvalues(w, h, 0, 1.0)
    np.testing.assert_allclose(brute.eq4_evaluate(w, h, pos, c[0], a[0], lam), u[0], atol=1e-10)


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("w,h", [(16, 16), (16, 8), (7, 5)])
def test_single_point_gives_constant(w, h):
    for p in (0, w * h - 1, (w * h) // 2):
        pos = np.array([p], dtype=np.uint16)
        np.testing.assert_allclose(oracle.block_direct(w, h, pos, [3.25]), 3.25, atol=1e-12)
        c, a, u = oracle.block_green(w, h, pos, [3.25])
        np.testing.assert_allclose(u[0], 3.25, atol=1e-12)
        assert abs(c[0, 0]) < 1e-12


def test_constant_data_gives_constant_and_zero_coefficients():
    rng = _rng(3)
    pos = np.sort(rng.choice(256, 20, replace=False)).astype(np.uint16)
    c, a, u = oracle.block_green(16, 16, pos, np.full(20, -7.5))
    np.testing.assert_allclose(u[0], -7.5, atol=1e-11)
    np.testing.assert_allclose(c[0], 0.0, atol=1e-11)


@pytest.mark.parametrize("w", [5, 16, 32])
def test_row_block_is_linear_interpolation(w):
    """On a w x 1 block the harmonic inpainting is piecewise-linear between
    the mask points and constant beyond the outermost ones (numpy.interp)."""
    rng = _rng(w)
    for K in (2, 3, max(2, w // 3)):
        pos = np.sort(rng.choice(w, K, replace=False))
        r = rng.uniform(-64, 64, K)
        ref = np.interp(np.arange(w), pos, r)
        np.testing.assert_allclose(oracle.block_direct(w, 1, pos.astype(np.uint16), r)[0], ref, atol=1e-10)
        np.testing.assert_allclose(oracle.block_direct(1, w, pos.astype(np.uint16), r)[:, 0], ref, atol=1e-10)
        np.testing.assert_allclose(oracle.block_green(w, 1, pos.astype(np.uint16), r)[2][0, 0], ref, atol=1e-10)


@pytest.mark.parametrize("w,h", [(16, 16), (16, 8), (9, 4)])
def test_two_edge_columns_give_ramp(w, h):
    """Full first and last columns with values 0 and w-1 give u(x,y) = x;
    rows give u = y (catches x/y swaps)."""
    pos = np.array(sorted([y * w for y in range(h)] + [y * w + w - 1 for y in range(h)]), np.uint16)
    r = np.array([0.0 if p % w == 0 else w - 1.0 for p in pos])
    ramp = np.tile(np.arange(w, dtype=float), (h, 1))
    np.testing.assert_allclose(oracle.block_direct(w, h, pos, r), ramp, atol=1e-10)
    np.testing.assert_allclose(oracle.block_green(w, h, pos, r)[2][0], ramp, atol=1e-10)
    pos = np.array(list(range(w)) + list(range((h - 1) * w, h * w)), np.uint16)
    r = np.array([0.0] * w + [h - 1.0] * w)
    ramp = np.tile(np.arange(h, dtype=float)[:, None], (1, w))
    np.testing.assert_allclose(oracle.block_green(w, h, pos, r)[2][0], ramp, atol=1e-10)


def test_empty_and_full_masks():
    """K = 0 gives u = 0 (reading); K = w*h gives u = r."""
    np.testing.assert_array_equal(oracle.block_direct(4, 3, np.zeros(0, np.uint16), []), 0.0)
    c, a, u = oracle.block_green(4, 3, np.zeros(0, np.uint16), np.zeros((1, 0)))
    np.testing.assert_array_equal(u, 0.0)
    r = np.arange(12, dtype=float) * 1.5 - 4
    np.testing.assert_allclose(oracle.block_direct(4, 3, np.arange(12), r).ravel(), r, atol=1e-12)
    np.testing.assert_allclose(oracle.block_green(4, 3, np.arange(12), r)[2][0].ravel(), r, atol=1e-10)


# -------------------------------------------------------------- invariants

@pytest.mark.parametrize("w,h", [(16, 16), (16, 12), (32, 32)])
def test_invariants(w, h):
    """Exact interpolation, maximum principle, harmonic off-mask, sum c = 0,
    c = A u at the mask points (A u = M c), a = block mean, linearity."""
    rng = _rng(w * h)
    N = w * h
    A = brute.neg_laplacian(w, h)
    for K in (3, N // 20, N // 5):
        pos = np.sort(rng.choice(N, K, replace=False)).astype(np.uint16)
        r = rng.uniform(-64, 64, (2, K))
        c, a, u = oracle.block_green(w, h, pos, r)
        for t in range(2):
            uf = u[t].ravel()
            np.testing.assert_allclose(uf[pos], r[t], atol=1e-9)
            assert r[t].min() - 1e-9 <= uf.min() and uf.max() <= r[t].max() + 1e-9
            Au = A @ uf
            off = np.setdiff1d(np.arange(N), pos)
            np.testing.assert_allclose(Au[off], 0.0, atol=1e-9)
            np.testing.assert_allclose(Au[pos], c[t], atol=1e-9)
            assert abs(c[t].sum()) < 1e-9
            assert abs(a[t] - uf.mean()) < 1e-9
        np.testing.assert_allclose(u[0] * 2.0 - u[1] * 0.5,
                                   oracle.block_green(w, h, pos, 2.0 * r[0] - 0.5 * r[1])[2][0], atol=1e-9)


def test_dihedral_equivariance():
    """Transposing / flipping a square block transposes / flips u."""
    rng = _rng(11)
    w = h = 8
    pos = np.sort(rng.choice(64, 9, replace=False))
    r = rng.uniform(-64, 64, 9)
    u = oracle.block_direct(w, h, pos.astype(np.uint16), r)
    x, y = pos % w, pos // w
    for xf, yf, tr, fn in [
        (x, y, True, lambda a: a.T),
        (w - 1 - x, y, False, lambda a: a[:, ::-1]),
        (x, h - 1 - y, False, lambda a: a[::-1, :]),
    ]:
        p2 = (xf * h + yf) if tr else (yf * w + xf)
        order = np.argsort(p2)
        u2 = oracle.block_green(w, h, p2[order].astype(np.uint16), r[order])[2][0]
        np.testing.assert_allclose(u2, fn(u), atol=1e-10)


# -------------------------------------------------------------- frames

def test_frame_matches_per_block_solves():
    """Frame decode = every block decoded alone and placed at its offset in
    its plane; blocks are independent images (Sec. 2.2).  Catches block order,
    plane offsets and the shared chroma value runs (Cr vs Cb)."""
    fr = synth.random_frame(70, 37, synth.YUV420, 16, (0.02, 0.2), seed=5)
    planes = oracle.decode(fr, method=oracle.DIRECT)
    ref = [np.full(p.shape, np.nan) for p in planes]
    for blk in fr.iter_blocks():
        for vp, vals in zip(blk["planes"], blk["values"]):
            u = brute.solve_eq1(blk["w"], blk["h"], blk["pos"], vals.astype(float),
                                brute.neg_laplacian(blk["w"], blk["h"]))
            ref[vp][blk["y0"]:blk["y0"] + blk["h"], blk["x0"]:blk["x0"] + blk["w"]] = u
    for p, q in zip(planes, ref):
        assert not np.isnan(q).any()
        np.testing.assert_allclose(p, q, atol=1e-9)


def test_frame_reproduces_field_at_mask_points():
    """Exact interpolation at frame level: u equals the drawn residual field at
    every mask pixel of every plane (pins value-run alignment)."""
    fr = synth.random_frame(100, 60, synth.YUV420, 16, (0.01, 0.1), seed=1)
    planes = oracle.decode(fr, method=oracle.GREEN)
    for blk in fr.iter_blocks():
        px = blk["x0"] + blk["pos"].astype(int) % blk["w"]
        py = blk["y0"] + blk["pos"].astype(int) // blk["w"]
        for vp in blk["planes"]:
            np.testing.assert_allclose(planes[vp][py, px],
                                       fr.fields[vp][py, px].astype(np.float32), atol=1e-9)


def test_frame_routes_agree_and_locality():
    fr = synth.config_frame(0)
    a = oracle.decode(fr, method=oracle.DIRECT)[0]
    b = oracle.decode(fr, method=oracle.GREEN)[0]
    np.testing.assert_allclose(a, b, atol=1e-9)
    # perturb the values of block 37 only
    fr2 = synth.config_frame(0)
    lo, hi = fr2.block_ptr[37], fr2.block_ptr[38]
    fr2.values = fr2.values.copy()
    fr2.values[lo:hi] += 10.0
    c = oracle.decode(fr2, method=oracle.DIRECT)[0]
    diff = np.abs(c - a) > 0
    by, bx = divmod(37, 16)
    expect = np.zeros_like(diff)
    expect[by * 16:(by + 1) * 16, bx * 16:(bx + 1) * 16] = True
    np.testing.assert_array_equal(diff, expect)


def test_separate_chroma_masks():
    fr = synth.random_frame(48, 40, synth.YUV420, 16, (0.05, 0.2), seed=9, chroma_shared=False)
    a = oracle.decode(fr, method=oracle.DIRECT)
    b = oracle.decode(fr, method=oracle.GREEN)
    for p, q in zip(a, b):
        np.testing.assert_allclose(p, q, atol=1e-9)


def test_planted_mistake_is_caught():
    """The pins are sharp: a perturbed table (a plausible wrong weight) breaks
    the pseudo-inverse pin by far more than its tolerance."""
    w, h = 4, 3
    G = oracle.green_matrix(w, h)
    P = np.linalg.pinv(brute.neg_laplacian(w, h))
    assert np.abs(G - P).max() < 1e-11
    lam = oracle.eigenvalues(w, h).ravel()
    C = np.kron(brute.dct_matrix(h), brute.dct_matrix(w))
    lam_bad = lam.copy()
    lam_bad[1] *= 1.01
    assert np.abs(C.T @ np.diag(lam_bad) @ C - P).max() > 1e-4


# ------------------------------------------------- stored coefficients

def test_dequant_codes():
    """Dead-zone reconstruction (Sec. 2.3): hand-computed values; catches a
    lost offset, a wrong sign for negative codes or a zero that comes back
    non-zero."""
    cases = [(0, 0.5, 0.5, 0.0), (3, 0.5, 0.5, 1.75), (-2, 0.5, 0.5, -1.25), (1, 2.0, 0.0, 2.0),
             (-127, 1.0, 0.25, -127.25), (127, 0.125, 0.0, 15.875), (0, 7.0, 0.9, 0.0)]
    for q, step, rho, want in cases:
        assert oracle.dequant([q], step, rho)[0] == want, (q, step, rho)


def _coef_identity(w, h, pos, c, a, u):
    """u solves A u = M c - mean_k(M c) with mean(u) = a, A = -L built by
    Kronecker products (no Green's table, no DCT); these fix u uniquely."""
    A = brute.neg_laplacian(w, h)
    mc = np.zeros(w * h)
    mc[np.asarray(pos, dtype=np.int64)] = c
    np.testing.assert_allclose(A @ u.ravel(), mc - mc.mean(), atol=1e-9 * max(1.0, np.abs(c).sum()))
    assert abs(u.mean() - a) <= 1e-10 * max(1.0, abs(a) + np.abs(u).max())


@pytest.mark.parametrize("fmt,shared", [(synth.GRAY, True), (synth.YUV420, True), (synth.YUV420, False)])
def test_coef_decode_solves_operator_equation(fmt, shared):
    """Every block of a frame decoded from codes satisfies A u = M c -
    mean(M c) and mean(u) = a (Eq. 2 with G the pseudo-inverse of A and the
    constant its null space), for ragged edge blocks, K = 0, K = w*h, shared
    and separate chroma masks; catches a wrong Green's weight or sign, a
    code read from the wrong run, a constant of the wrong block or plane."""
    W, H, b = 21, 13, 8
    # one empty and one full block in the Y plane
    rng = _rng(4)
    ms, fs = [], []
    dims = synth.plane_dims(W, H, fmt)
    for k, (pw, ph) in enumerate(dims):
        m = rng.uniform(size=(ph, pw)) < 0.3
        if k == 0:
            m[:8, :8] = False
            m[:8, 8:16] = True
        ms.append(m)
        fs.append(rng.uniform(-64, 64, (ph, pw)))
    if fmt == synth.YUV420 and shared:
        ms = ms[:2]
    fr = synth.pack_dense(W, H, fmt, b, ms, fs)
    q, consts = synth.coef_inputs(fr, 7)
    steps = (0.5, 0.25, 0.75)
    rho = 0.5
    planes = oracle.decode_coef(fr, q, consts, steps, rho)
    # walk the documented layout independently of the oracle
    bp = fr.block_ptr
    groups = [[0]] if fmt == synth.GRAY else ([[0], [1, 2]] if fr.chroma_shared else [[0], [1], [2]])
    cbase = np.concatenate([[0], np.cumsum(synth.plane_block_counts(W, H, fmt, b))])
    m = 0
    chroma_first = None
    runs = []
    for gp in groups:
        pw, ph = dims[gp[0]]
        if gp[0] == 1:
            chroma_first = m
        for k, (x0, y0, w, h) in enumerate(synth.block_grid(pw, ph, b)):
            runs.append((gp, k, x0, y0, w, h, m))
            m += 1
    nnz = bp[m]
    checked = 0
    for gp, k, x0, y0, w, h, mb in runs:
        lo, hi = bp[mb], bp[mb + 1]
        pos = fr.pos[lo:hi]
        for pl in gp:
            vb = nnz + (lo - bp[chroma_first]) if (pl == 2 and fr.chroma_shared) else lo
            codes = q[vb:vb + (hi - lo)].astype(np.float64)
            c = np.where(codes == 0, 0.0, np.sign(codes) * (np.abs(codes) + rho) * steps[pl])
            a = float(consts[cbase[pl] + k])
            u = planes[pl][y0:y0 + h, x0:x0 + w]
            _coef_identity(w, h, pos, c, a, u)
            checked += 1
    assert checked == sum(synth.plane_block_counts(W, H, fmt, b))


def test_coef_zero_codes_give_constant():
    """All codes zero: every block is its constant."""
    fr = synth.random_frame(24, 16, synth.YUV420, 8, (0.1, 0.4), seed=5)
    q = np.zeros(fr.values.size, np.int8)
    consts = np.arange(sum(synth.plane_block_counts(24, 16, synth.YUV420, 8)), dtype=np.float32) - 7.0
    planes = oracle.decode_coef(fr, q, consts, (1.0, 1.0, 1.0), 0.5)
    k = 0
    for pl, (pw, ph) in enumerate(synth.plane_dims(24, 16, synth.YUV420)):
        for (x0, y0, w, h) in synth.block_grid(pw, ph, 8):
            assert np.all(planes[pl][y0:y0 + h, x0:x0 + w] == consts[k])
            k += 1


def test_coef_round_trip_of_the_solve():
    """Coefficients taken from the plain definition (c = A u at the mask
    points of the Eq. (1) solution, a = its mean), stored with a fine step,
    decode back to that solution within the quantisation bound: the stored
    form is the same inpainting (Sec. 2.2, last paragraph)."""
    w = h = 8
    rng = _rng(12)
    pos = np.sort(rng.choice(w * h, 9, replace=False))
    r = rng.uniform(-64, 64, pos.size)
    u = brute.solve_eq1(w, h, pos, r, brute.operator(w, h, 1))
    c = (brute.neg_laplacian(w, h) @ u.ravel())[pos]
    step = np.abs(c).max() / 120.0
    qc = np.rint(c / step).astype(np.int8)
    fr = synth.pack_dense(w, h, synth.GRAY, 8, [np.isin(np.arange(w * h), pos).reshape(h, w)],
                          [u.reshape(h, w)])
    got = oracle.decode_coef(fr, qc, np.array([u.mean()], np.float32), (step,), 0.0)[0]
    G = np.linalg.pinv(brute.neg_laplacian(w, h))
    bound = 0.5 * step * np.abs(G).max() * pos.size + 1e-4
    assert np.abs(got - u.reshape(h, w)).max() <= bound


# ------------------------------------------------- coefficient encoder

def test_quant_codes():
    """Dead-zone quantisation (Sec. 2.3): hand-computed codes; catches a
    rounding instead of a floor, a lost dead zone, a wrong sign for negative
    coefficients or a missing cap at 127."""
    cases = [(0.3, 1.0, 0), (-0.99, 1.0, 0), (1.0, 1.0, 1), (-2.99, 1.0, -2), (3.75, 0.5, 7),
             (-3.75, 0.5, -7), (-200.0, 1.0, -127), (0.0, 0.25, 0), (1000.0, 0.125, 127), (0.5, 0.25, 2)]
    for c, step, want in cases:
        assert oracle.quant([c], step)[0] == want, (c, step)


def test_quant_inverts_dequant_intervals():
    """A code is the interval its reconstruction lies in: for rho in [0, 1)
    dequant(q) and c fall in the same interval [|q| step, (|q|+1) step) with
    the same sign, and q = 0 exactly when |c| < step."""
    rng = _rng(21)
    c = rng.normal(0, 20, 4000)
    step = 0.37
    q = oracle.quant(c, step)
    lo = oracle.dequant(q, step, 0.0)
    hi = oracle.dequant(q, step, 1.0 - 1e-12)
    nz = (q != 0) & (np.abs(q) < 127)
    assert np.all(np.abs(lo[nz]) <= np.abs(c[nz]) + 1e-12) and np.all(np.abs(c[nz]) < np.abs(hi[nz]) + 1e-9)
    assert np.all(np.sign(q[nz]) == np.sign(c[nz]))
    assert np.all((q == 0) == (np.abs(c) < step))


def _encode_frame(fmt, shared, seed):
    W, H, b = 21, 13, 8
    rng = _rng(seed)
    ms, fs = [], []
    dims = synth.plane_dims(W, H, fmt)
    for k, (pw, ph) in enumerate(dims):
        m = rng.uniform(size=(ph, pw)) < 0.3
        if k == 0:
            m[:8, :8] = False     # K = 0
            m[:8, 8:16] = True    # K = w*h
        ms.append(m)
        fs.append(rng.uniform(-64, 64, (ph, pw)))
    if fmt == synth.YUV420 and shared:
        ms = ms[:2]
    return synth.pack_dense(W, H, fmt, b, ms, fs)


@pytest.mark.parametrize("fmt,shared", [(synth.GRAY, True), (synth.YUV420, True), (synth.YUV420, False)])
def test_encode_coef_is_the_plain_solution(fmt, shared):
    """The encoder's c and a on every block are those of the plain
    definition: with u the Eq. (1) solution (dense Kronecker solve, no
    Green's table), c = (A u) at the mask points and a = mean(u) (0 for an
    empty block); the codes lie in c's quantiser interval.  Ragged edge
    blocks, K = 0, K = w*h, shared and separate chroma masks; catches a
    coefficient or constant written to the wrong run, block or plane."""
    fr = _encode_frame(fmt, shared, 22)
    W, H, b = fr.width, fr.height, fr.block_size
    steps = (0.5, 0.25, 0.75)
    code, cex, consts = oracle.encode_coef(fr, steps)
    dims = synth.plane_dims(W, H, fmt)
    bp = fr.block_ptr
    groups = [[0]] if fmt == synth.GRAY else ([[0], [1, 2]] if fr.chroma_shared else [[0], [1], [2]])
    cbase = np.concatenate([[0], np.cumsum(synth.plane_block_counts(W, H, fmt, b))])
    m, chroma_first, runs = 0, None, []
    for gp in groups:
        pw, ph = dims[gp[0]]
        if gp[0] == 1:
            chroma_first = m
        for k, (x0, y0, w, h) in enumerate(synth.block_grid(pw, ph, b)):
            runs.append((gp, k, w, h, m))
            m += 1
    nnz = bp[m]
    seen_full = seen_empty = 0
    for gp, k, w, h, mb in runs:
        lo, hi = bp[mb], bp[mb + 1]
        pos = np.asarray(fr.pos[lo:hi], dtype=np.int64)
        K = pos.size
        seen_full += K == w * h
        seen_empty += K == 0
        for pl in gp:
            vb = nnz + (lo - bp[chroma_first]) if (pl == 2 and fr.chroma_shared) else lo
            r = np.asarray(fr.values[vb:vb + K], dtype=np.float64)
            a = consts[cbase[pl] + k]
            if K == 0:
                assert a == 0.0
                continue
            u = brute.solve_eq1(w, h, pos, r, brute.operator(w, h, 1)).ravel()
            c_ref = (brute.neg_laplacian(w, h) @ u)[pos]
            np.testing.assert_allclose(cex[vb:vb + K], c_ref, atol=1e-8 * max(1.0, np.abs(c_ref).max()))
            assert abs(a - u.mean()) <= 1e-9 * max(1.0, np.abs(u).max())
            q = code[vb:vb + K].astype(np.int64)
            c = cex[vb:vb + K]
            st = steps[pl]
            assert np.all((q == 0) == (np.abs(c) < st))
            nz = (q != 0) & (np.abs(q) < 127)
            assert np.all(np.abs(q[nz]) * st <= np.abs(c[nz]) + 1e-12)
            assert np.all(np.abs(c[nz]) < (np.abs(q[nz]) + 1) * st)
            assert np.all(np.sign(q[nz]) == np.sign(c[nz]))
    assert seen_full >= 1 and seen_empty >= 1


def test_encode_decode_round_trip():
    """Codes and constants from the encoder decode (stored-coefficient
    decoder) to the plain-definition inpainting of the same mask and values
    within the quantisation bound: per pixel at most sum_i |c_i - c^_i|
    |G(x, x_i)| <= step * K * max|G| with rho = 0.5; a fine step brings the
    two together (Sec. 2.2's split reproduces the inpainting)."""
    fr = synth.random_frame(40, 24, synth.YUV420, 8, (0.05, 0.3), seed=23)
    ref = oracle.decode_flat(fr)
    cmax = np.abs(oracle.encode_coef(fr, (1.0, 1.0, 1.0))[1]).max()
    # steps that map every coefficient into [-127, 127] (no code saturates)
    for step in (cmax / 32.0, cmax / 127.0):
        steps = (step, step, step)
        code, _, consts = oracle.encode_coef(fr, steps)
        got = oracle.decode_coef_flat(fr, code, consts.astype(np.float32), steps, 0.5)
        G = np.linalg.pinv(brute.neg_laplacian(8, 8))
        Kmax = int(np.diff(fr.block_ptr).max())
        bound = step * Kmax * np.abs(G).max() + 1e-3
        err = np.abs(got - ref).max()
        assert err <= bound, (step, err, bound)
    assert err <= 0.5  # the fine step meets the decoder's acceptance bar


# ----------------------------------------- mask selection (subdivision)

@pytest.mark.parametrize("name", ["subdivide_5x1.txt", "subdivide_3x3.txt"])
def test_golden_subdivision(name):
    """Hand-derived subdivisions: catches a split at the wrong threshold side
    (strictly greater), a wrong mid-point, the wrong axis on a tie, or an
    error averaged over the wrong pixels."""
    rows = _read_golden(name)
    w, h = map(int, rows[0])
    r = np.array(rows[1:1 + h])
    for row in rows[1 + h:]:
        T, want = row[0], np.array(row[1:], dtype=bool).reshape(h, w)
        got = oracle.select_mask(w, h, synth.GRAY, 8, [r], True, (T, T))[0]
        assert np.array_equal(got, want), (name, T, got.astype(int))


def _corner_mask(W, H, b):
    m = np.zeros((H, W), bool)
    for (x0, y0, w, h) in synth.block_grid(W, H, b):
        for x in (x0, x0 + w - 1):
            for y in (y0, y0 + h - 1):
                m[y, x] = True
    return m


@pytest.mark.parametrize("b", [8, 16])
def test_subdivision_limits(b):
    """No split (threshold above every error) leaves exactly the corners of
    every block, ragged edge blocks included; splitting whenever possible
    (negative threshold) reaches every pixel; constant planes never split."""
    W, H = 2 * b + 5, b + 3
    rng = _rng(31)
    planes = [rng.uniform(-64, 64, (h, w)) for (w, h) in synth.plane_dims(W, H, synth.YUV420)]
    dims = synth.plane_dims(W, H, synth.YUV420)
    for shared in (True, False):
        ms = oracle.select_mask(W, H, synth.YUV420, b, planes, shared, (1e300, 1e300))
        for m, (pw, ph) in zip(ms, dims):
            assert np.array_equal(m, _corner_mask(pw, ph, b))
        ms = oracle.select_mask(W, H, synth.YUV420, b, planes, shared, (-1.0, -1.0))
        assert all(m.all() for m in ms)
    const = [np.full((h, w), 7.5) for (w, h) in dims]
    ms = oracle.select_mask(W, H, synth.YUV420, b, const, True, (1e-9, 1e-9))
    for m, (pw, ph) in zip(ms, dims):
        assert np.array_equal(m, _corner_mask(pw, ph, b))


def _subdivide_brute(r, T):
    """The subdivision rounds on one block with Eq. (1) solved by the dense
    Kronecker route (no Green's table): an independent inpainting and
    independent bookkeeping (rectangles as sets of their pixels)."""
    h, w = r.shape
    rects = [(0, w - 1, 0, h - 1)]
    while True:
        known = set()
        for x0, x1, y0, y1 in rects:
            known |= {(x0, y0), (x1, y0), (x0, y1), (x1, y1)}
        if len(known) == w * h:
            break
        pos = np.array(sorted(y * w + x for x, y in known))
        u = brute.solve_eq1(w, h, pos, r.ravel()[pos], brute.operator(w, h, 1)).reshape(h, w)
        new = []
        for x0, x1, y0, y1 in rects:
            e = ((u[y0:y1 + 1, x0:x1 + 1] - r[y0:y1 + 1, x0:x1 + 1]) ** 2).mean()
            gx, gy = x1 - x0, y1 - y0
            if e > T and max(gx, gy) >= 2:
                if gx >= gy:
                    m = (x0 + x1) // 2
                    new += [(x0, m, y0, y1), (m, x1, y0, y1)]
                else:
                    m = (y0 + y1) // 2
                    new += [(x0, x1, y0, m), (x0, x1, m, y1)]
            else:
                new.append((x0, x1, y0, y1))
        if len(new) == len(rects):
            break
        rects = new
    m = np.zeros((h, w), bool)
    for x0, x1, y0, y1 in rects:
        for x, y in ((x0, y0), (x1, y0), (x0, y1), (x1, y1)):
            m[y, x] = True
    return m


@pytest.mark.parametrize("w,h", [(8, 8), (5, 7), (8, 3), (2, 6)])
def test_subdivision_matches_brute_force(w, h):
    """Random blocks and thresholds: the oracle's masks equal the dense-solve
    re-run of the rounds (thresholds well away from every error, so FP64
    rounding cannot flip a decision)."""
    rng = _rng(32 + w * h)
    for trial in range(6):
        r = rng.uniform(-64, 64, (h, w)) if trial % 2 else \
            np.cumsum(rng.normal(0, 6, (h, w)), axis=1)
        for T in (2.0, 20.0, 150.0):
            got = oracle.select_mask(w, h, synth.GRAY, 8, [r], True, (T, T))[0]
            assert np.array_equal(got, _subdivide_brute(r, T)), (w, h, trial, T)


def test_subdivision_shared_chroma_averages_errors():
    """One chroma mask for both chroma planes (Sec. 2.3) is chosen on the
    mean of their errors: equal planes give the single-plane mask; a zero Cr
    plane halves the error, as doubling the threshold on Cb alone does."""
    W, H = 40, 24
    rng = _rng(33)
    dims = synth.plane_dims(W, H, synth.YUV420)
    y = rng.uniform(-64, 64, dims[0][::-1])
    cb = np.cumsum(rng.normal(0, 5, dims[1][::-1]), axis=1)
    T = 6.0
    sep = oracle.select_mask(W, H, synth.YUV420, 8, [y, cb, cb], False, (T, T))
    sh = oracle.select_mask(W, H, synth.YUV420, 8, [y, cb, cb], True, (T, T))
    assert np.array_equal(sh[1], sep[1]) and np.array_equal(sh[0], sep[0])
    sh0 = oracle.select_mask(W, H, synth.YUV420, 8, [y, cb, np.zeros_like(cb)], True, (T, T))
    sep2 = oracle.select_mask(W, H, synth.YUV420, 8, [y, cb, cb], False, (T, 2 * T))
    assert np.array_equal(sh0[1], sep2[1])


# ------------------------------------- global homogeneous diffusion inpainting

@pytest.mark.parametrize("W,H,d", [(7, 5, 0.3), (12, 9, 0.1), (16, 11, 0.05), (23, 14, 0.2)])
def test_homogeneous_equals_block_route(W, H, d):
    """Eq. (1) on the whole image is Eq. (1) on one W x H block: the sparse
    solve equals the banded-Cholesky route of the per-block oracle."""
    rng = _rng(W * 100 + H)
    m = rng.uniform(size=(H, W)) < d
    m[rng.integers(H), rng.integers(W)] = True
    f = rng.uniform(-64, 64, (H, W))
    pos = np.flatnonzero(m.ravel())
    ref = oracle.block_direct(W, H, pos, f.ravel()[pos])
    got = oracle.homogeneous_inpaint(m, f)
    np.testing.assert_allclose(got, ref, atol=1e-9)


def test_homogeneous_row_is_linear_interpolation():
    """One image row: linear interpolation between known pixels, constant
    continuation past the outermost ones (reflecting boundary)."""
    m = np.zeros((1, 12), bool)
    m[0, [2, 7, 9]] = True
    f = np.zeros((1, 12))
    f[0, [2, 7, 9]] = [4.0, -6.0, 10.0]
    u = oracle.homogeneous_inpaint(m, f)[0]
    want = np.array([4, 4, 4, 2, 0, -2, -4, -6, 2, 10, 10, 10], float)
    np.testing.assert_allclose(u, want, atol=1e-12)


def test_homogeneous_invariants():
    """Interpolation at the mask, A u = 0 off the mask (A = -L by Kronecker
    products), maximum principle, one known pixel gives a constant, an empty
    mask gives 0 (reading)."""
    rng = _rng(77)
    H, W = 19, 26
    m = rng.uniform(size=(H, W)) < 0.06
    f = rng.uniform(-64, 64, (H, W))
    u = oracle.homogeneous_inpaint(m, f)
    assert np.all(u[m] == f[m])
    Au = brute.neg_laplacian(W, H) @ u.ravel()
    assert np.abs(Au[~m.ravel()]).max() < 1e-9
    assert u.min() >= f[m].min() - 1e-9 and u.max() <= f[m].max() + 1e-9
    one = np.zeros((H, W), bool)
    one[3, 4] = True
    np.testing.assert_allclose(oracle.homogeneous_inpaint(one, f), f[3, 4], atol=1e-9)
    assert np.all(oracle.homogeneous_inpaint(np.zeros((H, W), bool), f) == 0)


# ------------------------------------------------- property-based checks

def test_routes_agree_on_random_blocks():
    """Hypothesis-drawn blocks (any shape up to 7x7, any non-empty point
    subset short of the whole block, any values): the plain definition
    (banded Cholesky of Eq. 1) and the Green's route (Eqs. 2-4, dense LU of
    the bordered system) give the same u, and c satisfies A u = M c - mean."""
    hyp = pytest.importorskip("hypothesis")
    st = hyp.strategies

    @hyp.settings(max_examples=60, deadline=None, derandomize=True)
    @hyp.given(st.integers(1, 7), st.integers(1, 7), st.data())
    def check(w, h, data):
        N = w * h
        if N < 2:
            return
        K = data.draw(st.integers(1, N - 1))
        pos = np.array(sorted(data.draw(st.lists(st.integers(0, N - 1), min_size=K, max_size=K, unique=True))),
                       dtype=np.uint16)
        r = np.array(data.draw(st.lists(st.floats(-64, 64, allow_nan=False), min_size=K, max_size=K)))
        u1 = oracle.block_direct(w, h, pos, r)
        c, a, u2 = oracle.block_green(w, h, pos, r)
        np.testing.assert_allclose(u2[0], u1, atol=1e-8 * max(1.0, np.abs(r).max()))
        _coef_identity(w, h, pos, c[0], a[0], u2[0])

    check()
