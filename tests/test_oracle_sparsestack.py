"""Pins for oracle.sparsestack (SparseStack, paper Sec. 2.2)."""

import math
import os

import numpy as np
import pytest

from oracle import sparsestack as ss

MASK = (1 << 64) - 1


def _golden_splitmix(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "splitmix64.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            vals = [int(v) for v in line.split()]
            rows.append((vals[0], vals[1:]))
    return rows


def test_splitmix64_published_outputs(golden_dir):
    gamma = 0x9E3779B97F4A7C15
    for seed, outs in _golden_splitmix(golden_dir):
        state = seed
        for expect in outs:
            got = int(ss.splitmix64(np.uint64(state)))
            assert got == expect
            state = (state + gamma) & MASK


def _py_splitmix(x):
    z = (x + 0x9E3779B97F4A7C15) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def _py_target(i, j, d, zeta, seed):
    """One nonzero of S from the counter spec, with Python integers."""
    base, extra = divmod(d, zeta)
    lens = [base + (1 if q < extra else 0) for q in range(zeta)]
    start = sum(lens[:j])
    h = _py_splitmix(seed ^ _py_splitmix((i * zeta + j) & MASK))
    row = start + (((h & 0xFFFFFFFF) * lens[j]) >> 32)
    sign = -1.0 if (h >> 63) else 1.0
    return row, sign


@pytest.mark.parametrize("d,zeta", [(200, 8), (37, 8), (9, 4), (5, 5), (7, 1)])
def test_piece_bounds(d, zeta):
    starts, lens = ss.piece_bounds(d, zeta)
    assert lens.sum() == d
    assert lens.max() - lens.min() <= 1
    assert list(lens) == sorted(lens, reverse=True)          # the longer pieces come first
    assert starts[0] == 0 and all(starts[1:] == np.cumsum(lens)[:-1])


def test_draw_matches_integer_spec_and_large_seeds():
    m, d, zeta = 300, 37, 8
    for seed in (0, 2002, (1 << 63) + 12345):
        rows, signs = ss.draw(m, d, zeta, seed)
        for i in range(0, m, 7):
            for j in range(zeta):
                r, s = _py_target(i, j, d, zeta, seed)
                assert rows[i, j] == r and signs[i, j] == s
    # an offset block of columns equals the same columns of a full draw
    rows_a, signs_a = ss.draw(100, d, zeta, 5, row0=200)
    rows_b, signs_b = ss.draw(300, d, zeta, 5)
    assert np.array_equal(rows_a, rows_b[200:]) and np.array_equal(signs_a, signs_b[200:])


def test_one_nonzero_per_piece():
    m, d, zeta = 5000, 203, 8
    rows, signs = ss.draw(m, d, zeta, 77)
    starts, lens = ss.piece_bounds(d, zeta)
    assert np.all(rows >= starts[None, :]) and np.all(rows < (starts + lens)[None, :])
    assert set(np.unique(signs)) == {-1.0, 1.0}
    S = ss.embedding(m, d, zeta, 77).toarray()
    assert np.array_equal((S != 0).sum(axis=0), np.full(m, zeta))


def test_positions_and_signs_uniform():
    """Positions uniform within each piece, signs fair (chi-square, fixed seed)."""
    m, d, zeta = 200_000, 64, 8
    rows, signs = ss.draw(m, d, zeta, 2024)
    starts, lens = ss.piece_bounds(d, zeta)
    for j in range(zeta):
        counts = np.bincount(rows[:, j] - starts[j], minlength=lens[j])
        expect = m / lens[j]
        chi2 = float(((counts - expect) ** 2 / expect).sum())
        dof = lens[j] - 1
        assert chi2 < dof + 6 * math.sqrt(2 * dof)
    frac_neg = float((signs < 0).mean())
    assert abs(frac_neg - 0.5) < 6 * math.sqrt(0.25 / signs.size)


def test_sketch_equals_dense_product_and_is_exact_for_integers():
    from workloads import integer_matrix
    m, n, d, zeta, seed = 700, 9, 40, 8, 31
    A = integer_matrix(m, n, 3)
    S = np.zeros((d, m))
    for i in range(m):
        for j in range(zeta):
            r, s = _py_target(i, j, d, zeta, seed)
            S[r, i] += s
    Y = ss.sketch(A, d, zeta, seed)
    exact = S @ A                        # integers: exact in FP64
    assert np.array_equal(Y, exact * (1.0 / math.sqrt(zeta)))
    Ac = integer_matrix(m, n, 4, is_complex=True)
    assert np.array_equal(ss.sketch(Ac, d, zeta, seed), (S @ Ac) * (1.0 / math.sqrt(zeta)))


def test_embedding_is_isometric_on_average_and_a_subspace_embedding():
    """Columns of zeta^{-1/2} S have unit norm, so E||Sx||^2 = ||x||^2.  The
    preconditioner P is unchanged up to a scalar when S is rescaled, so the
    distortion that matters is the scale-free one, eta' = (k^2-1)/(k^2+1) with
    k = sigma_max(SQ)/sigma_min(SQ): with d = 4n, zeta = 8 the drawn S embeds an
    n-dimensional subspace with eta' well below 1 (Def. 1.1, Fact
    fact:sketching_constructions)."""
    m, n, zeta = 20_000, 50, 8
    d = 4 * n
    S = ss.embedding(m, d, zeta, 9) * ss.scale_factor(zeta)
    col_norm2 = np.asarray(S.multiply(S).sum(axis=0)).ravel()
    assert np.allclose(col_norm2, 1.0, rtol=0, atol=4e-16)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((m, 400))
    X /= np.linalg.norm(X, axis=0)
    mean_sq = float(np.mean(np.linalg.norm(np.asarray(S @ X), axis=0) ** 2))
    assert abs(mean_sq - 1.0) < 0.02
    Q, _ = np.linalg.qr(rng.standard_normal((m, n)))
    sv = np.linalg.svd(np.asarray(S @ Q), compute_uv=False)
    k2 = (sv.max() / sv.min()) ** 2
    eta_scale_free = (k2 - 1.0) / (k2 + 1.0)
    assert 0.0 < eta_scale_free < 0.9
