"""Pins for oracle.eft against exact rational arithmetic."""

from fractions import Fraction

import numpy as np
import pytest

from oracle import eft

U = 2.0 ** -53


def _rand_wide(rng, size):
    return rng.standard_normal(size) * 2.0 ** rng.integers(-60, 60, size)


def test_two_sum_and_two_prod_are_error_free():
    rng = np.random.default_rng(0)
    a = _rand_wide(rng, 400)
    b = _rand_wide(rng, 400)
    s, e = eft.two_sum(a, b)
    p, f = eft.two_prod(a, b)
    for ai, bi, si, ei, pi, fi in zip(a, b, s, e, p, f):
        assert Fraction(ai) + Fraction(bi) == Fraction(si) + Fraction(ei)
        assert Fraction(ai) * Fraction(bi) == Fraction(pi) + Fraction(fi)


def _ill_conditioned(rng, n, cond_exp):
    """Dot products with heavy cancellation: big terms that cancel plus small ones."""
    x = rng.standard_normal(n) * 2.0 ** rng.integers(0, cond_exp, n)
    y = rng.standard_normal(n)
    half = n // 2
    x[half:2 * half] = -x[:half]
    y[half:2 * half] = y[:half] * (1 + rng.standard_normal(half) * 2.0 ** -40)
    return x, y


def test_dot2_error_bound_against_exact():
    """Ogita-Rump-Oishi Prop. 5.5: |res - x'y| <= u|x'y| + gamma_n^2 |x|'|y|."""
    rng = np.random.default_rng(1)
    plain_failures = 0
    for trial in range(40):
        n = int(rng.integers(2, 300))
        x, y = _ill_conditioned(rng, n, 50)
        exact = sum(Fraction(float(xi)) * Fraction(float(yi)) for xi, yi in zip(x, y))
        got = eft.dot2(x, y)
        gamma = n * U / (1 - n * U)
        absdot = float(np.sum(np.abs(x * y)))
        bound = U * abs(float(exact)) + gamma * gamma * absdot * 1.0001
        assert abs(Fraction(got) - exact) <= Fraction(bound)
        plain = float(np.dot(x, y))
        if abs(Fraction(plain) - exact) > Fraction(bound):
            plain_failures += 1
    assert plain_failures > 10          # the inputs are hard enough to matter


def test_matmul_real_and_complex_match_scalar_dot2_and_exact():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((70, 33)) * 2.0 ** rng.integers(-20, 20, (70, 33))
    W = rng.standard_normal((33, 3))
    got = eft.matmul(A, W, row_chunk=16)
    for i in range(70):
        for j in range(3):
            assert got[i, j] == eft.dot2(A[i], W[:, j])
    Ac = A + 1j * rng.standard_normal((70, 33))
    Wc = W + 1j * rng.standard_normal((33, 3))
    gc = eft.matmul(Ac, Wc, row_chunk=32)
    for i in range(0, 70, 9):
        for j in range(3):
            re = sum(Fraction(float(a.real)) * Fraction(float(w.real)) -
                     Fraction(float(a.imag)) * Fraction(float(w.imag)) for a, w in zip(Ac[i], Wc[:, j]))
            im = sum(Fraction(float(a.real)) * Fraction(float(w.imag)) +
                     Fraction(float(a.imag)) * Fraction(float(w.real)) for a, w in zip(Ac[i], Wc[:, j]))
            scale_r = float(np.sum(np.abs(Ac[i].real * Wc[:, j].real)) + np.sum(np.abs(Ac[i].imag * Wc[:, j].imag)))
            scale_i = float(np.sum(np.abs(Ac[i].real * Wc[:, j].imag)) + np.sum(np.abs(Ac[i].imag * Wc[:, j].real)))
            g = 66 * U
            assert abs(Fraction(float(gc[i, j].real)) - re) <= Fraction(U * abs(float(re)) + 2 * g * g * scale_r)
            assert abs(Fraction(float(gc[i, j].imag)) - im) <= Fraction(U * abs(float(im)) + 2 * g * g * scale_i)
    v = eft.matmul(A, W[:, 0])
    assert v.shape == (70,) and np.array_equal(v, got[:, 0])


def test_matmul_h_tree_dot2_against_exact():
    """A^* Y summed over the long axis with the pairwise TwoSum tree."""
    rng = np.random.default_rng(4)
    m, n = 3001, 7
    A = rng.standard_normal((m, n)) * 2.0 ** rng.integers(-30, 30, (m, n))
    y = rng.standard_normal(m)
    half = m // 2
    A[half:2 * half] = -A[:half]
    y[half:2 * half] = y[:half] * (1 + rng.standard_normal(half) * 2.0 ** -45)
    got = eft.matmul_h(A, y, row_chunk=500)
    g = 2 * np.log2(m) * U
    for c in range(n):
        exact = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(A[:, c], y))
        bound = U * abs(float(exact)) + g * g * float(np.sum(np.abs(A[:, c] * y)))
        assert abs(Fraction(float(got[c])) - exact) <= Fraction(bound)
    # plain summation misses that bound on these inputs
    plain = A.T @ y
    misses = sum(abs(Fraction(float(plain[c])) - sum(Fraction(float(a)) * Fraction(float(b))
                                                    for a, b in zip(A[:, c], y))) >
                 Fraction(U * 1e-3 * float(np.sum(np.abs(A[:, c] * y)))) for c in range(n))
    assert misses >= 1


def test_matmul_h_complex_against_exact():
    rng = np.random.default_rng(6)
    m, n = 257, 3
    A = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    Y = rng.standard_normal((m, 2)) + 1j * rng.standard_normal((m, 2))
    got = eft.matmul_h(A, Y, row_chunk=64)
    for c in range(n):
        for j in range(2):
            a, y = A[:, c], Y[:, j]
            re = sum(Fraction(float(p.real)) * Fraction(float(q.real)) + Fraction(float(p.imag)) * Fraction(float(q.imag))
                     for p, q in zip(a, y))
            im = sum(Fraction(float(p.real)) * Fraction(float(q.imag)) - Fraction(float(p.imag)) * Fraction(float(q.real))
                     for p, q in zip(a, y))
            sc = float(np.sum(np.abs(a) * np.abs(y))) * 2
            g = 2 * np.log2(2 * m) * U
            assert abs(Fraction(float(got[c, j].real)) - re) <= Fraction(U * abs(float(re)) + g * g * sc)
            assert abs(Fraction(float(got[c, j].imag)) - im) <= Fraction(U * abs(float(im)) + g * g * sc)
    assert np.allclose(got, A.conj().T @ Y, rtol=1e-12, atol=1e-12)


def test_c_forms_give_the_numpy_forms_bits():
    """oracle/eft_c.c performs the numpy forms' operations in the same order,
    so both give identical bits (real and complex, ragged row chunks, chunk
    boundaries across the stacked real and imaginary rows, every thread
    count)."""
    if not eft.have_c():
        from oracle import build as obuild
        obuild.build()
        eft._clib_handle = None
    assert eft.have_c()
    rng = np.random.default_rng(11)
    for (m, n, b, cp) in [(20001, 7, 3, False), (257, 3, 2, True), (5000, 40, 2, True), (16385, 33, 1, False),
                          (3, 5, 2, True), (1, 1, 1, False)]:
        A = rng.standard_normal((m, n)) * np.logspace(0, -12, n)[None, :]
        W = rng.standard_normal((n, b))
        Y = rng.standard_normal((m, b))
        if cp:
            A = A + 1j * rng.standard_normal((m, n))
            W = W + 1j * rng.standard_normal((n, b))
            Y = Y + 1j * rng.standard_normal((m, b))
        for nt in (1, 3):
            eft.set_threads(nt)
            assert np.array_equal(eft.matmul(A, W), eft._matmul_numpy(A, W))
            for rc in (64, 8192):
                assert np.array_equal(eft.matmul_h(A, Y, row_chunk=rc), eft._matmul_h_numpy(A, Y, row_chunk=rc))
    # a strided row view is read through its leading dimension
    A = rng.standard_normal((300, 40))
    W = rng.standard_normal((25, 2))
    assert np.array_equal(eft.matmul(A[:, :25], W), eft._matmul_numpy(A[:, :25], W))
    with pytest.raises(ValueError):
        eft.matmul_h(A, rng.standard_normal((299, 1)))
