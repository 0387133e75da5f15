"""Pins for oracle.eft against exact rational arithmetic."""

from fractions import Fraction

import numpy as np

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
