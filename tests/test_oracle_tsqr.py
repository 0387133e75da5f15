"""Pins for oracle.tsqr (blocked R factor + SVD of R) against dense LAPACK
and planted singular values."""

import numpy as np

from oracle import tsqr
from workloads import planted_numpy, spectrum_gap


def test_r_factor_matches_dense_qr_up_to_row_phases():
    rng = np.random.default_rng(11)
    A = rng.standard_normal((5003, 17)) + 1j * rng.standard_normal((5003, 17))
    R = tsqr.r_factor(A, row_block=700)
    Rd = np.linalg.qr(A, mode="r")
    # R^* R = A^* A determines R up to a unit phase per row
    ph = np.diag(Rd) / np.diag(R)
    assert np.allclose(np.abs(ph), 1.0, atol=1e-12)
    assert np.allclose(R * ph[:, None], Rd, atol=1e-11 * np.abs(Rd).max())
    assert np.allclose(np.tril(R, -1), 0.0)


def test_tall_svd_recovers_planted_spectrum_and_vectors():
    sig = spectrum_gap(30, 3, 1e-9, 100.0)
    A, V, s = planted_numpy(20_000, 30, sig, 5, is_complex=False)
    got_s, got_V = tsqr.tall_svd(A, row_block=3000)
    assert np.all(np.abs(got_s - s) <= 1e-14 * s[0] + 1e-13 * s)
    # the three smallest right vectors span the planted ones (gap 100)
    Vo = V[:, -3:]
    P = got_V[:, -3:]
    sin = np.linalg.norm(Vo - P @ (P.conj().T @ Vo), 2)
    assert sin <= 1e-6
    dense = np.linalg.svd(A, compute_uv=False)
    assert np.allclose(got_s, dense, rtol=0, atol=1e-14)
