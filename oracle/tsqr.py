"""Reference SVD of a tall matrix for checks at full size.

Test infrastructure only (see ``oracle/__init__``).

A = Q R by Householder QR of row blocks, the block R factors stacked and
factored again (a one-level TSQR), then the LAPACK SVD of the n x n R:
A = (Q U_R) Sigma V_R^*.  Householder QR is backward stable, so Sigma and V_R
are the singular data of a matrix within u*||A|| of A, with host memory of
about one row block beyond A itself.
"""

from __future__ import annotations

import numpy as np


def r_factor(A, row_block: int = 1 << 16) -> np.ndarray:
    A = np.asarray(A)
    m, n = A.shape
    rs = []
    for r0 in range(0, m, row_block):
        rs.append(np.linalg.qr(A[r0:r0 + row_block], mode="r"))
    Rst = np.vstack(rs)
    return np.linalg.qr(Rst, mode="r")


def tall_svd(A, row_block: int = 1 << 16):
    """(sigma descending, V with V[:, j] the j-th right singular vector)."""
    R = r_factor(A, row_block)
    _, s, Vh = np.linalg.svd(R)
    return s, Vh.conj().T
