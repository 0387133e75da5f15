"""SparseStack embedding S (paper Sec. 2.2) and the sketch S*A.

Test infrastructure only (see ``oracle/__init__``).

Definition (Sec. 2.2, "Choice of embedding"): S = zeta^{-1/2} [s_1 ... s_m];
each column s_i is cut into zeta equally sized pieces, and each piece holds one
entry +-1 at a uniformly random position.  The paper does not say how
"uniformly random" is drawn nor how pieces are sized when zeta does not divide
d; this package follows the counter spec below, which the HIP side implements
separately from the same text:

  pieces   len_j = floor(d/zeta) + (1 if j < d mod zeta else 0),
           start_j = sum_{l<j} len_l                      (j = 0..zeta-1)
  hash     h(i, j) = splitmix64(seed XOR splitmix64(i*zeta + j))  (64-bit wrap)
  position row(i, j) = start_j + floor((h mod 2^32) * len_j / 2^32)
  sign     -1 if bit 63 of h is set, else +1

splitmix64 is Steele, Lea and Flood's mixer (OOPSLA 2014, the generator of
java.util.SplittableRandom): z = x + 0x9E3779B97F4A7C15;
z = (z ^ z>>30) * 0xBF58476D1CE4E5B9; z = (z ^ z>>27) * 0x94D049BB133111EB;
return z ^ z>>31.

The sketch adds the +-1 rows exactly and applies the factor zeta^{-1/2} once
at the end, so an integer-valued A gives an exactly representable S*A before
the final scaling.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_MUL1 = np.uint64(0xBF58476D1CE4E5B9)
_MUL2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x) -> np.ndarray:
    """splitmix64 finaliser applied elementwise to uint64 counters."""
    z = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _MUL1
        z = (z ^ (z >> np.uint64(27))) * _MUL2
        return z ^ (z >> np.uint64(31))


def piece_bounds(d: int, zeta: int):
    """(starts, lens) of the zeta pieces of a length-d column."""
    if not (1 <= zeta <= d):
        raise ValueError("need 1 <= zeta <= d")
    base, extra = divmod(d, zeta)
    lens = np.array([base + (1 if j < extra else 0) for j in range(zeta)], dtype=np.int64)
    starts = np.zeros(zeta, dtype=np.int64)
    starts[1:] = np.cumsum(lens)[:-1]
    return starts, lens


def draw(m: int, d: int, zeta: int, seed: int, row0: int = 0):
    """Nonzero rows and signs of columns s_{row0} .. s_{row0+m-1}.

    Returns ``rows`` (m, zeta) int64 and ``signs`` (m, zeta) float64 in {-1, +1}.
    """
    starts, lens = piece_bounds(d, zeta)
    i = np.arange(row0, row0 + m, dtype=np.uint64)[:, None]
    j = np.arange(zeta, dtype=np.uint64)[None, :]
    with np.errstate(over="ignore"):
        ctr = i * np.uint64(zeta) + j
    h = splitmix64(np.uint64(seed) ^ splitmix64(ctr))
    off = ((h & np.uint64(0xFFFFFFFF)) * lens[None, :].astype(np.uint64)) >> np.uint64(32)
    rows = starts[None, :] + off.astype(np.int64)
    signs = np.where((h >> np.uint64(63)) == np.uint64(1), -1.0, 1.0)
    return rows, signs


def embedding(m: int, d: int, zeta: int, seed: int) -> sp.csr_matrix:
    """Unscaled S (entries +-1) as a d x m sparse matrix: S_paper = zeta^{-1/2} * this."""
    rows, signs = draw(m, d, zeta, seed)
    cols = np.repeat(np.arange(m, dtype=np.int64), zeta)
    return sp.csr_matrix((signs.ravel(), (rows.ravel(), cols)), shape=(d, m))


def scale_factor(zeta: int) -> float:
    """zeta^{-1/2} rounded once (IEEE sqrt and division are correctly rounded)."""
    return 1.0 / math.sqrt(zeta)


def sketch(A, d: int, zeta: int, seed: int) -> np.ndarray:
    """S*A (d x n): exact +-1 row accumulation, then one multiply by zeta^{-1/2}."""
    A = np.asarray(A)
    S = embedding(A.shape[0], d, zeta, seed)
    Y = np.asarray(S @ A)
    return Y * scale_factor(zeta)
