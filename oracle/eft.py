"""Error-free transformations and the compensated dot product Dot2.

Test infrastructure only (see ``oracle/__init__``).

Published algorithms, restated:
  TwoSum      Knuth (TAOCP vol. 2, 4.2.2): s = fl(a+b), e = (a+b) - s exactly.
  Split       Veltkamp/Dekker (Dekker 1971): a = hi + lo, each half fits in
              26 bits, with the factor 2^27 + 1.
  TwoProduct  Dekker (1971): p = fl(a*b), e = a*b - p exactly (no FMA needed).
  Dot2        Ogita, Rump and Oishi, SIAM J. Sci. Comput. 26(6), 2005, Alg. 5.3:
              the dot product computed as if in twice the working precision
              and rounded once; error <= u|x'y| + gamma_n^2 |x|'|y|.

Why the oracle needs Dot2: on tall matrices whose smallest singular values sit
far below ||A||, a plain FP64 product A*v is accurate only to about
u*||row||*||v|| per entry, which is far above |(Av)_i|; that rounding noise
alone moves the computed minimum singular vector by up to
u*||A||_F / (sqrt(m) * sigma_{n-1}) (Sec. 4, accuracy floors).  Computing the
products with A as Dot2 removes that floor on both the oracle and the GPU side.
"""

from __future__ import annotations

import numpy as np

_SPLITTER = 134217729.0  # 2^27 + 1


def two_sum(a, b):
    s = a + b
    z = s - a
    e = (a - (s - z)) + (b - z)
    return s, e


def split(a):
    c = _SPLITTER * a
    hi = c - (c - a)
    lo = a - hi
    return hi, lo


def two_prod(a, b):
    p = a * b
    ah, al = split(a)
    bh, bl = split(b)
    e = al * bl - (((p - ah * bh) - al * bh) - ah * bl)
    return p, e


def _two_prod_presplit(a, ah, al, b, bh, bl):
    p = a * b
    e = al * bl - (((p - ah * bh) - al * bh) - ah * bl)
    return p, e


def dot2(x, y) -> float:
    """Dot2 of two real vectors (Ogita-Rump-Oishi Alg. 5.3)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.size == 0:
        return 0.0
    p, s = two_prod(x[0], y[0])
    for i in range(1, x.size):
        h, r = two_prod(x[i], y[i])
        p, q = two_sum(p, h)
        s = s + (q + r)
    return float(p + s)


def _dot2_rows(XT: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Dot2 of every column of XT (L x rows) with y (L,): one result per row."""
    L, rows = XT.shape
    if L == 0:
        return np.zeros(rows)
    yh, yl = split(y)
    x0 = XT[0]
    x0h, x0l = split(x0)
    p, s = _two_prod_presplit(x0, x0h, x0l, y[0], yh[0], yl[0])
    for i in range(1, L):
        xi = XT[i]
        xh, xl = split(xi)
        h, r = _two_prod_presplit(xi, xh, xl, y[i], yh[i], yl[i])
        p, q = two_sum(p, h)
        s = s + (q + r)
    return p + s


def matmul(A, W, row_chunk: int = 16384) -> np.ndarray:
    """A @ W with every entry computed by Dot2 (real or complex A, W)."""
    A = np.asarray(A)
    W = np.asarray(W)
    vec = W.ndim == 1
    if vec:
        W = W[:, None]
    m, n = A.shape
    b = W.shape[1]
    cplx = np.iscomplexobj(A) or np.iscomplexobj(W)
    out = np.empty((m, b), dtype=np.complex128 if cplx else np.float64)
    for r0 in range(0, m, row_chunk):
        blk = A[r0:r0 + row_chunk]
        if cplx:
            blk = np.asarray(blk, dtype=np.complex128)
            # Re(a.w) = [Re a, Im a].[Re w, -Im w]; Im(a.w) = [Re a, Im a].[Im w, Re w]
            XT = np.ascontiguousarray(np.concatenate([blk.real, blk.imag], axis=1).T)
            for j in range(b):
                w = W[:, j].astype(np.complex128)
                re = _dot2_rows(XT, np.concatenate([w.real, -w.imag]))
                im = _dot2_rows(XT, np.concatenate([w.imag, w.real]))
                out[r0:r0 + blk.shape[0], j] = re + 1j * im
        else:
            XT = np.ascontiguousarray(np.asarray(blk, dtype=np.float64).T)
            for j in range(b):
                out[r0:r0 + blk.shape[0], j] = _dot2_rows(XT, W[:, j].astype(np.float64))
    return out[:, 0] if vec else out
