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

  Dot2 tree  The same transformations applied pairwise along the long axis
              (TwoSum of pairs, errors carried and summed in working
              precision): exact partial sums plus an error term, so the
              result is again within u|x'y| + O(log2(n) u^2) |x|'|y|.  Used for
              A^* Y, whose sums run over the m >> n rows.

Why the oracle needs Dot2: on tall matrices whose smallest singular values sit
far below ||A||, a plain FP64 product A*v is accurate only to about
u*||row||*||v|| per entry, which is far above |(Av)_i|; that rounding noise
alone moves the computed minimum singular vector by up to
u*||A||_F / (sqrt(m) * sigma_{n-1}) (Sec. 4, accuracy floors).  The residual
A^*(A v) - theta^2 v of the search direction has the same problem: computed
with a plain A^*, its rounding floor keeps two otherwise identical runs (two
sketch seeds) about 2e-9 apart in angle on a 6e4 x 200 matrix with
sigma_{n-1}/sigma_n = 10 and sigma_n = 1e-12, and about 6e-16 apart when A^* is
applied as Dot2 as well.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_SPLITTER = 134217729.0  # 2^27 + 1
_CLIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_eft_c.so")
_clib_handle = None


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


def _matmul_numpy(A, W, row_chunk: int = 16384) -> np.ndarray:
    """A @ W with every entry computed by Dot2 (real or complex A, W), in numpy."""
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


def _tree_sum(P: np.ndarray, E: np.ndarray):
    """Sum P + E along axis 0: TwoSum on pairs, errors carried in E (exact in P)."""
    while P.shape[0] > 1:
        if P.shape[0] % 2:
            P = np.concatenate([P, np.zeros_like(P[:1])], axis=0)
            E = np.concatenate([E, np.zeros_like(E[:1])], axis=0)
        s, t = two_sum(P[0::2], P[1::2])
        E = (E[0::2] + E[1::2]) + t
        P = s
    return P[0], E[0]


def _stacked_rows(parts, r0: int, r1: int) -> np.ndarray:
    """Rows r0:r1 of the vertical stack of ``parts`` (each rows x n), built
    without forming the whole stack."""
    out, base = [], 0
    for p in parts:
        lo, hi = max(r0, base), min(r1, base + p.shape[0])
        if lo < hi:
            out.append(p[lo - base:hi - base])
        base += p.shape[0]
    return out[0] if len(out) == 1 else np.concatenate(out, axis=0)


def _dot2_cols(parts, y: np.ndarray, row_chunk: int):
    """sum_r X[r, c] * y[r] for every column c, Dot2-class (real X, y), where X
    is the vertical stack of ``parts``; it is read in chunks of ``row_chunk``
    rows, so only one chunk of the stack is ever formed."""
    n = parts[0].shape[1]
    total = sum(p.shape[0] for p in parts)
    acc_s = np.zeros(n)
    acc_e = np.zeros(n)
    for r0 in range(0, total, row_chunk):
        blk = _stacked_rows(parts, r0, min(r0 + row_chunk, total))
        yb = y[r0:r0 + row_chunk][:, None]
        P, E = two_prod(blk, yb)
        ps, pe = _tree_sum(P, E)
        acc_s, t = two_sum(acc_s, ps)
        acc_e = acc_e + pe + t
    return acc_s + acc_e


class _Negated:
    """-M, negated one slice at a time (a row block of -A.imag on demand)."""

    def __init__(self, M):
        self.M = M
        self.shape = M.shape

    def __getitem__(self, idx):
        return -self.M[idx]


def _matmul_h_numpy(A, Y, row_chunk: int = 8192) -> np.ndarray:
    """A^* @ Y (A m x n, Y m x b) with every entry Dot2-class accurate, in numpy."""
    A = np.asarray(A)
    Y = np.asarray(Y)
    vec = Y.ndim == 1
    if vec:
        Y = Y[:, None]
    n, b = A.shape[1], Y.shape[1]
    cplx = np.iscomplexobj(A) or np.iscomplexobj(Y)
    out = np.empty((n, b), dtype=np.complex128 if cplx else np.float64)
    if cplx:
        A = np.asarray(A, dtype=np.complex128)
        # conj(a) y: Re = [ar; ai] . [yr; yi], Im = [ar; -ai] . [yi; yr] (sums over 2m terms)
        ar, ai = A.real, A.imag
        for j in range(b):
            y = Y[:, j].astype(np.complex128)
            re = _dot2_cols((ar, ai), np.concatenate([y.real, y.imag]), row_chunk)
            im = _dot2_cols((ar, _Negated(ai)), np.concatenate([y.imag, y.real]), row_chunk)
            out[:, j] = re + 1j * im
    else:
        for j in range(b):
            out[:, j] = _dot2_cols((np.asarray(A, dtype=np.float64),), Y[:, j].astype(np.float64), row_chunk)
    return out[:, 0] if vec else out


# ---------------------------------------------------------------- C forms
#
# ``oracle/eft_c.c`` performs the same operations in the same order as the
# numpy forms above (so the same bits; tests/test_oracle_eft.py checks it)
# with OpenMP threads over rows (A W) or columns (A^* Y).  The C forms are
# used when ``oracle/_eft_c.so`` is built (``oracle/build.py``).

def _clib():
    global _clib_handle
    if _clib_handle is None:
        if os.environ.get("RL_ORACLE_NUMPY") == "1" or not os.path.exists(_CLIB_PATH):
            _clib_handle = False
        else:
            lib = ctypes.CDLL(_CLIB_PATH)
            P, I64 = ctypes.c_void_p, ctypes.c_int64
            lib.eft_matmul.argtypes = [P, I64, I64, I64, P, I64, I64, ctypes.c_int, P, I64]
            lib.eft_matmul_h.argtypes = [P, I64, I64, I64, P, I64, I64, ctypes.c_int, I64, P, I64]
            lib.eft_set_threads.argtypes = [ctypes.c_int]
            lib.eft_get_threads.restype = ctypes.c_int
            _clib_handle = lib
    return _clib_handle or None


def have_c() -> bool:
    return _clib() is not None


def set_threads(nt: int) -> None:
    """Threads of the C forms (OpenMP); no effect on the numpy forms."""
    lib = _clib()
    if lib is not None:
        lib.eft_set_threads(int(nt))


def get_threads() -> int:
    lib = _clib()
    return int(lib.eft_get_threads()) if lib is not None else 1


def _as_rows(M, dt):
    """M as a C-ordered array of dtype dt whose rows may be strided."""
    M = np.asarray(M, dtype=dt)
    if M.ndim != 2 or M.strides[1] != M.itemsize or M.strides[0] % M.itemsize:
        M = np.ascontiguousarray(M)
    return M, M.strides[0] // M.itemsize


def matmul(A, W, row_chunk: int = 16384) -> np.ndarray:
    """A @ W with every entry computed by Dot2 (real or complex A, W)."""
    lib = _clib()
    if lib is None:
        return _matmul_numpy(A, W, row_chunk)
    A = np.asarray(A)
    W = np.asarray(W)
    vec = W.ndim == 1
    if vec:
        W = W[:, None]
    cplx = np.iscomplexobj(A) or np.iscomplexobj(W)
    dt = np.complex128 if cplx else np.float64
    A, lda = _as_rows(A, dt)
    W, ldw = _as_rows(W, dt)
    m, n = A.shape
    b = W.shape[1]
    if W.shape[0] != n:
        raise ValueError("matmul: W must have as many rows as A has columns")
    out = np.empty((m, b), dtype=dt)
    lib.eft_matmul(A.ctypes.data, m, n, lda, W.ctypes.data, b, ldw, int(cplx), out.ctypes.data, b)
    return out[:, 0] if vec else out


def matmul_h(A, Y, row_chunk: int = 8192) -> np.ndarray:
    """A^* @ Y (A m x n, Y m x b) with every entry Dot2-class accurate."""
    lib = _clib()
    if lib is None:
        return _matmul_h_numpy(A, Y, row_chunk)
    A = np.asarray(A)
    Y = np.asarray(Y)
    vec = Y.ndim == 1
    if vec:
        Y = Y[:, None]
    cplx = np.iscomplexobj(A) or np.iscomplexobj(Y)
    dt = np.complex128 if cplx else np.float64
    A, lda = _as_rows(A, dt)
    Y, ldy = _as_rows(Y, dt)
    m, n = A.shape
    b = Y.shape[1]
    if Y.shape[0] != m:
        raise ValueError("matmul_h: Y must have as many rows as A")
    out = np.empty((n, b), dtype=dt)
    lib.eft_matmul_h(A.ctypes.data, m, n, lda, Y.ctypes.data, b, ldy, int(cplx), int(row_chunk),
                     out.ctypes.data, b)
    return out[:, 0] if vec else out
