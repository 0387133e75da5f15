"""RLOBPCG, plain CPU FP64: the k smallest singular triplets of a tall A.

Test infrastructure only (see ``oracle/__init__``).

What is computed (Sec. 1, Sec. 2.1, Sec. 2.3): LOBPCG for the smallest
eigenpairs of the Gram matrix A^* A, preconditioned by P P^* = ((S A)^* S A)^{-1}
from a SparseStack sketch S A (Sec. 2.2), started from the sketch-and-solve
block (the smallest right singular vectors of S A), with the paper's stopping
rule.  b = 1 is Alg. rlopcg and b > 1 Alg. rlobpcg; both are the same
iteration on a block of width b.  The code is organised by the mathematical
pieces the method is built from, each a function below:

  sketch preconditioner   P, Sigma~(1,1) and the start block from S A
  rayleigh_ritz           Ritz pairs of A^* A on span(T) for an orthonormal T,
                          read off the SVD of the product A T (the Ritz values
                          are the singular values of A T)
  search_block            eq:search-direction: W = P P^* R, made orthonormal
                          and orthogonal to the current basis [V X] (two block
                          Gram-Schmidt projections, then Orth)
  previous_direction      eq:x-defining: the part of the new Ritz block that
                          lies outside the old V, as an orthonormal block X
                          with its product A X, both from the Ritz
                          coefficients (no product with A)
  residual                R = A^* (A V) - V Theta^2, one column per Ritz pair
  left_vectors            U-hat from the Ritz block's product A V

Each step of the loop builds the trial basis T = [V X W] (t = 3b columns; 2b
while X is still empty), applies Rayleigh-Ritz to it, keeps the b smallest
Ritz pairs as the new V, forms their residual, consults the stopping rule
(``oracle.termination``) and, if the loop goes on, the next X.

Readings where the paper is silent:
  * On the first step X is empty, so t = 2b, and the next X comes from the
    b x b block of coefficients of the old V.
  * Orth is the thin Householder QR (numpy/LAPACK); Normalize (Orth of one
    column) of a zero or non-finite vector returns e_1 and raises the
    ``degenerate`` flag.
  * Singular values come in descending order, as MATLAB's svd returns them;
    the output is sorted ascending.
  * ^* is the conjugate transpose throughout; S is real.
  * The b = 1 start keeps theta_0 = inf and v_0 unrotated (Alg. rlopcg); for
    b > 1 the start block is first rotated by Rayleigh-Ritz on span(V_0)
    (Alg. rlobpcg).
  * U-hat_j = A_V(:, j) / theta_j (zero, with the ``zero_theta`` flag, if
    theta_j = 0).  ``refresh=True`` (the default) recomputes A_V = A V-hat
    once at the end and rotates (V-hat, sigma, U-hat) by the SVD of that
    m x b block, so the outputs carry no drift of the maintained products;
    ``refresh=False`` returns the last Rayleigh-Ritz triplets as they are.
  * ``precond="qr"`` uses R from S A = Q R with P = R^{-1}; P P^* = (R^* R)^{-1}
    = ((S A)^* S A)^{-1} = V~ Sigma~^{-2} V~^*, the same operator as the SVD
    route (Sec. 1, footnote on QR), with V_0 taken from the SVD of R.
  * ``loop_precond`` swaps the loop's preconditioner for the diagonal one
    (P = diag(||A(:, i)||^{-1})) or none, keeping the sketch-and-solve start
    (Sec. 1.1 initialises every compared method with v_0).
  * ``orth="svqb"`` replaces Orth(W) after the two block projections by
    SVQB (Gram matrix, eigendecomposition), the faster, less stable option
    the paper names for this step.
  * ``lock=True`` (Sec. 2.3, the locking paragraph; soft locking): once column
    j of V meets eq:est_conv_criterion on its own (||R(:, j)|| <=
    Sigma~(1,1)^2 tau) it is locked for good.  A locked column stays in V and
    in every Rayleigh-Ritz step, but gets no search direction: W = P P^* R
    over the active columns only, and the next X is built from the active
    columns of the old V only, X = T C(:, 1:t-b) Orth(C(act, 1:t-b)^*) (the
    part of span{V_i(:, act)} outside the new V; with every column active
    this is eq:x-defining).  So t = b + a_X + a_W, and both added blocks are
    orthogonal to every column of V, the locked ones included.  The loop also
    ends (status 0) once every column is locked.
  * ``dot2=True`` computes every product with A (A V_0, A W, the refresh) and
    the residual's A^* A_V as Dot2-class sums (``oracle.eft``); without it the
    FP64 rounding floor of those products, not the iteration, limits the
    attainable angle on strongly graded spectra (Sec. 4, accuracy floors).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from . import eft, sparsestack, termination

EPS_MATLAB = 2.0 ** -52


def default_tau(n: int) -> float:
    """tau = 2 n^{1/2} eps_mach (Sec. 2.1), eps_mach = 2^-52 as in MATLAB."""
    return 2.0 * math.sqrt(n) * EPS_MATLAB


@dataclass
class RLResult:
    sigma: np.ndarray          # k smallest singular values, ascending
    V: np.ndarray              # n x k right singular vectors (matching sigma)
    U: np.ndarray              # m x k left singular vectors
    iters: int                 # loop iterations executed
    status: int                # 0 stopped by the rule, 1 hit max_iter
    sigma1: float              # Sigma~(1,1), the sketch's largest singular value
    theta_hist: list = field(default_factory=list)   # theta_j per iterate (length b)
    rnorm_hist: list = field(default_factory=list)   # ||r_j(:, c)|| per iterate
    degenerate: bool = False
    zero_theta: bool = False
    V_block: np.ndarray | None = None     # final block V (n x b), paper order
    theta_block: np.ndarray | None = None
    lock_hist: list = field(default_factory=list)    # active mask after each iterate (lock=True)


def _ct(M: np.ndarray) -> np.ndarray:
    return M.conj().T


# ---------------------------------------------------------------- orthonormal bases

def _orth(M: np.ndarray):
    """Orth (thin Householder QR); a single column is Normalize.  Returns the
    basis and whether Normalize met a zero (or non-finite) vector, in which
    case the basis is e_1."""
    if M.shape[1] == 1:
        nrm = np.linalg.norm(M[:, 0])
        if nrm == 0.0 or not np.isfinite(nrm):
            e = np.zeros_like(M)
            e[0, 0] = 1.0
            return e, True
        return M / nrm, False
    Q, _ = np.linalg.qr(M)
    return Q, False


def _svqb(M: np.ndarray):
    """Orth by SVQB (Stathopoulos and Wu, the faster alternative the paper
    names for the orthogonalisation step): G = M^* M scaled to unit diagonal,
    D G D = Z Lambda Z^*, result M D Z Lambda^{-1/2}.  Eigenvalues below
    eps * max(Lambda) are raised to that value (their safeguard); a zero
    column, or a block with no positive eigenvalue, falls back to Orth."""
    G = _ct(M) @ M
    dg = np.real(np.diag(G))
    if np.any(dg <= 0.0) or not np.all(np.isfinite(dg)):
        Q, _ = _orth(M)
        return Q, True
    dsc = 1.0 / np.sqrt(dg)
    lam, Z = np.linalg.eigh(dsc[:, None] * G * dsc[None, :])
    lmax = float(lam.max())
    if not lmax > 0.0:
        Q, _ = _orth(M)
        return Q, True
    lam = np.maximum(lam, EPS_MATLAB * lmax)
    return M @ (dsc[:, None] * Z / np.sqrt(lam)[None, :]), False


# ---------------------------------------------------------------- preconditioners

@dataclass
class _SketchData:
    sigma1: float          # Sigma~(1,1), the largest singular value of S A
    V0: np.ndarray         # the b smallest right singular vectors of S A (n x b)
    apply_prec: object     # R -> P P^* R


def _sketch_preconditioner(SA: np.ndarray, b: int, precond: str) -> _SketchData:
    """Sec. 1 step 2 and the sketch-and-solve start: from S A, the operator
    P P^* = ((S A)^* S A)^{-1}, Sigma~(1,1) and the smallest right singular
    subspace of S A.  "svd": P = V~ Sigma~^{-1} from the SVD of S A (the
    paper's route); "qr": P = R^{-1} from S A = Q R (the same operator)."""
    n = SA.shape[1]
    if precond == "svd":
        _, St, Vth = np.linalg.svd(SA, full_matrices=False)
        Vt = _ct(Vth)
        P = Vt / St[None, :]                                  # P = V~ Sigma~^{-1}

        def apply_prec(Rm):
            return P @ (_ct(P) @ Rm)
        return _SketchData(float(St[0]), Vt[:, n - b:].copy(), apply_prec)
    if precond == "qr":
        Rf = np.linalg.qr(SA, mode="r")
        _, Sr, Vrh = np.linalg.svd(Rf)

        def apply_prec(Rm):
            Z = sla.solve_triangular(Rf, Rm, trans="C", lower=False)
            return sla.solve_triangular(Rf, Z, lower=False)
        return _SketchData(float(Sr[0]), _ct(Vrh)[:, n - b:].copy(), apply_prec)
    raise ValueError(f"unknown precond {precond!r}")


def _loop_preconditioner(A: np.ndarray, kind: str, sketch_prec):
    """The preconditioner of the LOBPCG loop (Sec. 1.1's comparison methods):
    the sketch's, the diagonal P = diag(||A(:, i)||^{-1}) (P P^* =
    diag(||A(:, i)||^{-2}); a zero column keeps P(i, i) = 1), or none."""
    if kind == "sketch":
        return sketch_prec
    if kind == "diag":
        cn2 = np.sum(np.abs(A) ** 2, axis=0)
        dscale = np.where(cn2 > 0.0, 1.0 / np.where(cn2 > 0.0, cn2, 1.0), 1.0)

        def apply_prec(Rm):
            return dscale[:, None] * Rm
        return apply_prec
    if kind == "none":
        def apply_prec(Rm):
            return Rm.copy()
        return apply_prec
    raise ValueError(f"unknown loop_precond {kind!r}")


# ---------------------------------------------------------------- the LOBPCG pieces

def rayleigh_ritz(AT: np.ndarray):
    """Ritz data of A^* A on span(T), T orthonormal, from the product A T:
    A T = U_T Theta C^* gives the Ritz values Theta^2 (descending Theta) and
    the coefficients C of the Ritz vectors T C (Sec. 2.1, the SVD of A_T)."""
    _, Th, Ch = np.linalg.svd(AT, full_matrices=False)
    return Th, _ct(Ch)


def search_block(R: np.ndarray, apply_prec, basis: np.ndarray, orth_fn):
    """eq:search-direction: W = P P^* R, then two block projections against
    span(basis) (block classical Gram-Schmidt, twice) and an orthonormal basis
    of the result.  Returns W and Orth's degenerate flag."""
    W = apply_prec(R)
    W = W - basis @ (_ct(basis) @ W)
    return orth_fn(W - basis @ (_ct(basis) @ W))


def previous_direction(T: np.ndarray, AT: np.ndarray, C: np.ndarray, b: int, act=None):
    """eq:x-defining: X spans the components of the non-selected Ritz vectors
    along the old V, i.e. X = T C(:, 1:t-b) Q with Q = Orth(C(1:b, 1:t-b)^*),
    and A X = A_T C(:, 1:t-b) Q.  With a lock mask ``act`` only the active
    columns of the old V contribute: Q = Orth(C(act, 1:t-b)^*), one column
    of X per active index.  Returns X, A X and Orth's degenerate flag."""
    t = T.shape[1]
    rows = np.arange(b) if act is None else np.flatnonzero(act)
    Q, flag = _orth(_ct(C[rows, :t - b]))
    CX = C[:, :t - b] @ Q
    return T @ CX, AT @ CX, flag


def lock_update(act: np.ndarray, R: np.ndarray, sigma1: float, tau: float) -> np.ndarray:
    """Sec. 2.3 (locking): column j stays active until its residual meets
    eq:est_conv_criterion, ||R(:, j)|| <= Sigma~(1,1)^2 tau; a locked column
    never becomes active again."""
    return act & ~(np.linalg.norm(R, axis=0) <= sigma1 * sigma1 * tau)


def residual(AV: np.ndarray, V: np.ndarray, theta: np.ndarray, mulAh) -> np.ndarray:
    """R = A^* (A V) - V Theta^2 (Sec. 2.1; one column per Ritz pair)."""
    return mulAh(AV) - V * (theta * theta)[None, :]


def left_vectors(AV: np.ndarray, sig: np.ndarray):
    """U-hat(:, j) = A v_j / sigma_j; a zero sigma_j gives a zero column and
    the zero_theta flag."""
    zero = sig == 0.0
    U = np.where(zero[None, :], 0.0, AV / np.where(zero, 1.0, sig)[None, :])
    return U, bool(zero.any())


# ---------------------------------------------------------------- the solver

def rlobpcg(A, k: int, *, block: int | None = None, d: int | None = None,
            zeta: int = 8, seed: int = 0, tau: float | None = None,
            max_iter: int | None = None, rule: str = "paper", check_every: int = 5,
            precond: str = "svd", dot2: bool = True, refresh: bool = True,
            loop_precond: str = "sketch", orth: str = "cgs2", lock: bool = False,
            callback=None) -> RLResult:
    """Return the k smallest singular triplets of the tall matrix A."""
    A = np.asarray(A)
    if A.ndim != 2:
        raise ValueError("A must be a matrix")
    m, n = A.shape
    b = k if block is None else block
    d = 4 * n if d is None else d
    if not (1 <= k <= b) or 3 * b > n or n > m or d < n or not (1 <= zeta <= d):
        raise ValueError("need 1 <= k <= b, 3b <= n <= m, n <= d, 1 <= zeta <= d")
    cplx = np.iscomplexobj(A)
    dt = np.complex128 if cplx else np.float64
    A = A.astype(dt, copy=False)
    tau = default_tau(n) if tau is None else tau
    max_iter = (200 if b == 1 else 100) if max_iter is None else max_iter
    orth_fn = {"cgs2": _orth, "svqb": _svqb}.get(orth)
    if orth_fn is None:
        raise ValueError(f"unknown orth {orth!r}")

    def mulA(M):
        return eft.matmul(A, M) if dot2 else A @ M

    def mulAh(M):
        return eft.matmul_h(A, M) if dot2 else _ct(A) @ M

    # The sketch (Sec. 2.2), its preconditioner and the start block.
    sk = _sketch_preconditioner(sparsestack.sketch(A, d, zeta, seed), b, precond)
    apply_prec = _loop_preconditioner(A, loop_precond, sk.apply_prec)

    # Sketch-and-solve start.
    V = sk.V0
    AV = mulA(V)
    if b == 1:
        theta = np.array([np.inf])                            # theta_0 = inf
        th2 = np.array([np.vdot(AV[:, 0], AV[:, 0]).real])
        R = mulAh(AV) - V * th2[None, :]
    else:
        theta, C0 = rayleigh_ritz(AV)
        V = V @ C0
        AV = AV @ C0
        theta = theta.copy()
        R = residual(AV, V, theta, mulAh)
    X = np.zeros((n, 0), dtype=dt)
    AX = np.zeros((m, 0), dtype=dt)
    theta_hist = [theta.copy()]
    rnorm_hist = [np.linalg.norm(R, axis=0)]
    degenerate = False
    status = 1
    iters = 0
    # the lock mask (every column active without locking)
    act = np.ones(b, dtype=bool)
    if lock:
        act = lock_update(act, R, sk.sigma1, tau)
    lock_hist = [act.copy()]

    # LOBPCG on A^* A, preconditioned by P P^*, until the stopping rule holds.
    while iters < max_iter:
        if lock and not act.any():
            status = 0                                        # every column is locked
            break
        W, flag = search_block(R[:, act] if lock else R, apply_prec, np.hstack([V, X]), orth_fn)
        degenerate |= flag
        T = np.hstack([V, X, W])
        AT = np.hstack([AV, AX, mulA(W)])
        Th, C = rayleigh_ritz(AT)
        t = T.shape[1]
        Cv = C[:, t - b:]                                     # the b smallest Ritz pairs
        V = T @ Cv
        AV = AT @ Cv
        theta = Th[t - b:].copy()
        R = residual(AV, V, theta, mulAh)
        theta_hist.append(theta.copy())
        rnorm_hist.append(np.linalg.norm(R, axis=0))
        if callback is not None:
            callback(i=iters, T=T, AT=AT, C=C, Theta=Th, V=V, AV=AV, R=R, W=W, X=X, act=act.copy())
        iters += 1
        if termination.should_stop(iters - 1, theta_hist, rnorm_hist, sk.sigma1, tau,
                                   rule=rule, check_every=check_every):
            status = 0
            break
        if lock:
            act = lock_update(act, R, sk.sigma1, tau)
            lock_hist.append(act.copy())
            if not act.any():
                status = 0                                    # every column is locked
                break
        X, AX, flag = previous_direction(T, AT, C, b, act if lock else None)
        degenerate |= flag

    V_block, theta_block = V.copy(), theta.copy()
    if refresh:
        AV = mulA(V)
        Ur, Sr, Wh = np.linalg.svd(AV, full_matrices=False)
        V = V @ _ct(Wh)
        theta = Sr
        AV = Ur * Sr[None, :]
    # Ascending order; the first k of the block.
    order = np.argsort(theta, kind="stable")[:k]
    sig = theta[order]
    U, zero_theta = left_vectors(AV[:, order], sig)
    return RLResult(sigma=sig, V=V[:, order], U=U.astype(dt), iters=iters, status=status,
                    sigma1=sk.sigma1, theta_hist=theta_hist, rnorm_hist=rnorm_hist,
                    degenerate=degenerate, zero_theta=zero_theta,
                    V_block=V_block, theta_block=theta_block, lock_hist=lock_hist)
