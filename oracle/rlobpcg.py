"""RLOBPCG, plain CPU FP64 (paper Alg. rlopcg for b = 1, Alg. rlobpcg for b > 1).

Test infrastructure only (see ``oracle/__init__``).

Steps, in the paper's order and notation (Sec. 1 steps 1-4; Sec. 2.1; Sec. 2.3):
  1  S <- SparseStack (d x m, zeta nonzeros per column)        [Sec. 2.2]
  2  [~, Sigma~, V~] = svd(S A)                                 [Alg. rlopcg, sketch-and-SVD]
  3  P = V~ Sigma~^{-1};  V_0 = V~(:, n-b+1:n);  A_V = A V_0    [sketch-and-solve start]
     b = 1: theta_0 = inf, r_0 = A^* A_v - ||A_v||^2 v_0
     b > 1: Rayleigh-Ritz of A_V (its SVD) rotates V_0, A_V; R_0 = A^* A_V - V_0 Theta^2
  4  for i = 0 .. max_iter-1:
       W = P (P^* R)                                           [eq:search-direction]
       W <- W - [V X]([V X]^* W);  W <- Orth(W - [V X]([V X]^* W))   [CGS2 / BCGS2]
       T = [V X W];  A_T = [A_V A_X A W];  [~, Theta, C] = svd(A_T)  [Rayleigh-Ritz]
       V = T C(:, t-b+1:t);  A_V = A_T C(:, t-b+1:t)
       R = A^* A_V - V Theta_b^2
       stop? (oracle.termination)
       Q = Orth(C(1:b, 1:t-b)^*);  X = T C(:, 1:t-b) Q;  A_X = A_T C(:, 1:t-b) Q   [eq:x-defining]
  Output: sigma = Theta_b, V; here sorted ascending.

Readings where the paper is silent:
  * The loop is written once for all b; with b = 1 it is Alg. rlopcg line by
    line (Normalize is Orth of one column; the b = 1 start keeps theta_0 = inf).
  * On the first pass X is empty, so t = 2b, V takes the last b columns of C
    and Q = Orth(C(1:b, 1:b)^*).
  * Orth is the thin Householder QR (numpy/LAPACK); Normalize of a zero vector
    returns e_1 and raises the ``degenerate`` flag.
  * svd returns singular values in descending order, as MATLAB's does.
  * ^* is the conjugate transpose throughout; S is real.
  * U-hat_j = A_V(:, j) / theta_j (zero, with a flag, if theta_j = 0).
    ``refresh=True`` recomputes A_V = A V-hat once at the end and rotates
    (V-hat, sigma, U-hat) by the SVD of that m x b block.
  * ``precond="qr"`` uses R from S A = Q R with P = R^{-1}; P P^* = (R^* R)^{-1}
    = ((S A)^* S A)^{-1} = V~ Sigma~^{-2} V~^*, the same operator as the SVD
    route (Sec. 1, footnote on QR), with V_0 taken from the SVD of R.
  * ``loop_precond`` swaps the loop's preconditioner for the diagonal one
    (P = diag(||A(:, i)||^{-1})) or none, keeping the sketch-and-solve start
    (Sec. 1.1 initialises every compared method with v_0).
  * ``orth="svqb"`` replaces Orth(W) after the two block projections by
    SVQB (Gram matrix, eigendecomposition), the faster, less stable option
    the paper names for this step.
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


def _ct(M: np.ndarray) -> np.ndarray:
    return M.conj().T


def _orth(M: np.ndarray):
    """Orth (thin Householder QR); a single column is Normalize."""
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


def rlobpcg(A, k: int, *, block: int | None = None, d: int | None = None,
            zeta: int = 8, seed: int = 0, tau: float | None = None,
            max_iter: int | None = None, rule: str = "paper", check_every: int = 5,
            precond: str = "svd", dot2: bool = True, refresh: bool = False,
            loop_precond: str = "sketch", orth: str = "cgs2", callback=None) -> RLResult:
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

    def mulA(M):
        return eft.matmul(A, M) if dot2 else A @ M

    def mulAh(M):
        return eft.matmul_h(A, M) if dot2 else _ct(A) @ M

    # Steps 1-2: embedding, sketch, factorisation.
    SA = sparsestack.sketch(A, d, zeta, seed)
    if precond == "svd":
        _, St, Vth = np.linalg.svd(SA, full_matrices=False)
        Vt = _ct(Vth)
        sigma1 = float(St[0])
        P = Vt / St[None, :]                                  # P = V~ Sigma~^{-1}

        def apply_prec(Rm):
            return P @ (_ct(P) @ Rm)
        V = Vt[:, n - b:].copy()
    elif precond == "qr":
        Rf = np.linalg.qr(SA, mode="r")
        _, Sr, Vrh = np.linalg.svd(Rf)
        sigma1 = float(Sr[0])

        def apply_prec(Rm):
            Z = sla.solve_triangular(Rf, Rm, trans="C", lower=False)
            return sla.solve_triangular(Rf, Z, lower=False)
        V = _ct(Vrh)[:, n - b:].copy()
    else:
        raise ValueError(f"unknown precond {precond!r}")
    # The loop's preconditioner (Sec. 1.1, the comparison methods): the sketch
    # preconditioner above, the diagonal P = diag(||A(:, i)||^{-1}) (so
    # P P^* = diag(||A(:, i)||^{-2})), or none (P = I).  Every variant keeps
    # the sketch-and-solve start and Sigma~(1,1), as the paper's comparison
    # initialises all iterative methods with v_0.  A zero column keeps P(i,i) = 1.
    if loop_precond == "diag":
        cn2 = np.sum(np.abs(A) ** 2, axis=0)
        dscale = np.where(cn2 > 0.0, 1.0 / np.where(cn2 > 0.0, cn2, 1.0), 1.0)

        def apply_prec(Rm):
            return dscale[:, None] * Rm
    elif loop_precond == "none":
        def apply_prec(Rm):
            return Rm.copy()
    elif loop_precond != "sketch":
        raise ValueError(f"unknown loop_precond {loop_precond!r}")
    # Orth of W after the two block projections on [V X]: Householder QR
    # (the CGS2 of the paper yields the same orthonormal basis up to rounding
    # and column signs) or SVQB.
    if orth == "cgs2":
        orth_fn = _orth
    elif orth == "svqb":
        orth_fn = _svqb
    else:
        raise ValueError(f"unknown orth {orth!r}")

    # Step 3: sketch-and-solve start.
    AV = mulA(V)
    if b == 1:
        th2 = np.array([np.vdot(AV[:, 0], AV[:, 0]).real])
        theta = np.array([np.inf])                            # theta_0 = inf
    else:
        _, Th, Ch = np.linalg.svd(AV, full_matrices=False)
        C0 = _ct(Ch)
        V = V @ C0
        AV = AV @ C0
        theta = Th.copy()
        th2 = Th * Th
    R = mulAh(AV) - V * th2[None, :]
    X = np.zeros((n, 0), dtype=dt)
    AX = np.zeros((m, 0), dtype=dt)
    theta_hist = [theta.copy()]
    rnorm_hist = [np.linalg.norm(R, axis=0)]
    degenerate = False
    status = 1
    iters = 0

    # Step 4: LOBPCG on A^* A with preconditioner P P^*.
    for i in range(max_iter):
        W = apply_prec(R)
        B = np.hstack([V, X])
        W = W - B @ (_ct(B) @ W)
        W, flag = orth_fn(W - B @ (_ct(B) @ W))
        degenerate |= flag
        T = np.hstack([V, X, W])
        AT = np.hstack([AV, AX, mulA(W)])
        _, Th, Ch = np.linalg.svd(AT, full_matrices=False)
        C = _ct(Ch)
        t = T.shape[1]
        Cv = C[:, t - b:]
        V = T @ Cv
        AV = AT @ Cv
        theta = Th[t - b:].copy()
        R = mulAh(AV) - V * (theta * theta)[None, :]
        theta_hist.append(theta.copy())
        rnorm_hist.append(np.linalg.norm(R, axis=0))
        iters = i + 1
        if callback is not None:
            callback(i=i, T=T, AT=AT, C=C, Theta=Th, V=V, AV=AV, R=R, W=W)
        if termination.should_stop(i, theta_hist, rnorm_hist, sigma1, tau,
                                   rule=rule, check_every=check_every):
            status = 0
            break
        Q, flag = _orth(_ct(C[:b, :t - b]))
        degenerate |= flag
        CX = C[:, :t - b] @ Q
        X = T @ CX
        AX = AT @ CX

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
    Vk = V[:, order]
    zero = sig == 0.0
    U = np.where(zero[None, :], 0.0, AV[:, order] / np.where(zero, 1.0, sig)[None, :])
    return RLResult(sigma=sig, V=Vk, U=U.astype(dt), iters=iters, status=status,
                    sigma1=sigma1, theta_hist=theta_hist, rnorm_hist=rnorm_hist,
                    degenerate=degenerate, zero_theta=bool(zero.any()),
                    V_block=V_block, theta_block=theta_block)
