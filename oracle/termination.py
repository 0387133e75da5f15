"""Stopping rule of RLOBPCG (paper Sec. 2.1 "Stopping criteria", Alg. rlopcg).

Test infrastructure only (see ``oracle/__init__``).

History convention: ``theta[j]`` and ``rnorm[j]`` hold, for iterate j, the Ritz
values theta_j and residual column norms ||r_j|| (arrays of length b).  Loop
index i of the algorithm produces iterate i+1, so the check at loop index i
reads entries up to i+1.

Rules
  "paper"  (default for every block size) at loop indices i = 0 (mod 5):
           tol:   max_j ||r_{i+1}(:,j)|| <= Sigma~(1,1)^2 * tau  (eq:est_conv_criterion)
           stag1: 1.1 ||r_{i+1}|| >= ||r_{i-4}||                  (eq:stagnation-check)
           stag2: 1.1 (theta_{i-4} - theta_{i+1}) / theta_{i+1}
                    >= (theta_{i-9} - theta_{i-4}) / theta_{i-4}  (eq:stagnation-check)
           stop iff tol and stag1 and stag2, the stagnation checks holding for
           every column.
  "tol"    the tolerance alone, every iteration (the block algorithm as typeset).
  "none"   never stop early (run max_iter iterations).

With locking (Sec. 2.3, ``rlobpcg(lock=True)``) a column whose residual meets
the tolerance on its own is locked for good, and the loop also ends once
every column is locked (``first_stop_locked``).

Readings where the paper is silent or inconsistent:
  * The algorithm divides by theta_i in stag2 while eq:stagnation-check divides
    by the newest value; the equation is followed (theta_{i+1}).
  * An index below 0 is missing history, and a check with missing history
    counts as "not stagnated"; so the earliest stop is i = 10.
  * theta_{i+1} = 0 counts as stagnated for that column (theta cannot decrease
    further); a zero theta_{i-4} makes the right-hand side +inf.
"""

from __future__ import annotations

import math

import numpy as np

STAGNATION_LAG = 5
STAGNATION_FACTOR = 1.1


def _col_stag1(rn_new: float, rn_old: float) -> bool:
    return STAGNATION_FACTOR * rn_new >= rn_old


def _col_stag2(th_new: float, th_mid: float, th_old: float) -> bool:
    if th_new == 0.0:
        return True
    lhs = STAGNATION_FACTOR * (th_mid - th_new) / th_new
    rhs = math.inf if th_mid == 0.0 else (th_old - th_mid) / th_mid
    return bool(lhs >= rhs)


def should_stop(i: int, theta, rnorm, sigma1: float, tau: float, *,
                rule: str = "paper", check_every: int = 5) -> bool:
    """Decide whether loop index ``i`` ends the iteration."""
    if rule == "none":
        return False
    tol = float(np.max(np.asarray(rnorm[i + 1]))) <= sigma1 * sigma1 * tau
    if rule == "tol":
        return bool(tol)
    if rule != "paper":
        raise ValueError(f"unknown rule {rule!r}")
    if i % check_every != 0:
        return False
    if not tol:
        return False
    lag = STAGNATION_LAG
    j_new, j_mid, j_old = i + 1, i + 1 - lag, i + 1 - 2 * lag
    if j_mid < 0 or j_old < 0:
        return False
    r_new = np.asarray(rnorm[j_new], dtype=np.float64)
    r_mid = np.asarray(rnorm[j_mid], dtype=np.float64)
    t_new = np.asarray(theta[j_new], dtype=np.float64)
    t_mid = np.asarray(theta[j_mid], dtype=np.float64)
    t_old = np.asarray(theta[j_old], dtype=np.float64)
    for c in range(r_new.size):
        if not _col_stag1(float(r_new[c]), float(r_mid[c])):
            return False
        if not _col_stag2(float(t_new[c]), float(t_mid[c]), float(t_old[c])):
            return False
    return True


def first_stop(theta, rnorm, sigma1: float, tau: float, *, rule: str = "paper",
               check_every: int = 5, max_iter: int | None = None):
    """First loop index at which the rule fires on the given histories, or None."""
    last = len(theta) - 2 if max_iter is None else min(len(theta) - 2, max_iter - 1)
    for i in range(0, last + 1):
        if should_stop(i, theta, rnorm, sigma1, tau, rule=rule, check_every=check_every):
            return i
    return None


def locked_mask(act, rn, sigma1: float, tau: float):
    """The lock update of Sec. 2.3: column j stays active while ||r(:, j)|| >
    Sigma~(1,1)^2 tau; a locked column stays locked."""
    return np.asarray(act, dtype=bool) & ~(np.asarray(rn, dtype=np.float64) <= sigma1 * sigma1 * tau)


def first_stop_locked(theta, rnorm, sigma1: float, tau: float, *, rule: str = "paper",
                      check_every: int = 5, max_iter: int | None = None):
    """Where a solve with locking ends on the given histories: -1 if every
    column is locked by the start block's residual, else the first loop index
    at which the rule fires or, after the rule's check, the last active column
    locks; None if neither happens."""
    b = len(rnorm[0])
    act = locked_mask(np.ones(b, dtype=bool), rnorm[0], sigma1, tau)
    if not act.any():
        return -1
    last = len(theta) - 2 if max_iter is None else min(len(theta) - 2, max_iter - 1)
    for i in range(0, last + 1):
        if should_stop(i, theta, rnorm, sigma1, tau, rule=rule, check_every=check_every):
            return i
        act = locked_mask(act, rnorm[i + 1], sigma1, tau)
        if not act.any():
            return i
    return None
