"""Pins for oracle.termination against hand-derived cases (tests/golden)."""

import math
import os

import numpy as np

from oracle import termination as term

N_HIST = 60


def _series(recipe: str):
    kind, *args = recipe.split(":")
    vals = []
    for j in range(N_HIST):
        if kind == "const":
            v = float(args[0])
        elif kind == "geo":                      # a + r^j
            v = float(args[0]) + float(args[1]) ** j
        elif kind == "geo0":                     # a * r^j
            v = float(args[0]) * float(args[1]) ** j
        elif kind == "kink":                     # a + r^min(j, J)
            v = float(args[0]) + float(args[1]) ** min(j, int(args[2]))
        else:
            raise ValueError(kind)
        vals.append(v)
    return vals


def _cases(golden_dir):
    with open(os.path.join(golden_dir, "termination_cases.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            name, th, rn, thr, stop = [p.strip() for p in line.split("|")]
            ths = [_series(r) for r in th.split(",")]
            rns = [_series(r) for r in rn.split(",")]
            theta = [np.array([s[j] for s in ths]) for j in range(N_HIST)]
            rnorm = [np.array([s[j] for s in rns]) for j in range(N_HIST)]
            theta[0] = np.full(len(ths), math.inf)           # theta_0 = inf (b = 1 start)
            yield name, theta, rnorm, float(thr), (None if stop == "none" else int(stop))


def test_hand_derived_cases(golden_dir):
    seen = 0
    for name, theta, rnorm, thr, expect in _cases(golden_dir):
        got = term.first_stop(theta, rnorm, 1.0, thr)
        assert got == expect, name
        seen += 1
    assert seen == 8


def test_checks_only_every_fifth_iteration_and_tol_rule():
    theta = [np.array([math.inf])] + [np.array([1.0])] * 30
    rnorm = [np.array([1.0])] * 31
    assert all(not term.should_stop(i, theta, rnorm, 1.0, 1e-3) for i in range(29))
    # "tol": every iteration, tolerance only
    rn2 = [np.array([0.5 ** j]) for j in range(31)]
    assert term.first_stop(theta, rn2, 1.0, 0.5 ** 7, rule="tol") == 6
    assert term.first_stop(theta, rn2, 2.0, 0.5 ** 7 / 4.0, rule="tol") == 6   # Sigma~(1,1)^2 scales tau
    assert term.first_stop(theta, rnorm, 1.0, 1.0, rule="none") is None


def test_equation_denominator_is_newest_theta():
    """The algorithm text divides by theta_i, eq:stagnation-check by the newest
    value theta_{i+1}.  With theta_1 = 2, theta_6 = 1.5, theta_10 = 100,
    theta_11 = 1 the equation gives 1.1*0.5/1 = 0.55 >= (2-1.5)/1.5 (stop at
    i = 10) while the literal text gives 1.1*0.5/100 < 0.33 (no stop)."""
    vals = {1: 2.0, 6: 1.5, 10: 100.0, 11: 1.0}
    theta = [np.array([math.inf])] + [np.array([vals.get(j, 5.0)]) for j in range(1, 12)]
    rnorm = [np.array([1e-30])] * 12
    assert term.should_stop(10, theta, rnorm, 1.0, 1e-15)


def test_locked_stop_on_hand_built_histories():
    """Locking: columns lock one by one as their residual meets sigma1^2 tau;
    the solve ends at the loop index whose new residuals lock the last one,
    unless the rule fires first; all locked at the start gives -1."""
    thr = 1e-3
    theta = [[1.0, 2.0]] * 8
    rn = [[1.0, 1.0], [1e-4, 1.0], [1.0, 1.0], [1.0, 1e-4], [1.0, 1.0], [1.0, 1.0], [1.0, 1.0], [1.0, 1.0]]
    # column 0 locks at iterate 1 (loop index 0) and stays locked although its
    # residual grows again; column 1 locks at iterate 3 (loop index 2)
    assert term.first_stop_locked(theta, rn, 1.0, thr, rule="none") == 2
    assert term.first_stop(theta, rn, 1.0, thr, rule="none") is None
    # Sigma~(1,1)^2 scales the threshold: with sigma1 = 0.001 nothing locks
    assert term.first_stop_locked(theta, rn, 1e-3, thr, rule="none") is None
    # every column below the threshold at the start
    assert term.first_stop_locked(theta, [[1e-4, 1e-5]] + rn[1:], 1.0, thr, rule="none") == -1
    # the tol rule fires at loop index 0 only when both columns meet it at once
    rn2 = [[1.0, 1.0], [1e-4, 1e-4]] + rn[2:]
    assert term.first_stop_locked(theta, rn2, 1.0, thr, rule="tol") == 0
    m = term.locked_mask([True, True, False], [1e-4, 1.0, 1.0], 1.0, thr)
    assert m.tolist() == [False, True, False]
