"""Full RLOBPCG solves through the C-ABI against the CPU oracle.

Gates (per triplet): |sigma_gpu - sigma_oracle| <= 1e-12 ||A||,
||A v - sigma u|| <= 1e-12 ||A|| (checked in numpy), and a principal-angle
sine <= 1e-10 to the oracle's subspace where sigma_{n-k}/sigma_{n-k+1} >= 10.
The iteration count is decided by floating-point stagnation tests, so it is
not unique: the GPU's own stop is validated by re-evaluating the oracle's
stopping rule on the GPU's reported histories.
"""

import numpy as np
import pytest

from oracle import rlobpcg, termination
from workloads import planted_numpy, spectrum_gap, spectrum_logspace_tail, spectrum_nullspace

from .gpu_util import banner, sin_angle, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rl():
    import paper_2602_16797_amd as rl
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return rl


def _check(rl, A, k, *, seed, normA, block=None, gap_ok=True, rule="paper", max_iter=None, dot2=True,
           angle_tol=1e-10, oracle_dot2=None, d=None, oracle=None, refresh=True):
    """GPU solve (products with or without Dot2) against the oracle (with
    Dot2 unless oracle_dot2 says otherwise), on the gates of the module doc."""
    At = torch.from_numpy(A).cuda()
    kw = dict(seed=seed, rule=rule, dot2=dot2, refresh=refresh)
    if block is not None:
        kw["block"] = block
    if max_iter is not None:
        kw["max_iter"] = max_iter
    if d is not None:
        kw["d"] = d
    r = rl.rl_svds_smallest(At, k, **kw)
    sg, Vg, Ug = to_np(r.sigma), to_np(r.V), to_np(r.U)
    o = oracle if oracle is not None else rlobpcg(A, k, seed=seed, block=block, rule=rule, max_iter=max_iter, d=d,
                                                  dot2=dot2 if oracle_dot2 is None else oracle_dot2,
                                                  refresh=refresh)
    banner(f"  gpu iters {r.iters} status {r.status}; oracle iters {o.iters} status {o.status}; "
           f"sigma gpu {sg} oracle {o.sigma}")
    assert np.all(np.diff(sg) >= 0)
    assert np.max(np.abs(sg - o.sigma)) <= 1e-12 * normA
    res = A @ Vg - Ug * sg[None, :]
    assert np.linalg.norm(res, axis=0).max() <= 1e-12 * normA
    assert np.allclose(np.linalg.norm(Vg, axis=0), 1.0, atol=1e-12)
    if refresh and dot2:   # U-hat from the SVD of the fresh, compensated A V-hat: orthonormal columns
        assert np.linalg.norm(Ug.conj().T @ Ug - np.eye(k)) <= 1e-12
    if gap_ok:
        ang = sin_angle(Vg, o.V)
        banner(f"  sin angle to oracle {ang:.3e}")
        assert ang <= angle_tol
    # Sigma~(1,1): Lanczos estimate vs the oracle's exact SVD value
    assert abs(r.sigma1 - o.sigma1) <= 1e-10 * o.sigma1
    # the GPU stopped where the rule first fires on its own histories
    b = block or k
    tau = 2.0 * np.sqrt(A.shape[1]) * 2.0 ** -52
    th = [r.theta_hist[j] for j in range(r.iters + 1)]
    rn = [r.rnorm_hist[j] for j in range(r.iters + 1)]
    assert all(len(x) == b for x in th)
    first = termination.first_stop(th, rn, r.sigma1, tau, rule=rule)
    if r.status == 0:
        assert first == r.iters - 1
    else:
        assert first is None and r.iters == (max_iter if max_iter is not None else (200 if b == 1 else 100))
    return r, o


def test_cfg1_single_vector(rl):
    banner("parity cfg1 4000x50 k=1")
    A, _, s = planted_numpy(4000, 50, spectrum_logspace_tail(50, 1e-3, 1e-6), 1001)
    _check(rl, A, 1, seed=2001, normA=s[0])


def test_cfg2_regime_medium(rl):
    """The 1e-12-conditioned spectrum with a gap of 10 at the bottom, at a size
    the oracle finishes in seconds; plain FP64 would leave a ~1e-6 angle floor
    here, so both sides use Dot2 for the products with A."""
    banner("parity 60000x200 k=1, cond 1e12, gap 10")
    A, _, s = planted_numpy(60_000, 200, spectrum_gap(200, 1, 1e-12, 10.0), 1102)
    _check(rl, A, 1, seed=2102, normA=s[0])


@pytest.mark.parametrize("m,n,k,cplx,gamma", [(3000, 60, 3, False, 10.0), (2999, 61, 2, True, 10.0),
                                              (20000, 100, 5, False, 100.0)])
def test_block(rl, m, n, k, cplx, gamma):
    banner(f"parity block m={m} n={n} k={k} complex={cplx}")
    A, _, s = planted_numpy(m, n, spectrum_gap(n, k, 1e-9, gamma), 7 + m, is_complex=cplx)
    _check(rl, A, k, seed=3 + k, normA=s[0])


def test_trial_space_near_n(rl):
    """A served-stream shape whose trial space nearly fills the columns
    (n = 36, k = b = 10: t = 30): the search block lives in a 16-dimensional
    complement of [V X], so its orthonormalisation meets heavy cancellation
    (the paper's rule need not fire here: the oracle too runs to max_iter on
    this matrix)."""
    from workloads import request_spectrum, served_requests
    q = served_requests(count=256)[229]
    banner(f"parity served shape m={q.m} n={q.n} k={q.k}")
    A, _, s = planted_numpy(q.m, q.n, request_spectrum(q), q.data_seed)
    _check(rl, A, q.k, seed=q.sketch_seed, normA=s[0])


def test_complex_nullspace_small(rl):
    """cfg3's structure (rank n-k plus complex noise 1e-14) at a small size."""
    banner("parity complex nullspace 8000x60 k=4")
    A, _, s = planted_numpy(8000, 60, spectrum_nullspace(60, 4, 1e-4), 1303, is_complex=True, noise_std=1e-14)
    _check(rl, A, 4, seed=2303, normA=s[0])


@pytest.mark.parametrize("cplx", [False, True])
def test_without_refresh(rl, cplx):
    """refresh = 0: the last Rayleigh-Ritz triplets as they are (U-hat = A_V / theta
    from the maintained products), against the oracle's refresh=False."""
    banner(f"parity without refresh complex={cplx}")
    A, _, s = planted_numpy(4000, 60, spectrum_gap(60, 3, 1e-8, 10.0), 91 + cplx, is_complex=cplx)
    _check(rl, A, 3, seed=12, normA=s[0], refresh=False)


def test_oversampled_block(rl):
    banner("parity k=1 with block 3")
    A, _, s = planted_numpy(5000, 45, spectrum_gap(45, 1, 1e-8, 10.0), 77)
    _check(rl, A, 1, seed=9, block=3, normA=s[0])


@pytest.mark.parametrize("rule,max_iter", [("tol", None), ("none", 7)])
def test_other_stop_rules(rl, rule, max_iter):
    banner(f"parity rule={rule}")
    A, _, s = planted_numpy(3000, 40, spectrum_gap(40, 2, 1e-6, 10.0), 88)
    _check(rl, A, 2, seed=10, rule=rule, max_iter=max_iter, normA=s[0], gap_ok=(rule == "tol"))


def test_max_iter_zero_returns_the_start(rl):
    A, _, s = planted_numpy(2000, 30, spectrum_gap(30, 1, 1e-6, 10.0), 5)
    r = rl.rl_svds_smallest(torch.from_numpy(A).cuda(), 1, seed=1, max_iter=0)
    assert r.status == rl.RL_NOT_CONVERGED and r.iters == 0
    sg = to_np(r.sigma)
    assert s[-1] * 0.999 <= sg[0] <= s[-1] * 3.0       # the sketch-and-solve start (Fact prop:sketch_and_solve)


def test_argument_and_data_errors(rl):
    A = torch.zeros((100, 12), dtype=torch.float64, device="cuda")
    with pytest.raises(rl.RlError) as e:
        rl.rl_svds_smallest(A, 5)                        # 3b > n
    assert e.value.code == rl.RL_ERR_ARG
    with pytest.raises(rl.RlError) as e:
        rl.rl_svds_smallest(torch.zeros((10, 12), dtype=torch.float64, device="cuda"), 1)   # n > m
    assert e.value.code == rl.RL_ERR_ARG
    B = torch.randn((500, 12), dtype=torch.float64, device="cuda")
    B[17, 3] = float("nan")
    with pytest.raises(rl.RlError) as e:
        rl.rl_svds_smallest(B, 1)
    assert e.value.code == rl.RL_ERR_NONFINITE


def test_determinism(rl):
    A, _, s = planted_numpy(20000, 80, spectrum_gap(80, 2, 1e-8, 10.0), 21)
    At = torch.from_numpy(A).cuda()
    a = rl.rl_svds_smallest(At, 2, seed=4)
    b = rl.rl_svds_smallest(At, 2, seed=4)
    assert a.iters == b.iters
    assert torch.equal(a.sigma, b.sigma) and torch.equal(a.V, b.V) and torch.equal(a.U, b.U)
