"""The comparison methods of Sec. 1.1 on the GPU: LOBPCG with the diagonal
preconditioner P = diag(||A(:, i)||^{-1}) and with none, both from the
sketch-and-solve start, against the CPU oracle run with the same loop
preconditioner.

Gates: |sigma_gpu - sigma_oracle| <= 1e-12 ||A||, ||A v - sigma u|| <=
1e-12 ||A||, principal-angle sine <= 1e-10 (the planted gaps are >= 10), and
the first iterates' theta within 1e-8 relative of the oracle's (the GPU start
comes from inverse subspace iteration, equal to the oracle's SVD start up to
rounding on these gaps), which a wrong scaling of the residual changes at
the 1e-4 level.
"""

import numpy as np
import pytest

from oracle import rlobpcg

from .gpu_util import banner, sin_angle, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rl():
    import paper_2602_16797_amd as rl
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return rl


def _coherent(m, n, s, seed, colscale=None):
    """A = U diag(s) V^T with V close to the standard basis (the paper's easy
    problem shape); optional column scaling spreads the column norms."""
    rng = np.random.default_rng(seed)
    V, _ = np.linalg.qr(np.diag(rng.standard_normal(n)) + 1e-4 * rng.standard_normal((n, n)))
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    A = (U * s[None, :]) @ V.T
    if colscale is not None:
        A = A * colscale[None, :]
    return np.ascontiguousarray(A)


CASES = [
    # (loop_precond, m, n, smallest, column-norm spread, seed)
    ("diag", 4000, 50, 1e-7, None, 11),
    ("diag", 3001, 40, 1e-5, 100.0, 12),
    ("none", 4000, 50, 1e-2, None, 13),
]


@pytest.mark.parametrize("lp,m,n,smin,spread,seed", CASES)
def test_loop_precond_matches_oracle(rl, lp, m, n, smin, spread, seed):
    s = np.geomspace(1.0, 0.5, n)
    s[-1] = smin
    cs = None if spread is None else np.geomspace(1.0, spread, n)
    A = _coherent(m, n, s, seed, cs)
    normA = float(np.linalg.norm(A, 2))
    banner(f"loop_precond={lp} m={m} n={n} smin={smin} spread={spread}")
    r = rl.rl_svds_smallest(torch.from_numpy(A).cuda(), 1, seed=seed, loop_precond=lp)
    o = rlobpcg(A, 1, seed=seed, precond="qr", loop_precond=lp)
    sg, Vg, Ug = to_np(r.sigma), to_np(r.V), to_np(r.U)
    banner(f"  gpu iters {r.iters} status {r.status}; oracle iters {o.iters} status {o.status}; "
           f"sigma gpu {sg} oracle {o.sigma}")
    assert r.status == 0 and o.status == 0
    assert np.max(np.abs(sg - o.sigma)) <= 1e-12 * normA
    res = A @ Vg - Ug * sg[None, :]
    assert np.linalg.norm(res, axis=0).max() <= 1e-12 * normA
    assert sin_angle(Vg, o.V) <= 1e-10
    for j in (1, 2):
        tg, to = r.theta_hist[j][0], o.theta_hist[j][0]
        assert abs(tg - to) <= 1e-8 * abs(to), (j, tg, to)


def test_loop_precond_diag_counts_its_pass(rl):
    """The diagonal preconditioner reads A once more (its column norms).
    Passes over A: the sketch, the start block, one per iteration and the
    refresh (on by default), plus the column norms with the diagonal one."""
    s = np.geomspace(1.0, 0.5, 30)
    s[-1] = 1e-6
    A = torch.from_numpy(_coherent(2000, 30, s, 21)).cuda()
    a = rl.rl_svds_smallest(A, 1, seed=1, loop_precond="diag")
    b = rl.rl_svds_smallest(A, 1, seed=1)
    banner(f"  diag: {a.iters} iterations, {a.a_passes} passes; sketch: {b.iters}, {b.a_passes}")
    assert a.status == 0 and b.status == 0
    assert a.a_passes == a.iters + 4
    assert b.a_passes == b.iters + 3


def test_loop_precond_rejects_unknown_value(rl):
    A = torch.zeros((100, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(KeyError):
        rl.rl_svds_smallest(A, 1, loop_precond="jacobi")
