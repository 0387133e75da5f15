"""The served form (rl_server_*): continuous admission of solves of different
shapes under an HBM budget, results identical to solving each alone."""

import numpy as np
import pytest

from workloads import planted_numpy, spectrum_gap

from .gpu_util import banner

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rl():
    import paper_2602_16797_amd as rl
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return rl


def _requests(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for r in range(count):
        m = int(rng.integers(3000, 30000))
        n = int(rng.integers(20, 130))
        k = int(rng.integers(1, 4))
        k = max(1, min(k, n // 3))
        smin = 10.0 ** rng.uniform(-10, -4)
        A, _, _ = planted_numpy(m, n, spectrum_gap(n, k, smin, 10.0), 6000 + r)
        out.append((torch.from_numpy(A).cuda(), k, 7000 + r))
    return out


def test_served_results_equal_alone(rl):
    reqs = _requests(12, 11)
    alone = []
    for A, k, seed in reqs:
        r = rl.rl_svds_smallest(A, k, seed=seed)
        alone.append((r.sigma.clone(), r.V.clone(), r.U.clone(), r.status))
    torch.cuda.synchronize()
    with rl.Server(hbm_budget_bytes=8 << 30, max_inflight=4) as srv:
        tickets = [srv.submit(A, k, seed=seed) for A, k, seed in reqs]
        got = [srv.wait(t) for t in tickets]
    for i, (g, a) in enumerate(zip(got, alone)):
        banner(f"request {i}: m={reqs[i][0].shape[0]} n={reqs[i][0].shape[1]} k={reqs[i][1]} "
               f"iters {g.iters} queued {g.queued_us:.0f} us run {g.run_us:.0f} us")
        assert g.status == a[3]
        # same kernels in the same launch configuration: bitwise equal
        assert torch.equal(g.sigma, a[0]) and torch.equal(g.V, a[1]) and torch.equal(g.U, a[2])


def test_admission_by_budget(rl):
    reqs = _requests(6, 12)
    sizes = []
    with rl.Server(hbm_budget_bytes=1 << 40, max_inflight=1) as probe:
        for A, k, seed in reqs:
            sizes.append(probe.wait(probe.submit(A, k, seed=seed)).workspace_bytes)
    budget = max(sizes) + min(sizes) // 2     # at most one large solve fits at a time
    with rl.Server(hbm_budget_bytes=budget, max_inflight=6) as srv:
        tickets = [srv.submit(A, k, seed=seed) for A, k, seed in reqs]
        res = [srv.wait(t) for t in tickets]
    assert all(r.status in (rl.RL_OK, rl.RL_NOT_CONVERGED) for r in res)
    # later requests waited for memory: the budget held them back
    assert max(r.queued_us for r in res[1:]) > 0.0
    with rl.Server(hbm_budget_bytes=min(sizes) // 2, max_inflight=2) as small:
        with pytest.raises(rl.RlError) as e:
            small.submit(*reqs[0][:2], seed=reqs[0][2])
        assert e.value.code == rl.RL_ERR_ADMISSION


def test_submit_argument_errors(rl):
    A = torch.zeros((100, 30), dtype=torch.float64, device="cuda")
    with rl.Server(hbm_budget_bytes=1 << 30, max_inflight=2) as srv:
        with pytest.raises(rl.RlError) as e:
            srv.submit(A, 11)                   # 3b > n
        assert e.value.code == rl.RL_ERR_ARG
        # a zero matrix has a singular sketch: the solve's own error comes back
        t = srv.submit(A, 1, seed=1)
        with pytest.raises(rl.RlError) as e2:
            srv.wait(t)
        assert e2.value.code == rl.RL_ERR_NONFINITE
