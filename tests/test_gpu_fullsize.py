"""Full-size solves in the launch configuration bench.py times (the
10^6 x 200 k = 1 and 2*10^6 x 500 k = 5 workloads), checked by properties
that hold at any size and by sampled rows the oracle recomputes:

* status 0 (the paper's stopping rule fired),
* sigma within 1e-12 ||A|| of the planted values (A = U diag(s) V^T by
  construction),
* ||A v - sigma u|| <= 1e-12 ||A|| for every returned triplet (device FP64
  product, a check only),
* V orthonormal to 1e-12, and the subspace within 1e-6 of the planted right
  singular vectors: the stored A is U diag(s) V^T rounded entry by entry,
  which moves the singular vectors of sigma_min = 1e-12 (gap 10) by about
  1e-8, more than any FP64 reference could resolve, so this only rules out a
  wrong vector; the residual gate is the accuracy check,
* on 64 sampled rows, the oracle's compensated product A[rows] v equals
  sigma u[rows] to 1e-12 ||A||.
"""

import numpy as np
import pytest

from oracle import eft
from workloads import planted_torch, spectrum_gap

from .gpu_util import banner, sin_angle, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rl():
    import paper_2602_16797_amd as rl
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return rl


CASES = [
    # (m, n, k, d, data seed, sketch seed, smallest, gap) as the bench workloads
    (1_000_000, 200, 1, 800, 1002, 2002, 1e-12, 10.0),
    (2_000_000, 500, 5, 2000, 1004, 2004, 1e-10, 100.0),
]


@pytest.mark.parametrize("m,n,k,d,dseed,sseed,smin,gap", CASES)
def test_full_size_workload(rl, m, n, k, d, dseed, sseed, smin, gap):
    banner(f"full size m={m} n={n} k={k}")
    sig = spectrum_gap(n, k, smin, gap)
    A, Vp, s = planted_torch(m, n, sig, dseed, device="cuda")
    torch.cuda.synchronize()
    r = rl.rl_svds_smallest(A, k, seed=sseed, d=d, zeta=8)
    torch.cuda.synchronize()
    normA = float(np.max(sig))
    banner(f"  iters {r.iters} status {r.status} sigma {to_np(r.sigma)}")
    assert r.status == 0
    sg = to_np(r.sigma)
    assert np.max(np.abs(sg - np.sort(sig)[:k])) <= 1e-12 * normA
    with torch.no_grad():
        res = torch.linalg.norm(A @ r.V - r.U * r.sigma[None, :], dim=0).max().item()
    assert res <= 1e-12 * normA
    Vg = to_np(r.V)
    assert np.linalg.norm(Vg.T @ Vg - np.eye(k)) <= 1e-12
    Vplant = to_np(Vp)
    order = np.argsort(sig)[:k]
    ang = sin_angle(Vg, Vplant[:, order])
    banner(f"  residual {res:.2e}; sin angle to the planted vectors {ang:.2e}")
    assert ang <= 1e-6
    rows = np.random.default_rng(7).choice(m, size=64, replace=False)
    Arows = to_np(A[torch.from_numpy(rows).cuda()])
    Av = eft.matmul(Arows, Vg)
    Ug = to_np(r.U)[rows]
    assert np.max(np.abs(Av - Ug * sg[None, :])) <= 1e-12 * normA
    del A
    torch.cuda.empty_cache()


def test_full_size_single_vector_against_the_oracle(rl):
    """The 10^6 x 200, k = 1 workload solved by the oracle as well (its
    compensated products run in C threads): the GPU's sigma within
    1e-12 ||A|| and its vector within a principal-angle sine of 1e-10 of the
    oracle's, both sides working on the same stored A."""
    from oracle import eft as oeft
    from oracle import rlobpcg
    m, n, k, d, dseed, sseed, smin, gap = CASES[0]
    banner(f"full size against the oracle m={m} n={n} k={k} (oracle threads {oeft.get_threads()})")
    sig = spectrum_gap(n, k, smin, gap)
    A, _, _ = planted_torch(m, n, sig, dseed, device="cuda")
    torch.cuda.synchronize()
    r = rl.rl_svds_smallest(A, k, seed=sseed, d=d, zeta=8)
    sg, Vg = to_np(r.sigma), to_np(r.V)
    Ah = to_np(A)
    del A
    torch.cuda.empty_cache()
    o = rlobpcg(Ah, k, seed=sseed, d=d, zeta=8)
    ang = sin_angle(Vg, o.V)
    banner(f"  gpu iters {r.iters} oracle iters {o.iters}; sigma gpu {sg} oracle {o.sigma}; sin angle {ang:.2e}")
    assert o.status == 0 and r.status == 0
    assert np.max(np.abs(sg - o.sigma)) <= 1e-12 * float(np.max(sig))
    assert ang <= 1e-10
