"""SVQB as the Orth of the loop's orthogonalisation step on the GPU
(rl_opts.orth = RL_ORTH_SVQB), against the CPU oracle run with orth="svqb".

Gates: |sigma_gpu - sigma_oracle| <= 1e-12 ||A||, ||A v - sigma u|| <=
1e-12 ||A||, principal-angle sine <= 1e-10 to the oracle's subspace (the
planted gaps are 10), and the same triplets as the default CGS2 solve.  The
stopping rule may fire at different iterations (or not before max_iter) with
SVQB, so iteration counts are not compared.
"""

import numpy as np
import pytest

from oracle import rlobpcg
from workloads import planted_numpy, spectrum_gap

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
    # (m, n, k, complex, seed)
    (3000, 40, 3, False, 31),
    (2001, 30, 1, False, 32),
    (2500, 36, 2, True, 33),
]


@pytest.mark.parametrize("m,n,k,cplx,seed", CASES)
def test_svqb_matches_oracle(rl, m, n, k, cplx, seed):
    s = spectrum_gap(n, k, 1e-6, 10.0)
    A, _, s = planted_numpy(m, n, s, seed, is_complex=cplx)
    normA = float(s[0])
    banner(f"svqb m={m} n={n} k={k} complex={cplx}")
    At = torch.from_numpy(A).cuda()
    r = rl.rl_svds_smallest(At, k, seed=seed, orth="svqb")
    c = rl.rl_svds_smallest(At, k, seed=seed)
    o = rlobpcg(A, k, seed=seed, precond="qr", orth="svqb")
    sg, Vg, Ug = to_np(r.sigma), to_np(r.V), to_np(r.U)
    banner(f"  gpu iters {r.iters} status {r.status}; cgs2 iters {c.iters}; oracle iters {o.iters} "
           f"status {o.status}; sigma gpu {sg} oracle {o.sigma}")
    assert np.max(np.abs(sg - o.sigma)) <= 1e-12 * normA
    assert np.max(np.abs(sg - to_np(c.sigma))) <= 1e-12 * normA
    res = A @ Vg - Ug * sg[None, :]
    assert np.linalg.norm(res, axis=0).max() <= 1e-12 * normA
    assert sin_angle(Vg, o.V) <= 1e-10
    assert sin_angle(Vg, to_np(c.V)) <= 1e-10


def test_svqb_rejects_unknown_value(rl):
    A = torch.zeros((100, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(KeyError):
        rl.rl_svds_smallest(A, 1, orth="mgs")
