"""Full solves on the wide and wide-block paths against the CPU oracle.

* The complex null-space workload's structure (rank n - 10 plus complex
  Gaussian noise of std 1e-14, k = b = 10, sketch d = 3n) at 8000 x 400, so
  the solve runs the kernels of the 10^6 x 1000 workload: the complex sketch
  QR above n = 256, the wide complex pass (compensated sums on the vector
  units, or plain sums on the matrix cores), TSQR of the 30-column trial
  basis, and the Rayleigh-Ritz, panel and orthogonalisation kernels at
  b = 10.  The oracle uses compensated products either way; the plain-sum
  GPU path must still meet every gate (its rounding moves the null space's
  vectors by about u ||A||_F / (sqrt(m) sigma_{n-10}) = 1e-13 here).
* Real blocks of 8 and 10 vectors at n = 300 (the column-split pass and the
  column-wave TSQR at t = 24 and 30).
* Real n in (1024, 2048], where the pass runs plain sums on the matrix cores
  and the Lanczos estimate holds two vector entries per thread: a gapped
  spectrum (sigma_{n-k+1} = 1e-4 below a drop of 10, so plain products move
  the vectors by about u sqrt(n) / 1e-3 and the angle gate holds), and the
  clustered spectrum of the block-size study (Sec. 5.2) at reduced m, where
  the bottom gap is 9e-5 relative and only sigma, the residual and the
  stopping rule are gated.  The oracle uses plain products too.

Gates as in test_gpu_parity: |sigma - sigma_oracle| <= 1e-12 ||A||, the
residual ||A v - sigma u|| <= 1e-12 ||A||, the principal-angle sine to the
oracle's subspace <= 1e-10, and the GPU's stop re-derived from its own
histories by the oracle's stopping rule.
"""

import pytest

from oracle import rlobpcg
from workloads import planted_numpy, spectrum_clustered, spectrum_gap, spectrum_nullspace

from .gpu_util import banner
from .test_gpu_parity import _check

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rl():
    import paper_2602_16797_amd as rl
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return rl


@pytest.fixture(scope="module")
def nullspace_8000x400():
    """The input and the oracle's solve (compensated products), shared by both GPU variants."""
    A, _, s = planted_numpy(8000, 400, spectrum_nullspace(400, 10, 1e-4), 1313, is_complex=True, noise_std=1e-14)
    return A, s, rlobpcg(A, 10, seed=2313, d=1200, dot2=True)


@pytest.mark.parametrize("dot2", [True, False])
def test_complex_nullspace_block10_wide(rl, nullspace_8000x400, dot2):
    A, s, o = nullspace_8000x400
    banner(f"parity complex nullspace 8000x400 k=b=10 d=3n, GPU dot2={dot2}")
    _check(rl, A, 10, seed=2313, normA=s[0], dot2=dot2, d=1200, oracle=o)


@pytest.mark.parametrize("k", [8, 10])
def test_real_block_wide(rl, k):
    banner(f"parity real 20000x300 k=b={k}")
    A, _, s = planted_numpy(20_000, 300, spectrum_gap(300, k, 1e-8, 10.0), 1400 + k)
    _check(rl, A, k, seed=2400 + k, normA=s[0])


@pytest.mark.parametrize("m,n,k,b", [(12_000, 1100, 1, 1), (8000, 2048, 3, 5)])
def test_real_wide_plain(rl, m, n, k, b):
    banner(f"parity real {m}x{n} k={k} b={b}, plain products (matrix-core pass)")
    A, _, s = planted_numpy(m, n, spectrum_gap(n, k, 1e-4, 10.0), 1500 + n)
    _check(rl, A, k, seed=2500 + n, normA=s[0], block=b, dot2=False)


@pytest.mark.parametrize("b", [1, 3])
def test_real_clustered_wide(rl, b):
    banner(f"parity real 10000x2000 clustered spectrum (Sec. 5.2) k=1 b={b}, plain products")
    A, _, s = planted_numpy(10_000, 2000, spectrum_clustered(2000), 1600)
    _check(rl, A, 1, seed=2600, normA=s[0], block=b, dot2=False, gap_ok=False)


def test_complex_wide_plain_without_refresh(rl):
    """The late-residual loop (A W, the Rayleigh-Ritz, then A^* A_{V_{i+1}}
    on its own) with refresh = 0: U-hat comes from the A_V buffer of the last
    Rayleigh-Ritz, which the two-buffer scheme must find after a stop between
    host checks."""
    banner("parity complex 6000x300 k=3 plain products, refresh off (late-residual loop)")
    A, _, s = planted_numpy(6000, 300, spectrum_gap(300, 3, 1e-4, 10.0), 1700, is_complex=True)
    _check(rl, A, 3, seed=2700, normA=s[0], dot2=False, refresh=False)


def test_complex_wide_plain_locked(rl):
    """Locking on the late-residual loop: the Gram pass after the
    Rayleigh-Ritz, then the lock update, against the oracle's locked solve."""
    from oracle import termination
    from oracle.rlobpcg import default_tau
    from .gpu_util import sin_angle, to_np
    import numpy as np
    banner("parity complex 6000x300 k=4 plain products, locking (late-residual loop)")
    n, k = 300, 4
    A, _, s = planted_numpy(6000, n, spectrum_gap(n, k, 1e-3, 10.0), 1710, is_complex=True)
    r = rl.rl_svds_smallest(torch.from_numpy(A).cuda(), k, seed=2710, dot2=False, lock=True)
    o = rlobpcg(A, k, seed=2710, dot2=False, lock=True)
    banner(f"  gpu iters {r.iters} status {r.status} locked {r.n_locked}; oracle iters {o.iters}")
    sg, Vg, Ug = to_np(r.sigma), to_np(r.V), to_np(r.U)
    assert np.max(np.abs(sg - o.sigma)) <= 1e-12 * s[0]
    assert np.linalg.norm(A @ Vg - Ug * sg[None, :], axis=0).max() <= 1e-12 * s[0]
    assert sin_angle(Vg, o.V) <= 1e-8
    tau = default_tau(n)
    th = [r.theta_hist[j] for j in range(r.iters + 1)]
    rn = [r.rnorm_hist[j] for j in range(r.iters + 1)]
    assert r.status == 0 and termination.first_stop_locked(th, rn, r.sigma1, tau) == r.iters - 1
