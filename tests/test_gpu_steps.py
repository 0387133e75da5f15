"""Step-level parity of the HIP kernels through the C-ABI step entry points."""

import numpy as np
import pytest

from oracle import eft, sparsestack
from workloads import integer_matrix

from .gpu_util import banner, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def rl():
    import paper_2602_16797_amd as rl
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return rl


@pytest.mark.parametrize("m,n,d,zeta,cplx", [(10007, 37, 150, 8, False), (4096, 64, 256, 8, False),
                                             (3001, 19, 77, 4, True), (2500, 10, 3000, 8, False),
                                             (700, 9, 9, 9, False), (1234, 5, 40, 1, True)])
def test_sketch_bit_exact_on_integers(rl, m, n, d, zeta, cplx):
    banner(f"sketch integer m={m} n={n} d={d} zeta={zeta} complex={cplx}")
    A = integer_matrix(m, n, 7 + m, is_complex=cplx)
    Y = to_np(rl.rl_step_sketch(torch.from_numpy(A).cuda(), d, zeta, 1234 + d))
    Yo = sparsestack.sketch(A, d, zeta, 1234 + d)
    assert np.array_equal(Y, Yo)


def test_sketch_float_close_and_deterministic(rl):
    banner("sketch float 200000x120, d=480")
    rng = np.random.default_rng(3)
    A = rng.standard_normal((200_000, 120))
    At = torch.from_numpy(A).cuda()
    Y1 = to_np(rl.rl_step_sketch(At, 480, 8, 99))
    Y2 = to_np(rl.rl_step_sketch(At, 480, 8, 99))
    assert np.array_equal(Y1, Y2)                     # fixed reduction order
    Yo = sparsestack.sketch(A, 480, 8, 99)
    S = sparsestack.embedding(200_000, 480, 8, 99)
    scale = abs(S) @ np.abs(A) / np.sqrt(8)           # sum of |terms| per entry
    assert np.all(np.abs(Y1 - Yo) <= 2 * 200_000 * U * scale + 1e-300)


def test_sketch_strided_lda(rl):
    A = integer_matrix(999, 40, 5)
    At = torch.from_numpy(A).cuda()[:, 3:33]           # lda = 40, n = 30
    Y = to_np(rl.rl_step_sketch(At, 64, 8, 5))
    assert np.array_equal(Y, sparsestack.sketch(A[:, 3:33], 64, 8, 5))


@pytest.mark.parametrize("d,n,cplx", [(800, 200, False), (150, 37, False), (96, 33, True), (64, 64, False),
                                      (3000, 70, True), (1024, 300, False), (500, 100, True), (256, 256, True),
                                      (65, 60, False), (2000, 500, False), (1536, 512, True), (3000, 1000, True),
                                      (3500, 300, False),
                                      # sketches over 4096 rows: panels factored in leaves
                                      (6000, 700, False), (8000, 2000, False), (4500, 64, True)])
def test_qr_and_inverse(rl, d, n, cplx):
    banner(f"qr d={d} n={n} complex={cplx}")
    rng = np.random.default_rng(d + n)
    Y = rng.standard_normal((d, n)) * np.logspace(0, -6, n)[None, :]
    if cplx:
        Y = Y + 1j * rng.standard_normal((d, n)) * np.logspace(0, -6, n)[None, :]
    R, Rinv = rl.rl_step_qr(torch.from_numpy(Y).cuda())
    R, Rinv = to_np(R), to_np(Rinv)
    assert np.all(np.abs(np.tril(R, -1)) == 0) and np.all(np.abs(np.tril(Rinv, -1)) == 0)
    assert np.all(np.abs(np.diag(R).imag) == 0) if cplx else True
    Rn = np.linalg.qr(Y, mode="r")
    ph = np.diag(Rn) / np.diag(R)
    assert np.allclose(np.abs(ph), 1.0, rtol=1e-10)
    Radj = ph[:, None] * R
    # rows of R agree with LAPACK's up to a unit phase (R is unique up to phases)
    assert np.linalg.norm(Radj - Rn) <= 1e-12 * np.linalg.norm(Rn) * np.sqrt(n)
    # Q = Y R^{-1} is orthonormal and R^{-1} inverts R
    Q = Y @ Rinv
    assert np.linalg.norm(Q.conj().T @ Q - np.eye(n)) <= 1e-10
    assert np.linalg.norm(R @ Rinv - np.eye(n)) <= 1e-10


@pytest.mark.parametrize("m,n,b,cplx,dot2", [(5003, 37, 1, False, False), (5003, 37, 1, False, True),
                                             (20000, 200, 1, False, True), (7777, 513, 5, False, True),
                                             (3000, 256, 3, False, False), (2049, 65, 2, True, False),
                                             (2049, 65, 2, True, True), (1500, 1000, 10, True, False), (999, 1024, 10, False, True),
                                             (17, 130, 3, False, True), (40_000, 300, 4, False, True),
                                             (30_000, 500, 5, False, False), (1001, 301, 1, True, False),
                                             (5000, 1024, 10, True, False),
                                             # real plain sums on the matrix cores past n = 1024
                                             (5000, 2048, 10, False, False), (3001, 1026, 1, False, False),
                                             (777, 1500, 5, False, False)])
def test_astream(rl, m, n, b, cplx, dot2):
    banner(f"astream m={m} n={n} b={b} complex={cplx} dot2={dot2}")
    rng = np.random.default_rng(m + n + b)
    A = rng.standard_normal((m, n))
    W = rng.standard_normal((n, b))
    if cplx:
        A = A + 1j * rng.standard_normal((m, n))
        W = W + 1j * rng.standard_normal((n, b))
    AW, G = rl.rl_step_astream(torch.from_numpy(A).cuda(), torch.from_numpy(W).cuda(), dot2=dot2)
    AW, G = to_np(AW), to_np(G)
    if dot2:
        ref = eft.matmul(A, W)
        tol = 2 * U * np.abs(ref) + 4 * (n * U) ** 2 * (np.abs(A) @ np.abs(W))
        assert np.all(np.abs(AW - ref) <= tol)
    else:
        bound = 2 * n * U * (np.abs(A) @ np.abs(W))
        assert np.all(np.abs(AW - A @ W) <= bound)
    Gref = A.conj().T @ AW
    gb = 2 * m * U * (np.abs(A).T @ np.abs(AW))
    assert np.all(np.abs(G - Gref) <= gb)
    if dot2:   # A^* AW is a Dot2-class sum too
        G2 = eft.matmul_h(A, AW)
        gb2 = 2 * U * np.abs(G2) + 4 * (np.log2(2 * m) * U) ** 2 * (np.abs(A).T @ np.abs(AW))
        assert np.all(np.abs(G - G2) <= gb2)


def _rand(rng, shape, cplx):
    x = rng.standard_normal(shape)
    return x + 1j * rng.standard_normal(shape) if cplx else x


# one case per kernel family: real column-pair rows (n <= 256, b <= 2, even
# lda), real column split, complex column split (b split into vector groups,
# remainders of 1, 2 and 3), real generic (odd lda)
@pytest.mark.parametrize("m,n,b,cplx,dot2,with_x", [
    (5003, 37, 1, False, True, True), (20000, 200, 2, False, False, True),
    (4001, 700, 7, False, True, True), (3000, 1024, 10, False, False, False),
    (2049, 65, 2, True, True, True), (3001, 1000, 10, True, True, True), (3001, 1000, 10, True, False, True),
    (5000, 777, 7, True, False, False), (1234, 1024, 5, True, True, True), (40, 64, 3, True, False, True),
    (7777, 513, 5, False, True, True),
    # complex plain sums on the matrix cores: odd n (a ragged last k block),
    # n just above 256, b = 1 and b = 8 (one N tile), fewer rows than a tile
    (3001, 301, 1, True, False, True), (977, 257, 8, True, False, True), (33, 600, 3, True, False, False),
    (20_011, 1000, 10, True, False, True),
    # real plain sums on the matrix cores, 1024 < n <= 2048 (even): a ragged
    # last k block (n % 16 != 0), b = 1, 3, 8 and 10, fewer rows than a tile
    (4001, 1100, 3, False, False, True), (20_011, 2000, 10, False, False, True),
    (33, 1202, 8, False, False, False), (3000, 2048, 1, False, False, True)])
def test_astream_iter(rl, m, n, b, cplx, dot2, with_x):
    """Iteration form of the pass: A W and A^* [A_V A_X A_W] from one read of A."""
    banner(f"astream_iter m={m} n={n} b={b} complex={cplx} dot2={dot2} AX={with_x}")
    rng = np.random.default_rng(7 * m + n + b)
    A, W = _rand(rng, (m, n), cplx), _rand(rng, (n, b), cplx)
    AV, AX = _rand(rng, (m, b), cplx), _rand(rng, (m, b), cplx)
    dev = lambda x: torch.from_numpy(x).cuda()
    AW, G3 = rl.rl_step_astream_iter(dev(A), dev(W), dev(AV), dev(AX) if with_x else None, dot2=dot2)
    AW, G3 = to_np(AW), to_np(G3)
    absA = np.abs(A)
    if dot2:
        ref = eft.matmul(A, W)
        assert np.all(np.abs(AW - ref) <= 2 * U * np.abs(ref) + 4 * (n * U) ** 2 * (absA @ np.abs(W)))
    else:
        assert np.all(np.abs(AW - A @ W) <= 2 * n * U * (absA @ np.abs(W)))
    # block 0: A^* A_V (Dot2-class with dot2), block 1: A^* A_X or zero,
    # block 2: A^* A_W of the returned A_W
    if dot2:
        G1 = eft.matmul_h(A, AV)
        assert np.all(np.abs(G3[0] - G1) <= 2 * U * np.abs(G1)
                      + 4 * (np.log2(2 * m) * U) ** 2 * (absA.T @ np.abs(AV)))
    else:
        assert np.all(np.abs(G3[0] - A.conj().T @ AV) <= 2 * m * U * (absA.T @ np.abs(AV)))
    if with_x:
        assert np.all(np.abs(G3[1] - A.conj().T @ AX) <= 2 * m * U * (absA.T @ np.abs(AX)))
    else:
        assert np.all(G3[1] == 0)
    assert np.all(np.abs(G3[2] - A.conj().T @ AW) <= 2 * m * U * (absA.T @ np.abs(AW)))


@pytest.mark.parametrize("n,cplx,dot2,odd_lda", [(1025, False, False, False), (1100, False, True, False),
                                                (1100, True, False, False), (1100, False, False, True),
                                                (2050, False, False, False)])
def test_astream_wide_shapes_no_kernel_takes(rl, n, cplx, dot2, odd_lda):
    """Past n = 1024 only real, even n <= 2048, plain sums and 16-byte aligned
    rows have a pass kernel; every other shape is refused before any launch."""
    banner(f"astream refuses n={n} complex={cplx} dot2={dot2} odd lda={odd_lda}")
    m, b = 64, 3
    dt = torch.complex128 if cplx else torch.float64
    if odd_lda:
        A = torch.zeros((m, n + 1), dtype=dt, device="cuda")[:, :n]
    else:
        A = torch.zeros((m, n), dtype=dt, device="cuda")
    W = torch.zeros((n, b), dtype=dt, device="cuda")
    with pytest.raises(rl.RlError) as e:
        rl.rl_step_astream(A, W, dot2=dot2)
    assert e.value.code == rl.RL_ERR_UNSUPPORTED


def test_astream_misaligned_complex(rl):
    """A complex A whose base address is 8 bytes off a 16-byte boundary takes
    the generic complex kernel; same results as the aligned copy."""
    m, n, b = 3001, 300, 3
    rng = np.random.default_rng(99)
    A, W = _rand(rng, (m, n), True), _rand(rng, (n, b), True)
    AV = _rand(rng, (m, b), True)
    buf = torch.zeros(2 * m * n + 1, dtype=torch.float64, device="cuda")
    view = buf[1:].view(m, n, 2)
    view.copy_(torch.from_numpy(np.stack([A.real, A.imag], axis=-1)).cuda())
    Wd, AVd = torch.from_numpy(W).cuda(), torch.from_numpy(AV).cuda()
    AW = torch.empty((m, b), dtype=torch.complex128, device="cuda")
    G3 = torch.empty((3, n, b), dtype=torch.complex128, device="cuda")
    h = rl.handle(0)
    ptr = buf.data_ptr() + 8
    assert ptr % 16 == 8
    import ctypes
    rc = h.lib.rl_step_astream_iter(h.h, 1, m, n, ctypes.c_void_p(ptr), n, b, ctypes.c_void_p(Wd.data_ptr()),
                                    ctypes.c_void_p(AVd.data_ptr()), None, ctypes.c_void_p(AW.data_ptr()),
                                    ctypes.c_void_p(G3.data_ptr()), 0)
    assert rc == rl.RL_OK
    torch.cuda.synchronize()
    AW2, G32 = rl.rl_step_astream_iter(torch.from_numpy(A).cuda(), Wd, AVd, None, dot2=False)
    AW, G3, AW2, G32 = to_np(AW), to_np(G3), to_np(AW2), to_np(G32)
    absA = np.abs(A)
    bound = 2 * n * U * (absA @ np.abs(W))
    assert np.all(np.abs(AW - A @ W) <= bound) and np.all(np.abs(AW2 - A @ W) <= bound)
    assert np.all(np.abs(G3[0] - A.conj().T @ AV) <= 2 * m * U * (absA.T @ np.abs(AV)))
    assert np.all(G3[1] == 0)


def test_astream_cancellation_needs_dot2(rl):
    """On a graded A with A w tiny, Dot2 gives A w to full relative accuracy."""
    m, n = 4000, 200
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((m, n)))
    Vq, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.logspace(0, -12, n)
    A = (Q * s) @ Vq.T
    w = Vq[:, -1:].copy()
    AW, _ = rl.rl_step_astream(torch.from_numpy(A).cuda(), torch.from_numpy(w).cuda(), dot2=True)
    ref = eft.matmul(A, w)
    assert np.max(np.abs(to_np(AW) - ref) / np.abs(ref)) <= 4 * U + 1e-13


@pytest.mark.parametrize("m,t,cplx", [(100_000, 3, False), (20_000, 15, False), (5000, 30, True),
                                      (777, 2, False), (300, 1, True), (4096, 32, False),
                                      (1_000_000, 3, False), (20, 16, False), (64, 16, True), (65, 8, False),
                                      (123_457, 6, True), (40_000, 16, False),
                                      # column-wave kernel (16 < t <= 32): one tile, several tiles,
                                      # several levels of stacked factors
                                      (17, 17, True), (31, 31, False), (129, 18, False), (1000, 20, True),
                                      (50_000, 32, True), (300_000, 24, False), (200_000, 30, True),
                                      (1_000_000, 30, False)])
def test_tall_svd(rl, m, t, cplx):
    banner(f"tall svd m={m} t={t} complex={cplx}")
    rng = np.random.default_rng(m + t)
    Qa, _ = np.linalg.qr(rng.standard_normal((m, t)) + (1j * rng.standard_normal((m, t)) if cplx else 0))
    Qb, _ = np.linalg.qr(rng.standard_normal((t, t)) + (1j * rng.standard_normal((t, t)) if cplx else 0))
    s = np.logspace(0, -10, t)
    P = (Qa * s) @ Qb.conj().T
    sg, C = rl.rl_step_tall_svd(torch.from_numpy(np.ascontiguousarray(P)).cuda())
    sg, C = to_np(sg), to_np(C)
    assert np.all(np.abs(sg - s) <= 1e-12 * s + 1e-15 * s[0])   # graded: relative accuracy
    assert np.linalg.norm(C.conj().T @ C - np.eye(t)) <= 1e-12
    # ||P c_j|| = sigma_j (normwise-accurate singular pairs); the check's own
    # rounding (forming P, the m-term norms) grows with m, so the bound is the
    # larger of 1e-14 and twice what LAPACK's QR + SVD of the same P reaches
    Rl = np.linalg.qr(P, mode="r")
    _, sl, Vlh = np.linalg.svd(Rl)
    ref = np.max(np.abs(np.linalg.norm(P @ Vlh.conj().T, axis=0) - sl))
    assert np.all(np.abs(np.linalg.norm(P @ C, axis=0) - sg) <= max(1e-14 * s[0], 2 * ref))


# The search block's orthonormalisation (S5): two block projections against
# [V X], then Orth.  Register-resident kernel (real n <= 2048, complex
# n <= 1024, b <= 10; one to eight rows per thread, ragged tails) and the
# global-memory kernel (complex n > 1024, b > 10); no X, no projection.
@pytest.mark.parametrize("n,b,cplx,proj,with_x", [
    (200, 1, False, True, True), (1000, 10, True, True, True), (500, 5, False, True, True),
    (2000, 10, False, True, True), (1500, 3, True, True, True), (300, 7, True, True, False),
    (257, 4, False, False, False), (64, 16, False, True, True), (1025, 2, False, True, True),
    (33, 9, True, True, True)])
def test_orth_step(rl, n, b, cplx, proj, with_x):
    from oracle.rlobpcg import _orth, search_block
    banner(f"orth step n={n} b={b} complex={cplx} project={proj} with_x={with_x}")
    rng = np.random.default_rng(1000 * n + b)
    nb = (2 if with_x else 1) * b if proj else 0
    Y, _ = np.linalg.qr(_rand(rng, (n, max(nb, 1)), cplx))
    basis = Y[:, :nb]
    # graded columns with components along [V X] up to 10^4.5 times the part
    # the projections keep (column scaling does not change the Q factor)
    W = _rand(rng, (n, b), cplx) * np.logspace(0, -3, b)
    if nb:
        W = W + basis @ (10.0 * _rand(rng, (nb, b), cplx))
    dev = lambda M: torch.from_numpy(np.ascontiguousarray(M)).cuda()
    V = dev(basis[:, :b]) if proj else None
    X = dev(basis[:, b:2 * b]) if proj and with_x else None
    Q, deg = rl.rl_step_orth(dev(W), V, X)
    Q = to_np(Q)
    Qo, flag = search_block(W, lambda M: M, basis, _orth)
    assert not deg and not flag
    assert np.linalg.norm(Q.conj().T @ Q - np.eye(b)) <= 1e-13
    if nb:
        assert np.linalg.norm(basis.conj().T @ Q) <= 1e-13
    # the same orthonormal basis column by column (QR's Q is unique up to a
    # unit-modulus factor per column).  Any projection leaves an error of
    # about u ||w_j|| in the kept part, so a column agrees to about
    # u ||w_j|| / ||(I - Y Y^*) w_j||: the bound scales with the largest such
    # ratio (kappa), with room for the sqrt(n b) growth of the sums
    Wp = W - basis @ (basis.conj().T @ W) if nb else W
    kappa = float(np.max(np.linalg.norm(W, axis=0) / np.linalg.norm(Wp, axis=0)))
    tol = 64 * U * np.sqrt(n * b) * kappa + 1e-13
    ph = np.einsum("ij,ij->j", Qo.conj(), Q)
    assert np.all(np.abs(np.abs(ph) - 1.0) <= tol)
    assert np.linalg.norm(Q - Qo * (ph / np.abs(ph))) <= tol


@pytest.mark.parametrize("n,b,cplx", [(300, 1, False), (400, 4, True), (1500, 3, True), (2000, 6, False)])
def test_orth_step_degenerate(rl, n, b, cplx):
    """A zero last column: the flag is raised, the column is completed by a
    unit vector projected against [V X] and the earlier columns; the other
    columns are the oracle's."""
    from oracle.rlobpcg import _orth, search_block
    banner(f"orth step degenerate n={n} b={b} complex={cplx}")
    rng = np.random.default_rng(77 + n + b)
    Y, _ = np.linalg.qr(_rand(rng, (n, 2 * b), cplx))
    W = _rand(rng, (n, b), cplx)
    W[:, -1] = 0.0
    dev = lambda M: torch.from_numpy(np.ascontiguousarray(M)).cuda()
    Q, deg = rl.rl_step_orth(dev(W), dev(Y[:, :b]), dev(Y[:, b:]))
    Q = to_np(Q)
    assert deg
    assert np.linalg.norm(Q.conj().T @ Q - np.eye(b)) <= 1e-13
    assert np.linalg.norm(Y.conj().T @ Q) <= 1e-13
    if b > 1:
        Qo, _ = search_block(W[:, :-1], lambda M: M, Y, _orth)
        ph = np.einsum("ij,ij->j", Qo.conj(), Q[:, :-1])
        assert np.linalg.norm(Q[:, :-1] - Qo * (ph / np.abs(ph))) <= 1e-10
