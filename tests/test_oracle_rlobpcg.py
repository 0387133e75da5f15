"""Pins for oracle.rlobpcg: dense SVD on small inputs, planted spectra, the
theory's inequalities (Fact prop:randomized_preconditioning, Fact
prop:sketch_and_solve, eq:lobpcg_psd_compare, Thm. thm:rlobpcg_convergence),
LOBPCG invariants and exact transformations of A."""

import math

import numpy as np
import pytest

from oracle import rlobpcg, sparsestack
from oracle.rlobpcg import default_tau
from workloads import planted_numpy, spectrum_gap, spectrum_logspace_tail

U = 2.0 ** -53


def _sin_angle(Va, Vb):
    """Largest principal angle sine between span(Va) and span(Vb)."""
    Qa, _ = np.linalg.qr(Va)
    Qb, _ = np.linalg.qr(Vb)
    return float(np.linalg.norm(Qb - Qa @ (Qa.conj().T @ Qb), 2))


@pytest.fixture(scope="module")
def cfg1():
    s = spectrum_logspace_tail(50, 1e-3, 1e-6)
    A, V, s = planted_numpy(4000, 50, s, 1001)
    return A, V, s


def _dense(A):
    _, sv, Vh = np.linalg.svd(A, full_matrices=False)
    return sv, Vh.conj().T


def test_default_tau_and_arguments():
    assert default_tau(100) == 2.0 * 10.0 * 2.0 ** -52
    A = np.zeros((10, 6))
    for bad in (dict(k=0), dict(k=3, block=2), dict(k=3)):
        with pytest.raises(ValueError):
            rlobpcg(A, **bad)
    with pytest.raises(ValueError):
        rlobpcg(np.zeros((5, 6)), 1)


def test_single_vector_vs_dense_svd_and_planted(cfg1):
    A, Vp, s = cfg1
    sv, Vd = _dense(A)
    r = rlobpcg(A, 1, seed=2001)
    assert r.status == 0
    assert abs(r.sigma[0] - sv[-1]) <= 1e-12 * sv[0]
    assert abs(r.sigma[0] - s[-1]) <= 1e-12 * sv[0]
    assert _sin_angle(r.V, Vd[:, -1:]) <= 1e-10
    # backward-stable floors the paper compares against (Sec. 4): RLOBPCG beats them
    gap_abs = (sv[-2] - sv[-1]) / sv[0]
    assert abs(r.sigma[0] - sv[-1]) / sv[-1] <= U * sv[0] / sv[-1]
    assert _sin_angle(r.V, Vd[:, -1:]) <= U / gap_abs
    # left vector: A v = sigma u with a unit u
    assert np.linalg.norm(A @ r.V[:, 0] - r.sigma[0] * r.U[:, 0]) <= 1e-12 * sv[0]
    assert abs(np.linalg.norm(r.U[:, 0]) - 1.0) < 1e-8


@pytest.mark.parametrize("is_complex", [False, True])
def test_block_vs_dense_svd(is_complex):
    m, n, k = (3000, 60, 3) if not is_complex else (2000, 42, 2)
    s = spectrum_gap(n, k, 1e-9, 10.0)
    A, _, s = planted_numpy(m, n, s, 7 + is_complex, is_complex=is_complex)
    sv, Vd = _dense(A)
    r = rlobpcg(A, k, seed=3, max_iter=60)
    assert np.all(np.diff(r.sigma) >= 0)
    assert np.max(np.abs(r.sigma - sv[::-1][:k])) <= 1e-12 * sv[0]
    assert _sin_angle(r.V, Vd[:, -k:]) <= 1e-10
    res = A @ r.V - r.U * r.sigma[None, :]
    assert np.linalg.norm(res, axis=0).max() <= 1e-12 * sv[0]


def _eta_scale_free(A, d, zeta, seed):
    """Distortion of S on range(A), after the best rescaling of S."""
    Qa, _ = np.linalg.qr(A)
    SQ = sparsestack.sketch(Qa, d, zeta, seed)
    sv = np.linalg.svd(SQ, compute_uv=False)
    c2 = 2.0 / (sv.max() ** 2 + sv.min() ** 2)          # best scale: 1-eta = c2 smin^2
    return 1.0 - c2 * sv.min() ** 2, c2


def test_randomized_preconditioning_and_sketch_and_solve_bounds():
    """Fact prop:randomized_preconditioning: sigma(AP)^2 in [1/(1+eta), 1/(1-eta)];
    Fact prop:sketch_and_solve: ||A v_0||^2 <= (1+eta)/(1-eta) sigma_min^2."""
    m, n, d, zeta, seed = 6000, 40, 160, 8, 11
    s = spectrum_gap(n, 1, 1e-8, 10.0)
    A, _, s = planted_numpy(m, n, s, 5)
    eta, c2 = _eta_scale_free(A, d, zeta, seed)
    assert 0 < eta < 1
    SA = sparsestack.sketch(A, d, zeta, seed) * math.sqrt(c2)
    _, St, Vth = np.linalg.svd(SA, full_matrices=False)
    P = Vth.T / St[None, :]
    sap = np.linalg.svd(A @ P, compute_uv=False) ** 2
    assert sap.min() >= 1 / (1 + eta) * (1 - 1e-6)
    assert sap.max() <= 1 / (1 - eta) * (1 + 1e-6)
    v0 = Vth.T[:, -1]
    assert np.linalg.norm(A @ v0) ** 2 <= (1 + eta) / (1 - eta) * s[-1] ** 2 * (1 + 1e-6)


def test_convergence_theorem_bound_single_vector():
    """Thm. thm:rlobpcg_convergence: with eta < gap/(2+gap),
    (||A v_k||^2 - sigma_n^2)/sigma_n^2 <= C gap q^{2k} (until the FP64 floor)."""
    m, n, d, zeta, seed = 8000, 40, 160, 8, 17
    s = spectrum_gap(n, 1, 1e-6, 10.0)
    A, _, s = planted_numpy(m, n, s, 23)
    eta, _ = _eta_scale_free(A, d, zeta, seed)
    gap = (s[-2] ** 2 - s[-1] ** 2) / s[-1] ** 2
    assert eta < gap / (2 + gap)
    C = 2 * eta / ((1 - eta) * gap - 2 * eta)
    q = eta + (1 - eta) / (1 + gap)
    sv = np.linalg.svd(A, compute_uv=False)
    r = rlobpcg(A, 1, d=d, zeta=zeta, seed=seed, rule="none", max_iter=25)
    floor = 1e3 * U * sv[0] / sv[-1]
    for kk, th in enumerate(r.theta_hist[1:], start=1):
        rel = (th[0] ** 2 - sv[-1] ** 2) / sv[-1] ** 2
        assert rel <= C * gap * q ** (2 * kk) + floor


def test_lobpcg_step_beats_steepest_descent_and_invariants():
    """eq:lobpcg_psd_compare: the minimiser over span{v_old, v, w} is at least as
    good as over span{v, w}; T orthonormal; Ritz values monotone; Galerkin
    V^* R ~ 0; maintained A_T equals A T up to rounding drift."""
    m, n, k = 3000, 45, 2
    s = spectrum_gap(n, k, 1e-7, 10.0)
    A, _, s = planted_numpy(m, n, s, 41)
    normA = s[0]
    log = []

    def cb(**kw):
        log.append({key: np.array(v, copy=True) for key, v in kw.items() if key != "i"})

    r = rlobpcg(A, k, seed=5, rule="none", max_iter=12, callback=cb)
    prev = r.theta_hist[0]
    for it, st in enumerate(log):
        T, AT, C, V, AV, R = st["T"], st["AT"], st["C"], st["V"], st["AV"], st["R"]
        b = V.shape[1]
        t = T.shape[1]
        assert np.linalg.norm(T.conj().T @ T - np.eye(t)) <= 1e-13
        # PSD trial space: [V_i, W_i] = first b and last b columns of T
        psd = np.hstack([AT[:, :b], AT[:, t - b:]])
        psd_min = np.linalg.svd(psd, compute_uv=False)[::-1][:b]
        theta = np.sort(r.theta_hist[it + 1])
        assert np.all(theta <= psd_min * (1 + 1e-10) + 1e3 * U * normA)
        assert np.all(theta <= np.sort(prev) * (1 + 1e-10) + 1e3 * U * normA)
        prev = r.theta_hist[it + 1]
        assert np.linalg.norm(V.conj().T @ R) <= 1e3 * U * np.linalg.norm(AT, 2) ** 2 * t
        drift = np.linalg.norm(AT - A @ T, 2)
        assert drift <= 50 * (it + 1) * U * normA * math.sqrt(n)


def test_exact_transformations():
    m, n = 3000, 40
    s = spectrum_gap(n, 1, 1e-7, 10.0)
    A, _, s = planted_numpy(m, n, s, 51)
    base = rlobpcg(A, 1, seed=6)
    # scaling A by c scales sigma by |c|, same V
    sc = rlobpcg(-4.0 * A, 1, seed=6)
    assert abs(sc.sigma[0] - 4.0 * base.sigma[0]) <= 1e-12 * 4.0 * s[0]
    assert _sin_angle(sc.V, base.V) <= 1e-10
    # a column permutation permutes V's rows
    perm = np.random.default_rng(0).permutation(n)
    pc = rlobpcg(A[:, perm], 1, seed=6)
    assert abs(pc.sigma[0] - base.sigma[0]) <= 1e-12 * s[0]
    assert _sin_angle(pc.V, base.V[perm]) <= 1e-10
    # a real A passed as complex gives the same triplet
    cc = rlobpcg(A.astype(np.complex128), 1, seed=6)
    assert abs(cc.sigma[0] - base.sigma[0]) <= 1e-12 * s[0]
    assert _sin_angle(cc.V, base.V.astype(np.complex128)) <= 1e-10
    # a row permutation changes the sketch, not the answer
    rp = rlobpcg(A[np.random.default_rng(1).permutation(m)], 1, seed=6)
    assert abs(rp.sigma[0] - base.sigma[0]) <= 1e-12 * s[0]
    assert _sin_angle(rp.V, base.V) <= 1e-10


def test_qr_preconditioner_is_the_same_operator():
    """P P^* from the SVD route equals (R^* R)^{-1} from the QR route
    (Sec. 1, footnote), and both routes reach the same triplets."""
    m, n, d = 2000, 30, 120
    s = spectrum_gap(n, 2, 1e-5, 10.0)
    A, _, s = planted_numpy(m, n, s, 61)
    SA = sparsestack.sketch(A, d, 8, 4)
    _, St, Vth = np.linalg.svd(SA, full_matrices=False)
    P = Vth.T / St[None, :]
    R = np.linalg.qr(SA, mode="r")
    Rinv = np.linalg.inv(R)
    M1, M2 = P @ P.T, Rinv @ Rinv.T
    assert np.linalg.norm(M1 - M2) <= 1e-10 * np.linalg.norm(M1)
    a = rlobpcg(A, 2, d=d, seed=4, precond="svd")
    b = rlobpcg(A, 2, d=d, seed=4, precond="qr")
    assert np.max(np.abs(a.sigma - b.sigma)) <= 1e-12 * s[0]
    assert _sin_angle(a.V, b.V) <= 1e-10


def test_block_of_one_equals_single_vector_start():
    """With b = 1 the start is v_0 = V~(:, n) with theta_0 = inf (Alg. rlopcg);
    the first iterate's theta equals the minimum over span{v_0, w_0}."""
    m, n = 2000, 30
    s = spectrum_gap(n, 1, 1e-6, 10.0)
    A, _, s = planted_numpy(m, n, s, 71)
    r = rlobpcg(A, 1, seed=2, rule="none", max_iter=3)
    assert math.isinf(r.theta_hist[0][0])
    SA = sparsestack.sketch(A, 4 * n, 8, 2)
    v0 = np.linalg.svd(SA)[2][-1]
    r0 = A.T @ (A @ v0) - np.linalg.norm(A @ v0) ** 2 * v0
    assert abs(np.linalg.norm(r0) - r.rnorm_hist[0][0]) <= 1e-6 * np.linalg.norm(r0)


@pytest.mark.parametrize("lp", ["diag", "none"])
def test_loop_precond_first_step_minimises_over_span(lp):
    """The comparison methods of Sec. 1.1 (LOBPCG with P = diag(||A(:, i)||^{-1})
    and with no preconditioner) keep the sketch-and-solve start v_0; their
    first iterate minimises ||A z|| / ||z|| over span{v_0, P P^* r_0}, checked
    against the smallest singular value of A on that 2-dimensional span.
    Column norms spread over three decades so a wrong power or axis of the
    diagonal scaling changes the span."""
    m, n = 2000, 30
    s = spectrum_gap(n, 1, 1e-6, 10.0)
    A0, _, _ = planted_numpy(m, n, s, 73)
    A = A0 * np.logspace(0, 3, n)[None, :]
    r = rlobpcg(A, 1, seed=2, rule="none", max_iter=1, loop_precond=lp)
    SA = sparsestack.sketch(A, 4 * n, 8, 2)
    v0 = np.linalg.svd(SA)[2][-1]
    Av0 = A @ v0
    r0 = A.T @ Av0 - (Av0 @ Av0) * v0
    w0 = r0 / np.sum(A * A, axis=0) if lp == "diag" else r0
    Q, _ = np.linalg.qr(np.stack([v0, w0], axis=1))
    expect = np.linalg.svd(A @ Q, compute_uv=False)[-1]
    assert abs(r.theta_hist[1][0] - expect) <= 1e-9 * expect


def test_loop_precond_diag_converges_on_coherent_problem():
    """On the paper's easy problem shape (right singular vectors close to the
    standard basis, sigma geometric from 1 to 0.1 and a gap to 1e-7) the
    diagonally preconditioned loop reaches the dense SVD's smallest triplet."""
    rng = np.random.default_rng(5)
    m, n = 3000, 40
    V, _ = np.linalg.qr(np.diag(rng.standard_normal(n)) + 1e-4 * rng.standard_normal((n, n)))
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    s = np.geomspace(1.0, 0.1, n)
    s[-1] = 1e-7
    A = (U * s[None, :]) @ V.T
    r = rlobpcg(A, 1, seed=3, loop_precond="diag")
    sv, Vd = _dense(A)
    assert r.status == 0
    assert abs(r.sigma[0] - sv[-1]) <= 1e-12 * sv[0]
    assert _sin_angle(r.V, Vd[:, -1:]) <= 1e-8


def test_loop_precond_rejects_unknown():
    A = np.random.default_rng(0).standard_normal((200, 12))
    with pytest.raises(ValueError):
        rlobpcg(A, 1, loop_precond="jacobi")


def test_svqb_is_an_orthonormal_basis_of_the_same_span():
    """SVQB returns orthonormal columns spanning span(W) (checked against the
    Householder QR basis); its loss of orthogonality grows like eps * cond^2
    (Stathopoulos and Wu), so an ill-conditioned block stays within that."""
    from oracle.rlobpcg import _svqb
    rng = np.random.default_rng(9)
    W = rng.standard_normal((60, 5)) * np.array([1.0, 3.0, 0.5, 10.0, 2.0])[None, :]
    Q, flag = _svqb(W)
    assert not flag
    assert np.linalg.norm(Q.T @ Q - np.eye(5)) <= 1e-14
    assert _sin_angle(Q, W) <= 1e-14
    U, _ = np.linalg.qr(rng.standard_normal((60, 4)))
    Vt, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    Wc = (U * np.array([1.0, 1e-2, 1e-4, 1e-6])[None, :]) @ Vt.T
    Qc, _ = _svqb(Wc)
    assert np.linalg.norm(Qc.T @ Qc - np.eye(4)) <= 1e3 * 2.0 ** -52 * 1e12
    assert _sin_angle(Qc[:, :], Wc) <= 1e-4
    Zc = np.zeros((20, 3)) + 1j * 0.0
    Zc[:, 0] = 1.0
    _, flag = _svqb(Zc)
    assert flag                                    # zero columns fall back to Orth


def test_svqb_solve_reaches_dense_triplets():
    """RLOBPCG with SVQB in the orthogonalisation step converges to the dense
    SVD's smallest triplets on a block problem with a gap.  (Here the paper's
    stagnation test does not fire before max_iter with SVQB, while it stops
    the CGS2 run at iteration 81: the triplets are reached either way.)"""
    m, n, k = 3000, 40, 3
    s = spectrum_gap(n, k, 1e-6, 10.0)
    A, _, s = planted_numpy(m, n, s, 77)
    r = rlobpcg(A, k, seed=4, orth="svqb")
    sv, Vd = _dense(A)
    assert np.max(np.abs(r.sigma - sv[::-1][:k])) <= 1e-12 * sv[0]
    assert _sin_angle(r.V, Vd[:, -k:]) <= 1e-10
    with pytest.raises(ValueError):
        rlobpcg(A, k, orth="mgs")


def test_normalize_of_a_zero_vector_is_e1_with_the_flag():
    """Orth of one column (Normalize): a zero or non-finite vector gives e_1
    and raises the degenerate flag; any other vector is scaled to unit norm."""
    from oracle.rlobpcg import _orth
    for bad in (np.zeros((7, 1)), np.zeros((7, 1), dtype=np.complex128), np.full((7, 1), np.nan)):
        q, flag = _orth(bad)
        assert flag
        assert q.shape == (7, 1) and q[0, 0] == 1.0 and np.count_nonzero(q) == 1
    x = np.arange(1.0, 8.0)[:, None] * (1 - 2j)
    q, flag = _orth(x)
    assert not flag
    assert abs(np.linalg.norm(q) - 1.0) <= 1e-15
    assert np.linalg.norm(q - x / np.linalg.norm(x)) <= 1e-15


def test_previous_direction_when_the_old_block_does_not_mix():
    """eq:x-defining with C(1:b, 1:t-b) = 0: the old V is itself the selected
    Ritz vector, Q = Orth(0) = e_1 with the degenerate flag, and X = T C(:, 1)
    is still a unit vector orthogonal to the new V, with A X = A_T C(:, 1)."""
    from oracle.rlobpcg import previous_direction
    rng = np.random.default_rng(3)
    T, _ = np.linalg.qr(rng.standard_normal((20, 3)))
    AT = rng.standard_normal((50, 3))
    c, s = math.cos(0.3), math.sin(0.3)
    C = np.array([[0.0, 0.0, 1.0], [c, s, 0.0], [-s, c, 0.0]])      # orthogonal, C(1, 1:2) = 0
    X, AX, flag = previous_direction(T, AT, C, 1)
    assert flag
    assert np.allclose(X[:, 0], T @ C[:, 0], atol=1e-15, rtol=0)
    assert np.allclose(AX[:, 0], AT @ C[:, 0], atol=1e-15, rtol=0)
    assert abs(np.linalg.norm(X) - 1.0) <= 1e-14
    assert abs(float(X[:, 0] @ (T @ C[:, 2]))) <= 1e-14
    # with a mixing block the same call needs no fallback
    C2, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    X2, _, flag2 = previous_direction(T, AT, C2, 1)
    assert not flag2 and abs(np.linalg.norm(X2) - 1.0) <= 1e-14


def test_left_vectors_of_a_zero_singular_value():
    """U-hat(:, j) = A v_j / sigma_j, and a zero sigma_j gives a zero column
    with the zero_theta flag instead of a division by zero."""
    from oracle.rlobpcg import left_vectors
    AV = np.array([[3.0, 0.0], [4.0, 0.0], [0.0, 0.0]])
    U, flag = left_vectors(AV, np.array([5.0, 0.0]))
    assert flag
    assert np.array_equal(U[:, 1], np.zeros(3))
    assert np.allclose(U[:, 0], [0.6, 0.8, 0.0], rtol=0, atol=1e-16)
    _, flag = left_vectors(AV[:, :1], np.array([5.0]))
    assert not flag


def test_refresh_recomputes_the_product_and_rotates():
    """refresh=True recomputes A V-hat from V-hat and rotates (V-hat, sigma,
    U-hat) by the SVD of that m x b block.  The maintained A_V is corrupted
    after the last step, so only a real recomputation meets the residual
    gate; the refreshed triplets then match the dense SVD, U-hat has
    orthonormal columns, and V-hat spans the final Ritz block."""
    m, n, k = 3000, 60, 3
    A, _, s = planted_numpy(m, n, spectrum_gap(n, k, 1e-9, 10.0), 7)
    sv, Vd = _dense(A)
    last = 59

    def corrupt(**kw):
        if kw["i"] == last:
            kw["AV"][:] += 1e-6 * np.random.default_rng(0).standard_normal(kw["AV"].shape)

    plain = rlobpcg(A, k, seed=3, rule="none", max_iter=last + 1, callback=corrupt, refresh=False)
    res_plain = np.linalg.norm(A @ plain.V - plain.U * plain.sigma[None, :], axis=0).max()
    assert res_plain > 1e-9                               # U-hat came from the corrupted A_V
    r = rlobpcg(A, k, seed=3, rule="none", max_iter=last + 1, callback=corrupt, refresh=True)
    res = np.linalg.norm(A @ r.V - r.U * r.sigma[None, :], axis=0).max()
    assert res <= 1e-12 * sv[0]
    assert np.all(np.diff(r.sigma) >= 0)
    assert np.max(np.abs(r.sigma - sv[::-1][:k])) <= 1e-12 * sv[0]
    assert np.linalg.norm(r.U.conj().T @ r.U - np.eye(k)) <= 1e-13
    assert _sin_angle(r.V, r.V_block) <= 1e-13
    assert _sin_angle(r.V, Vd[:, -k:]) <= 1e-10
    # the rotation diagonalises A^* A on the block: V-hat^* A^* A V-hat = Sigma^2
    G = (A @ r.V).conj().T @ (A @ r.V)
    assert np.linalg.norm(G - np.diag(r.sigma ** 2)) <= 1e-12 * sv[0] ** 2


# ---------------------------------------------------------------- locking (Sec. 2.3)

def _davis_kahan(A, V, sig, sv, k):
    """Davis-Kahan sin-theta bound for span(V) against the k smallest right
    singular vectors of A: sqrt(k) max_j ||A^* A v_j - sigma_j^2 v_j|| /
    (sigma_{n-k}^2 - max_j sigma_j^2), the residual recomputed here from
    the returned triplets with compensated products (their error, about
    u ||A|| ||A v|| + u sigma^2, is covered by the allowance added)."""
    from oracle import eft
    AV = eft.matmul(A, V)
    R = eft.matmul_h(A, AV) - V * (sig * sig)[None, :]
    res = float(np.linalg.norm(R, axis=0).max()) + 8 * U * (sv[0] * float(np.linalg.norm(AV))
                                                             + float(np.max(sig)) ** 2)
    gap = sv[-k - 1] ** 2 - float(np.max(sig)) ** 2
    return math.sqrt(k) * res / gap


@pytest.mark.parametrize("cplx", [False, True])
def test_lock_solve_matches_dense_svd(cplx):
    """Locked solve: sigma to 1e-12 ||A|| of the dense SVD, residual gate, and
    the subspace inside the Davis-Kahan bound its own residual gives; the
    columns lock at different iterations and the solve ends when the last
    one does."""
    m, n, k = 3000, 60, 3
    A, _, s = planted_numpy(m, n, spectrum_logspace_tail(n, 1e-3, 1e-6), 13, is_complex=cplx)
    sv, Vd = _dense(A)
    r = rlobpcg(A, k, seed=3, lock=True)
    counts = [int(a.sum()) for a in r.lock_hist]
    assert r.status == 0 and counts[-1] == 0
    assert len(set(counts)) > 2                          # staggered locks
    assert np.max(np.abs(r.sigma - np.sort(sv)[:k])) <= 1e-12 * sv[0]
    assert np.linalg.norm(A @ r.V - r.U * r.sigma[None, :], axis=0).max() <= 1e-12 * sv[0]
    bound = _davis_kahan(A, r.V, r.sigma, sv, k)
    assert bound < 1e-6
    assert _sin_angle(r.V, Vd[:, -k:]) <= bound


def test_lock_search_blocks_are_orthogonal_to_every_column_of_v():
    """Every step's trial basis [V X W] is orthonormal, so X and W are
    orthogonal to all of V, the locked columns included (the property the
    paper gives locking); W has one column per active index and X one per
    active index of the previous step."""
    m, n, k = 3000, 60, 3
    A, _, _ = planted_numpy(m, n, spectrum_logspace_tail(n, 1e-3, 1e-6), 13)
    log = []

    def cb(**kw):
        log.append((kw["T"].copy(), kw["W"].shape[1], kw["X"].shape[1], kw["act"].copy()))

    r = rlobpcg(A, k, seed=3, lock=True, callback=cb)
    saw_locked = False
    for i, (T, nw, nx, act) in enumerate(log):
        b = k
        assert nw == int(act.sum())
        assert nx in (0, nw)
        assert T.shape[1] == b + nx + nw
        assert np.linalg.norm(T.conj().T @ T - np.eye(T.shape[1])) <= 1e-12
        if not act.all():
            saw_locked = True
            locked = T[:, :b][:, ~act]
            assert np.abs(locked.conj().T @ T[:, b:]).max() <= 1e-13
    assert saw_locked and len(log) == r.iters


def test_lock_decisions_follow_the_criterion():
    """The lock mask only shrinks, a column locks exactly when its residual
    first meets Sigma~(1,1)^2 tau, and the stop is where the last one locks
    (re-derived from the histories alone)."""
    from oracle import termination
    m, n, k = 3000, 60, 3
    A, _, _ = planted_numpy(m, n, spectrum_logspace_tail(n, 1e-3, 1e-6), 13)
    r = rlobpcg(A, k, seed=3, lock=True)
    thr = r.sigma1 ** 2 * default_tau(n)
    act = np.ones(k, dtype=bool)
    for j, (mask, rn) in enumerate(zip(r.lock_hist, r.rnorm_hist)):
        want = act & ~(np.asarray(rn) <= thr)
        assert mask.tolist() == want.tolist()
        act = want
    assert termination.first_stop_locked(r.theta_hist, r.rnorm_hist, r.sigma1, default_tau(n)) == r.iters - 1


def test_lock_without_converged_columns_is_the_plain_iteration():
    """With a tolerance no column can meet, locking changes nothing: the
    same bits as the solve without it."""
    m, n, k = 2000, 45, 3
    A, _, _ = planted_numpy(m, n, spectrum_gap(n, k, 1e-6, 10.0), 21)
    a = rlobpcg(A, k, seed=4, lock=False, rule="none", max_iter=15, tau=1e-40)
    b = rlobpcg(A, k, seed=4, lock=True, rule="none", max_iter=15, tau=1e-40)
    assert np.array_equal(a.sigma, b.sigma) and np.array_equal(a.V, b.V) and np.array_equal(a.U, b.U)
    assert np.array_equal(np.array(a.theta_hist), np.array(b.theta_hist))
    assert all(h.all() for h in b.lock_hist)


def test_lock_uses_fewer_search_columns_at_equal_sigma():
    """Locked columns get no search direction: fewer columns of W in all
    (fewer products with A) for the same sigma to 1e-12 ||A||."""
    m, n, k = 3000, 60, 3
    A, _, s = planted_numpy(m, n, spectrum_logspace_tail(n, 1e-3, 1e-6), 13)
    cols = {}
    res = {}
    for lock in (False, True):
        w = []
        res[lock] = rlobpcg(A, k, seed=3, lock=lock, callback=lambda **kw: w.append(kw["W"].shape[1]))
        cols[lock] = sum(w)
    assert cols[True] < cols[False]
    assert np.max(np.abs(res[True].sigma - res[False].sigma)) <= 1e-12 * s[0]
