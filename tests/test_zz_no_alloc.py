"""The allocation-free pass entry point (rl_step_astream_iter_noalloc)
against the allocating one (rl_step_astream_iter), through the C-ABI.

Both run the same kernels in the same launch configuration, so the outputs
must agree bit for bit.  Two calls in a row, the second on a smaller input,
check that the shared static scratch is reused correctly (nothing from the
first call leaks into the second); a shape whose partial sums need more than
the scratch holds is rejected before anything is enqueued."""

import pytest

from .gpu_util import banner

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rl():
    import paper_2602_16797_amd as rl
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return rl


def _inputs(m, n, b, cplx, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    dt = torch.complex128 if cplx else torch.float64
    A = torch.randn((m, n), dtype=dt, device="cuda", generator=g)
    W, _ = torch.linalg.qr(torch.randn((n, b), dtype=dt, device="cuda", generator=g))
    AV = torch.randn((m, b), dtype=dt, device="cuda", generator=g) * 1e-3
    AX = torch.randn((m, b), dtype=dt, device="cuda", generator=g) * 1e-2
    return A, W.contiguous(), AV, AX


@pytest.mark.parametrize("cplx", [False, True])
def test_noalloc_pass_equals_the_allocating_pass_twice(rl, cplx):
    shapes = [(200_000, 200, 1), (30_011, 96, 3)] if not cplx else [(20_000, 64, 2), (9_001, 40, 3)]
    for i, (m, n, b) in enumerate(shapes):
        banner(f"noalloc pass call {i}: {m}x{n} b={b} complex={cplx}")
        A, W, AV, AX = _inputs(m, n, b, cplx, 100 + i)
        aw_ref, g_ref = rl.rl_step_astream_iter(A, W, AV, AX, dot2=True)
        aw, g3 = rl.rl_step_astream_iter_noalloc(A, W, AV, AX, dot2=True)
        torch.cuda.synchronize()
        assert torch.equal(aw, aw_ref)
        assert torch.equal(g3, g_ref)
        # and against a plain product, loosely (the allocating pass has its own parity tests)
        ref = A @ W
        assert torch.allclose(aw, ref, rtol=1e-12, atol=1e-12 * float(ref.abs().max()))


def test_noalloc_pass_into_caller_buffers_without_x(rl):
    m, n, b = 50_000, 128, 2
    A, W, AV, _ = _inputs(m, n, b, False, 7)
    AW = torch.full((m, b), float("nan"), dtype=A.dtype, device="cuda")
    G3 = torch.full((3, n, b), float("nan"), dtype=A.dtype, device="cuda")
    aw_ref, g_ref = rl.rl_step_astream_iter(A, W, AV, None, dot2=False)
    rl.rl_step_astream_iter_noalloc(A, W, AV, None, dot2=False, AW=AW, G3=G3)
    torch.cuda.synchronize()
    assert torch.equal(AW, aw_ref) and torch.equal(G3, g_ref)
    assert torch.count_nonzero(G3[1]) == 0                  # no previous direction: the middle block is zero


def test_noalloc_pass_rejects_a_shape_beyond_its_scratch(rl):
    m, n, b = 200_000, 1024, 10
    A = torch.zeros((m, n), dtype=torch.float64, device="cuda")
    W = torch.zeros((n, b), dtype=torch.float64, device="cuda")
    AV = torch.zeros((m, b), dtype=torch.float64, device="cuda")
    with pytest.raises(rl.RlError) as e:
        rl.rl_step_astream_iter_noalloc(A, W, AV)
    assert e.value.code == rl.RL_ERR_SCRATCH
