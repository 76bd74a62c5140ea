"""The allocation-free SVD entry point against the allocating one, through the C ABI.

Two calls in a row share the device's fixed workspace (the second with a smaller
input sees what the first left in it); each result must equal tnfem_prim_svd's on
the same input and factor the input to LAPACK's singular values.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2501_12151_amd import tnfem  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _graded(rng, m, n):
    c = min(m, n)
    U, _ = np.linalg.qr(rng.standard_normal((m, c)))
    V, _ = np.linalg.qr(rng.standard_normal((n, c)))
    return (U * np.logspace(0, -10, c)) @ V.T


def _svd(fn, m, n, A):
    c = min(m, n)
    dU = torch.full((m, c), np.nan, dtype=torch.float64, device="cuda")
    dS = torch.full((c,), np.nan, dtype=torch.float64, device="cuda")
    dV = torch.full((c, n), np.nan, dtype=torch.float64, device="cuda")
    fn(m, n, dev(A), dU, dS, dV, stream=torch.cuda.current_stream())
    return host(dU), host(dS), host(dV)


def test_noalloc_svd_equals_allocating_svd_on_consecutive_calls():
    ctx = tnfem.Context(0, stream=torch.cuda.current_stream())
    try:
        rng = np.random.default_rng(11)
        # the first call fills most of the workspace (blocked QR of a tall matrix, the
        # 1024-thread Jacobi kernel); the second, smaller and wide, reuses it
        cases = [(1024, 132, rng.standard_normal((1024, 132))), (40, 300, _graded(rng, 40, 300))]
        for m, n, A in cases:
            print(f"noalloc svd m={m} n={n}", flush=True)
            assert 0 < tnfem.svd_noalloc_doubles(m, n) <= tnfem.NOALLOC_SCRATCH_BYTES // 8
            U0, S0, V0 = _svd(ctx.svd, m, n, A)
            U1, S1, V1 = _svd(ctx.svd_noalloc, m, n, A)
            scale = np.linalg.norm(A, 2)
            tol = 1e-13 * max(m, n)
            for a, b in ((U0, U1), (V0, V1)):
                assert np.abs(a - b).max() <= tol
            assert np.abs(S0 - S1).max() <= tol * scale
            Sl = np.linalg.svd(A, compute_uv=False)
            assert np.abs(S1 - Sl).max() <= 1e-13 * scale * max(m, n)
            assert np.linalg.norm((U1 * S1) @ V1 - A) <= 1e-13 * scale * max(m, n)
    finally:
        ctx.close()


def test_noalloc_svd_rejects_shapes_beyond_its_workspace():
    ctx = tnfem.Context(0, stream=torch.cuda.current_stream())
    try:
        m, n = 2048, 256
        assert tnfem.svd_noalloc_doubles(m, n) > tnfem.NOALLOC_SCRATCH_BYTES // 8
        t = torch.zeros(8, dtype=torch.float64, device="cuda")
        # rejected on the host before anything is launched (the buffers are never touched)
        with pytest.raises(tnfem.TnfemError) as e:
            ctx.svd_noalloc(m, n, t, t, t, t, stream=torch.cuda.current_stream())
        assert e.value.code == tnfem.EINVAL
    finally:
        ctx.close()
