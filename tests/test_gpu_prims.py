"""GPU parity of the sweep's building blocks against the oracle / LAPACK."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import amen as oamen  # noqa: E402
from paper_2501_12151_amd import tnfem, workloads  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def ctx():
    c = tnfem.Context(0, stream=torch.cuda.current_stream())
    yield c
    c.close()


# every column in registers for m <= 512 and n <= 80 (1 / 2 / 4 / 8 rows per lane, 1 / 2 / 3 / 5
# columns per wavefront: (1, 1), (8, 8), (64, 16), (37, 5), wide (5, 37) and (64, 80), (128, 64),
# (200, 40), (256, 36), (300, 80), (480, 33), (512, 16), (512, 72)); wider: the padded LDS layout
# ((100, 250)); beyond LDS: blocked for 256 < m <= 2048 and n >= 32 ((300, 256), (513, 65),
# (1024, 132), (1600, 200)), else 8 / 16 / 32 rows per lane ((700, 24), (1500, 20)); taller than
# 2048 rows (the plain global-memory variant)
QR_SHAPES = [(1, 1), (8, 8), (64, 16), (256, 36), (1024, 132), (37, 5), (5, 37), (300, 256), (1600, 200),
             (100, 250), (2100, 40), (513, 65), (200, 40), (128, 64), (512, 16), (700, 24), (1500, 20),
             (512, 72), (300, 80), (64, 80), (480, 33)]


@pytest.mark.parametrize("m,n", QR_SHAPES)
def test_qr_matches_definition(ctx, m, n):
    print(f"qr m={m} n={n}", flush=True)
    rng = np.random.default_rng(m * 1000 + n)
    A = rng.standard_normal((m, n))
    c = min(m, n)
    dA, dQ, dR = dev(A), torch.zeros((m, c), dtype=torch.float64, device="cuda"), torch.zeros((c, n), dtype=torch.float64, device="cuda")
    ctx.qr(m, n, dA, dQ, dR, stream=torch.cuda.current_stream())
    Q, R = host(dQ), host(dR)
    assert np.linalg.norm(Q @ R - A) <= 1e-13 * np.linalg.norm(A) * max(1, np.sqrt(n))
    assert np.abs(Q.T @ Q - np.eye(c)).max() <= 1e-13 * max(m, 1)
    assert np.all(np.tril(R, -1) == 0)
    Rl = np.linalg.qr(A)[1]
    assert np.allclose(np.abs(np.diag(R)), np.abs(np.diag(Rl)), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("m,n", [(700, 60), (40, 12), (500, 60)])
def test_qr_rank_deficient(ctx, m, n):
    """Zero and repeated columns (zero reflectors): Q R = A and Q orthonormal still hold."""
    print(f"qr deficient m={m} n={n}", flush=True)
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n))
    A[:, 3] = 0.0
    A[:, 7] = A[:, 1]
    A[:, n - 1] = 2.0 * A[:, 0]
    c = min(m, n)
    dA, dQ, dR = dev(A), torch.zeros((m, c), dtype=torch.float64, device="cuda"), torch.zeros((c, n), dtype=torch.float64, device="cuda")
    ctx.qr(m, n, dA, dQ, dR, stream=torch.cuda.current_stream())
    Q, R = host(dQ), host(dR)
    assert np.linalg.norm(Q @ R - A) <= 1e-13 * np.linalg.norm(A) * np.sqrt(n)
    assert np.abs(Q.T @ Q - np.eye(c)).max() <= 1e-13 * m
    assert np.all(np.tril(R, -1) == 0)


SVD_CASES = [(1, 1, "rand"), (16, 8, "rand"), (256, 32, "rand"), (512, 68, "rand"), (40, 40, "graded"),
             (128, 64, "lowrank"), (1024, 132, "rand"), (7, 30, "rand"), (64, 64, "zero"), (100, 63, "rand"),
             (70, 17, "graded"), (300, 100, "graded"), (200, 140, "rand"), (400, 120, "lowrank"),
             (137, 137, "graded")]


@pytest.mark.parametrize("m,n,kind", SVD_CASES)
def test_svd_matches_lapack(ctx, m, n, kind):
    print(f"svd m={m} n={n} {kind}", flush=True)
    rng = np.random.default_rng(7 + m + n)
    if kind == "rand":
        A = rng.standard_normal((m, n))
    elif kind == "graded":
        c = min(m, n)
        U, _ = np.linalg.qr(rng.standard_normal((m, c)))
        V, _ = np.linalg.qr(rng.standard_normal((n, c)))
        A = (U * np.logspace(0, -12, c)) @ V.T
    elif kind == "lowrank":
        A = rng.standard_normal((m, 5)) @ rng.standard_normal((5, n))
    else:
        A = np.zeros((m, n))
    c = min(m, n)
    dU = torch.zeros((m, c), dtype=torch.float64, device="cuda")
    dS = torch.zeros(c, dtype=torch.float64, device="cuda")
    dV = torch.zeros((c, n), dtype=torch.float64, device="cuda")
    ctx.svd(m, n, dev(A), dU, dS, dV, stream=torch.cuda.current_stream())
    U, S, Vt = host(dU), host(dS), host(dV)
    Sl = np.linalg.svd(A, compute_uv=False)
    scale = max(Sl[0], 1e-300)
    assert np.all(np.diff(S) <= 1e-14 * scale)  # descending
    assert np.abs(S - Sl).max() <= 1e-13 * scale * max(1, np.sqrt(n))
    # singular vectors of numerically nonzero singular values are orthonormal on both sides
    # (the factor from the Jacobi rotations is orthogonal throughout; vectors of zero
    # singular values carry no weight in U S V^T)
    keep = S > 1e-10 * scale
    if kind != "zero":
        assert np.linalg.norm((U * S) @ Vt - A) <= 1e-13 * np.linalg.norm(A) * max(1, np.sqrt(n))
    if keep.any():
        assert np.abs(U[:, keep].T @ U[:, keep] - np.eye(keep.sum())).max() <= 1e-11
        assert np.abs(Vt[keep] @ Vt[keep].T - np.eye(keep.sum())).max() <= 1e-11
    if m >= n:
        assert np.abs(U.T @ U - np.eye(c)).max() <= 1e-11


def _core(Ac, k, rev):
    K = len(Ac)
    return Ac[K - 1 - k].transpose(3, 1, 2, 0) if rev else Ac[k]


PROBS = {"2d": workloads.small_2d(), "3d": workloads.cube_body_force(4)}


@pytest.fixture(scope="module")
def problems(ctx):
    out = {}
    for name, prob in PROBS.items():
        out[name] = (tnfem.Problem(ctx, prob), tnfem.export_operator(prob))
    yield out
    for P, _ in out.values():
        P.close()


APPLY_CASES = [(name, k, rev, ranks) for name, K in (("2d", 6), ("3d", 5)) for k in range(K) for rev in (0, 1)
               for ranks in ((4, 4, 4, 4), (5, 7, 33, 17))]


@pytest.mark.parametrize("name,k,rev,ranks", APPLY_CASES)
def test_local_apply_and_interface_update_match_oracle(problems, name, k, rev, ranks):
    print(f"apply {name} k={k} rev={rev} ranks={ranks}", flush=True)
    P, Ac = problems[name]
    A = _core(Ac, k, rev)
    Rl, n, _, Rr = A.shape
    p, q, s, t = ranks
    rng = np.random.default_rng(hash((name, k, rev, ranks)) % 2 ** 32)
    L = rng.standard_normal((p, Rl, q))
    x = rng.standard_normal((q, n, s))
    Rt = rng.standard_normal((t, Rr, s))
    y = torch.zeros((p, n, t), dtype=torch.float64, device="cuda")
    P.local_apply(k, rev, p, q, s, t, dev(L), dev(x), dev(Rt), y, stream=torch.cuda.current_stream())
    ref = oamen.local_apply(L, A, x, Rt)
    got = host(y)
    # element by element against the FP64 rounding bound of the contraction chain:
    # |err| <= (depth + 6) u sum |L||A||x||R|, depth = every summed index's extent
    U64 = 2.0 ** -53
    yabs = oamen.local_apply(np.abs(L), np.abs(A), np.abs(x), np.abs(Rt))
    depth = q + Rl * n + s + Rr
    assert np.all(np.abs(got - ref) <= (depth + 6) * U64 * yabs + 1e-300)
    W = rng.standard_normal((p, n, t))
    Ln = torch.zeros((t, Rr, s), dtype=torch.float64, device="cuda")
    P.env_update(k, rev, p, q, s, t, dev(W), dev(L), dev(x), Ln, stream=torch.cuda.current_stream())
    ref2 = oamen.env_A(L, W, A, x)
    eabs = oamen.env_A(np.abs(L), np.abs(W), np.abs(A), np.abs(x))
    depth2 = p + n + Rl * n + q
    assert np.all(np.abs(host(Ln) - ref2) <= (depth2 + 6) * U64 * eabs + 1e-300)
