"""GPU AMEn solves against the oracle sweep and the sparse direct solve."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import amen as oamen, fem, qtt, tt  # noqa: E402
from paper_2501_12151_amd import tnfem, workloads  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = tnfem.Context(0)
    yield c
    c.close()


def _nodal_tt(D, d, rank, seed):
    """Seeded TT of nodal force values f0 (levels, then component)."""
    rng = np.random.default_rng(seed)
    modes = [2 ** D] * d + [D]
    ranks = [1] + [rank] * d + [1]
    return [rng.standard_normal((ranks[k], modes[k], ranks[k + 1])) for k in range(d + 1)]


SMALL = [
    dict(dim=2, level=3, E=1.0, nu=0.3, clamp=[(0, 0)], tractions=[(0, 1, [1.0, 0.0])]),
    dict(dim=2, level=4, E=3.0, nu=0.2, clamp=[(0, 0)], body_force=[0.0, -1.0]),
    dict(dim=3, level=2, E=1.0, nu=0.3, clamp=[(0, 0)], body_force=[0.0, 0.0, -1.0]),
    dict(dim=3, level=3, E=1.0, nu=0.45, clamp=[(2, 0)], tractions=[(2, 1, [0.0, 0.0, -1.0])]),
    dict(dim=3, level=3, E=1.0, nu=0.3, clamp=[(a, s) for a in range(3) for s in (0, 1)], manufactured_c=[0.3, -1.0, 0.5]),
    # anisotropic materials (constant Voigt stiffness; one also in slabs)
    dict(dim=2, level=4, E=1.0, nu=0.3, clamp=[(0, 0)], tractions=[(0, 1, [1.0, 0.3])],
         stiffness_voigt=workloads.random_anisotropic_voigt(2, 1)),
    dict(dim=3, level=3, E=2.0, nu=0.3, clamp=[(2, 0)], tractions=[(2, 1, [0.0, 0.0, -1.0])],
         layered_E=(2, [2.0, 2.0, 20.0, 20.0, 2.0, 2.0, 20.0]), stiffness_voigt=workloads.orthotropic_voigt(3, 1.0, 3.0, 0.5)),
    # quadrilateral domain (Alg. 1 in full: a trapezoid, slanted side loaded)
    dict(dim=2, level=4, E=1.0, nu=0.3, quad=[[0.0, 0.0], [2.0, 0.0], [0.0, 1.0], [1.4, 0.7]], clamp=[(0, 0)],
         tractions=[(0, 1, [0.3, -1.0])], body_force=[0.0, -0.5]),
    # heterogeneous material: a stiff disk inclusion as a per-element field
    dict(dim=2, level=4, E=1.0, nu=0.3, clamp=[(1, 0)], body_force=[0.0, -1.0],
         elem_weight=np.where(np.add.outer(((np.arange(15) + 0.5) / 15 - 0.55) ** 2,
                                           ((np.arange(15) + 0.5) / 15 - 0.45) ** 2) < 0.09, 10.0, 1.0)),
    # nodal load f0 given as a TT (Alg. 2 input)
    dict(dim=3, level=3, E=1.0, nu=0.3, clamp=[(0, 0)], f_nodal_tt=_nodal_tt(3, 3, 2, seed=5)),
    dict(dim=2, level=4, E=1.0, nu=0.3, clamp=[(1, 0)], f_nodal_tt=_nodal_tt(2, 4, 3, seed=6)),
]


@pytest.mark.parametrize("case", range(len(SMALL)))
def test_unconstrained_solve_equals_direct_and_oracle(ctx, case):
    prob = SMALL[case]
    print(f"solve small case {case}: {dict((k, v) for k, v in prob.items() if k not in ('f_nodal_tt', 'elem_weight'))}",
          flush=True)
    A, b, grid, _ = fem.build_system(prob)
    u = qtt.to_qtt_order(fem.direct_solve(A, b), prob["dim"], prob["level"])
    P = tnfem.Problem(ctx, prob)
    opts = dict(rank_cap=200, tol=1e-10, max_sweeps=30)
    U, st, rc = P.solve(**opts)
    assert rc == tnfem.OK, st
    ug = tt.tt_full(U.cores)
    assert np.linalg.norm(ug - u) <= 1e-8 * np.linalg.norm(u)
    X, ost = oamen.amen_solve(qtt.assemble_operator(prob), qtt.assemble_load(prob),
                              oamen.Options(tol=1e-10, rank_cap=200, max_sweeps=30))
    assert np.linalg.norm(ug - tt.tt_full(X)) <= 1e-8 * np.linalg.norm(u)
    assert st["sweeps"] == ost.sweeps


def test_small_2d_capped_matches_oracle(ctx):
    """The 32 x 32 workload with rank cap 16: GPU sweep and oracle sweep agree."""
    prob = workloads.small_2d()
    P = tnfem.Problem(ctx, prob)
    U, st, rc = P.solve(rank_cap=16, tol=1e-8, max_sweeps=20)
    X, ost = oamen.amen_solve(qtt.assemble_operator(prob), qtt.assemble_load(prob),
                              oamen.Options(tol=1e-8, rank_cap=16, max_sweeps=20))
    ug, uo = tt.tt_full(U.cores), tt.tt_full(X)
    rel = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    print(f"capped 2D: gpu sweeps={st['sweeps']} cg={st['cg_iters']} oracle cg={ost.cg_iters} rel.diff={rel:.2e}")
    assert rel <= 1e-6
    assert st["max_rank"] <= 16


def test_solve_is_deterministic(ctx):
    prob = SMALL[3]
    P = tnfem.Problem(ctx, prob)
    a = P.solve(rank_cap=32, tol=1e-9)[0].cores
    b = P.solve(rank_cap=32, tol=1e-9)[0].cores
    for x, y in zip(a, b):
        assert np.array_equal(x, y)



@pytest.mark.parametrize("prob", [
    dict(workloads.layered_cube(3), clamp=[(2, 0), (0, 0)]),
    dict(dim=2, level=5, E=1.0, nu=0.3, clamp=[(1, 0)], tractions=[(1, 1, [0.0, -1.0])],
         layered_E=(1, np.where((np.arange(31) >> 2) & 1, 10.0, 1.0).tolist())),
])
def test_layered_material_solve_equals_direct(prob):
    """Slab-wise Young's modulus: the GPU sweep with an unbinding rank cap reaches the direct solve."""
    A, b, grid, _ = fem.build_system(prob)
    u = qtt.to_qtt_order(fem.direct_solve(A, b), prob["dim"], prob["level"])
    ctx = tnfem.Context(0)
    P = tnfem.Problem(ctx, prob)
    U, st, rc = P.solve(rank_cap=200, tol=1e-10, max_sweeps=40)
    rel = np.linalg.norm(tt.tt_full(U.cores).reshape(-1) - u) / np.linalg.norm(u)
    print(f"layered {prob['dim']}D level {prob['level']}: rel.err vs direct {rel:.2e}, sweeps {st['sweeps']}", flush=True)
    assert rel <= 1e-8
    P.close()
    ctx.close()


def test_anisotropic_material_reproduces_linear_field_at_level_6(ctx):
    """Patch test at 3 x 2^18 dofs: a fully anisotropic material clamped at x = 0 and loaded by
    the face tractions sigma . n of the constant stress of u_i = g_i x is solved exactly by
    that linear field (Q1 reproduces it); checked at 4096 random nodes."""
    D, d = 3, 6
    Cv = np.asarray(workloads.random_anisotropic_voigt(3, 7))
    grad = np.array([0.7, -0.4, 0.25])
    C = fem.voigt_to_tensor(Cv, D)
    Gm = np.zeros((D, D))
    Gm[:, 0] = grad
    sig = np.einsum("ijkl,kl->ij", C, 0.5 * (Gm + Gm.T))
    tr = [(0, 1, list(sig[:, 0]))] + [(a, s, list((1 if s else -1) * sig[:, a])) for a in (1, 2) for s in (0, 1)]
    prob = dict(dim=D, level=d, E=1.0, nu=0.3, clamp=[(0, 0)], tractions=tr, stiffness_voigt=Cv.tolist())
    P = tnfem.Problem(ctx, prob)
    U, st, rc = P.solve(rank_cap=32, tol=1e-10, max_sweeps=30)
    rng = np.random.default_rng(3)
    nodes = rng.integers(0, 2 ** d, size=(4096, D))
    comp = rng.integers(0, D, size=4096)
    idx = np.zeros((4096, d + 1), dtype=np.int64)
    for l in range(d):
        idx[:, l] = sum(((nodes[:, a] >> (d - 1 - l)) & 1) << (D - 1 - a) for a in range(D))
    idx[:, d] = comp
    x = nodes[:, 0] / (2 ** d - 1)
    exact = grad[comp] * x
    got = U.eval(idx)
    err = np.abs(got - exact).max() / np.abs(exact).max()
    print(f"anisotropic linear field, level {d}: max rel error {err:.2e}, max rank {st['max_rank']}, "
          f"sweeps {st['sweeps']}", flush=True)
    assert err <= 1e-8
    P.close()


def test_torch_allocator_hooks_hold_the_device_memory():
    """With allocator hooks bound to torch's caching allocator every device byte of the
    problem and its solve comes from torch (and returns to it), and the result equals the
    solve on the library's own allocations bit for bit."""
    import torch

    prob = SMALL[3]
    ctx0 = tnfem.Context(0)
    P0 = tnfem.Problem(ctx0, prob)
    ref = P0.solve(rank_cap=32, tol=1e-9)[0].cores
    P0.close()
    ctx0.close()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    ctx = tnfem.Context(0, stream=torch.cuda.current_stream(), allocator="torch")
    P = tnfem.Problem(ctx, prob)
    U, st, rc = P.solve(rank_cap=32, tol=1e-9)
    held = torch.cuda.memory_allocated() - base
    print(f"torch allocator holds {held} bytes for the problem and its workspace", flush=True)
    assert held > 1 << 20
    for x, y in zip(U.cores, ref):
        assert np.array_equal(x, y)
    P.close()
    ctx.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base


def test_interpreter_exit_with_open_device_objects():
    """A process that leaves a context (with torch's allocator), a problem and a solution open
    exits cleanly: the binding closes them in an exit handler, problems before their context,
    while torch and the HIP runtime are still up."""
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import torch\n"
            "from paper_2501_12151_amd import tnfem\n"
            "ctx = tnfem.Context(0, stream=torch.cuda.current_stream(), allocator='torch')\n"
            "ctx2 = tnfem.Context(0)\n"
            "P = tnfem.Problem(ctx, dict(dim=3, level=3, E=1.0, nu=0.3, clamp=[(0, 0)], body_force=[0, 0, -1.0]))\n"
            "Q = tnfem.Problem(ctx2, dict(dim=2, level=4, E=1.0, nu=0.3, clamp=[(0, 0)], body_force=[0, -1.0]))\n"
            "u = P.solve(rank_cap=16, max_sweeps=4)[0]\n"
            "v = Q.solve(rank_cap=16, max_sweeps=4)[0]\n"
            "print('left open', flush=True)\n") % root
    r = subprocess.run([sys.executable, "-u", "-c", code], capture_output=True, text=True, timeout=300)
    print(r.stdout[-400:], r.stderr[-400:], flush=True)
    assert r.returncode == 0 and "left open" in r.stdout
