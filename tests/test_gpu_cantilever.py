"""The experiment of Sec. 6 on the GPU: the aluminium cantilever (20 m x 1 m, plane stress,
E = 68 GPa, nu = 0.33, clamped at x = 0, self-weight).

* Level 8 (131k dofs): the TT solve equals the sparse direct solve of the oracle to 1e-5, and
  so do its tip deflection and strain energy (b.u / 2 in TT format).
* Levels 10 and 12 (2.1M and 33.6M dofs, beyond a direct solve): the tip deflection is within
  0.5% of the Euler-Bernoulli value 3 rho g L_x^4 / (2 E L_y^2) of Sec. 6 (shear deformation
  adds about 0.2% at this slenderness; the direct solves at levels 5..9 approach it from below),
  and the two energies agree to 2e-3.  Without a preconditioner for the local systems the
  sweep stagnates at these levels (the local solves stop at their iteration limit): between
  40 and 80 half-sweeps the level-12 energy moves by a few 1e-4 either way, more than the
  discretisation changes it between levels 10 and 12, so its sign is not tested.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import fem, qtt, tt  # noqa: E402
from paper_2501_12151_amd import tnfem, workloads  # noqa: E402

OPTS = dict(rank_cap=64, tol=1e-10, max_sweeps=40, rho=8)


def _euler_bernoulli(prob):
    Lx, Ly = prob["extent"]
    return 3 * workloads.CANTILEVER_RHO * workloads.CANTILEVER_G * Lx ** 4 / (2 * prob["E"] * Ly ** 2)


def _tip(u, level):
    n = 2 ** level
    iy = np.arange(n, dtype=np.int64) if level <= 8 else np.unique(np.linspace(0, n - 1, 257).astype(np.int64))
    idx = np.zeros((iy.size, level + 1), dtype=np.int64)
    for l in range(level):
        idx[:, l] = (((n - 1) >> (level - 1 - l)) & 1) * 2 + ((iy >> (level - 1 - l)) & 1)
    idx[:, level] = 1
    return float(np.abs(u.eval(idx)).max())


@pytest.fixture(scope="module")
def ctx():
    c = tnfem.Context(0)
    yield c
    c.close()


def test_cantilever_level8_equals_direct_solve(ctx):
    prob = workloads.cantilever(8)
    A, b, grid, info = fem.build_system(prob)
    u = fem.direct_solve(A, b)
    uq = qtt.to_qtt_order(u, 2, 8)
    P = tnfem.Problem(ctx, prob)
    U, st, rc = P.solve(**OPTS)
    ug = tt.tt_full(U.cores).reshape(-1)
    rel = np.linalg.norm(ug - uq) / np.linalg.norm(uq)
    tip_direct = np.abs(u[grid.n_nodes:].reshape(grid.n, grid.n)[-1]).max()
    tip = _tip(U, 8)
    B = tnfem.TT.from_cores(tnfem.export_load(prob))
    energy = 0.5 * B.dot(U)
    print(f"level 8: rel.diff vs direct {rel:.2e}, tip {tip:.6e} / direct {tip_direct:.6e}, energy {energy:.6e} / "
          f"{0.5 * b @ u:.6e}, max rank {st['max_rank']}", flush=True)
    # on this slender, ill-conditioned problem the sweep settles 1e-7 to 1e-5 from the
    # direct solve depending on rounding in the truncations (3e-7 and 6.5e-6 measured with
    # two SVD orderings); more half-sweeps do not close the gap
    assert rel <= 1e-5
    assert tip == pytest.approx(tip_direct, rel=1e-5)
    assert energy == pytest.approx(0.5 * b @ u, rel=1e-5)
    assert abs(tip / _euler_bernoulli(prob) - 1) <= 5e-3
    P.close()


def test_cantilever_fine_levels_meet_euler_bernoulli(ctx):
    energies = []
    for d in (10, 12):
        prob = workloads.cantilever(d)
        P = tnfem.Problem(ctx, prob)
        U, st, rc = P.solve(**OPTS)
        tip = _tip(U, d)
        B = tnfem.TT.from_cores(tnfem.export_load(prob))
        energies.append(0.5 * B.dot(U))
        ratio = tip / _euler_bernoulli(prob)
        print(f"level {d}: {2 * 4 ** d} dofs, tip / Euler-Bernoulli {ratio:.5f}, energy {energies[-1]:.6e}, "
              f"{st['seconds']:.2f} s, max rank {st['max_rank']}", flush=True)
        assert abs(ratio - 1) <= 5e-3
        P.close()
    assert abs(energies[1] / energies[0] - 1) <= 2e-3
