"""Shared launches across requests: a lockstep batch gives every problem its alone result, bit for bit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2501_12151_amd import tnfem  # noqa: E402


def _problems_3d(level):
    return [
        dict(dim=3, level=level, E=1.0, nu=0.3, clamp=[(0, 0)], body_force=[0.0, 0.0, -1.0]),
        dict(dim=3, level=level, E=7.5, nu=0.22, clamp=[(0, 0)], tractions=[(0, 1, [0.3, -1.1, 0.4])]),
        dict(dim=3, level=level, E=0.4, nu=0.41, clamp=[(2, 0)], tractions=[(2, 1, [0.0, 0.0, -1.0])]),
        dict(dim=3, level=level, E=2.0, nu=0.3, clamp=[(a, s) for a in range(3) for s in (0, 1)],
             manufactured_c=[0.5, -1.2, 0.8]),
        dict(dim=3, level=level, E=1.3, nu=0.35, clamp=[(0, 0), (1, 1)], body_force=[1.0, 0.5, 0.0]),
    ]


def _problems_2d(level):
    return [
        dict(dim=2, level=level, E=1.0, nu=0.3, clamp=[(0, 0)], tractions=[(0, 1, [1.0, 0.0])]),
        dict(dim=2, level=level, E=3.0, nu=0.25, plane_stress=True, clamp=[(0, 0)], body_force=[0.0, -1.0]),
        dict(dim=2, level=level, E=0.7, nu=0.4, clamp=[(1, 0)], tractions=[(1, 1, [0.2, -0.6])]),
    ]


def _same(a, b):
    ca, cb = a.cores, b.cores
    return len(ca) == len(cb) and all(x.shape == y.shape and np.array_equal(x, y) for x, y in zip(ca, cb))


@pytest.mark.parametrize("which,level,opts", [
    ("3d", 4, dict(rank_cap=24, tol=1e-8, max_sweeps=10)),
    ("3d", 5, dict(rank_cap=32, tol=1e-6, max_sweeps=8)),
    ("2d", 6, dict(rank_cap=32, tol=1e-9, max_sweeps=20)),
    ("3d", 3, dict(rank_cap=64, tol=1e-8, max_sweeps=40)),  # converge at different half-sweeps
])
def test_batch_equals_alone_bitwise(which, level, opts):
    descs = _problems_3d(level) if which == "3d" else _problems_2d(level)
    print(f"batch {which} level {level} ({len(descs)} problems) {opts}", flush=True)
    ctx = tnfem.Context(0)
    probs = [tnfem.Problem(ctx, d) for d in descs]
    alone = [p.solve(**opts) for p in probs]
    batch = tnfem.solve_batch(probs, **opts)
    for i, ((ua, sa, ra), (ub, sb, rb)) in enumerate(zip(alone, batch)):
        print(f"  problem {i}: sweeps {sa['sweeps']}/{sb['sweeps']} cg {sa['cg_iters']}/{sb['cg_iters']} "
              f"res {sa['final_max_res']:.2e} status {ra}/{rb}", flush=True)
        assert rb == ra
        assert sb["sweeps"] == sa["sweeps"] and sb["cg_iters"] == sa["cg_iters"]
        assert sb["local_applies"] == sa["local_applies"]
        assert _same(ub, ua), f"problem {i} differs from its alone solve"
    # a second batch on the same problems reproduces the first
    again = tnfem.solve_batch(probs, **opts)
    for (ub, _, _), (uc, _, _) in zip(batch, again):
        assert _same(ub, uc)
    for p in probs:
        p.close()
    ctx.close()


def test_batch_rejects_mixed_levels_and_low_precision():
    ctx = tnfem.Context(0)
    a = tnfem.Problem(ctx, _problems_3d(3)[0])
    b = tnfem.Problem(ctx, _problems_3d(4)[0])
    with pytest.raises(tnfem.TnfemError, match="same dimension and level"):
        tnfem.solve_batch([a, b], rank_cap=8, max_sweeps=2)
    with pytest.raises(tnfem.TnfemError, match="FP64"):
        tnfem.solve_batch([a], rank_cap=8, max_sweeps=2, precision=1)
    a.close()
    b.close()
    ctx.close()
