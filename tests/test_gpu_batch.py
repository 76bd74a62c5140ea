"""Shared launches across requests: a lockstep batch gives every problem its alone result, bit for bit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import amen as oamen, fem, qtt, tt  # noqa: E402
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
    # low-precision local applies with the per-request FP64 refinement (restarts, fallbacks)
    ("3d", 4, dict(rank_cap=24, tol=1e-8, max_sweeps=10, precision=1)),
    ("3d", 5, dict(rank_cap=40, tol=1e-6, max_sweeps=8, precision=1)),
    ("2d", 6, dict(rank_cap=32, tol=1e-9, max_sweeps=20, precision=2)),
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
        assert sb["refinements"] == sa["refinements"] and sb["precision_fallbacks"] == sa["precision_fallbacks"]
        assert _same(ub, ua), f"problem {i} differs from its alone solve"
    # a second batch on the same problems reproduces the first
    again = tnfem.solve_batch(probs, **opts)
    for (ub, _, _), (uc, _, _) in zip(batch, again):
        assert _same(ub, uc)
    for p in probs:
        p.close()
    ctx.close()


def test_batch_rejects_mixed_levels_and_outer_refinement():
    ctx = tnfem.Context(0)
    a = tnfem.Problem(ctx, _problems_3d(3)[0])
    b = tnfem.Problem(ctx, _problems_3d(4)[0])
    with pytest.raises(tnfem.TnfemError, match="same dimension and level"):
        tnfem.solve_batch([a, b], rank_cap=8, max_sweeps=2)
    with pytest.raises(tnfem.TnfemError, match="outer refinement"):
        tnfem.solve_batch([a], rank_cap=8, max_sweeps=2, precision=1, ir_max=1)
    a.close()
    b.close()
    ctx.close()


ORACLE_OPTS = dict(rank_cap=64, tol=1e-10, max_sweeps=30)


def _oracle_and_direct(prob, opts):
    A, b, _, _ = fem.build_system(prob)
    u = qtt.to_qtt_order(fem.direct_solve(A, b), prob["dim"], prob["level"])
    X, ost = oamen.amen_solve(qtt.assemble_operator(prob), qtt.assemble_load(prob),
                              oamen.Options(tol=opts["tol"], rank_cap=opts["rank_cap"], max_sweeps=opts["max_sweeps"]))
    return u, tt.tt_full(X).reshape(-1), ost


@pytest.mark.parametrize("which,level,precision", [("3d", 3, 0), ("2d", 5, 0), ("3d", 3, 1), ("2d", 5, 2)])
def test_batch_matches_oracle_and_direct_solve(which, level, precision):
    """Every problem of a lockstep batch reaches the oracle sweep's and the direct solve's
    solution (unbinding cap, tight tolerance), with the oracle's half-sweep count; with
    FP32 / BF16 local applies the FP64 refinement of every local solve gives the same."""
    descs = _problems_3d(level) if which == "3d" else _problems_2d(level)
    ctx = tnfem.Context(0)
    probs = [tnfem.Problem(ctx, d) for d in descs]
    batch = tnfem.solve_batch(probs, precision=precision, **ORACLE_OPTS)
    for i, (d, (ub, sb, rb)) in enumerate(zip(descs, batch)):
        u, uo, ost = _oracle_and_direct(d, ORACLE_OPTS)
        ug = tt.tt_full(ub.cores).reshape(-1)
        e_d = np.linalg.norm(ug - u) / np.linalg.norm(u)
        e_o = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
        print(f"  problem {i}: sweeps {sb['sweeps']} / oracle {ost.sweeps}, vs direct {e_d:.2e}, vs oracle {e_o:.2e}",
              flush=True)
        assert rb == tnfem.OK
        # FP64 takes the oracle's half-sweep count; refined low-precision local solves
        # meet the same local tolerance from slightly different residuals, so the stop
        # rule may fire one half-sweep apart
        assert sb["sweeps"] == ost.sweeps if precision == 0 else abs(sb["sweeps"] - ost.sweeps) <= 1
        assert e_d <= 1e-8 and e_o <= 1e-8
    for p in probs:
        p.close()
    ctx.close()
