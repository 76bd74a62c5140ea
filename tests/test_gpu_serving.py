"""Serving: results alone equal results in a mix; admission by HBM budget."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import amen as oamen, fem, qtt, tt  # noqa: E402
from paper_2501_12151_amd import tnfem, workloads  # noqa: E402

MIX = [
    (workloads.small_2d(), dict(rank_cap=16, tol=1e-8, max_sweeps=12)),
    (dict(dim=3, level=4, E=2.0, nu=0.25, clamp=[(0, 0)], tractions=[(0, 1, [0.3, -1.0, 0.5])]),
     dict(rank_cap=32, tol=1e-6, max_sweeps=8)),
    (dict(dim=2, level=6, E=0.5, nu=0.4, clamp=[(0, 0)], tractions=[(0, 1, [1.0, 0.2])]),
     dict(rank_cap=32, tol=1e-6, max_sweeps=10)),
    (workloads.cube_body_force(5), dict(rank_cap=32, tol=1e-6, max_sweeps=6)),
]


def _cores(res):
    return [c.copy() for c in res[0].cores]


def test_alone_equals_in_mix():
    alone = []
    srv = tnfem.Server(0, slots=1)
    for prob, opt in MIX:
        print(f"alone: {prob}", flush=True)
        alone.append(_cores(srv.poll(srv.submit(prob, **opt))))
    srv.close()
    srv = tnfem.Server(0, slots=4)
    tickets = []
    for rep in range(3):
        for j, (prob, opt) in enumerate(MIX):
            tickets.append((j, srv.submit(prob, **opt)))
    info_seen = srv.info()
    results = [(j, srv.poll(t)) for j, t in tickets]
    info = srv.info()
    srv.close()
    print("server info", info_seen, info, flush=True)
    assert info["completed"] == len(tickets)
    assert info["peak_running"] >= 2  # requests overlapped on the device
    for j, res in results:
        got = _cores(res)
        assert len(got) == len(alone[j])
        for a, b in zip(got, alone[j]):
            assert np.array_equal(a, b)  # bitwise: no cross-request interaction
        assert res[3] > 0  # latency measured


def test_budget_rejects_and_serialises():
    srv = tnfem.Server(0, slots=2, hbm_budget_bytes=1 << 20)
    t = srv.submit(MIX[0][0], **MIX[0][1])
    with pytest.raises(tnfem.TnfemError) as e:
        srv.poll(t)
    assert e.value.code == tnfem.EBUDGET
    srv.close()
    # measure one request's device footprint, then allow 1.5 of them: one at a time
    srv = tnfem.Server(0, slots=1)
    srv.poll(srv.submit(MIX[0][0], **MIX[0][1]))
    one = srv.info()["peak_bytes"]
    srv.close()
    budget = int(1.5 * one)
    srv = tnfem.Server(0, slots=4, hbm_budget_bytes=budget)
    ts = [srv.submit(MIX[0][0], **MIX[0][1]) for _ in range(4)]
    outs = [srv.poll(t) for t in ts]
    info = srv.info()
    srv.close()
    print("small budget info", info, flush=True)
    assert info["peak_bytes"] <= budget
    assert info["peak_running"] == 1
    assert info["completed"] == 4
    ref = _cores(outs[0])
    assert len(ref) == MIX[0][0]["level"] + 1
    for o in outs:
        got = _cores(o)
        assert len(got) == len(ref) > 0  # every request came back with its whole TT
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)


def _bucket_requests():
    rng = np.random.default_rng(3)
    out = []
    for _ in range(6):
        out.append(dict(dim=3, level=5, E=float(10 ** rng.uniform(-1, 1)), nu=float(rng.uniform(0.2, 0.45)),
                        clamp=[(0, 0)], tractions=[(0, 1, [float(v) for v in rng.standard_normal(3)])]))
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_server_batches_one_bucket_and_results_equal_alone(precision):
    """A queued bucket runs as one lockstep batch and every result equals the request
    alone, in FP64 and with FP32 local applies (FP64-refined local solves)."""
    opts = dict(rank_cap=32, tol=1e-6, max_sweeps=6, precision=precision)
    reqs = _bucket_requests()
    ctx = tnfem.Context(0)
    alone = []
    for d in reqs:
        P = tnfem.Problem(ctx, d)
        alone.append([c.copy() for c in P.solve(**opts)[0].cores])
        P.close()
    ctx.close()
    blocker = (workloads.cube_body_force(6), dict(rank_cap=32, tol=1e-6, max_sweeps=6))
    for max_batch, expect in [(8, 6), (1, 1)]:
        srv = tnfem.Server(0, slots=1)
        srv.set_max_batch(max_batch)
        tb = srv.submit(blocker[0], **blocker[1])  # keeps the one slot busy while the bucket queues
        ts = [srv.submit(d, **opts) for d in reqs]
        outs = [srv.poll(t) for t in ts]
        srv.poll(tb)
        info = srv.info()
        srv.close()
        print(f"max_batch {max_batch}: {info}", flush=True)
        assert info["peak_batch"] == expect
        assert info["batched_requests"] == (6 if expect > 1 else 0)
        for o, a in zip(outs, alone):
            got = [c.copy() for c in o[0].cores]
            assert len(got) == len(a)
            for x, y in zip(got, a):
                assert np.array_equal(x, y)
            assert o[3] > 0


def test_served_results_match_oracle_and_direct_solve():
    """Requests of different dimensions, levels and materials served together (overlapping
    slots, lockstep batches of a bucket) reach the oracle sweep's and the direct solve's
    solution (unbinding cap, tight tolerance)."""
    opts = dict(rank_cap=64, tol=1e-10, max_sweeps=30)
    reqs = [
        dict(dim=2, level=5, E=1.0, nu=0.3, clamp=[(0, 0)], tractions=[(0, 1, [1.0, 0.0])]),
        dict(dim=2, level=5, E=4.0, nu=0.2, clamp=[(0, 0)], tractions=[(0, 1, [-0.3, 0.8])]),
        dict(dim=3, level=3, E=2.0, nu=0.25, clamp=[(0, 0)], tractions=[(0, 1, [0.3, -1.0, 0.5])]),
        dict(dim=3, level=3, E=0.5, nu=0.4, clamp=[(0, 0)], body_force=[0.0, 0.0, -1.0]),
        dict(dim=2, level=4, E=1.0, nu=0.35, plane_stress=True, clamp=[(1, 0)], body_force=[0.0, -1.0]),
    ]
    srv = tnfem.Server(0, slots=3)
    tickets = [srv.submit(p, **opts) for p in reqs]
    results = [srv.poll(t) for t in tickets]
    info = srv.info()
    srv.close()
    assert info["completed"] == len(reqs)
    for i, (prob, res) in enumerate(zip(reqs, results)):
        A, b, _, _ = fem.build_system(prob)
        u = qtt.to_qtt_order(fem.direct_solve(A, b), prob["dim"], prob["level"])
        X, ost = oamen.amen_solve(qtt.assemble_operator(prob), qtt.assemble_load(prob),
                                  oamen.Options(tol=opts["tol"], rank_cap=opts["rank_cap"],
                                                max_sweeps=opts["max_sweeps"]))
        ug = tt.tt_full(res[0].cores).reshape(-1)
        uo = tt.tt_full(X).reshape(-1)
        e_d = np.linalg.norm(ug - u) / np.linalg.norm(u)
        e_o = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
        print(f"  request {i}: sweeps {res[1]['sweeps']} / oracle {ost.sweeps}, vs direct {e_d:.2e}, "
              f"vs oracle {e_o:.2e}", flush=True)
        assert res[2] == tnfem.OK and res[1]["sweeps"] == ost.sweeps
        assert e_d <= 1e-8 and e_o <= 1e-8
