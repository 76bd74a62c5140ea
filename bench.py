#!/usr/bin/env python3
"""Throughput of the QTT AMEn elasticity solve on one MI355X.

One step = one complete solve (initial orthogonalisation, half-sweeps of local
CG solves, SVD truncation, residual enrichment, QR, interface updates) of the
3D unit-cube workload: 128^3 nodes (QTT level 7, 6.3 M dofs), E = 1, nu = 0.3,
face x = 0 clamped, uniform body force (0, 0, -1), FP64, TT rank cap 32.  The
operator and load are assembled and resident on the device before timing.

Prints one JSON line (see the repository documentation for the fields).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "solves/s + p50/p99 latency at 1e-6 rel. error; contraction TFLOP/s vs peak"
PEAK_FP64_MFMA_TFLOPS = 78.6
# HBM bytes per launch of fused_apply32_kernel<0> on the cube128 workload: FETCH_SIZE and
# WRITE_SIZE per dispatch, each scaled by what the counter reads for a 256 MiB copy
# (profiles/fused_apply_cube128_f64_cap32.md).  Valid while that kernel is unchanged.
FUSED_APPLY_TRAFFIC_BYTES = 4264407.6

WORKLOADS = {
    # name: (problem factory args, solve options, description)
    "cube128": dict(level=7, opts=dict(rank_cap=32, tol=1e-6, max_sweeps=16),
                    desc="3D unit cube 128^3 nodes (QTT level 7), body force (0,0,-1), x=0 clamped, E=1, nu=0.3, "
                         "FP64, rank cap 32"),
    "square32": dict(level=5, opts=dict(rank_cap=16, tol=1e-8, max_sweeps=20),
                     desc="2D plane strain 32x32 nodes (QTT level 5), x-traction 1 on x=1, x=0 clamped, E=1, nu=0.3, "
                          "FP64, rank cap 16"),
}


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def problem_for(name):
    from paper_2501_12151_amd import workloads

    if name == "cube128":
        return workloads.cube_body_force(WORKLOADS[name]["level"])
    return workloads.small_2d()


def cpu_baseline(name, gpu_applies, budget_s=20.0):
    """The oracle sweep timed on the host, on a bounded sample of the same solve.

    The oracle runs the same solve (same options) until about budget_s seconds
    have passed (checked between half-sweeps); its time is scaled by the ratio of
    the GPU solve's local operator applications to the oracle's.  The sampled
    early half-sweeps run at lower ranks than the later ones, so the estimate
    favours the oracle.
    """
    from threadpoolctl import threadpool_info

    from oracle import amen, qtt

    prob = problem_for(name)
    o = WORKLOADS[name]["opts"]
    A = qtt.assemble_operator(prob)
    b = qtt.assemble_load(prob)
    opt = amen.Options(tol=o["tol"], rank_cap=o["rank_cap"], max_sweeps=o["max_sweeps"])
    t0 = time.perf_counter()
    _, st = amen.amen_solve(A, b, opt, after_half_sweep=lambda s: time.perf_counter() - t0 > budget_s)
    t1 = time.perf_counter()
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    per_solve = (t1 - t0) * max(gpu_applies, 1) / max(st.applies, 1)
    return {
        "value": 1.0 / per_solve,
        "unit": "solves/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"first {st.sweeps} of {o['max_sweeps']} half-sweeps of the same solve in {t1 - t0:.1f} s "
                  f"({st.applies} local operator applications); scaled by the GPU solve's {gpu_applies} applications",
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cube128", choices=sorted(WORKLOADS) + ["serving"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the high-rank reference solves")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 10 device-to-device copies of MIB MiB (to calibrate HBM byte counters)")
    ap.add_argument("--requests", type=int, default=256, help="serving: number of requests")
    ap.add_argument("--slots", type=int, default=8, help="serving: worker slots")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solve is not sharded across GPUs.",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        import torch

        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_copy": {"read": 8 * n, "write": 8 * n}, "copies": 10}))
        return

    from paper_2501_12151_amd import tnfem

    if args.workload == "serving":
        serving(args)
        return
    wl = WORKLOADS[args.workload]
    prob = problem_for(args.workload)
    opts = dict(wl["opts"])
    ctx = tnfem.Context(0)
    P = tnfem.Problem(ctx, prob)
    info = P.info()
    for i in range(args.warmup):
        _, st, rc = P.solve(**opts)
        print(f"warmup {i}: {st['seconds']:.3f} s sweeps={st['sweeps']} res={st['final_max_res']:.2e}",
              file=sys.stderr, flush=True)
    lat, stats = [], []
    t_begin = time.perf_counter()
    for i in range(args.steps):
        t0 = time.perf_counter()
        u, st, rc = P.solve(**opts)
        lat.append(time.perf_counter() - t0)
        stats.append(st)
        print(f"step {i}: {lat[-1]:.3f} s sweeps={st['sweeps']} cg={st['cg_iters']} res={st['final_max_res']:.2e}",
              file=sys.stderr, flush=True)
    total = time.perf_counter() - t_begin
    st = stats[-1]
    roof = None
    if not args.no_profile:
        roof = roofline(P, opts)
    accuracy = None
    if not args.no_accuracy:
        accuracy = accuracy_vs_reference(P, u, opts)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.workload, st["local_applies"])
    value = args.steps / total
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": wl["desc"],
            "dofs": prob["dim"] * 2 ** (prob["dim"] * prob["level"]),
            "mpo_ranks": info["mpo_ranks"],
            "rank_cap": opts["rank_cap"],
            "tol": opts["tol"],
            "max_sweeps": opts["max_sweeps"],
        },
        "latency_ms": {"p50": 1e3 * percentile(lat, 0.5), "p99": 1e3 * percentile(lat, 0.99)},
        "solve": {
            "sweeps": st["sweeps"], "converged": bool(st["converged"]), "final_max_local_residual": st["final_max_res"],
            "cg_iters": st["cg_iters"], "max_rank": st["max_rank"], "counted_flops": st["flops"],
            "median_latency_s": statistics.median(lat),
        },
        "accuracy": accuracy,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def roofline(P, opts):
    """Live roofline of the dominant contraction kernel, the fused local apply (row a2):
    one more solve with per-launch HIP events on the library stream around every
    contraction launch.  achieved = algorithmic flops of the launches that did work
    (sparse-operator term counts at the actual ranks) / summed event time of all its
    launches; the all-contraction rate (grouped GEMMs included) is reported beside it."""
    _, pst, _ = P.solve(profile=1, **opts)
    ms, fl, nl = pst["apply_kernel_ms"], pst["apply_kernel_flops"], pst["apply_kernel_launches"]
    achieved = fl / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    cms, cfl, cnl = pst["contraction_ms"], pst["contraction_flops"], pst["contraction_launches"]
    return {
        "bound": "mfma",
        "kernel": "fused_apply32_kernel<0> (fused local operator apply, FP64 MFMA, ranks <= 32)",
        "achieved": achieved,
        "peak": PEAK_FP64_MFMA_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP64_MFMA_TFLOPS,
        "traffic": FUSED_APPLY_TRAFFIC_BYTES if opts.get("precision", 0) == 0 else None,
        "traffic_unit": "bytes per launch (PMC, copy-calibrated)",
        "launches_per_solve": nl,
        "avg_launch_us": 1e3 * ms / max(nl, 1),
        "flops_per_launch": fl / max(nl, 1),
        "all_contractions": {
            "kernels": "fused_apply32_kernel<0> + gemm_grouped_kernel<*>",
            "launches_per_solve": cnl, "ms_per_solve": cms,
            "tflops": cfl / (cms * 1e-3) / 1e12 if cms > 0 else 0.0,
        },
    }


def accuracy_vs_reference(P, u, opts, ref_caps=(64, 96), ref_sweeps=30):
    """Relative displacement error of the timed solve against high-rank FP64 solves of the
    same problem, computed by the library in TT format (no densification).  The two
    references differ only in their rank cap; their mutual difference bounds how far the
    larger one is from converged."""
    refs = {}
    for cap in ref_caps:
        r, rst, _ = P.solve(rank_cap=cap, tol=1e-9, max_sweeps=ref_sweeps)
        refs[cap] = (r, rst)
        print(f"reference cap {cap}: {rst['seconds']:.2f} s, max local residual {rst['final_max_res']:.2e}",
              file=sys.stderr, flush=True)
    top = refs[ref_caps[-1]][0]
    err = u.rel_diff(top)
    ref_gap = refs[ref_caps[0]][0].rel_diff(top)
    return {
        "rel_error_vs_reference": err,
        "reference": f"same problem, FP64, rank cap {ref_caps[-1]}, tol 1e-9, {ref_sweeps} half-sweeps "
                     f"(max local residual {refs[ref_caps[-1]][1]['final_max_res']:.2e})",
        "reference_cap_gap": {"caps": list(ref_caps), "rel_diff": ref_gap},
        "target": 1e-6,
        "meets_target": bool(err <= 1e-6),
        "rank_cap_of_timed_solve": opts["rank_cap"],
    }


def serving(args):
    """Serving stream: Poisson arrivals of mixed 2D/3D requests; throughput and p50/p99 latency."""
    from paper_2501_12151_amd import tnfem, workloads

    def opts_for(cap):
        return dict(rank_cap=cap, tol=1e-6, max_sweeps=12)

    # closed loop: all requests at once -> saturation throughput
    sat_reqs = workloads.serving_stream(min(64, args.requests), seed=1, rate=1.0)
    srv = tnfem.Server(0, slots=args.slots)
    t0 = time.perf_counter()
    ts = [srv.submit(p, **opts_for(c)) for _, p, c in sat_reqs]
    for t in ts:
        srv.poll(t)
    sat = len(ts) / (time.perf_counter() - t0)
    srv.close()
    print(f"closed loop: {len(ts)} requests, {sat:.2f} solves/s", file=sys.stderr, flush=True)
    rate = 0.8 * sat
    reqs = workloads.serving_stream(args.requests, seed=0, rate=rate)
    srv = tnfem.Server(0, slots=args.slots)
    lat, tickets = [], []
    t0 = time.perf_counter()
    for arrival, p, c in reqs:
        now = time.perf_counter() - t0
        if arrival > now:
            time.sleep(arrival - now)
        tickets.append(srv.submit(p, **opts_for(c)))
    for t in tickets:
        _, st, rc, l = srv.poll(t)
        lat.append(l)
    elapsed = time.perf_counter() - t0
    info = srv.info()
    srv.close()
    out = {
        "metric": METRIC,
        "value": len(tickets) / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": len(tickets),
        "warmup": 0,
        "ms_per_step": 1e3 * elapsed / len(tickets),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"serving stream: {len(tickets)} requests, Poisson arrivals at 0.8 x closed-loop "
                               f"rate ({rate:.2f}/s), 2D/3D, levels 6..10, caps 32..64, {args.slots} slots",
                   "closed_loop_solves_per_s": sat},
        "latency_ms": {"p50": 1e3 * percentile(lat, 0.5), "p99": 1e3 * percentile(lat, 0.99)},
        "server": info,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
