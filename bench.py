#!/usr/bin/env python3
"""Throughput of the QTT AMEn elasticity solve on one MI355X.

One step = one complete solve (initial orthogonalisation, half-sweeps of local
CG solves, SVD truncation, residual enrichment, QR, interface updates).  The
default workload is the 3D unit cube with 1024^3 nodes (QTT level 10, 3.2e9
dofs), all faces clamped, load of the manufactured field u_i = c_i sin(pi x)
sin(pi y) sin(pi z) with c ~ N(0, 1) (seed 0), E = 1, nu = 0.3, TT rank cap 64,
solved in FP64 (FP64 MFMA); the mixed-precision solve (FP32 local applies on MFMA
refined in FP64) of the same problem is timed beside it.  The operator and load
are assembled and resident on the device before timing.  The oracle solves the
same problem on the host cores; its solution is the accuracy reference.

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
# Counter summaries of the fused local apply: HBM bytes per launch (FETCH_SIZE + WRITE_SIZE
# per dispatch, copy-calibrated, averaged over every fused-apply launch of one solve), keyed
# by (workload, precision).  Each file states the command that produced it and holds one line
# "traffic_bytes_per_launch: <bytes>"; a summary is valid while the kernels it covers are.
TRAFFIC_SUMMARIES = {
    ("cube1024", 1): "fused_apply_cube1024_f32_cap64.md",
    ("cube1024", 0): "fused_apply_cube1024_f64_cap64.md",
}

PEAKS = {0: 78.6, 1: 157.3, 2: 2500.0}  # dense MFMA TFLOP/s: FP64, FP32, BF16
DTYPES = {0: "f64", 1: "f32 (FP32 MFMA local applies, FP64 refinement)",
          2: "bf16 (BF16 MFMA local applies, FP32 accumulate, FP64 refinement)"}
DTYPE_TAGS = {0: "f64", 1: "f32/f64", 2: "bf16/f64"}

WORKLOADS = {
    # refs: solve options of the FP64 reference solves for the accuracy block (the last one is
    # the reference; the difference of the two bounds how far it is from converged)
    # the cap binds: 30 half-sweeps with enrichment rank 8 bring the solve within 1.1x of the
    # cap-32 error floor (6.0e-4 against 5.4e-4 after 40; 5.4e-3 after 16 with rank 4)
    "cube128": dict(level=7, opts=dict(rank_cap=32, tol=1e-8, max_sweeps=30, rho=8),
                    refs=[dict(rank_cap=64, tol=1e-9, max_sweeps=30), dict(rank_cap=96, tol=1e-9, max_sweeps=30)],
                    desc="3D unit cube 128^3 nodes (QTT level 7), body force (0,0,-1), x=0 clamped, E=1, nu=0.3, "
                         "rank cap 32"),
    # the oracle runs this whole solve on the host (about a minute) as the accuracy reference;
    # enrichment rank 8 grows the ranks twice as fast as 4, so 16 half-sweeps reach what 24 did
    # (2.7e-7 from the cap-96 reference in FP64, 14% less time)
    "cube1024": dict(level=10, opts=dict(rank_cap=64, tol=1e-6, max_sweeps=16, rho=8), oracle_full=True,
                     refs=[dict(rank_cap=64, tol=1e-8, max_sweeps=40), dict(rank_cap=96, tol=1e-9, max_sweeps=40)],
                     desc="3D unit cube 1024^3 nodes (QTT level 10), all faces clamped, load of the manufactured field "
                          "u_i = c_i sin(pi x) sin(pi y) sin(pi z), c ~ N(0,1) (seed 0), E=1, nu=0.3, rank cap 64"),
    # the discrete solution needs ranks above 128: at cap 128 the sweep settles about 3e-6
    # from the converged solution; enrichment rank 8 reaches the cap in 16 half-sweeps
    "layered512": dict(level=9, opts=dict(rank_cap=128, tol=1e-8, max_sweeps=30, rho=8),
                       refs=[dict(rank_cap=160, tol=1e-10, max_sweeps=40, rho=12),
                             dict(rank_cap=192, tol=1e-10, max_sweeps=40, rho=8)],
                       desc="3D unit cube 512^3 nodes (QTT level 9), 8 slabs along z alternating E=1 and E=10, "
                            "nu=0.3, base z=0 clamped, top pressure 1.0, rank cap 128"),
    "square32": dict(level=5, opts=dict(rank_cap=16, tol=1e-8, max_sweeps=20),
                     refs=[dict(rank_cap=64, tol=1e-10, max_sweeps=30)],
                     desc="2D plane strain 32x32 nodes (QTT level 5), x-traction 1 on x=1, x=0 clamped, E=1, nu=0.3, "
                          "rank cap 16"),
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
    if name == "cube1024":
        return workloads.cube_manufactured(WORKLOADS[name]["level"])
    if name == "layered512":
        return workloads.layered_cube(WORKLOADS[name]["level"])
    return workloads.small_2d()


def manufactured_field_cores(level, c):
    """QTT of the nodal field u_i = c_i sin(pi x) sin(pi y) sin(pi z), x = ix / (2^level - 1),
    levels most significant bit first, mode (bx 2 + by) 2 + bz, component core last: each axis
    carries the state [cos phi, sin phi] of its partial angle and a bit b of weight w rotates
    it by b w, so every level core is a Kronecker product of three 2 x 2 rotations (rank 8)."""
    import numpy as np

    h = 1.0 / (2 ** level - 1)
    cores = []
    for k in range(level):
        w = np.pi * h * 2 ** (level - 1 - k)
        rot = [np.array([[np.cos(b * w), np.sin(b * w)], [-np.sin(b * w), np.cos(b * w)]]) for b in (0, 1)]
        core = np.zeros((8, 8, 8))
        for m in range(8):
            bx, by, bz = (m >> 2) & 1, (m >> 1) & 1, m & 1
            core[:, m, :] = np.kron(np.kron(rot[bx], rot[by]), rot[bz])
        if k == 0:
            core = core[:1]  # start state (cos 0, sin 0) on every axis: row index 0
        cores.append(core)
    comp = np.zeros((8, 3, 1))
    comp[7, :, 0] = c  # sin component on all three axes
    cores.append(comp)
    return cores


def cpu_baseline(name, opts, gpu_applies, full, budget_s=20.0):
    """The oracle timed on the host cores; returns (baseline dict, oracle solution cores or None).

    full: the oracle runs the whole solve with the timed solve's options (FP64) and its
    solution becomes the accuracy reference.  Otherwise it runs until about budget_s
    seconds have passed (checked between half-sweeps) and its time is scaled by the ratio
    of the GPU solve's local operator applications to the oracle's; the sampled early
    half-sweeps run at lower ranks than the later ones, so that estimate favours the oracle.
    Assembly is not timed.
    """
    from threadpoolctl import threadpool_info

    from oracle import amen, qtt

    prob = problem_for(name)
    A = qtt.assemble_operator(prob)
    b = qtt.assemble_load(prob)
    opt = amen.Options(tol=opts["tol"], rank_cap=opts["rank_cap"], max_sweeps=opts["max_sweeps"],
                       rho=opts.get("rho", 4))
    stop = None if full else (lambda s: time.perf_counter() - t0 > budget_s)
    t0 = time.perf_counter()
    X, st = amen.amen_solve(A, b, opt, after_half_sweep=stop)
    t1 = time.perf_counter()
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    whole = full or st.sweeps >= opts["max_sweeps"]
    per_solve = (t1 - t0) if whole else (t1 - t0) * max(gpu_applies, 1) / max(st.applies, 1)
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    sample = (f"the whole solve ({st.sweeps} half-sweeps, {st.applies} local operator applications) in "
              f"{t1 - t0:.1f} s" if whole else
              f"first {st.sweeps} of {opts['max_sweeps']} half-sweeps of the same solve in {t1 - t0:.1f} s "
              f"({st.applies} local operator applications); scaled by the GPU solve's {gpu_applies} applications")
    out = {
        "value": 1.0 / per_solve,
        "unit": "solves/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": sample + "; FP64 numpy/LAPACK, assembly not timed",
        "cpu_model": cpu_model,
        "nproc": os.cpu_count(),
    }
    return out, (X if whole else None)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cube1024", choices=sorted(WORKLOADS) + ["serving", "cantilever"])
    ap.add_argument("--levels", default="6,8,10,12,14,16,18,20", help="cantilever: grid levels")
    ap.add_argument("--precision", type=int, default=0, choices=(0, 1, 2),
                    help="0 FP64; 1 FP32 local applies; 2 BF16 local applies (both refined in FP64)")
    ap.add_argument("--ir-max", type=int, default=0, help="outer FP64 refinement steps after the solve (0: none)")
    ap.add_argument("--ir-sweeps", type=int, default=4, help="half-sweeps of each correction solve")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle (and its accuracy reference)")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the GPU's high-rank reference solves")
    ap.add_argument("--no-side-solver", "--no-fp64-solver", dest="no_side_solver", action="store_true",
                    help="do not time the other precision beside (FP32 applies beside FP64, FP64 beside the rest)")
    ap.add_argument("--mfma-calibration", type=int, default=0, metavar="N",
                    help="only run 10 FP64 and 10 FP32 N x N matrix products (to calibrate MFMA counters)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 10 device-to-device copies of MIB MiB (to calibrate HBM byte counters)")
    ap.add_argument("--requests", type=int, default=256, help="serving: number of requests")
    ap.add_argument("--slots", type=int, default=8, help="serving: worker slots")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solve is not sharded across GPUs.",
              file=sys.stderr)
        sys.exit(2)

    if args.mfma_calibration:
        import torch

        n = args.mfma_calibration
        for dt in (torch.float64, torch.float32):
            a = torch.ones((n, n), dtype=dt, device="cuda")
            b = torch.ones((n, n), dtype=dt, device="cuda")
            for _ in range(10):
                c = a @ b
            torch.cuda.synchronize()
            del c
        print(json.dumps({"mfma_calibration_flops_per_matmul": 2 * n ** 3, "matmuls_per_dtype": 10,
                          "dtypes": ["f64", "f32"]}))
        return

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
    if args.workload == "cantilever":
        cantilever(args)
        return
    wl = WORKLOADS[args.workload]
    prob = problem_for(args.workload)
    opts = dict(wl["opts"], precision=args.precision)
    if args.ir_max > 0:
        opts.update(ir_max=args.ir_max, ir_sweeps=args.ir_sweeps, ir_tol=0.1 * opts["tol"])
    ctx = tnfem.Context(0)
    P = tnfem.Problem(ctx, prob)
    info = P.info()

    def timed(o, label):
        for i in range(args.warmup):
            _, st, rc = P.solve(**o)
            print(f"{label} warmup {i}: {st['seconds']:.3f} s sweeps={st['sweeps']} res={st['final_max_res']:.2e}",
                  file=sys.stderr, flush=True)
        lat, stats, u = [], [], None
        t_begin = time.perf_counter()
        for i in range(args.steps):
            if u is not None:
                u.close()
            t0 = time.perf_counter()
            u, st, rc = P.solve(**o)
            lat.append(time.perf_counter() - t0)
            stats.append(st)
            print(f"{label} step {i}: {lat[-1]:.3f} s sweeps={st['sweeps']} cg={st['cg_iters']} "
                  f"res={st['final_max_res']:.2e}", file=sys.stderr, flush=True)
        return u, stats[-1], lat, time.perf_counter() - t_begin

    u, st, lat, total = timed(opts, DTYPES[args.precision].split(" ")[0])
    # the other precision, timed the same way: FP32 local applies beside an FP64
    # headline, plain FP64 beside a low-precision one
    side_prec = 1 if args.precision == 0 else 0
    side_key = "mixed_precision_solver" if side_prec else "fp64_solver"
    u_side, side = None, None
    if not args.no_side_solver:
        o2 = dict({k: v for k, v in opts.items() if not k.startswith("ir_")}, precision=side_prec)
        u_side, st2, lat2, total2 = timed(o2, DTYPES[side_prec].split(" ")[0])
        side = {"dtype": DTYPE_TAGS[side_prec], "value": args.steps / total2, "unit": "solves/s",
                "ms_per_step": 1e3 * total2 / args.steps,
                "latency_ms": {"p50": 1e3 * percentile(lat2, 0.5), "p99": 1e3 * percentile(lat2, 0.99)},
                "cg_iters": st2["cg_iters"], "counted_flops": st2["flops"],
                "low_precision_flops": st2["low_precision_flops"], "refinements": st2["refinements"],
                "speed_of_this_line_vs_headline": (args.steps / total2) / (args.steps / total)}
    roof = None
    if not args.no_profile:
        roof = roofline(P, opts, args.workload)
    cpu, oracle_cores = None, None
    if not args.no_cpu_baseline:
        cpu, oracle_cores = cpu_baseline(args.workload, opts, st["local_applies"], full=wl.get("oracle_full", False))
    accuracy = accuracy_block(P, u, u_side, side_key, oracle_cores, opts, args.workload, prob,
                              refs=not args.no_accuracy)
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
        "dtype": DTYPE_TAGS[args.precision],
        "data": "synthetic",
        "config": {
            "workload": wl["desc"] + ", " + DTYPES[args.precision],
            "dofs": prob["dim"] * 2 ** (prob["dim"] * prob["level"]),
            "mpo_ranks": info["mpo_ranks"],
            "rank_cap": opts["rank_cap"],
            "tol": opts["tol"],
            "max_sweeps": opts["max_sweeps"],
            "rho": opts.get("rho", 4),
        },
        "latency_ms": {"p50": 1e3 * percentile(lat, 0.5), "p99": 1e3 * percentile(lat, 0.99)},
        "solve": {
            "sweeps": st["sweeps"], "converged": bool(st["converged"]), "final_max_local_residual": st["final_max_res"],
            "cg_iters": st["cg_iters"], "max_rank": st["max_rank"], "counted_flops": st["flops"],
            "low_precision_flops": st["low_precision_flops"], "refinements": st["refinements"],
            "precision_fallbacks": st["precision_fallbacks"],
            "median_latency_s": statistics.median(lat),
        },
        side_key: side,
        "accuracy": accuracy,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def traffic_from_summary(workload, precision):
    """HBM bytes per fused-apply launch from the committed counter summary of this workload
    and precision (None when there is none)."""
    name = TRAFFIC_SUMMARIES.get((workload, precision))
    if not name:
        return None, None
    path = os.path.join(ROOT, "profiles", name)
    try:
        with open(path) as f:
            for ln in f:
                if ln.startswith("traffic_bytes_per_launch:"):
                    return float(ln.split(":", 1)[1]), "profiles/" + name
    except OSError:
        pass
    return None, None


def mfma_busy_from_summary(workload, precision):
    """MFMA busy % per contraction kernel from the committed counter summary (None if absent)."""
    key = f"mfma_busy_pct[{workload},{precision}]:"
    path = os.path.join(ROOT, "profiles", "mfma_utilisation_contractions.md")
    try:
        with open(path) as f:
            for ln in f:
                if ln.startswith(key):
                    vals = dict(tok.split("=") for tok in ln[len(key):].split())
                    return {"busy_pct": {k: float(v) for k, v in vals.items()},
                            "source": "profiles/mfma_utilisation_contractions.md"}
    except OSError:
        pass
    return None


def roofline(P, opts, workload):
    """Live roofline of the dominant contraction kernel, the fused local apply (row a2):
    one more solve with start/stop events stamped by every contraction dispatch.
    achieved = algorithmic flops of the launches that did work (nonzero-term counts at the
    actual ranks) / summed duration of all its launches; the all-contraction rate
    (grouped GEMMs included) is reported beside it."""
    prec = opts.get("precision", 0)
    _, pst, _ = P.solve(profile=1, **opts)
    ms, fl, nl = pst["apply_kernel_ms"], pst["apply_kernel_flops"], pst["apply_kernel_launches"]
    achieved = fl / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    cms, cfl, cnl = pst["contraction_ms"], pst["contraction_flops"], pst["contraction_launches"]
    cap = opts["rank_cap"]
    kinds = ["fused_apply32_kernel"] + \
        ((["fused_apply16_kernel"] if prec != 2 else []) + ["fused_apply64_kernel"] if cap > 32 else []) + \
        (["slot_product_kernel + slot_apply_kernel"] if cap > 64 else [])
    kname = " / ".join(f"{k}<{prec}>" for k in kinds)
    if len(kinds) > 1:
        kname += " (by the ranks of each core step)"
    what = {0: "FP64 MFMA", 1: "FP32 MFMA, FP32 accumulate", 2: "BF16 MFMA, FP32 accumulate"}[prec]
    traffic, src = traffic_from_summary(workload, prec)
    return {
        "bound": "mfma",
        "kernel": f"{kname} (fused local operator apply, {what})",
        "achieved": achieved,
        "peak": PEAKS[prec],
        "unit": "TFLOP/s",
        "frac": achieved / PEAKS[prec],
        "traffic": traffic,
        "traffic_unit": "bytes per launch (PMC FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "traffic_source": src,
        "mfma_counters": mfma_busy_from_summary(workload, prec),
        "launches_per_solve": nl,
        "avg_launch_us": 1e3 * ms / max(nl, 1),
        "flops_per_launch": fl / max(nl, 1),
        "all_contractions": {
            "kernels": f"{kname} + gemm_grouped_kernel<*> / gemm_multi_kernel<*>",
            "launches_per_solve": cnl, "ms_per_solve": cms,
            "tflops": cfl / (cms * 1e-3) / 1e12 if cms > 0 else 0.0,
        },
    }


def accuracy_block(P, u, u_side, side_key, oracle_cores, opts, name, prob, refs=True):
    """Relative displacement errors of the timed solve, computed by the library in TT format
    (no densification): against the oracle's FP64 solve of the same problem with the same
    options (when the oracle ran the whole solve), against FP64 GPU solves with larger rank
    caps / tighter tolerances (their mutual difference bounds how far the last one is from
    converged), against the solve of the other precision timed beside it (`side_key`), and
    for the manufactured load against the closed-form field (which adds the O(h^2)
    discretisation error)."""
    from paper_2501_12151_amd import tnfem

    def label(o):
        return f"cap {o['rank_cap']} tol {o['tol']:g}" + (f" rho {o['rho']}" if "rho" in o else "")

    out = {"target": 1e-6, "rank_cap_of_timed_solve": opts["rank_cap"]}
    judged = None
    if oracle_cores is not None:
        ref = tnfem.TT.from_cores(oracle_cores)
        err = u.rel_diff(ref)
        out["rel_error_vs_oracle"] = err
        out["oracle"] = (f"the oracle's FP64 AMEn solve of the same problem on the host, {label(opts)}, "
                         f"{opts['max_sweeps']} half-sweeps")
        if u_side is not None:
            out[side_key + "_rel_error_vs_oracle"] = u_side.rel_diff(ref)
        judged = ("oracle", err)
    top = None
    if refs:
        rs = []
        for ro in WORKLOADS[name]["refs"]:
            r, rst, _ = P.solve(**ro)
            rs.append((r, rst, ro))
            print(f"reference {label(ro)}: {rst['seconds']:.2f} s, max local residual {rst['final_max_res']:.2e}",
                  file=sys.stderr, flush=True)
        top, tst, ro = rs[-1]
        err = u.rel_diff(top)
        out["rel_error_vs_fp64_reference"] = err
        out["fp64_reference"] = (f"same problem, FP64 on the GPU, {label(ro)}, {ro['max_sweeps']} half-sweeps "
                                 f"(max local residual {tst['final_max_res']:.2e}, max rank {tst['max_rank']})")
        if len(rs) > 1:
            out["fp64_reference_gap"] = {"between": [label(o) for _, _, o in rs], "rel_diff": rs[0][0].rel_diff(top)}
        if oracle_cores is not None:
            out["oracle_vs_fp64_reference"] = tnfem.TT.from_cores(oracle_cores).rel_diff(top)
        if judged is None:
            judged = ("fp64_reference", err)
    if u_side is not None:
        out["rel_diff_vs_" + side_key] = u.rel_diff(u_side)
    if "manufactured_c" in prob:
        exact = tnfem.TT.from_cores(manufactured_field_cores(prob["level"], prob["manufactured_c"]))
        out["rel_error_vs_closed_form"] = u.rel_diff(exact)
        if top is not None:
            out["fp64_reference_vs_closed_form"] = top.rel_diff(exact)
    if judged is not None:
        out["meets_target"] = bool(judged[1] <= 1e-6)
        out["judged_against"] = judged[0]
    return out


CANTILEVER_OPTS = dict(rank_cap=64, tol=1e-10, max_sweeps=40, rho=8)


def cantilever_tip(u, level):
    """Largest |u_y| over 257 nodes of the free end x = L_x (the tip carries the largest
    deflection), read from the TT by point evaluation."""
    import numpy as np

    n = 2 ** level
    iy = np.unique(np.linspace(0, n - 1, 257).astype(np.int64))
    idx = np.zeros((iy.size, level + 1), dtype=np.int64)
    for l in range(level):
        idx[:, l] = (((n - 1) >> (level - 1 - l)) & 1) * 2 + ((iy >> (level - 1 - l)) & 1)
    idx[:, level] = 1
    return float(np.abs(u.eval(idx)).max())


def cantilever(args):
    """The experiment of Sec. 6: the aluminium cantilever at increasing grid levels; per level
    the solve time, the tip deflection against the Euler-Bernoulli value 3 rho g L_x^4 /
    (2 E L_y^2), the strain energy b.u / 2, and the storage of u, b and the operator in TT
    format against the dense vector / sparse matrix they replace."""
    from paper_2501_12151_amd import tnfem, workloads

    rho, g = workloads.CANTILEVER_RHO, workloads.CANTILEVER_G
    levels = [int(x) for x in args.levels.split(",")]
    ctx = tnfem.Context(0)
    rows = []
    for d in levels:
        prob = workloads.cantilever(d)
        Lx, Ly = prob["extent"]
        ymax = 3 * rho * g * Lx ** 4 / (2 * prob["E"] * Ly ** 2)
        P = tnfem.Problem(ctx, prob)
        b = tnfem.TT.from_cores(tnfem.export_load(prob))
        Ac = tnfem.export_operator(prob)
        for _ in range(args.warmup):
            P.solve(**CANTILEVER_OPTS)[0].close()
        lat, u, st = [], None, None
        for _ in range(args.steps):
            if u is not None:
                u.close()
            t0 = time.perf_counter()
            u, st, rc = P.solve(**CANTILEVER_OPTS)
            lat.append(time.perf_counter() - t0)
        tip = cantilever_tip(u, d)
        ndof = 2 * 4 ** d
        row = {
            "level": d, "dofs": ndof, "solve_ms_p50": 1e3 * percentile(lat, 0.5), "sweeps": st["sweeps"],
            "converged": bool(st["converged"]), "max_rank": st["max_rank"],
            "tip_deflection_m": tip, "euler_bernoulli_m": ymax, "tip_rel_error": abs(tip - ymax) / ymax,
            "strain_energy_J_per_m": 0.5 * b.dot(u),
            "tt_bytes": {"u": 8 * sum(c.size for c in u.cores), "b": 8 * sum(c.size for c in b.cores),
                         "operator_cores": 8 * sum(c.size for c in Ac),
                         "operator_nonzeros": int(sum(int((c != 0).sum()) for c in Ac))},
            "dense_bytes": {"u": 8 * ndof, "b": 8 * ndof, "sparse_K_csr": 12 * 18 * ndof},
        }
        print(f"cantilever level {d}: {row['solve_ms_p50']:.1f} ms, tip {tip:.5e} m ({tip / ymax:.5f} of "
              f"Euler-Bernoulli), energy {row['strain_energy_J_per_m']:.5e}", file=sys.stderr, flush=True)
        rows.append(row)
        u.close()
        b.close()
        P.close()
    ctx.close()
    top = rows[-1]
    out = {
        "metric": METRIC,
        "value": 1e3 / top["solve_ms_p50"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": top["solve_ms_p50"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"aluminium cantilever 20 m x 1 m, plane stress, E = 68 GPa, nu = 0.33, self-weight "
                               f"rho g = {rho * g:g} N/m^3, x = 0 clamped; levels {levels} (value: finest level)",
                   "solve_options": CANTILEVER_OPTS},
        "levels": rows,
    }
    print(json.dumps(out), flush=True)


SERVING_REF = dict(rank_cap=96, tol=1e-9, max_sweeps=30)


def serving_accuracy(reqs, kept):
    """Relative displacement error of sampled served solutions against FP64 reference solves
    of the same problems at a larger rank cap (computed by the library in TT format)."""
    from paper_2501_12151_amd import tnfem

    ctx = tnfem.Context(0)
    rows = []
    for i in sorted(kept):
        u = kept[i]
        _, prob, cap = reqs[i]
        P = tnfem.Problem(ctx, prob)
        ref, rst, _ = P.solve(**SERVING_REF)
        err = u.rel_diff(ref) if u is not None else float("nan")
        rows.append({"request": i, "dim": prob["dim"], "level": prob["level"], "rank_cap": cap, "rel_error": err})
        print(f"accuracy sample {i}: {prob['dim']}D level {prob['level']} cap {cap}: {err:.2e}", file=sys.stderr,
              flush=True)
        ref.close()
        if u is not None:
            u.close()
        P.close()
    ctx.close()
    errs = [r["rel_error"] for r in rows]
    return {
        "reference": "same problem, FP64, rank cap {rank_cap}, tol {tol:g}, {max_sweeps} half-sweeps".format(
            **SERVING_REF),
        "sample": len(rows),
        "rel_error_p50": percentile(errs, 0.5),
        "rel_error_max": max(errs) if errs else None,
        "meets_target": sum(1 for e in errs if e <= 1e-6),
        "target": 1e-6,
        "requests": rows,
    }


def serving_run(args, precision):
    """One serving measurement at the given local-apply precision: a closed loop (64
    requests at once, saturation throughput), then the Poisson stream at 0.8 x that rate.
    Returns the stream's figures and the solutions kept for the accuracy sample."""
    from paper_2501_12151_amd import tnfem, workloads

    # enrichment rank 8 and 20 half-sweeps: 3D requests end near their cap's error floor
    # (12 half-sweeps with rank 4 stop at 2e-2 .. 8e-2 from the reference)
    def opts_for(cap):
        return dict(rank_cap=cap, tol=1e-8, max_sweeps=20, rho=8, precision=precision)

    sat_reqs = workloads.serving_stream(min(64, args.requests), seed=1, rate=1.0)
    srv = tnfem.Server(0, slots=args.slots)
    t0 = time.perf_counter()
    ts = [srv.submit(p, **opts_for(c)) for _, p, c in sat_reqs]
    for t in ts:
        srv.poll(t)
    sat = len(ts) / (time.perf_counter() - t0)
    srv.close()
    print(f"{DTYPE_TAGS[precision]} closed loop: {len(ts)} requests, {sat:.2f} solves/s", file=sys.stderr, flush=True)
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
    # every (n/8)-th request keeps its solution for the accuracy sample
    sample = set(range(0, len(tickets), max(1, len(tickets) // 8)))
    kept = {}
    for i, t in enumerate(tickets):
        u, st, rc, l = srv.poll(t)
        lat.append(l)
        if i in sample:
            kept[i] = u
        elif u is not None:
            u.close()
    elapsed = time.perf_counter() - t0
    info = srv.info()
    srv.close()
    return dict(sat=sat, rate=rate, n=len(tickets), elapsed=elapsed, lat=lat, info=info), reqs, kept


def serving(args):
    """Serving stream: Poisson arrivals of mixed 2D/3D requests; throughput and p50/p99 latency.
    With --precision 1 or 2 (low-precision local applies, FP64-refined local solves, lockstep
    batches as in FP64) the plain FP64 stream is measured the same way beside it."""
    r, reqs, kept = serving_run(args, args.precision)
    accuracy = serving_accuracy(reqs, kept)
    fp64 = None
    if args.precision != 0 and not args.no_side_solver:
        r64, _, kept64 = serving_run(args, 0)
        for u in kept64.values():
            if u is not None:
                u.close()
        fp64 = {"value": r64["n"] / r64["elapsed"], "unit": "solves/s", "closed_loop_solves_per_s": r64["sat"],
                "latency_ms": {"p50": 1e3 * percentile(r64["lat"], 0.5), "p99": 1e3 * percentile(r64["lat"], 0.99)},
                "server": r64["info"]}
    out = {
        "metric": METRIC,
        "value": r["n"] / r["elapsed"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": r["n"],
        "warmup": 0,
        "ms_per_step": 1e3 * r["elapsed"] / r["n"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE_TAGS[args.precision],
        "data": "synthetic",
        "config": {"workload": f"serving stream: {r['n']} requests, Poisson arrivals at 0.8 x closed-loop "
                               f"rate ({r['rate']:.2f}/s), 2D/3D, levels 6..10, caps 32..64, {args.slots} slots, "
                               f"{DTYPES[args.precision]}",
                   "closed_loop_solves_per_s": r["sat"]},
        "latency_ms": {"p50": 1e3 * percentile(r["lat"], 0.5), "p99": 1e3 * percentile(r["lat"], 0.99)},
        "server": r["info"],
        "accuracy": accuracy,
        "fp64_serving": fp64,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
