#!/usr/bin/env python3
"""Benchmark: transformed Radau IIA linear solves per second on one MI355X.

Workload (default): s = 3 Radau IIA on a periodic 64 x 64 quad mesh with
randomly permuted elements, 64 x 64 blocks (DG p = 3, 4 components),
5 blocks per row, shared Jacobian, FP64, stage-coupled block ILU(0),
GMRES(30), relative true-residual tolerance 1e-10, dt = 0.1.  Synthetic
values of the shape and distribution of the paper's DG Jacobians.

One step = one full linear solve of the hot path with the operator already
resident in HBM: operator ingest (block relayout), block ILU(0)
factorization, and preconditioned GMRES to tolerance.  The level schedule
is built once per sparsity pattern (setup) and reused, as within a Newton
loop.

Prints one JSON line.  It reports every kernel family of the step (BSR
matvec, preconditioner sweeps, factorization, Arnoldi) against its roofline
from HIP events recorded around each launch group inside the timed region,
with `roofline` naming the family that takes the most time; the other five
cells of the workload (dt in {0.01, 0.1, 1.0} x coupled / shifted
uncoupled); the untransformed operator beside the transformed one; one
Newton time step (linear and nonlinear) and the DIRK comparison steps; and
the CPU oracle on the same workload, single-threaded and on all host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s
FP64_PEAK_TFS = 78.6    # MI355X dense FP64 matrix-core peak, TFLOP/s


def matvec_bytes(s, T, m, nnzb, nJ=1, w=8):
    """Algorithmic bytes of one multi-stage matvec: every Jacobian block and
    mass block once, the input and output stage vectors once, the BSR
    indices once."""
    return (nJ * nnzb * m * m * w + T * m * m * w + 2 * s * T * m * 8
            + 4 * (T + 1) + 4 * nnzb)


def sweep_bytes(s, T, m, nnzb, coupled, w=8):
    """Algorithmic bytes of one preconditioner application (both sweeps):
    off-diagonal Jacobian blocks once (lower ones forward, upper ones
    backward), every pivot inverse twice, and four stage-vector passes; the
    coupled form adds each stored cross-stage block once (C_kl with k, l >= 1:
    the ones in stage row or column 0 are multiples of M) and the mass block
    once per direction."""
    r_blocks = nnzb - T
    cross = ((s - 1) * (s - 2) + 2) * T * m * m * w if coupled and s > 1 else 0
    return r_blocks * m * m * w + 2 * s * T * m * m * w + cross + 4 * s * T * m * 8


def factor_flops(s, T, m, row_ptr, col_idx, coupled):
    """FP64 flops of one block ILU(0) factorization as the kernels run it:
    per stage and element, two m x m products per lower neighbour
    (P_j^{-1} J_ji, then J_ij X) and one Gauss-Jordan inversion, each 2 m^3;
    the coupled form adds, per element, the stage rounds' products (2 for
    the first stage, (s-1-k)(s-k) for stage k >= 1)."""
    import numpy as np
    rows = np.repeat(np.arange(T), np.diff(row_ptr))
    lower = int(np.sum(np.asarray(col_idx) < rows))
    m3 = 2.0 * m ** 3
    fl = s * (2 * lower + T) * m3
    if coupled and s > 1:
        fl += T * (2 + sum((s - 1 - k) * (s - k) for k in range(1, s))) * m3
    return fl


def arnoldi_bytes(s, T, m, j):
    """Algorithmic bytes of Arnoldi step j (CGS2: three basis passes over
    j + 1 vectors, the work vector read and written, the new basis vector)."""
    return (3 * (j + 1) + 5) * s * T * m * 8


def untransformed_bytes(s, T, m, nnzb, nJ=1, form="blocks", w=8):
    """Algorithmic bytes of the untransformed operator: block by block, each
    of the s^2 blocks streams its stage Jacobian (and M on the diagonal) and
    reads x_l, writes y_k; fused, each Jacobian row and M once."""
    if form == "blocks":
        return s * s * nnzb * m * m * w + s * T * m * m * w + 2 * s * s * T * m * 8
    return matvec_bytes(s, T, m, nnzb, nJ, w)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_matvec_s3_64x64_m64_hbm_traffic.txt")
TRAFFIC_SOURCES = ["paper_1701_07181_amd/csrc/k_matvec.hip", "paper_1701_07181_amd/csrc/irk_device.h"]
SWEEP_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweep_s3_64x64_m64_coupled_hbm_traffic.txt")
SWEEP_TRAFFIC_SOURCES = ["paper_1701_07181_amd/csrc/k_sweep.hip", "paper_1701_07181_amd/csrc/k_sweep_flow.hip",
                         "paper_1701_07181_amd/csrc/sweep_item.h", "paper_1701_07181_amd/csrc/irk_device.h"]
FACTOR_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_factor_s3_64x64_m64_coupled_counters.txt")
FACTOR_TRAFFIC_SOURCES = ["paper_1701_07181_amd/csrc/k_factor.hip", "paper_1701_07181_amd/csrc/dense64.h",
                          "paper_1701_07181_amd/csrc/irk_device.h"]


def _counter_traffic(path, sources):
    """HBM bytes per launch (group) from a committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes scaled by a known-size copy), or None
    when the kernel sources have changed since the counters were taken."""
    import hashlib
    try:
        txt = open(path).read()
    except OSError:
        return None
    vals = dict(l.split(":", 1) for l in txt.splitlines()
                if l.startswith(("traffic_bytes_per_launch:", "source_sha256:")))
    vals.update({l.split(":", 1)[0][len("factor "):]: l.split(":", 1)[1] for l in txt.splitlines()
                 if l.startswith(("factor traffic_bytes_per_launch:", "factor source_sha256:"))})
    h = hashlib.sha256()
    for p in sources:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    if vals.get("source_sha256", "").split()[0:1] != [h.hexdigest()]:
        return None
    return int(vals["traffic_bytes_per_launch"])


def measured_traffic():
    """HBM bytes per k_matvec launch (see _counter_traffic)."""
    return _counter_traffic(TRAFFIC_FILE, TRAFFIC_SOURCES)


def sweep_traffic():
    """HBM bytes per preconditioner application (all sweep levels)."""
    return _counter_traffic(SWEEP_TRAFFIC_FILE, SWEEP_TRAFFIC_SOURCES)


def factor_traffic():
    """HBM bytes per factorization (all wavefronts: k_factor_flow, the
    asynchronous factorization of the timed steps)."""
    return _counter_traffic(FACTOR_TRAFFIC_FILE, FACTOR_TRAFFIC_SOURCES)


def _log(msg):
    print("# " + msg, file=sys.stderr, flush=True)


def run_mixed(args):
    """16^3 periodic hex mesh, m = 135, s = 3, dt = 0.5: plain FP64 GMRES
    against the FP64 refinement loop with FP32 matvec and FP32 / BF16 /
    FP16-scaled factors, all to a true relative residual of 1e-8.  One step
    = factor + solve, operator resident."""
    import torch
    import dgsynth
    import paper_1701_07181_amd as irk
    steps = max(1, args.steps)
    sy = dgsynth.config_system("cfg2")
    rhs = torch.as_tensor(sy.rhs).cuda()
    results = []
    x_ref = None
    for name, mv, fp in [("fp64", "fp64", "fp64"), ("fp32", "fp32", "fp32"),
                         ("bf16", "fp32", "bf16"), ("fp16s", "fp32", "fp16s")]:
        opts = irk.Options(pc="uncoupled_shifted", matvec_prec=mv, factor_prec=fp, rtol=1e-8,
                           restart=30)
        sol = irk.Solver(sy, opts)
        sol.factor()
        sol.autotune()
        for _ in range(max(1, args.warmup)):
            sol.factor()
            x, info = sol.solve(rhs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            sol.factor(wait=False)
            x, info = sol.solve(rhs)
        torch.cuda.synchronize()
        dt_s = (time.perf_counter() - t0) / steps
        if x_ref is None:
            x_ref = x.clone()
        err = float(torch.linalg.norm(x - x_ref) / torch.linalg.norm(x_ref))
        results.append({"variant": name, "solves_per_s": round(1.0 / dt_s, 3),
                        "ms_per_solve": round(dt_s * 1e3, 2), "ms_factor": round(info["ms_factor"], 2),
                        "iters": info["iters"], "outer_iters": info["outer_iters"],
                        "rel_res_true": info["rel_res_true"], "rel_diff_vs_fp64": err,
                        "converged": info["converged"]})
        _log(f"mixed {name}: {results[-1]}")
        sol.close()
        del sol
        torch.cuda.empty_cache()
    return {"metric": "IRK solves/s at 1e-8 rel residual", "mode": "mixed", "unit": "solves/s",
            "data": "synthetic",
            "config": {"workload": "s=3 Radau IIA, periodic 16^3 hex mesh (T=4096), m=135, 7 blocks "
                                   "per row, shifted uncoupled block ILU(0), GMRES(30), rtol 1e-8, dt=0.5",
                       "steps": steps},
            "results": results}


def _build_systems(specs, torch):
    systems = []
    for q, sp in enumerate(specs):
        sy = sp.build()
        sy.J = torch.from_numpy(sy.J).cuda()
        sy.M = torch.from_numpy(sy.M).cuda()
        sy.rhs = torch.from_numpy(sy.rhs).cuda()
        systems.append(sy)
    torch.cuda.synchronize()
    return systems


def run_batched(args):
    """256 independent systems of uneven size (2D periodic N in 4..32, p in
    1..4, s in 2..4, dt log-uniform): FP32-inner / FP64-outer to 1e-8.  One
    step = one batched factorization of every system + one batched solve of
    all of them; compared with the same solvers factored and solved one by
    one and with plain FP64 one by one."""
    import torch
    import dgsynth
    import paper_1701_07181_amd as irk
    count = args.count or 256
    specs = dgsynth.batch_specs(count)
    t0 = time.time()
    systems = _build_systems(specs, torch)
    elems = sum(sy.T for sy in systems)
    _log(f"built {count} systems ({elems} elements) in {time.time() - t0:.1f}s")
    mixed = irk.Options(pc="uncoupled_shifted", matvec_prec="fp32", factor_prec="fp32", rtol=1e-8,
                        restart=30)
    plain = irk.Options(pc="uncoupled_shifted", rtol=1e-8, restart=30)
    res = {}
    xs = None
    xs_by_label = {}
    legs = set(args.legs.split(",")) if args.legs else {f"{a}_{b}" for a in ("mixed", "fp64")
                                                          for b in ("batched", "one_by_one")}
    for label, opts in [("mixed", mixed), ("fp64", plain)]:
        if not any(l.startswith(label) for l in legs):
            continue
        solvers = [irk.Solver(sy, opts) for sy in systems]
        # launch shapes per problem class: timed on the first system of each
        # class, then taken from the process-wide table
        tuned = 0
        for so in solvers:
            so.factor()
            tuned += 1 - so.autotune()["from_cache"]
        _log(f"batched {label}: {tuned} problem classes timed by the autotuner")
        batch = irk.Batch(count, elems)
        modes = [md for md in ("batched", "one_by_one") if f"{label}_{md}" in legs]
        for mode in modes:
            def step():
                nonlocal xs
                if mode == "batched":
                    irk.factor_batched(batch, solvers)
                    xs, infos, st = irk.solve_batched(batch, solvers, [sy.rhs for sy in systems])
                else:
                    for s in solvers:
                        s.factor()
                    infos = [s.solve(sy.rhs)[1] for s, sy in zip(solvers, systems)]
                return infos
            step()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(max(1, args.steps)):
                infos = step()
            torch.cuda.synchronize()
            el = (time.perf_counter() - t1) / max(1, args.steps)
            res[f"{label}_{mode}"] = {"solves_per_s": round(count / el, 2), "ms_per_step": round(el * 1e3, 2),
                                      "converged": sum(bool(i["converged"]) for i in infos),
                                      "mean_iters": round(sum(i["iters"] for i in infos) / count, 2),
                                      "max_rel_res": max(i["rel_res_true"] for i in infos)}
            if mode == "batched":
                xs_by_label[label] = [x.clone() for x in xs]
            _log(f"batched {label} {mode}: {res[f'{label}_{mode}']}")
        for s in solvers:
            s.close()
        if batch:
            batch.close()
        torch.cuda.empty_cache()
    # like for like: mixed against FP64, both batched and both one by one;
    # the mixed solutions against the FP64 ones (both at a true residual of 1e-8)
    for mode in ("batched", "one_by_one"):
        if f"mixed_{mode}" in res and f"fp64_{mode}" in res:
            res[f"mixed_over_fp64_{mode}"] = round(res[f"mixed_{mode}"]["solves_per_s"] /
                                                   res[f"fp64_{mode}"]["solves_per_s"], 3)
    if "mixed" in xs_by_label and "fp64" in xs_by_label:
        diffs = [float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
                 for a, b in zip(xs_by_label["mixed"], xs_by_label["fp64"])]
        res["mixed_vs_fp64_rel_diff_max"] = max(diffs)
    return {"metric": "IRK solves/s at 1e-8 rel residual", "mode": "batched", "unit": "solves/s",
            "data": "synthetic",
            "config": {"workload": f"{count} systems: 2D periodic NxN, N in 4..32, DG p in 1..4 "
                                   "(m = 4(p+1)^2), s in 2..4, dt log-uniform [0.01, 1], shifted "
                                   "uncoupled block ILU(0), GMRES(30), rtol 1e-8",
                       "elements": elems, "steps": max(1, args.steps)},
            "results": res}


def run_serve(args):
    """Poisson arrivals of solve requests (75 % 2D periodic N x N, N up to 64,
    p 1..4; 25 % 3D N^3, N up to 16, p 2; s 2..4; 30 % re-use a resident
    operator), served by the continuous-batching loop to a true residual of
    1e-8.  Legs: FP32 inner / FP64 outer, plain FP64, BF16-factor inner.
    Each leg first measures its saturation rate (every request present at
    t = 0), then serves Poisson arrivals at fixed fractions of that rate.
    The stream replays 200 generated (operator, right-hand side)
    specifications with fresh right-hand sides; each replay's operators
    count as new (set up and factored again), which keeps input generation
    within two minutes."""
    import numpy as np
    import torch
    import dgsynth
    import paper_1701_07181_amd as irk
    from paper_1701_07181_amd.serve import Request, Server, latency_stats
    count = args.count or 600
    NB = 200
    N2max, N3max = 64, 16
    stream = dgsynth.serve_requests(min(count, NB), N2max=N2max, N3max=N3max)
    systems, reqs_base = {}, []
    t0 = time.time()
    for rid in range(count):
        spec, reuse_of, rhs_seed = stream[rid % NB]
        rep = rid // NB
        base = rid % NB if reuse_of is None else reuse_of
        if base not in systems:
            sy = spec.build()
            sy.J = torch.from_numpy(sy.J).cuda()
            sy.M = torch.from_numpy(sy.M).cuda()
            systems[base] = sy
        sy = systems[base]
        rhs = torch.from_numpy(dgsynth.fresh_rhs((*rhs_seed, rep), sy.s, sy.T, sy.m)).cuda()
        reqs_base.append((rid, base + NB * rep, sy, rhs))
    torch.cuda.synchronize()
    elems = [sy.T for sy in systems.values()]
    _log(f"built {len(systems)} operators for {count} requests in {time.time() - t0:.1f}s "
         f"(elements per operator {min(elems)}..{max(elems)})")
    legs = [("fp32_inner", irk.Options(pc="uncoupled_shifted", matvec_prec="fp32", factor_prec="fp32",
                                       rtol=1e-8, restart=30), (0.25, 0.5, 0.75, 0.9)),
            ("fp64", irk.Options(pc="uncoupled_shifted", rtol=1e-8, restart=30), (0.25, 0.5, 0.75, 0.9)),
            ("bf16_inner", irk.Options(pc="uncoupled_shifted", matvec_prec="fp32", factor_prec="bf16",
                                       rtol=1e-8, restart=30), (0.5,))]
    out = {}
    rng = np.random.default_rng(4242)

    def serve(opts, arrivals, tag):
        reqs = [Request(rid, op, sy, rhs, float(a)) for (rid, op, sy, rhs), a in zip(reqs_base, arrivals)]
        srv = Server(opts, capacity=64, max_elements=1 << 20, budget_bytes=120 << 30)
        results = srv.run(reqs, progress=lambda d, n: _log(f"serve {tag}: {d}/{n} done"))
        st = latency_stats(results)
        st["stalls"], st["evictions"] = srv.stalls, srv.evictions
        srv.close()
        torch.cuda.empty_cache()
        return st

    for label, opts, fracs in legs:
        sat = serve(opts, np.zeros(count), f"{label} saturation")
        sat_rate = sat["solves_per_s"]
        _log(f"serve {label} saturation: {sat}")
        points = []
        for fr in fracs:
            qps = fr * sat_rate
            arr = np.cumsum(rng.exponential(1.0 / qps, size=count))
            st = serve(opts, arr, f"{label} {fr:.2f} x saturation")
            st["offered_qps"] = round(qps, 2)
            st["fraction_of_saturation"] = fr
            points.append(st)
            _log(f"serve {label} {fr:.2f} x saturation: {st}")
        out[label] = {"saturation": sat, "points": points}
    out["fp32_inner_over_fp64_saturation"] = round(out["fp32_inner"]["saturation"]["solves_per_s"] /
                                                   out["fp64"]["saturation"]["solves_per_s"], 3)
    out["bf16_inner_over_fp64_saturation"] = round(out["bf16_inner"]["saturation"]["solves_per_s"] /
                                                   out["fp64"]["saturation"]["solves_per_s"], 3)
    return {"metric": "IRK solves/s at 1e-8 rel residual; p99 latency", "mode": "serve",
            "unit": "solves/s", "data": "synthetic",
            "config": {"workload": f"{count} requests per point, 75% 2D N<={N2max} p 1..4, 25% 3D "
                                   f"N<={N3max} p=2, s 2..4, 30% operator re-use, shifted uncoupled "
                                   "block ILU(0), rtol 1e-8, capacity 64, Poisson arrivals at 0.25 / "
                                   "0.5 / 0.75 / 0.9 of each leg's measured saturation rate, "
                                   f"{NB} generated specifications replayed with fresh right-hand "
                                   "sides (replayed operators set up and factored again), 120 GiB "
                                   "workspace pool"},
            "legs": out}


def family_report(prof, elapsed, sy, pc, iters, N):
    """Per kernel family: time in the timed region, its share, the average
    launch group, and the fraction of its roofline (HBM for the matvec,
    sweeps and Arnoldi; FP64 for the factorization).  Returns (families,
    roofline of the family with the most time)."""
    fam = {}
    tot = elapsed * 1e3
    if prof["matvec_count"]:
        ms = prof["matvec_ms"] / prof["matvec_count"]
        by = matvec_bytes(sy.s, sy.T, sy.m, sy.nnzb)
        ach = by / (ms * 1e-3) / 1e9
        fam["matvec"] = {"kernel": "k_matvec (BSR multi-stage matvec, FP64)", "bound": "hbm",
                         "total_ms": round(prof["matvec_ms"], 3), "share": round(prof["matvec_ms"] / tot, 4),
                         "launches": prof["matvec_count"], "avg_launch_us": round(ms * 1e3, 2),
                         "bytes_per_launch": by, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                         "traffic": measured_traffic() if N == 64 else None}
    if prof["pc_count"]:
        ms = prof["pc_ms"] / prof["pc_count"]
        by = sweep_bytes(sy.s, sy.T, sy.m, sy.nnzb, pc == "coupled")
        ach = by / (ms * 1e-3) / 1e9
        fam["sweeps"] = {"kernel": "k_sweep / k_sweep_flow (block ILU(0) forward + backward sweeps, "
                                   "all levels of one preconditioner application, FP64)", "bound": "hbm",
                         "total_ms": round(prof["pc_ms"], 3), "share": round(prof["pc_ms"] / tot, 4),
                         "launches": prof["pc_count"], "avg_launch_us": round(ms * 1e3, 2),
                         "bytes_per_launch": by, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                         "traffic": sweep_traffic() if N == 64 and pc == "coupled" else None}
    if prof["factor_count"]:
        ms = prof["factor_ms"] / prof["factor_count"]
        fl = factor_flops(sy.s, sy.T, sy.m, sy.row_ptr, sy.col_idx, pc == "coupled")
        ach = fl / (ms * 1e-3) / 1e12
        fam["factor"] = {"kernel": "k_factor_flow / k_factor_task (block ILU(0) factorization, all "
                                   "stage/level wavefronts, FP64 matrix-core products and Gauss-Jordan "
                                   "inverses)",
                         "bound": "mfma",
                         "total_ms": round(prof["factor_ms"], 3), "share": round(prof["factor_ms"] / tot, 4),
                         "launches": prof["factor_count"], "avg_launch_us": round(ms * 1e3, 2),
                         "flops_per_launch": fl, "achieved": round(ach, 2), "peak": FP64_PEAK_TFS,
                         "unit": "TFLOP/s", "frac": round(ach / FP64_PEAK_TFS, 4),
                         "traffic": factor_traffic() if N == 64 and pc == "coupled" else None}
    if prof["orth_count"]:
        ms = prof["orth_ms"] / prof["orth_count"]
        # steps j = 0 .. iters-1 of one cycle per solve (GMRES(30) never restarts here)
        it = max(1, iters[0])
        by = sum(arnoldi_bytes(sy.s, sy.T, sy.m, j) for j in range(it)) / it
        ach = by / (ms * 1e-3) / 1e9
        fam["arnoldi"] = {"kernel": "k_cgs / k_cgs_finish / k_scale (CGS2 Arnoldi step + Givens)",
                          "bound": "hbm", "total_ms": round(prof["orth_ms"], 3),
                          "share": round(prof["orth_ms"] / tot, 4), "launches": prof["orth_count"],
                          "avg_launch_us": round(ms * 1e3, 2), "bytes_per_launch": int(by),
                          "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None}
    dom = max(fam, key=lambda k: fam[k]["total_ms"])
    f = fam[dom]
    roof = {"bound": f["bound"], "achieved": f["achieved"], "peak": f["peak"], "unit": f["unit"],
            "frac": f["frac"], "traffic": f["traffic"], "kernel": f["kernel"], "family": dom,
            "share_of_step": f["share"], "avg_launch_us": f["avg_launch_us"], "launches": f["launches"]}
    roof["bytes_per_launch" if "bytes_per_launch" in f else "flops_per_launch"] = \
        f.get("bytes_per_launch", f.get("flops_per_launch"))
    return fam, roof


def run_cells(sy, args, skip, irk, torch):
    """The other cells of the workload (dt x preconditioner), each timed over
    a few steps of ingest + factor + solve after one warm-up step."""
    out = []
    rhs = torch.as_tensor(sy.rhs).cuda()
    for pc in ("coupled", "uncoupled_shifted"):
        for dt in (0.01, 0.1, 1.0):
            if (dt, pc) == skip:
                continue
            sol = irk.Solver(sy, irk.Options(pc=pc, rtol=1e-10, restart=30), dt=dt)
            sol.factor()
            sol.autotune()
            Jd, Md = sol.J, sol.M

            def step():
                sol.update_values(Jd, Md, dt)
                sol.factor(wait=False)
                return sol.solve(rhs)[1]
            step()
            torch.cuda.synchronize()
            n = 4
            t0 = time.perf_counter()
            infos = [step() for _ in range(n)]
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / n
            assert all(i["converged"] for i in infos), (dt, pc)
            out.append({"dt": dt, "pc": pc, "solves_per_s": round(1.0 / el, 3),
                        "ms_per_step": round(el * 1e3, 3), "iters": infos[-1]["iters"],
                        "equiv_mults": infos[-1]["equiv_mults"],
                        "ms_factor": round(infos[-1]["ms_factor"], 3),
                        "rel_res_true": infos[-1]["rel_res_true"]})
            _log(f"cell dt={dt} {pc}: {out[-1]}")
            sol.close()
            del sol
            torch.cuda.empty_cache()
    return out


def run_extras(solver, sy, irk, torch):
    """The untransformed operator beside the transformed one (Table 2), one
    Newton time step (linear f; nonlinear f with per-stage Jacobians), and
    the DIRK comparison steps at equal order, on the same mesh and blocks."""
    import numpy as np
    out = {}
    x = torch.as_tensor(np.random.default_rng(5).standard_normal(sy.s * sy.T * sy.m)).cuda()
    reps = 10
    solver.profile(True)
    for _ in range(reps):
        solver.apply_operator(x)
    mv = solver.profile_read()
    res = {"transformed": {"avg_us": round(mv["matvec_ms"] / mv["matvec_count"] * 1e3, 2),
                           "bytes": matvec_bytes(sy.s, sy.T, sy.m, sy.nnzb)}}
    for form in ("blocks", "fused"):
        solver.profile(True)
        for _ in range(reps):
            solver.apply_operator_untransformed(x, form=form)
        pr = solver.profile_read()
        us = pr["untr_ms"] / pr["untr_count"] * 1e3
        by = untransformed_bytes(sy.s, sy.T, sy.m, sy.nnzb, form=form)
        res[f"untransformed_{form}"] = {"avg_us": round(us, 2), "bytes": by,
                                        "achieved_GBs": round(by / (us * 1e-6) / 1e9, 1)}
    res["ratio_blocks_over_transformed"] = round(res["untransformed_blocks"]["avg_us"]
                                                 / res["transformed"]["avg_us"], 3)
    solver.profile(False)
    out["untransformed_operator"] = res
    _log(f"untransformed: {res}")

    rng = np.random.default_rng(77)
    n = sy.T * sy.m
    u0 = torch.as_tensor(rng.standard_normal(n)).cuda()
    g = torch.as_tensor(rng.standard_normal(n)).cuda()
    dt = 0.1
    steps = {}
    # linear f = J u + cos(2 t) g with the workload's operator; the step
    # re-factors (a new Jacobian per step, as in a Newton loop)
    lin = irk.Solver(sy, irk.Options(pc="coupled", rtol=1e-10), dt=dt)
    lin.step(u0, g=g, omega=2.0, newton_tol=1e-8)
    lin.update_values(lin.J, lin.M, dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, inf = lin.step(u0, g=g, omega=2.0, newton_tol=1e-8)
    torch.cuda.synchronize()
    steps["radau35_linear"] = {"ms": round((time.perf_counter() - t0) * 1e3, 2), **{
        k: inf[k] for k in ("newton_iters", "gmres_iters", "equiv_mults", "factorizations")}}
    lin.close()
    # nonlinear f = J u + cos(2 t) g - 0.3 u^3: per-stage Jacobians (nJ = s)
    J3 = np.repeat(np.asarray(sy.J), sy.s, axis=0)
    sy3 = type(sy)(**{**sy.__dict__, "J": J3, "nJ": sy.s})
    nl = irk.Solver(sy3, irk.Options(pc="coupled", rtol=1e-10), dt=dt)
    del J3
    nl.step(u0, g=g, omega=2.0, eps=0.3, newton_tol=1e-8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, inf = nl.step(u0, g=g, omega=2.0, eps=0.3, newton_tol=1e-8)
    torch.cuda.synchronize()
    steps["radau35_nonlinear"] = {"ms": round((time.perf_counter() - t0) * 1e3, 2), **{
        k: inf[k] for k in ("newton_iters", "gmres_iters", "equiv_mults", "factorizations")}}
    nl.close()
    del nl, sy3
    torch.cuda.empty_cache()
    # equal-order comparison of one linear step each (factorization included):
    # RADAU23 vs DIRK33 (order 3), RADAU35 vs ESDIRK65 (order 5)
    cmp = {}
    for name, kind, arg in (("RADAU23", "radau", 2), ("DIRK33", "dirk", "DIRK33"),
                            ("RADAU35", "radau", 3), ("ESDIRK65", "dirk", "ESDIRK65")):
        if kind == "radau":
            so = irk.Solver(sy, irk.Options(pc="coupled", rtol=1e-10), s=arg, dt=dt)
            run = lambda: so.step(u0, g=g, omega=2.0, newton_tol=1e-8)
        else:
            A, _, _ = irk.dirk_tableau(arg)
            so = irk.Solver(sy, irk.Options(pc="coupled", rtol=1e-10), A=np.array([[A[-1, -1]]]),
                            s=1, dt=dt)
            run = lambda: so.dirk_step(A, u0, g=g, omega=2.0, newton_tol=1e-8)
        run()
        so.update_values(so.J, so.M, dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u1, inf = run()
        torch.cuda.synchronize()
        cmp[name] = {"ms": round((time.perf_counter() - t0) * 1e3, 2), **{
            k: inf[k] for k in ("newton_iters", "gmres_iters", "equiv_mults", "factorizations")}}
        so.close()
        torch.cuda.empty_cache()
    steps["equal_order_comparison"] = cmp
    out["time_step"] = steps
    _log(f"time steps: {steps}")
    return out


def cpu_baselines(sy, pc):
    """The oracle on the same workload: one full solve single-threaded and one
    with the OpenMP build on all host cores (a child process, so the two
    builds do not meet in one process; it uses no GPU)."""
    import subprocess
    import oracle
    A, _, _ = oracle.radau_iia(sy.s)
    P = oracle.Problem(sy)
    tc = time.perf_counter()
    xo, io = oracle.solve(P, A, sy.rhs, pc=pc, rtol=1e-10, orth="cgs2")
    t1 = time.perf_counter() - tc
    single = {"value": round(1.0 / t1, 5), "unit": "solves/s", "cores": 1, "kind": "oracle",
              "sample": f"one full solve of the same workload (factor + GMRES, {io['iters']} "
                        f"iterations), plain FP64 C loops, single thread, {t1:.1f} s"}
    code = ("import sys, time, os; sys.path.insert(0, %r)\n"
            "import oracle, dgsynth\n"
            "oracle.use_openmp(True)\n"
            "sy = dgsynth.config_system('cfg1', dt=%r, N=%d)\n"
            "A, _, _ = oracle.radau_iia(sy.s)\n"
            "P = oracle.Problem(sy)\n"
            "t = time.perf_counter()\n"
            "x, i = oracle.solve(P, A, sy.rhs, pc=%r, rtol=1e-10, orth='cgs2')\n"
            "print(time.perf_counter() - t, i['iters'])\n") % (ROOT, sy.dt, int(round(sy.T ** 0.5)), pc)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    allc = None
    if r.returncode == 0:
        tall, its = r.stdout.split()[-2:]
        tall = float(tall)
        model = ""
        try:
            lines = subprocess.run(["lscpu"], capture_output=True, text=True).stdout.splitlines()
            info = {l.split(":", 1)[0].strip(): l.split(":", 1)[1].strip() for l in lines if ":" in l}
            model = f"{info.get('Model name', '?')}, {info.get('Socket(s)', '?')} socket(s), " \
                    f"{info.get('CPU(s)', '?')} CPUs"
        except OSError:
            pass
        allc = {"value": round(1.0 / tall, 5), "unit": "solves/s", "cores": threads, "kind": "oracle",
                "sample": f"one full solve of the same workload ({its} iterations), the oracle's "
                          f"OpenMP build (matvec rows, per-pivot row updates of the ILU(0), "
                          f"uncoupled stages, GMRES vector loops) on {threads} threads, {tall:.1f} s; "
                          f"nproc {os.cpu_count()}; {model}"}
    else:
        _log("all-cores oracle run failed: " + r.stderr[-400:])
    return (allc or single), (single if allc else None)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--pc", default="coupled", choices=["coupled", "uncoupled_shifted", "uncoupled"])
    ap.add_argument("--dt", type=float, default=0.1)
    ap.add_argument("--N", type=int, default=64, help="mesh side (64 = the full workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cells", action="store_true", help="skip the other dt / preconditioner cells")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the untransformed operator, time-step and DIRK measurements")
    ap.add_argument("--no-profile", action="store_true", help="no HIP events around kernels")
    ap.add_argument("--mode", default="headline", choices=["headline", "mixed", "batched", "serve"],
                    help="headline: the FP64 64x64 workload (default); mixed: the 16^3 hex m=135 "
                         "workload in FP64 and the three reduced-precision inner forms; batched: "
                         "256 uneven systems solved together vs one by one; serve: a request "
                         "stream at several arrival rates")
    ap.add_argument("--count", type=int, default=0, help="systems / requests for batched and serve")
    ap.add_argument("--legs", default="", help="batched mode: comma list of legs to run "
                    "(mixed_batched, mixed_one_by_one, fp64_batched, fp64_one_by_one; default all)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (the "
                         "known-size kernel that scales the HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for {args.gpus}); "
              "multi-GPU sharding is a design note, not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import dgsynth
    import paper_1701_07181_amd as irk

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 3}), flush=True)
        return
    if args.mode != "headline":
        out = {"mixed": run_mixed, "batched": run_batched, "serve": run_serve}[args.mode](args)
        print(json.dumps(out), flush=True)
        return
    t0 = time.time()
    sy = dgsynth.config_system("cfg1", dt=args.dt, N=args.N)
    print(f"# generated T={sy.T} m={sy.m} s={sy.s} nnzb={sy.nnzb} in {time.time()-t0:.1f}s",
          file=sys.stderr, flush=True)
    opts = irk.Options(pc=args.pc, rtol=1e-10, restart=30)
    solver = irk.Solver(sy, opts)
    Jd, Md = solver.J, solver.M
    # launch shapes timed once on this system (setup, like the level schedule)
    solver.factor()
    tune = solver.autotune()
    print(f"# autotune: {tune}", file=sys.stderr, flush=True)
    rhs = torch.as_tensor(sy.rhs).cuda()
    stream = solver.stream

    def step():
        solver.update_values(Jd, Md, args.dt)
        solver.factor(wait=False)     # the solve's first state read covers it
        x, info = solver.solve(rhs)
        return info

    for _ in range(args.warmup):
        info = step()
        print(f"# warmup: iters={info['iters']} rel_res={info['rel_res_true']:.2e}",
              file=sys.stderr, flush=True)
    # the timed steps (no profiling events in them)
    lat = []
    infos = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        infos.append(step())
        lat.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    for k in range(args.steps):
        print(f"# step {k}: {lat[k]:.2f} ms iters={infos[k]['iters']}", file=sys.stderr, flush=True)
    ms_per_step = elapsed * 1e3 / args.steps
    value = args.steps / elapsed
    # the same number of steps again with HIP events on the solver's stream
    # around every launch group, for the per-kernel figures (the events add a
    # few microseconds per group, so these steps are timed on their own)
    prof, elapsed_prof = None, None
    if not args.no_profile:
        solver.profile(True)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for k in range(args.steps):
            infos.append(step())
        torch.cuda.synchronize()
        elapsed_prof = time.perf_counter() - tp
        prof = solver.profile_read()
        solver.profile(False)

    assert all(i["converged"] for i in infos), "a timed solve did not converge"
    iters = [i["iters"] for i in infos]
    res = max(i["rel_res_true"] for i in infos)

    fam, roof = family_report(prof, elapsed_prof, sy, args.pc, iters, args.N) if prof else ({}, None)
    extra = {"kernels": fam} if fam else {}
    if prof:
        extra["profiled_steps"] = {"steps": args.steps, "ms_per_step": round(elapsed_prof * 1e3 / args.steps, 3),
                                   "note": "the per-kernel figures come from these steps, run after the "
                                           "timed ones with HIP events around every launch group"}
    if not args.no_cells:
        extra["cells"] = run_cells(sy, args, (args.dt, args.pc), irk, torch)
    if not args.no_extras:
        extra.update(run_extras(solver, sy, irk, torch))
    cpu, cpu1 = (None, None) if args.no_cpu_baseline else cpu_baselines(sy, args.pc)
    if cpu1:
        extra["cpu_baseline_single_thread"] = cpu1

    out = {
        "metric": "IRK solves/s at 1e-8 rel residual; BSR matvec GB/s vs HBM peak; p99 latency",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"s=3 Radau IIA, periodic {args.N}x{args.N} quad mesh "
                               f"(T={sy.T}), m={sy.m}, shared J, FP64, {args.pc} block ILU(0), "
                               f"GMRES(30), rtol 1e-10, dt={args.dt}",
                   "s": sy.s, "T": sy.T, "m": sy.m, "nnzb": sy.nnzb, "pc": args.pc,
                   "dt": args.dt, "rtol": 1e-10, "restart": 30},
        "roofline": roof,
        "cpu_baseline": cpu,
        "autotune": {k: tune[k] for k in ("matvec_teams", "sweep_big_min", "sweep_teams", "sweep_big_form",
                                              "sweep_flow", "sweep_chain_max", "sweep_split")},
        "iters": {"min": min(iters), "max": max(iters)},
        "equiv_mults": iters[0] * sy.s,
        "rel_res_true_max": res,
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3)},
        **extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
