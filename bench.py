"""Benchmark of the M-ABD per-step solve on one MI355X.

Default workload: the 1,048,576-body ball-jointed chain (body 0 pinned,
h = 1e-2 s, one Newton iteration per step), plain FP64.  A step is one pass
of the whole hot path: per-body co-rotated solve and polar decomposition, dual
assembly, chain dual solve, primal back-projection and state update.

Prints one JSON line with body-steps/s (dynamic bodies x steps / wall time of
the timed mabd_step call), the live per-kernel roofline of the dominant kernel
(HIP events on the stream the kernels run on), the KKT residual reached (FP64
oracle verification of one GPU step), and the FP64 oracle timed on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FORMS = {0: "plain FP64", 1: "FP32 bulk + FP64 factor + FP64 refinement"}

# Algorithmic HBM bytes per body (or joint) that each kernel must move at
# minimum (FP64): state q, qdot read (192 B) and written (192 B), per-row
# anchors of both ends and the side flags (49 B), shape index (4 B),
# multipliers written (24 B).  Intermediate data the design itself moves (the
# packed tiles' survivors and factors, ~38 B and ~45 B per body) is not
# counted, so `achieved` understates the bytes the kernels move.
ALG_BYTES = {
    "chain_reduce": 192 + 49 + 4,
    "chain_apply": 192 + 49 + 4 + 192 + 24,
}
# Precision form 1: its tile kernels move different data per pass (FP32
# solve: q, qdot; corrections: q and the FP64 residual), so only the FP64
# residual kernel is priced: q, qdot, dq read (288 B), anchors, flags and shape
# index (53 B), multipliers read (24 B), residuals written (96 + 24 B).
ALG_BYTES_F1 = {"chain_resid": 288 + 53 + 24 + 120}
JOINT_ROWS = (3, 5, 4, 5)  # ball, hinge, universal, prismatic


def generic_parts(asm):
    """Masks of the bodies and joints outside the fused chain path: the
    library takes a component (dynamic bodies connected by joints) as a
    chain when it is acyclic, every joint is a ball joint, every body carries
    at most two joints and there are at least two joints (one Newton
    iteration); everything else is solved on the generic path."""
    import numpy as np
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    n, m = int(asm.n), int(asm.m)
    dyn = np.asarray(asm.pinned) == 0
    ja, jb = np.asarray(asm.ja, np.int64), np.asarray(asm.jb, np.int64)
    da = (ja >= 0) & dyn[np.clip(ja, 0, None)]
    db = (jb >= 0) & dyn[np.clip(jb, 0, None)]
    two = da & db
    g = coo_matrix((np.ones(int(two.sum())), (ja[two], jb[two])), shape=(n, n))
    _, comp = connected_components(g, directed=False)
    jcomp = np.where(da, comp[np.clip(ja, 0, None)], comp[np.clip(jb, 0, None)])
    inc = np.bincount(ja[da], minlength=n) + np.bincount(jb[db], minlength=n)
    nc = int(comp.max()) + 1 if n else 0
    nb = np.bincount(comp[dyn], minlength=nc)
    nj = np.bincount(jcomp, minlength=nc)
    edges = np.bincount(jcomp, weights=da.astype(int) + db.astype(int), minlength=nc)
    nonball = np.bincount(jcomp, weights=(np.asarray(asm.jtype) != 0).astype(int), minlength=nc)
    maxinc = np.zeros(nc, int)
    np.maximum.at(maxinc, comp[dyn], inc[dyn])
    chain = (edges == nb + nj - 1) & (nonball == 0) & (maxinc <= 2) & (nj >= 2)
    return dyn & ~chain[comp], ~chain[jcomp]


def generic_alg_bytes(asm, phase):
    """Algorithmic HBM bytes per launch of a kernel group of the generic
    (tree) path, FP64, counted over the bodies and joints outside the fused
    chain path (generic_parts).  A joint row
    on one dynamic side is 12 doubles (96 B); a body's state q, qdot is 192 B,
    its rotation 72 B, its local solve 96 B, its shape index 4 B; a joint's
    record is 200 B, its values C and multipliers 8 B per row.
      body:  q, qdot, shape index read; R and u written.
      joint: records, both sides' A, t and R read (168 B per dynamic side);
             rows and C written.
      tree:  u and shape index read per body, every row and C read, the
             multipliers written (the clique matrices are intermediate).
      apply: rows and multipliers of the incident joints, R, u, shape index
             and q, qdot read; q, qdot written."""
    import numpy as np

    dyn = np.asarray(asm.pinned) == 0
    bmask, jmask = generic_parts(asm)
    nb = int(bmask.sum())
    rows = np.asarray(JOINT_ROWS)[np.asarray(asm.jtype, int)] if asm.m else np.zeros(0, int)
    ja, jb = np.asarray(asm.ja), np.asarray(asm.jb)
    sides = ((ja >= 0) & dyn[np.clip(ja, 0, None)]).astype(int) + ((jb >= 0) & dyn[np.clip(jb, 0, None)]).astype(int)
    rows, sides = rows * jmask, sides * jmask
    side_rows = int((rows * sides).sum())
    nrows = int(rows.sum())
    if phase == "body":
        return nb * (192 + 4 + 72 + 96)
    if phase == "joint":
        return int(jmask.sum()) * 200 + int(sides.sum()) * 168 + side_rows * 96 + nrows * 8
    if phase == "tree":
        return nb * (96 + 4) + side_rows * 96 + nrows * 16
    if phase == "apply":
        return nb * (72 + 96 + 4 + 192 + 192) + side_rows * (96 + 8)
    return None
# HBM bytes per launch of the dominant kernel measured with rocprofv3 --pmc
# (FETCH_SIZE x2.000 + WRITE_SIZE x1.000, scales from a plain 512 MiB copy),
# keyed by workload, kernel, tile threads and tile packing, together with the
# SHA-256 (first 16 hex digits) of the kernel source the counters were taken
# on: once that source changes the figure is stale and `traffic` is null.
PMC_TRAFFIC = {
    # profiles/chain1m_fp64_kernels.md: FETCH_SIZE 149,036.9 KiB x2.000,
    # WRITE_SIZE 221,791.7 KiB x1.000 per dispatch of the packed apply kernel
    ("chain1m", "chain_apply", 64, 1): ("0a0ad516dddf1630", 532342272),
}
PMC_SOURCE = os.path.join(ROOT, "paper_2603_08079_amd", "csrc", "k_chain.hip")


def source_sha16(path):
    import hashlib

    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def host_cpu():
    """Model name and logical CPU count of the host (for the CPU baseline)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return model, os.cpu_count(), usable


def slice_bodies(asm, nb):
    """Bodies [0, nb) of an assembly with the joints among them (a prefix of
    the chain workload is the same chain, shorter)."""
    import dataclasses

    import numpy as np

    jm = (np.where(asm.ja >= 0, asm.ja, 0) < nb) & (np.where(asm.jb >= 0, asm.jb, 0) < nb)
    return dataclasses.replace(
        asm, name=f"{asm.name}[:{nb}]", dims=asm.dims[:nb], density=asm.density[:nb],
        k_orth=asm.k_orth[:nb], pinned=asm.pinned[:nb], q0=asm.q0[:nb], qd0=asm.qd0[:nb],
        poisson=None if asm.poisson is None else asm.poisson[:nb], jtype=asm.jtype[jm],
        ja=asm.ja[jm], jb=asm.jb[jm], pa=asm.pa[jm], pb=asm.pb[jm], axis=asm.axis[jm],
        cp_len=asm.cp_len[jm], meta={})


def cpu_baseline(asm, wrench, q, qd, workload, nb, steps, body_solve=0, network=False, tol=1e-10,
                 max_iters=200000):
    """The FP64 oracle (the same C source, built -O3 -march=native for this
    host) timed on `steps` steps of a bounded sample of the workload: its
    first `nb` bodies, from the benchmark's final state.  Two legs: one
    thread (the paper's design point) and OpenMP over the per-body phases on
    the host's cores (the chain / tree eliminations stay serial).  Workloads
    with loops or networks take the oracle's block-Jacobi PCG to the same
    tolerance on one step of a sample of at most 4,096 bodies (its direct
    solvers are dense at that point; one such step is ~10 s)."""
    import ctypes
    import tempfile

    import numpy as np

    import oracle

    if network:
        nb, steps = min(nb, 4096), min(steps, 1)
    sub = slice_bodies(asm, nb)
    w = None if wrench is None else wrench[:nb]
    n_dyn = int((sub.pinned == 0).sum())
    legs = {}
    with tempfile.TemporaryDirectory() as td:
        for name, omp in (("single_thread", False), ("openmp", True)):
            L = oracle.load(oracle.build_native(os.path.join(td, f"ora_{name}.so"), omp))
            threads = 1
            if omp:
                try:
                    threads = int(ctypes.CDLL("libgomp.so.1").omp_get_max_threads())
                except OSError:
                    threads = os.cpu_count()
            sysm = oracle.System(sub, wrench=w, L=L, body_solve=body_solve)
            qq, qqd = q[:nb].copy(), qd[:nb].copy()
            t0 = time.perf_counter()
            for _ in range(steps):
                if network:
                    qq, qqd, _, _ = sysm.step(sub.h, qq, qqd, solver=oracle.PCG, tol=tol, max_iters=max_iters)
                else:
                    qq, qqd, _, _ = sysm.step(sub.h, qq, qqd)
            dt = time.perf_counter() - t0
            legs[name] = {"body_steps_per_s": round(n_dyn * steps / dt, 1), "threads": threads,
                          "seconds": round(dt, 2)}
    model, ncpu, usable = host_cpu()
    best = max(legs, key=lambda k: legs[k]["body_steps_per_s"])
    return {"value": legs[best]["body_steps_per_s"], "unit": "body-steps/s",
            "cores": legs[best]["threads"], "kind": "oracle",
            "sample": f"{steps} steps of the first {nb} bodies ({n_dyn} dynamic) of the {workload} "
                      f"workload from the benchmark's final state; FP64 oracle built -O3 "
                      f"-march=native" + (f", block-Jacobi PCG to {tol:g}" if network else "") +
                      f"; value = the faster leg ({best})",
            "legs": legs, "cpu_model": model, "nproc": ncpu, "usable_cpus": usable}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="chain1m")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kkt-check", action="store_true")
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed repeats of --steps steps; the median is reported")
    ap.add_argument("--cpu-sample-bodies", type=int, default=131072,
                    help="CPU baseline: bodies of the workload's prefix the oracle steps")
    ap.add_argument("--cpu-sample-steps", type=int, default=10)
    ap.add_argument("--kkt-tol", type=float, default=1e-10, help="PCG stopping tolerance")
    ap.add_argument("--max-iters", type=int, default=200000, help="PCG iteration cap")
    ap.add_argument("--precision", choices=("auto", "0", "1"), default="auto",
                    help="0 plain FP64, 1 FP32 bulk + FP64 factor + FP64 refinement (chains, and "
                         "trees in contexts without loops or networks), auto: time both where form "
                         "1 applies and report the faster")
    ap.add_argument("--ir-tol", type=float, default=1e-12,
                    help="precision 1: target KKT residual of the refinement")
    ap.add_argument("--body-solve", type=int, choices=(0, 1), default=0,
                    help="1: bodies without joints take the polar-free solve (Alg. 1)")
    ap.add_argument("--path-solver", type=int, choices=(0, 1), default=1,
                    help="0: tree components that are paths go through the tree contraction "
                         "instead of the path solver")
    ap.add_argument("--wrenches", action="store_true",
                    help="apply a seeded wind-like load at every step: force 0.2 m g along +x with "
                         "2 %% noise, torques of 1 %% of m g times the body size")
    ap.add_argument("--copy-calibration-mb", type=float, default=0.0,
                    help="only run a plain device-to-device copy of this many MB (5 times), "
                         "to calibrate HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; "
              "run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration_mb > 0:
        n = int(args.copy_calibration_mb * (1 << 20)) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        # achieved HBM rate of a plain copy (bytes read + written): the
        # practical ceiling next to the 8 TB/s of the specification
        print(json.dumps({"copy_bytes_per_launch": 8 * n, "launches": 6, "ms_per_copy": round(ms, 4),
                          "read_plus_write_GBps": round(2 * 8 * n / (ms * 1e-3) / 1e9, 1)}), flush=True)
        return

    import mabd_inputs as mi
    import paper_2603_08079_amd as pk

    torch.cuda.set_device(0)
    # a stream of our own (default priority): the step graphs are captured on it
    stream = torch.cuda.Stream()
    asm = mi.config(args.workload)
    h = asm.h

    wrench = None
    if args.wrenches:
        rng = np.random.default_rng(7)
        mg = 9.8 * asm.density * asm.dims.prod(axis=1)
        wrench = np.zeros((asm.n, 6))
        wrench[:, :3] = 0.01 * rng.normal(size=(asm.n, 3)) * (mg * asm.dims.max(axis=1))[:, None]
        wrench[:, 3:] = 0.02 * rng.normal(size=(asm.n, 3)) * mg[:, None]
        wrench[:, 3] += 0.2 * mg

    def make(precision, **kw):
        tol = args.ir_tol if precision == 1 else args.kkt_tol
        c = pk.Context(asm, stream=stream.cuda_stream, precision=precision, kkt_tol=tol,
                       max_iters=args.max_iters, body_solve=args.body_solve,
                       path_solver=args.path_solver, **kw)
        if wrench is not None:
            c.set_wrenches(wrench)
        return c

    def run(c, nsteps):
        try:
            c.step(h, nsteps)
            return None
        except pk.MabdError as e:  # PCG stopped at its iteration cap: report, do not hide
            if e.status != pk.ERR_NOT_CONVERGED:
                raise
            return str(e)

    def timed(c, restart):
        """--repeats timed regions of exactly --steps steps, each bracketed by
        a device synchronisation; the median region is reported.  With
        `restart` (contexts with tree components) every region times the same
        steps of the workload's trajectory, steps [warmup, warmup + steps):
        before it (untimed) the state goes back to the workload's initial
        state and the warmup steps run again, since on the random trees a few
        light links carry subtrees thousands of times their mass and leave
        the small-deformation regime after some tens of steps.  Otherwise the
        regions follow each other on one trajectory after one warmup
        (restarting measured 0.305-0.310 against 0.289 ms/step on the 1M
        chain, on one box)."""
        reps = []
        if not restart and args.warmup:
            run(c, args.warmup)
        for _ in range(max(1, args.repeats)):
            if restart:
                c.set_state(asm.q0, asm.qd0)
                if args.warmup:
                    run(c, args.warmup)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            t0 = time.perf_counter()
            nc = run(c, args.steps)
            e1.record(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            st_ = c.stats()  # also reads the outcome of the queued steps
            if st_["last_status"] not in (0, pk.ERR_NOT_CONVERGED):
                raise RuntimeError(f"step failed with status {st_['last_status']}")
            if st_["last_status"] == pk.ERR_NOT_CONVERGED and nc is None:
                nc = "NOT_CONVERGED"
            reps.append({"wall": wall, "gpu_ms": e0.elapsed_time(e1), "stats": st_, "notconv": nc})
        reps.sort(key=lambda r: r["wall"])
        med = dict(reps[len(reps) // 2])
        med["walls_ms"] = [round(r["wall"] * 1e3, 4) for r in reps]
        return med

    ctx = make(0)
    st0 = ctx.stats()
    n_dyn = st0["n_dyn"]
    print(f"# workload {args.workload}: {asm.n} bodies ({n_dyn} dynamic), {asm.m} joints, "
          f"chains {st0['n_chain']} trees {st0['n_tree']} graphs {st0['n_graph']}",
          file=sys.stderr, flush=True)
    forms = {}
    restart = st0["n_tree"] > 0
    if args.precision in ("auto", "0"):
        forms[0] = timed(ctx, restart)
    # form 1 covers chain components and, in contexts without loop or
    # network components, tree components
    form1 = st0["n_chain"] or (st0["n_tree"] and not st0["n_graph"] and not st0["n_loop"])
    if args.precision in ("auto", "1") and form1:
        ctx1 = make(1)
        forms[1] = timed(ctx1, restart)
        if args.precision == "1":
            ctx.close()
            ctx = ctx1
        else:
            ctx1.close()
    for p_, r_ in forms.items():
        s_ = r_["stats"]
        print(f"# precision {p_}: {args.steps} steps in {r_['wall'] * 1e3:.3f} ms (graph replay "
              f"{s_['graph_replay']}, chain tile threads {s_['tile_threads']}"
              + (" packed" if s_['tile_packed'] else "")
              + (f", sweeps {s_['ir_sweeps']}, device kkt {s_['kkt']:.3e})" if p_ == 1 else ")"),
              file=sys.stderr, flush=True)
    # the chosen form: the faster one (both reach the FP64 KKT residual)
    chosen = min(forms, key=lambda k: forms[k]["wall"])
    if chosen == 1 and args.precision == "auto":
        ctx.close()
        ctx = make(1)
        run(ctx, args.warmup + args.steps)
    res = forms[chosen]
    wall, gpu_ms, st, notconv = res["wall"], res["gpu_ms"], res["stats"], res["notconv"]
    value = n_dyn * args.steps / wall

    # Per-kernel durations: the same steps again on a second context whose
    # kernel groups are bracketed by HIP events on the stream they run on.
    psteps = min(args.steps, 10)
    prof = make(chosen, diagnostics=2)
    run(prof, 1)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    run(prof, psteps)
    prof_ms = (time.perf_counter() - tp) * 1e3 / psteps
    sp = prof.stats()
    prof.close()
    phases = pk.StepStats.PHASES
    per_launch = {phases[i]: sp["phase_ms"][i] / sp["phase_calls"][i]
                  for i in range(len(phases)) if sp["phase_calls"][i]}
    dom = max(per_launch, key=lambda k: per_launch[k] * sp["phase_calls"][phases.index(k)])
    roof = None
    ab = ALG_BYTES if chosen == 0 else ALG_BYTES_F1
    alg = ab[dom] * n_dyn if dom in ab else None
    if alg is None and chosen == 0 and not st0["n_graph"]:
        alg = generic_alg_bytes(asm, dom)
    if alg is not None:
        ach = alg / (per_launch[dom] * 1e-3) / 1e9
        key = (args.workload, dom, st["tile_threads"], st["tile_packed"])
        traffic = None
        if chosen == 0 and key in PMC_TRAFFIC:
            sha, nbytes = PMC_TRAFFIC[key]
            traffic = nbytes if sha == source_sha16(PMC_SOURCE) else None
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "avg_launch_ms": round(per_launch[dom], 4),
                "alg_bytes_per_launch": alg,
                "timing": f"HIP events around each launch, {psteps} steps, eager launches "
                          f"({prof_ms:.4f} ms/step)"}
    print(f"# per-launch ms: { {k: round(v, 4) for k, v in per_launch.items()} }",
          file=sys.stderr, flush=True)

    kkt = None
    cpu = None
    if not args.no_kkt_check or not args.no_cpu_baseline:
        import oracle

        s = oracle.System(asm, wrench=wrench, body_solve=args.body_solve)
        q_n, qd_n = ctx.state()
    if not args.no_kkt_check:
        # one more GPU step from the current (moving) state, verified by the
        # oracle's FP64 back-projection of the GPU multipliers
        kkt_notconv = run(ctx, 1)
        lam = ctx.multipliers()
        q1, qd1 = ctx.state()
        dres = ctx.residual() if st["n_graph"] == 0 or kkt_notconv is None else None
        qo, qdo, diag = s.finish(h, q_n, qd_n, lam)
        kkt = {"rho_p": float(diag[oracle.RHO_P]), "rho_d": float(diag[oracle.RHO_D]),
               "kkt": float(diag[oracle.KKT]),
               "state_rel_err": float(np.abs(q1 - qo).max() / max(1.0, np.abs(qo).max())),
               "vel_rel_err": float(np.abs(qd1 - qdo).max() / max(1e-300, np.abs(qdo).max())),
               "pcg_not_converged": kkt_notconv,
               "device_residual": dres}
    if not args.no_cpu_baseline:
        network = bool(st0["n_graph"] or st0["n_loop"])
        cpu = cpu_baseline(asm, wrench, q_n, qd_n, args.workload,
                           min(args.cpu_sample_bodies, asm.n), args.cpu_sample_steps,
                           body_solve=args.body_solve, network=network, tol=args.kkt_tol,
                           max_iters=args.max_iters)
        print(f"# cpu baseline {cpu}", file=sys.stderr, flush=True)
        # (networks: the oracle's direct solvers are dense, so no full step)
        if kkt is not None and asm.n <= 2_000_000 and not network:
            # the oracle's own full step from the same state: the KKT residual
            # its direct FP64 solve reaches there
            qo1, qdo1, lam_o, diag_o = s.step(h, q_n, qd_n)
            kkt["oracle_rho_p"] = float(diag_o[oracle.RHO_P])
            kkt["oracle_rho_d"] = float(diag_o[oracle.RHO_D])
            kkt["oracle_kkt"] = float(diag_o[oracle.KKT])
            kkt["state_rel_err_vs_oracle_solve"] = float(
                np.abs(q1 - qo1).max() / max(1.0, np.abs(qo1).max()))
    if kkt is not None:
        print(f"# kkt check {kkt}", file=sys.stderr, flush=True)

    out = {
        "metric": "body-steps/sec at fixed KKT residual (plain FP64 vs chosen form), 1M-link chain",
        "value": round(value, 1), "unit": "body-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "gpu_ms_per_step": round(gpu_ms / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if chosen == 0 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "bodies": asm.n, "dynamic_bodies": n_dyn,
                   "joints": asm.m, "h": h, "newton_iters": 1, "wrenches": bool(args.wrenches),
                   "body_solve": args.body_solve, "path_solver": args.path_solver,
                   "form": FORMS[chosen], "graph_replay": bool(st["graph_replay"]),
                   "chain_tile_threads": st["tile_threads"],
                   "chain_tiles_packed": bool(st["tile_packed"])},
        "repeats": {"count": max(1, args.repeats), "statistic": "median",
                    "restart_from_initial_state": restart,
                    "walls_ms": res["walls_ms"]},
        "forms": {FORMS[k]: {"ms_per_step": round(v["wall"] * 1e3 / args.steps, 4),
                             "body_steps_per_s": round(n_dyn * args.steps / v["wall"], 1),
                             **({"ir_sweeps_last_step": v["stats"]["ir_sweeps"],
                                 "device_kkt_last_step": v["stats"]["kkt"],
                                 "ir_tol": args.ir_tol} if k == 1 else {})}
                  for k, v in forms.items()},
        "kkt": kkt, "roofline": roof, "cpu_baseline": cpu,
    }
    if st["n_graph"]:
        out["pcg"] = {"iters_last_step": st["pcg_iters"], "rel_residual_last_step": st["rho_d"],
                      "kkt_tol": args.kkt_tol, "max_iters": args.max_iters,
                      "not_converged": notconv}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
