"""Training and evaluation of the learned PCG warm start (warm_start = 2).

    python -m paper_2603_08079_amd.gnn_train train --out w.bin [--n 2000 --seeds 0-19 --steps 10]
    python -m paper_2603_08079_amd.gnn_train eval --weights w.bin [--n 2000 --seeds 100-104 --steps 5]
    python -m paper_2603_08079_amd.gnn_train budget --weights w.bin [--n 100000 --seed 100 --iters 3000]

Workload: seeded random geometric graphs of 0.2 m cubes (ball joints to at
most 4 nearest neighbours within 1.5 m, 1 % pinned, body density of 100,000
bodies in a 50 m cube).  `train` steps each training seed with previous-step
PCG starts and, before every step, runs Adam on the energy loss of that
step's dual system; the weights carry over from seed to seed.  `eval`
reports PCG iterations and time to the tolerance for cold, previous-step and
learned starts on held-out seeds; `budget` compares the residual each start
reaches after a fixed number of iterations (for sizes where the tolerance is
out of reach).  Everything runs in the library on the GPU; this script only
drives it and prints one JSON line per command.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

import mabd_inputs as mi
import paper_2603_08079_amd as pk

MODES = {0: "cold", 1: "previous", 2: "learned"}


def _seeds(spec: str):
    out = []
    for part in spec.split(","):
        if "-" in part:
            a, b = part.split("-")
            out += list(range(int(a), int(b) + 1))
        else:
            out.append(int(part))
    return out


def _step(ctx, h):
    t = time.perf_counter()
    try:
        ctx.step(h, 1)
        ok = True
    except pk.MabdError as e:
        if e.status != pk.ERR_NOT_CONVERGED:
            raise
        ok = False
    return ok, time.perf_counter() - t


def train(args):
    params = None
    log = []
    t0 = time.perf_counter()
    for seed in _seeds(args.seeds):
        asm = mi.rgg(args.n, seed=seed)
        ctx = pk.Context(asm, warm_start=1, kkt_tol=args.tol, max_iters=args.max_iters)
        if params is None:
            ctx.gnn_init(args.init_seed)
        else:
            ctx.gnn_params(set_to=params)
        for s in range(args.steps):
            l0, l1 = ctx.gnn_train(asm.h, args.iters, args.lr)
            ok, dt = _step(ctx, asm.h)
            st = ctx.stats()
            log.append({"seed": seed, "step": s, "loss_before": l0, "loss_after": l1,
                        "pcg_iters": st["pcg_iters"], "converged": ok})
            print(f"# seed {seed} step {s}: loss {l0:.4f} -> {l1:.4f}, pcg {st['pcg_iters']} "
                  f"({dt * 1e3:.0f} ms)", file=sys.stderr, flush=True)
            if not ok:
                break
        params = ctx.gnn_params()
        ctx.gnn_save(args.out)
        ctx.close()
    print(json.dumps({"command": "train", "n": args.n, "seeds": args.seeds, "steps": args.steps,
                      "iters_per_step": args.iters, "lr": args.lr, "tol": args.tol,
                      "seconds": round(time.perf_counter() - t0, 1), "weights": args.out,
                      "first_loss": log[0]["loss_before"] if log else None,
                      "last_loss": log[-1]["loss_after"] if log else None}), flush=True)


def evaluate(args):
    rows = {m: [] for m in MODES.values()}
    times = {m: [] for m in MODES.values()}
    acc = []
    for seed in _seeds(args.seeds):
        asm = mi.rgg(args.n, seed=seed)
        for mode, name in MODES.items():
            ctx = pk.Context(asm, warm_start=mode, kkt_tol=args.tol, max_iters=args.max_iters)
            if mode == 2:
                ctx.gnn_load(args.weights)
            for s in range(args.steps):
                ok, dt = _step(ctx, asm.h)
                st = ctx.stats()
                rows[name].append(st["pcg_iters"] if ok else None)
                times[name].append(dt)
                if mode == 2:
                    acc.append(st["warm_accepted"])
                print(f"# seed {seed} {name} step {s}: {st['pcg_iters']} iterations, "
                      f"{dt * 1e3:.0f} ms, converged {ok}", file=sys.stderr, flush=True)
                if not ok:
                    break
            ctx.close()

    def summary(name):
        it = [x for x in rows[name] if x is not None]
        return {"steps": len(rows[name]), "not_converged": sum(x is None for x in rows[name]),
                "mean_iters": float(np.mean(it)) if it else None,
                "mean_iters_first_step": float(np.mean(rows[name][::args.steps])) if it else None,
                "mean_ms": round(1e3 * float(np.mean(times[name])), 2)}

    print(json.dumps({"command": "eval", "n": args.n, "seeds": args.seeds, "steps": args.steps,
                      "tol": args.tol, **{m: summary(m) for m in MODES.values()},
                      "learned_accepted": float(np.mean(acc)) if acc else None}), flush=True)


def budget(args):
    asm = mi.rgg(args.n, seed=args.seed)
    out = {"command": "budget", "n": args.n, "seed": args.seed, "iters": args.iters}
    for mode, name in MODES.items():
        ctx = pk.Context(asm, warm_start=mode, kkt_tol=1e-30, max_iters=args.iters)
        if mode == 2:
            ctx.gnn_load(args.weights)
        res = []
        for s in range(args.steps):
            ok, dt = _step(ctx, asm.h)  # never converges: reports the residual at the cap
            st = ctx.stats()
            res.append(st["rho_d"])
            print(f"# {name} step {s}: residual {st['rho_d']:.3e} after {st['pcg_iters']} "
                  f"iterations ({dt * 1e3:.0f} ms)", file=sys.stderr, flush=True)
        out[name] = res
        ctx.close()
    print(json.dumps(out), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(prog="gnn_train")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--out", required=True)
    t.add_argument("--n", type=int, default=2000)
    t.add_argument("--seeds", default="0-19")
    t.add_argument("--steps", type=int, default=10)
    t.add_argument("--iters", type=int, default=20, help="Adam steps per simulation step")
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--tol", type=float, default=1e-6)
    t.add_argument("--max-iters", type=int, default=200000)
    t.add_argument("--init-seed", type=int, default=0)
    e = sub.add_parser("eval")
    e.add_argument("--weights", required=True)
    e.add_argument("--n", type=int, default=2000)
    e.add_argument("--seeds", default="100-104")
    e.add_argument("--steps", type=int, default=5)
    e.add_argument("--tol", type=float, default=1e-6)
    e.add_argument("--max-iters", type=int, default=200000)
    b = sub.add_parser("budget")
    b.add_argument("--weights", required=True)
    b.add_argument("--n", type=int, default=100000)
    b.add_argument("--seed", type=int, default=100)
    b.add_argument("--iters", type=int, default=3000)
    b.add_argument("--steps", type=int, default=1)
    args = ap.parse_args(argv)
    {"train": train, "eval": evaluate, "budget": budget}[args.cmd](args)


if __name__ == "__main__":
    main()
