#!/usr/bin/env python3
"""Benchmark: GTEPS to the least fixpoint of one energy game on one MI355X.

A step is one eg_solve of the whole game (init, every round to the fixpoint,
result conversion and copy to the host) on a game already resident in device
memory.  value = relaxed edges over the K timed steps / their wall time / 1e9.

The default workload is the uniform random game (n = 2^20, out-degree 16,
weights uniform in [-1000, 1000], owners Bernoulli(0.5), seed 2).  Synthetic,
seeded input: the paper's instances are not available.

Also reported:
  roofline      the round kernels' algorithmic bytes over their device time,
                against the 8 TB/s HBM peak; `traffic` from committed rocprofv3
                counter summaries when they match the current kernel source;
  cpu_baseline  the CPU oracle (sequential FIFO worklist, one core) on a
                bounded sample of the same game: its first lifts, ~15 s of work;
  seeded        the same game solved with TOP seeding (exact; changes the
                work, so it is reported apart from `value`), and whether its
                credits equal the plain solve's;
  rmat_lift     full-frontier lift rounds of the R-MAT scale-22 game (every
                vertex active): round-kernel time and algorithmic bytes
                against the 8 TB/s HBM peak, unsliced and target-sliced;
  serving       the first --serve-games games of the serving stream (n
                log-uniform in [1e3, 1e5], out-degree U{2..16}, W log-uniform in
                [10, 1000]): one-game-at-a-time solves, the batched server's
                closed-loop capacity, and Poisson arrivals at 0.8x that capacity
                and at 1.2x (overload), with p50/p99 latency (arrival to result).

Flags: --gpus N (only 1 is supported: the solver runs on one GPU),
--steps K, --warmup W, --config {uniform,plain,rmat,torus}, --no-cpu-baseline,
--cpu-seconds S (length of the oracle's bounded sample, default 15),
--sweep R (instead of solves: R full-frontier lift rounds from the least
fixpoint, every vertex lifted and none changing),
--max-rounds M (profiling only: stops each solve after M rounds; the line is
then marked partial), --serve-games G (0 = no serving report), --shape k=v,...
(launch-shape fields overriding the tuned ones), --no-seeded, --no-rmat-lift,
--rmat-sweeps R (full-frontier rounds timed per R-MAT variant); for profiling,
--rmat-only and --serving-only run one leg and print its JSON, and
--copy-calibration only copies 1 GiB three times (the counter scale).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "GTEPS to fixpoint (1 game); batched games/sec with p50/p99 latency"
KERNEL_SRC = os.path.join(ROOT, "paper_1710_03647_amd", "csrc", "eg_kernels.hip")
TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_game(name):
    from paper_1710_03647_amd import synth

    if name == "uniform":
        g = synth.gen_uniform_full()
        desc = "uniform random game: n=1048576, out-degree 16, weights uniform in [-1000,1000], owners Bernoulli(0.5), seed 2"
    elif name == "plain":
        g = synth.gen_plain()
        desc = "plain game: n=1000, out-degree 4, weights uniform in [-10,10], owners Bernoulli(0.5), seed 1"
    elif name == "rmat":
        g = synth.gen_rmat_full()
        desc = "R-MAT scale 22, edge factor 16, (.57,.19,.19,.05), sink self-loops, weights in [-10000,10000], seed 3"
    elif name == "torus":
        g = synth.gen_torus_full()
        desc = "2048x2048 directed torus, weights uniform in [-100,100]+2, owners Bernoulli(0.5), seed 4"
    else:
        raise SystemExit(f"unknown config {name}")
    return g, desc


def kernel_hash():
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def traffic_for(config):
    """HBM bytes per round launch from the committed counter summary, if it was
    taken on the current kernel source."""
    if not os.path.exists(TRAFFIC):
        return None
    try:
        t = json.load(open(TRAFFIC))
    except ValueError:
        return None
    e = t.get(config)
    if not e or e.get("kernel_sha") != kernel_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(game, seconds):
    from oracle import oracle

    oracle.build()
    probe = oracle.solve(game, max_lifts=200_000)
    t0 = time.perf_counter()
    probe = oracle.solve(game, max_lifts=200_000)
    dt = time.perf_counter() - t0
    lifts = max(200_000, int(200_000 * seconds / max(dt, 1e-6)))
    t0 = time.perf_counter()
    r = oracle.solve(game, max_lifts=lifts)
    dt = time.perf_counter() - t0
    done = "to the fixpoint" if r.status == 0 else f"its first {r.lifts} lifts"
    return {"value": r.relaxed_edges / dt / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"sequential FIFO worklist on the same game, {done} ({r.relaxed_edges} relaxed edges, "
                      f"{dt:.1f} s, one thread)"}


def poisson_run(ctx, synth, games, rate):
    """Submit `games` at Poisson arrivals of `rate` games/s; per-game latency
    (arrival to result) and the wall time until the last result."""
    arrivals = synth.poisson_arrivals(len(games), rate)
    t0 = time.perf_counter()
    tickets = []
    for g, a in zip(games, arrivals):
        d = a - (time.perf_counter() - t0)
        if d > 0:
            time.sleep(d)
        tickets.append(ctx.submit(g))
    lat = []
    for g, t in zip(games, tickets):
        rc, f, st = ctx.wait(t, g.n)
        lat.append(st["t_latency"])
    return lat, time.perf_counter() - t0


def serving_report(eg, synth, count):
    """One-at-a-time vs batched serving on the first `count` stream games; Poisson
    arrivals at 0.8x the batched closed-loop capacity, and an overload run at 1.2x."""
    import numpy as np

    games = [synth.gen_stream_game(i) for i in range(count)]
    with eg.Context(0) as ctx:
        t0 = time.perf_counter()
        for g in games:
            with ctx.create(g) as h:
                h.solve()
        t_one = time.perf_counter() - t0
    log(f"[bench] serving: one at a time {count / t_one:.2f} games/s ({t_one:.1f} s)")
    res = {"games": count, "workload": f"first {count} games of the serving stream (seed 5)",
           "one_at_a_time_games_per_s": count / t_one}
    with eg.Context(0, hbm_budget_bytes=16 << 30) as ctx:
        t0 = time.perf_counter()
        tickets = [ctx.submit(g) for g in games]
        for g, t in zip(games, tickets):
            ctx.wait(t, g.n)
        t_cap = time.perf_counter() - t0
        cap = count / t_cap
        log(f"[bench] serving: batched closed loop {cap:.2f} games/s ({t_cap:.1f} s)")
        rate = 0.8 * cap
        lat, t_poi = poisson_run(ctx, synth, games, rate)
        lat_o, t_over = poisson_run(ctx, synth, games, 1.2 * cap)
    res.update({"batched_capacity_games_per_s": cap, "poisson_rate_per_s": rate,
                "poisson_games_per_s": count / t_poi,
                "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
                "overload_rate_per_s": 1.2 * cap, "overload_games_per_s": count / t_over,
                "overload_p50_latency_s": float(np.percentile(lat_o, 50)),
                "overload_p99_latency_s": float(np.percentile(lat_o, 99)),
                "batched_vs_one_at_a_time": cap / (count / t_one)})
    log(f"[bench] serving: Poisson {rate:.2f}/s -> p50 {res['p50_latency_s']:.3f} s, p99 {res['p99_latency_s']:.3f} s")
    log(f"[bench] serving: overload {1.2 * cap:.2f}/s -> p50 {res['overload_p50_latency_s']:.3f} s, "
        f"p99 {res['overload_p99_latency_s']:.3f} s")
    return res


def seeded_leg(eg, game, stream, shape, plain_out):
    """The same game solved with TOP seeding (exact: the credits must equal the
    plain solve's bit for bit); reported beside the plain path because it
    changes the work."""
    import numpy as np

    with eg.Context(0, stream=stream, top_seeding=1, **shape) as ctx:
        with ctx.create(game) as g:
            g.solve()  # warm
            f, st, rc = g.solve()
    same = bool(np.array_equal(f, plain_out))
    log(f"[bench] seeded: t_solve {st['t_solve'] * 1e3:.2f} ms, rounds {st['rounds']}, seeded {st['seeded']}, "
        f"identical to the plain solve: {same}")
    return {"t_solve_s": st["t_solve"], "rounds": st["rounds"], "relaxed_edges": st["relaxed_edges"],
            "gteps": st["relaxed_edges"] / st["t_solve"] / 1e9 if st["t_solve"] else None,
            "seeded_vertices": st["seeded"], "seed_passes": st["seed_passes"], "identical_to_plain": same}


def least_fixpoint(eg, game, stream, shape):
    """The credits of `game` from a solve with TOP seeding (exact)."""
    with eg.Context(0, stream=stream, top_seeding=1, **shape) as ctx:
        with ctx.create(game) as g:
            f, st, rc = g.solve()
    return f


def strategy_timing(g, game, reps=5):
    """Player 0's strategy read off the least fixpoint (one kernel), against the
    HBM roofline.  Algorithmic bytes: per vertex its caller-to-internal id, two
    row starts, f(v) and the choice written (4 + 8 + 8 + 4); per edge scanned up
    to the first witness, the {target, weight} pair and f(target) (8 + 8)."""
    import numpy as np

    g.strategy()
    ts = []
    for _ in range(reps):
        choice, t = g.strategy()
        ts.append(t)
    t = min(ts)
    scanned = int(np.sum(choice[choice >= 0].astype(np.int64) + 1))
    nbytes = game.n * 24.0 + scanned * 16.0
    gbps = nbytes / t / 1e9
    log(f"[bench] strategy: {t * 1e6:.1f} us, {scanned} edges scanned, {gbps:.0f} GB/s = {gbps / HBM_PEAK_GBPS:.3f} of peak")
    return {"us": t * 1e6, "player0_choices": int(np.sum(choice >= 0)), "edges_scanned": scanned,
            "model_bytes": nbytes, "achieved": gbps, "frac": gbps / HBM_PEAK_GBPS}


def rmat_lift_leg(eg, stream, sweeps):
    """Full-frontier lift rounds of the R-MAT scale-22 game: every vertex is
    lifted from the least fixpoint, so nothing changes and the round is the
    lift alone (edge stream, gathers of f, reductions), against the HBM
    roofline."""
    from paper_1710_03647_amd import synth, tune

    t0 = time.perf_counter()
    game = synth.gen_rmat_full()
    log(f"[bench] rmat lift: generated R-MAT 22 in {time.perf_counter() - t0:.1f} s")
    res = {"workload": "R-MAT scale 22, edge factor 16: full-frontier lift rounds from the least fixpoint (every "
                       "vertex lifted, none changes), int64 values", "n": game.n, "m": game.m}
    base = tune.config_for(game)
    fstar = least_fixpoint(eg, game, stream, base)
    for label, over in (("unsliced", {}), ("unsliced, tiles not cut", {"seg_edges": -1}),
                        ("sliced", {"partition": 2})):
        shape = dict(base, **over)
        with eg.Context(0, stream=stream, **shape) as ctx:
            with ctx.create(game) as g:
                g.set_measure(fstar)
                for _ in range(2):
                    g.solve(max_rounds=1, resume=True, allow_timeout=True)
                kt = mb = 0.0
                for _ in range(sweeps):
                    f, st, rc = g.solve(max_rounds=1, resume=True, allow_timeout=True)
                    kt += st["t_round_kernels"]
                    mb += st["model_bytes"]
                if not over and rc == eg.EG_OK:
                    res["strategy"] = strategy_timing(g, game)
        us = kt / sweeps * 1e6
        gbps = mb / kt / 1e9
        res[label] = {"us_per_round": us, "model_bytes_per_round": mb / sweeps, "achieved": gbps,
                      "frac": gbps / HBM_PEAK_GBPS, "shape": shape}
        log(f"[bench] rmat lift ({label}): {us:.1f} us per round, {gbps:.0f} GB/s = {gbps / HBM_PEAK_GBPS:.3f} of peak")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--config", default="uniform")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--sweep", type=int, default=0)
    ap.add_argument("--max-rounds", type=int, default=0)
    ap.add_argument("--serve-games", type=int, default=32)
    ap.add_argument("--shape", default="", help="launch-shape overrides, e.g. partition=1,blocks_per_cu=4")
    ap.add_argument("--no-seeded", action="store_true")
    ap.add_argument("--no-rmat-lift", action="store_true")
    ap.add_argument("--rmat-sweeps", type=int, default=10)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB on the device three times (scales the FETCH_SIZE/WRITE_SIZE counters)")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving report and print its JSON")
    ap.add_argument("--rmat-only", action="store_true",
                    help="run only the R-MAT lift and strategy leg and print its JSON (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; the solver runs on one GPU "
              f"(games are independent: several GPUs would serve separate games)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1710_03647_amd import eg

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.int32, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print("copied 3 x 1 GiB", flush=True)
        return
    if args.serving_only:
        from paper_1710_03647_amd import synth as _synth

        print(json.dumps({"serving": serving_report(eg, _synth, args.serve_games)}), flush=True)
        return
    if args.rmat_only:
        print(json.dumps({"rmat_lift": rmat_lift_leg(eg, stream, args.rmat_sweeps)}), flush=True)
        return
    game, desc = make_game(args.config)
    info = eg.check(game)
    log(f"[bench] {desc}: n={game.n} m={game.m} bound={info['bound']} value_bits={info['value_bits']}")

    from paper_1710_03647_amd import tune

    shape = tune.config_for(game)
    for kv in filter(None, args.shape.split(",")):
        k, v = kv.split("=")
        if k not in tune.DEFAULTS:
            raise SystemExit(f"unknown launch-shape field {k}")
        shape[k] = int(v)
    log(f"[bench] launch shape: {shape}")
    ctx = eg.Context(0, stream=stream, **shape)
    # kernels loaded once, untimed (a small game)
    from paper_1710_03647_amd import synth

    with ctx.create(synth.gen_plain()) as g0:
        g0.solve()
    t0 = time.perf_counter()
    g = ctx.create(game)
    log(f"[bench] create: {time.perf_counter() - t0:.2f} s (upload {g.create_stats['t_upload'] * 1e3:.1f} ms, "
        f"reverse CSR {g.create_stats['t_rcsr'] * 1e3:.1f} ms)")
    out = np.empty(game.n, dtype=np.int64)
    partial = bool(args.max_rounds)

    if args.sweep:  # full-frontier rounds from the least fixpoint: the lift alone
        g.set_measure(least_fixpoint(eg, game, stream, shape))

    def step():
        if args.sweep:
            f, st, rc = g.solve(out=out, max_rounds=1, resume=True, allow_timeout=True)
        else:
            f, st, rc = g.solve(out=out, max_rounds=args.max_rounds, allow_timeout=partial)
        return st

    for i in range(args.warmup):
        st = step()
        log(f"[bench] warmup {i}: {st['t_solve']:.3f} s, rounds {st['rounds']}")
    steps = args.sweep or args.steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    agg = dict(relaxed_edges=0, rounds=0, t_round_kernels=0.0, launched_rounds=0, model_bytes=0.0, lifts=0)
    for i in range(steps):
        st = step()
        for k in agg:
            agg[k] += st[k]
        if not args.sweep:
            log(f"[bench] step {i}: t_solve {st['t_solve']:.3f} s, rounds {st['rounds']} "
                f"(dense {st['dense_rounds']}), relaxed edges {st['relaxed_edges']}, "
                f"kernel time {st['t_round_kernels']:.3f} s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    value = agg["relaxed_edges"] / wall / 1e9
    achieved = agg["model_bytes"] / agg["t_round_kernels"] / 1e9 if agg["t_round_kernels"] else 0.0
    traffic = traffic_for(args.config)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32" if info["value_bits"] == 32 else "int64",
        "data": "synthetic",
        "config": {"workload": desc, "n": game.n, "m": game.m, "W": game.W, "bound": info["bound"],
                   "mode": "full-frontier lift rounds" if args.sweep else "solve to fixpoint",
                   "rounds_per_step": agg["rounds"] / steps, "launch_shape": shape},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": "round kernels of the solve (one launch per round; all-vertex dense rounds dominate)",
                     "bytes_per_launch": agg["model_bytes"] / max(1, agg["launched_rounds"]),
                     "us_per_launch": agg["t_round_kernels"] / max(1, agg["launched_rounds"]) * 1e6},
    }
    if partial:
        line["partial"] = f"solves stopped after {args.max_rounds} rounds (profiling run)"
    if not args.sweep and not partial and not args.no_seeded:
        line["seeded"] = seeded_leg(eg, game, stream, shape, out)
    g.destroy()
    ctx.close()
    if not args.sweep and not partial and not args.no_rmat_lift:
        line["rmat_lift"] = rmat_lift_leg(eg, stream, args.rmat_sweeps)
    if args.serve_games and not args.sweep and not partial:
        line["serving"] = serving_report(eg, synth, args.serve_games)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(game, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
