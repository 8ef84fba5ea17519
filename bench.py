#!/usr/bin/env python3
"""Benchmark: GTEPS to the least fixpoint of one energy game on one MI355X.

Headline workload (the default --config rmat): the R-MAT scale-22 game (n =
4,194,304, edge factor 16, (a,b,c,d) = (.57,.19,.19,.05), every sink given one
0-weight self-loop, weights uniform in [-10000, 10000], owners Bernoulli(0.5),
int64 values, seed 3).  Synthetic, seeded input: the paper's instances are not
available.

A step is one exact solve of the resident game to the least fixpoint
(eg_solve: init, TOP seeding passes, every round, result conversion and the
copy of the n credits to the host) with TOP seeding on (--mode seeded; the
plain iteration needs on the order of n rounds on this game).  value = relaxed
edges over the K timed steps / their wall time / 1e9; ms_per_step is the time
to solution.  Every step must return the same credits.

Also reported (each leg once, after the timed steps, each under a time cap):
  roofline      the round kernels of the timed steps: their algorithmic bytes
                over their device time (HIP events on the solve's stream),
                against the 8 TB/s HBM peak; `traffic` from the committed
                rocprofv3 counter table when it was taken on the current kernels;
  step_parts    where a step's time goes: seeding passes, round kernels, the
                rest (init, host sync, result copy);
  rmat_lift     full-frontier lift rounds of the same game from its least
                fixpoint (every vertex lifted, none changes: the lift alone;
                all-vertex rounds where the shape allows them), against the
                HBM roofline, in place (cut tiles), per-XCD sliced and
                slice-major; and player 0's strategy kernel;
  work_options  the same seeded solve with the player-1 frontier filter and
                with the component schedule: rounds, lifts, time, credits;
  uniform       the uniform random game (n = 2^20, out-degree 16, weights in
                [-1000, 1000], seed 2): one plain solve to the fixpoint (no
                seeding) and one seeded solve, credits compared;
  serving       the first --serve-games (32) games of the serving stream (n
                log-uniform in [1e3, 1e5], out-degree U{2..16}, W log-uniform in
                [10, 1000]), TOP seeding on: one-game-at-a-time solves, the
                batched server's closed-loop capacity under an HBM budget of a
                quarter of the games' footprints (all games, and the typical
                ones that solve alone within 0.5 s), Poisson arrivals at 0.8x that
                capacity and at 1.2x (overload) with p50/p99 latency (arrival to
                result), and whether every game's credits are the same alone
                and in each mix;
  cpu_baseline  the CPU oracle (sequential FIFO worklist, one thread) on the
                same game: its relaxed edges per second over a bounded sample
                of lifts (about --cpu-seconds of work), with the host's core
                count and CPU model.

Flags: --gpus N (only 1 is supported: the solver runs on one GPU), --steps K,
--warmup W, --config {rmat,uniform,plain,torus}, --mode {seeded,plain},
--no-cpu-baseline, --cpu-seconds S (length of the oracle's sample, default
15), --serve-games G (0 = no serving report), --shape k=v,... (launch-shape
fields overriding the tuned ones), --no-uniform, --no-rmat-lift,
--rmat-sweeps R (full-frontier rounds timed per launch shape), --budget-s T
(wall-clock cap of the legs after the timed steps: a leg that would start
later is skipped and named in `skipped`), --max-rounds M (profiling only:
stops each solve after M rounds; the line is then marked partial); for
profiling, --rmat-only and --serving-only run one leg and print its JSON,
--no-legs stops after the timed steps, and --copy-calibration only copies
1 GiB three times (the counter scale).
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
T_START = time.perf_counter()


def log(*a):
    print(f"[bench {time.perf_counter() - T_START:7.1f}s]", *a, file=sys.stderr, flush=True)


DESC = {
    "rmat": "R-MAT scale 22, edge factor 16, (.57,.19,.19,.05), sink 0-self-loops, weights in [-10000,10000], "
            "owners Bernoulli(0.5), seed 3",
    "uniform": "uniform random game: n=1048576, out-degree 16, weights in [-1000,1000], owners Bernoulli(0.5), seed 2",
    "plain": "plain game: n=1000, out-degree 4, weights in [-10,10], owners Bernoulli(0.5), seed 1",
    "torus": "2048x2048 directed torus, weights in [-100,100]+2, owners Bernoulli(0.5), seed 4",
}


def make_game(name):
    from paper_1710_03647_amd import synth

    gen = {"rmat": synth.gen_rmat_full, "uniform": synth.gen_uniform_full, "plain": synth.gen_plain,
           "torus": synth.gen_torus_full}
    if name not in gen:
        raise SystemExit(f"unknown config {name}")
    t0 = time.perf_counter()
    g = gen[name]()
    log(f"generated {name}: n={g.n} m={g.m} in {time.perf_counter() - t0:.1f} s")
    return g, DESC[name]


def kernel_hash():
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def traffic_for(key):
    """HBM bytes per launch from the committed counter table, if it was taken on
    the current kernel source (else None)."""
    if not os.path.exists(TRAFFIC):
        return None
    try:
        t = json.load(open(TRAFFIC))
    except ValueError:
        return None
    e = t.get(key)
    if not e or e.get("kernel_sha") != kernel_hash():
        return None
    return e.get("bytes_per_launch")


def host_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return os.cpu_count() or 0, model


def cpu_baseline(game, seconds):
    """The oracle's relaxed edges per second over a bounded sample: two runs with
    different lift budgets, so that the predecessor-list build and the set-up
    (in both) cancel out of the rate."""
    from oracle import oracle

    oracle.build()
    small = 100_000
    t0 = time.perf_counter()
    a = oracle.solve(game, max_lifts=small)
    t_a = time.perf_counter() - t0
    # a first guess of the rate from the small run, refined by a second probe
    probe = 20 * small
    t0 = time.perf_counter()
    b = oracle.solve(game, max_lifts=probe)
    t_b = time.perf_counter() - t0
    rate = (b.lifts - a.lifts) / max(t_b - t_a, 1e-3)
    lifts = max(probe, int(rate * seconds))
    t0 = time.perf_counter()
    r = oracle.solve(game, max_lifts=lifts)
    t_r = time.perf_counter() - t0
    edges = r.relaxed_edges - a.relaxed_edges
    dt = max(t_r - t_a, 1e-6)
    cores, model = host_info()
    done = "to the fixpoint" if r.status == 0 else f"its first {r.lifts} lifts"
    return {"value": edges / dt / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "host_cores": cores, "cpu_model": model,
            "sample": f"sequential FIFO worklist (one thread) on the same game, {done}: {edges} relaxed edges in "
                      f"{dt:.1f} s beyond its first {a.lifts} lifts (set-up and predecessor lists excluded by "
                      f"differencing). The oracle follows one FIFO order of single lifts; the device runs "
                      f"rounds with TOP seeding, so the two do different amounts of work to the fixpoint and "
                      f"this rate is context, not a like-for-like time"}


def poisson_run(ctx, synth, games, rate):
    """Submit `games` at Poisson arrivals of `rate` games/s; per-game latency
    (arrival to result), the wall time until the last result, the credits."""
    arrivals = synth.poisson_arrivals(len(games), rate)
    t0 = time.perf_counter()
    tickets = []
    for g, a in zip(games, arrivals):
        d = a - (time.perf_counter() - t0)
        if d > 0:
            time.sleep(d)
        tickets.append(ctx.submit(g))
    lat, outs = [], []
    for g, t in zip(games, tickets):
        rc, f, st = ctx.wait(t, g.n)
        lat.append(st["t_latency"])
        outs.append(f)
    return lat, time.perf_counter() - t0, outs


def closed_loop(eg, ctx, games, alone):
    """Every game submitted at once, every result awaited: wall time, games
    that waited for admission, whether each result equals the game's alone."""
    import numpy as np

    t0 = time.perf_counter()
    tickets = [ctx.submit(g) for g in games]
    queued, same = 0, True
    for g, t, a in zip(games, tickets, alone):
        rc, f, st = ctx.wait(t, g.n)
        same &= bool(np.array_equal(f, a))
        queued += st["t_queue"] > 1e-3
    return time.perf_counter() - t0, queued, same


def serving_report(eg, synth, count):
    """One-at-a-time vs batched serving on the first `count` stream games, both
    with TOP seeding; the HBM budget of the server is a quarter of the games'
    summed footprints (at least three times the largest one), so admission
    waits for memory.  Closed loop on all of them and on the typical ones
    (those that solve alone within 0.5 s: a slow trap's time is its own serial
    rounds, whatever it shares the device with); Poisson arrivals at 0.8x the
    closed-loop capacity, and an overload run at 1.2x; every game's credits
    compared alone and in each mix."""
    import numpy as np

    from paper_1710_03647_amd import tune

    games = [synth.gen_stream_game(i) for i in range(count)]
    feet = [eg.check(g)["device_bytes"] for g in games]
    need = sum(feet)
    serve_shape = tune.serving_config()
    # the server's footprint of a game also holds its upload and seeding scratch
    budget_bytes = max(need // 4, 3 * max(feet))
    alone, t_alone = [], []
    with eg.Context(0, top_seeding=1) as ctx:
        for i, g in enumerate(games):
            t0 = time.perf_counter()
            with ctx.create(g) as h:
                alone.append(h.solve()[0].copy())
            t_alone.append(time.perf_counter() - t0)
            if i % 8 == 7:
                log(f"serving: {i + 1} of {count} games solved one at a time ({sum(t_alone):.1f} s)")
    t_one = sum(t_alone)
    typical = [i for i, t in enumerate(t_alone) if t <= 0.5]
    t_one_typ = sum(t_alone[i] for i in typical)
    log(f"serving: one at a time {count / t_one:.2f} games/s ({t_one:.1f} s); {len(typical)} typical games "
        f"{len(typical) / t_one_typ:.2f} games/s")
    res = {"games": count, "workload": f"first {count} games of the serving stream (seed 5)",
           "mode": "TOP seeding on, one at a time (eg_solve) and served (eg_submit)",
           "hbm_budget_bytes": budget_bytes, "footprint_sum_bytes": need, "server_shape": serve_shape,
           "one_at_a_time_games_per_s": count / t_one,
           "slow_games": {i: round(t, 2) for i, t in enumerate(t_alone) if t > 0.5}}
    with eg.Context(0, hbm_budget_bytes=budget_bytes, top_seeding=1, **serve_shape) as ctx:
        t_cap, queued, same = closed_loop(eg, ctx, games, alone)
        cap = count / t_cap
        log(f"serving: batched closed loop {cap:.2f} games/s ({t_cap:.1f} s), {queued} waited for admission")
        tg = [games[i] for i in typical]
        t_typ, queued_typ, same_typ = closed_loop(eg, ctx, tg, [alone[i] for i in typical])
        same &= same_typ
        log(f"serving: typical games batched {len(tg) / t_typ:.2f} games/s against {len(tg) / t_one_typ:.2f} "
            f"one at a time")
        rate = 0.8 * cap
        lat, t_poi, outs = poisson_run(ctx, synth, games, rate)
        same &= all(np.array_equal(f, a) for f, a in zip(outs, alone))
        log(f"serving: Poisson run done ({t_poi:.1f} s)")
        lat_o, t_over, outs = poisson_run(ctx, synth, games, 1.2 * cap)
        same &= all(np.array_equal(f, a) for f, a in zip(outs, alone))
    res.update({"batched_capacity_games_per_s": cap, "closed_loop_games_waiting_for_admission": queued,
                "batched_vs_one_at_a_time": cap / (count / t_one),
                "typical_games": len(tg),
                "typical_one_at_a_time_games_per_s": len(tg) / t_one_typ,
                "typical_batched_games_per_s": len(tg) / t_typ,
                "typical_batched_vs_one_at_a_time": (len(tg) / t_typ) / (len(tg) / t_one_typ),
                "typical_games_waiting_for_admission": queued_typ,
                "poisson_rate_per_s": rate, "poisson_games_per_s": count / t_poi,
                "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
                "overload_rate_per_s": 1.2 * cap, "overload_games_per_s": count / t_over,
                "overload_p50_latency_s": float(np.percentile(lat_o, 50)),
                "overload_p99_latency_s": float(np.percentile(lat_o, 99)),
                "alone_equals_mix": same})
    log(f"serving: Poisson {rate:.2f}/s -> p50 {res['p50_latency_s']:.3f} s, p99 {res['p99_latency_s']:.3f} s; "
        f"overload {1.2 * cap:.2f}/s -> p50 {res['overload_p50_latency_s']:.3f} s, "
        f"p99 {res['overload_p99_latency_s']:.3f} s; alone == mix: {same}")
    return res


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
    log(f"strategy: {t * 1e6:.1f} us, {scanned} edges scanned, {gbps:.0f} GB/s = {gbps / HBM_PEAK_GBPS:.3f} of peak")
    return {"us": t * 1e6, "player0_choices": int(np.sum(choice >= 0)), "edges_scanned": scanned,
            "model_bytes": nbytes, "achieved": gbps, "frac": gbps / HBM_PEAK_GBPS}


def lift_sweeps(eg, game, fstar, stream, shape, sweeps):
    """Full-frontier rounds from the least fixpoint in one launch shape: each is
    one round kernel with every vertex active and no value changing."""
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
            strat = strategy_timing(g, game) if not shape.get("partition") and shape.get("hub_cache", 0) >= 0 else None
    us = kt / sweeps * 1e6
    gbps = mb / kt / 1e9
    return {"us_per_round": us, "model_bytes_per_round": mb / sweeps, "achieved": gbps,
            "frac": gbps / HBM_PEAK_GBPS, "shape": shape}, strat


def rmat_lift_leg(eg, game, fstar, stream, base, sweeps):
    """Full-frontier lift rounds of the R-MAT scale-22 game: every vertex is
    lifted from the least fixpoint, so nothing changes and the round is the
    lift alone (edge stream, gathers of f, reductions), against the HBM
    roofline: in place (cut tiles, with and without the LDS copy of the
    hubs), per-XCD sliced and slice-major, in the tuned occupancy."""
    res = {"workload": "R-MAT scale 22, edge factor 16: full-frontier lift rounds from the least fixpoint (every "
                       "vertex lifted, none changes), int64 values", "n": game.n, "m": game.m}
    for label, over in (("in_place", {"partition": 0}), ("in_place_no_hub_cache", {"partition": 0, "hub_cache": -1}),
                        ("sliced", {"partition": 2}), ("slice_major", {"partition": 3})):
        r, strat = lift_sweeps(eg, game, fstar, stream, dict(base, **over), sweeps)
        res[label] = r
        if strat:
            res["strategy"] = strat
        log(f"rmat lift ({label}): {r['us_per_round']:.1f} us per round, {r['achieved']:.0f} GB/s = "
            f"{r['frac']:.3f} of peak")
    return res


def work_options_leg(eg, game, want, stream, shape):
    """The options that change the work and never the credits, on the R-MAT
    game with TOP seeding: the player-1 frontier filter (Alg. 1's predecessor
    test) and the component schedule (Sec. 6's refinement), each against the
    plain seeded solve: rounds, lifts, scanned predecessors, device time, and
    whether the credits are the same."""
    import numpy as np

    out = {}
    for label, over in (("seeded", {}), ("p1_filter", {"p1_filter": 1}), ("scc_schedule", {"scc_schedule": 1})):
        with eg.Context(0, stream=stream, top_seeding=1, **dict(shape, **over)) as ctx:
            with ctx.create(game) as g:
                f, st, _ = g.solve()  # the component schedule finds the components here
                f, st, _ = g.solve()
        out[label] = {"rounds": st["rounds"], "lifts": st["lifts"], "scanned_preds": st["scanned_preds"],
                      "filtered_preds": st["filtered_preds"], "t_solve_ms": st["t_solve"] * 1e3,
                      "identical": bool(np.array_equal(f, want))}
        if label == "scc_schedule":
            out[label].update({"components": st["scc_components"], "levels": st["scc_levels"]})
        log(f"work options ({label}): {st['t_solve'] * 1e3:.2f} ms, {st['rounds']} rounds, {st['lifts']} lifts, "
            f"identical {out[label]['identical']}")
    return out


def uniform_leg(eg, stream, budget_s):
    """The uniform game: one plain solve to the fixpoint and one seeded solve."""
    import numpy as np

    from paper_1710_03647_amd import synth, tune

    game = synth.gen_uniform_full()
    shape = tune.config_for(game)
    out = {"workload": DESC["uniform"], "n": game.n, "m": game.m}
    with eg.Context(0, stream=stream, time_budget_s=budget_s, **shape) as ctx:
        with ctx.create(game) as g:
            t0 = time.perf_counter()
            f_plain, st, rc = g.solve(allow_timeout=True)
            wall = time.perf_counter() - t0
    out["plain"] = {"finished": rc == eg.EG_OK, "wall_s": wall, "t_solve_s": st["t_solve"], "rounds": st["rounds"],
                    "relaxed_edges": st["relaxed_edges"], "gteps": st["relaxed_edges"] / wall / 1e9,
                    "round_kernel_gbps": st["model_bytes"] / max(st["t_round_kernels"], 1e-9) / 1e9}
    log(f"uniform plain: {wall:.2f} s, {st['rounds']} rounds, {out['plain']['gteps']:.1f} GTEPS, finished {rc == 0}")
    with eg.Context(0, stream=stream, top_seeding=1, **shape) as ctx:
        with ctx.create(game) as g:
            g.solve()
            t0 = time.perf_counter()
            f_seed, st, rc = g.solve()
            wall = time.perf_counter() - t0
    out["seeded"] = {"wall_s": wall, "t_solve_s": st["t_solve"], "rounds": st["rounds"], "seeded": st["seeded"],
                     "identical_to_plain": bool(np.array_equal(f_seed, f_plain)) if out["plain"]["finished"] else None}
    log(f"uniform seeded: {wall * 1e3:.2f} ms, {st['rounds']} rounds, identical {out['seeded']['identical_to_plain']}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="rmat")
    ap.add_argument("--mode", default="seeded", choices=["seeded", "plain"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--serve-games", type=int, default=32)
    ap.add_argument("--shape", default="", help="launch-shape overrides, e.g. blocks_per_cu=4")
    ap.add_argument("--no-uniform", action="store_true")
    ap.add_argument("--no-rmat-lift", action="store_true")
    ap.add_argument("--rmat-sweeps", type=int, default=10)
    ap.add_argument("--budget-s", type=float, default=420.0)
    ap.add_argument("--max-rounds", type=int, default=0)
    ap.add_argument("--no-legs", action="store_true",
                    help="only the timed steps and their line (profiling the headline kernels)")
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

    from paper_1710_03647_amd import eg, synth, tune

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
        print(json.dumps({"serving": serving_report(eg, synth, args.serve_games)}), flush=True)
        return

    game, desc = make_game(args.config)
    info = eg.check(game)
    shape = tune.config_for(game)
    for kv in filter(None, args.shape.split(",")):
        k, v = kv.split("=")
        if k not in tune.DEFAULTS:
            raise SystemExit(f"unknown launch-shape field {k}")
        shape[k] = int(v)
    seeded = args.mode == "seeded"
    log(f"{desc}: bound={info['bound']} value_bits={info['value_bits']}; launch shape {shape}; mode {args.mode}")
    if args.rmat_only:
        fstar = None
        with eg.Context(0, stream=stream, top_seeding=1, **shape) as c:
            with c.create(game) as g:
                fstar = g.solve()[0].copy()
        print(json.dumps({"rmat_lift": rmat_lift_leg(eg, game, fstar, stream, shape, args.rmat_sweeps)}), flush=True)
        return

    ctx = eg.Context(0, stream=stream, top_seeding=1 if seeded else 0, **shape)
    with ctx.create(synth.gen_plain()) as g0:  # kernels loaded once, untimed
        g0.solve()
    t0 = time.perf_counter()
    g = ctx.create(game)
    log(f"create: {time.perf_counter() - t0:.2f} s (upload {g.create_stats['t_upload'] * 1e3:.1f} ms, "
        f"reverse CSR {g.create_stats['t_rcsr'] * 1e3:.1f} ms, sliced copy {g.create_stats['t_slices'] * 1e3:.1f} ms)")
    # pinned host memory for the credits (the caller's choice of buffer: the
    # device-to-host copy then runs at full PCIe rate); one buffer per timed
    # step (up to KEEP), so that the steps are compared with the warm-up's
    # credits after the timed region
    KEEP = 32
    outs = [torch.empty(game.n, dtype=torch.int64, pin_memory=True).numpy()
            for _ in range(max(1, min(args.steps, KEEP)))]
    out = outs[0]
    first = None
    partial = bool(args.max_rounds)

    def step(buf):
        f, st, rc = g.solve(out=buf, max_rounds=args.max_rounds, allow_timeout=partial)
        return st

    for i in range(args.warmup):
        st = step(out)
        if first is None:
            first = out.copy()
        log(f"warmup {i}: t_solve {st['t_solve'] * 1e3:.2f} ms, rounds {st['rounds']}")
    torch.cuda.synchronize()
    keys = ("relaxed_edges", "rounds", "t_round_kernels", "launched_rounds", "model_bytes", "lifts", "t_seed",
            "t_solve", "t_d2h", "seeded")
    agg = {k: 0 for k in keys}
    t0 = time.perf_counter()
    for i in range(args.steps):
        st = step(outs[i % len(outs)])
        for k in keys:
            agg[k] += st[k]
        log(f"step {i}: t_solve {st['t_solve'] * 1e3:.2f} ms (seeding {st['t_seed'] * 1e3:.2f}, round kernels "
            f"{st['t_round_kernels'] * 1e3:.2f}), rounds {st['rounds']}, relaxed edges {st['relaxed_edges']}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # every kept step's credits against the first solve's (the last KEEP steps
    # when there are more)
    if first is None:
        first = outs[0].copy()
    same = partial or all(bool(np.array_equal(o, first)) for o in outs[:min(args.steps, len(outs))])
    steps = max(1, args.steps)

    value = agg["relaxed_edges"] / wall / 1e9
    achieved = agg["model_bytes"] / agg["t_round_kernels"] / 1e9 if agg["t_round_kernels"] else 0.0
    traffic = traffic_for(f"{args.config}-{args.mode}")
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32" if info["value_bits"] == 32 else "int64",
        "data": "synthetic",
        "config": {"workload": desc, "n": game.n, "m": game.m, "W": game.W, "bound": info["bound"],
                   "mode": ("exact solve to the least fixpoint with TOP seeding (seeding time included), "
                            "credits copied to the host" if seeded else
                            "exact solve to the least fixpoint (plain iteration), credits copied to the host"),
                   "rounds_per_step": agg["rounds"] / steps, "seeded_vertices_per_step": agg["seeded"] / steps,
                   "launch_shape": shape},
        "steps_identical": same,
        "step_parts_ms": {"seeding": agg["t_seed"] / steps * 1e3,
                          "round_kernels": agg["t_round_kernels"] / steps * 1e3,
                          "device_solve": agg["t_solve"] / steps * 1e3,
                          "result_copy": agg["t_d2h"] / steps * 1e3},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": "round kernels of the timed solves (one launch per round)",
                     "launches_per_step": agg["launched_rounds"] / steps,
                     "bytes_per_launch": agg["model_bytes"] / max(1, agg["launched_rounds"]),
                     "us_per_launch": agg["t_round_kernels"] / max(1, agg["launched_rounds"]) * 1e6},
    }
    if partial:
        line["partial"] = f"solves stopped after {args.max_rounds} rounds (profiling run)"
    log(f"headline: {value:.2f} GTEPS, {wall / steps * 1e3:.2f} ms per step, roofline {achieved:.0f} GB/s "
        f"({achieved / HBM_PEAK_GBPS:.3f})")
    g.destroy()
    ctx.close()

    if args.no_legs:
        line["skipped"] = ["all legs (--no-legs)"]
        print(json.dumps(line), flush=True)
        return
    skipped = []
    t_legs = time.perf_counter()

    def within(name, need_s):
        left = args.budget_s - (time.perf_counter() - t_legs)
        if left < need_s:
            skipped.append(name)
            log(f"skipping {name}: {left:.0f} s left of the legs' budget")
            return False
        return True

    if not partial and args.config == "rmat" and not args.no_rmat_lift and within("rmat_lift", 30):
        line["rmat_lift"] = rmat_lift_leg(eg, game, first, stream, shape, args.rmat_sweeps)
    if not partial and args.config == "rmat" and args.mode == "seeded" and within("work_options", 30):
        line["work_options"] = work_options_leg(eg, game, first, stream, shape)
    if not partial and not args.no_uniform and args.config != "uniform" and within("uniform", 150):
        line["uniform"] = uniform_leg(eg, stream, budget_s=100.0)
    if args.serve_games and not partial and within("serving", 120):
        line["serving"] = serving_report(eg, synth, args.serve_games)
    if not args.no_cpu_baseline and within("cpu_baseline", 3 * args.cpu_seconds):
        line["cpu_baseline"] = cpu_baseline(game, args.cpu_seconds)
    if skipped:
        line["skipped"] = skipped
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
