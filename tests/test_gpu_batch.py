"""Batched iteration and serving (continuous batching) against the oracle and
against one-game solves: every game's credits are the same alone and in the
mix, whatever else shares the device."""
import time

import numpy as np
import pytest

import pins
from paper_1710_03647_amd import eg, synth

pytestmark = pytest.mark.gpu
GiB = 1 << 30


def mix_games():
    games = [synth.gen_stream_game(i, scale_n=0.05) for i in range(10)]
    games += [synth.gen_plain(), synth.gen_torus(16, seed=5), synth.gen_rmat(10, 8, wlim=300, seed=9)]
    games += [synth.gen_random_small(900 + i, n_max=7) for i in range(6)]
    games.append(pins.cf8_game(300))
    games.append(synth.gen_rmat(12, 16, wlim=40000, seed=5))  # 64-bit values
    return games


def test_solve_batch_matches_oracle(oracle_mod):
    games = mix_games()
    with eg.Context(0, hbm_budget_bytes=2 * GiB) as ctx:
        res = ctx.solve_batch(games)
    for g, (f, st) in zip(games, res):
        pins.expect_equal(f, oracle_mod.solve(g).f, g.name)
        assert st["t_latency"] >= st["t_solve"] >= 0


def test_serving_alone_equals_mix(oracle_mod):
    games = mix_games()
    alone = []
    with eg.Context(0) as ctx:
        for g in games:
            h = ctx.create(g)
            alone.append(h.solve()[0])
            h.destroy()
    with eg.Context(0, hbm_budget_bytes=2 * GiB, max_slots=8) as ctx:
        tickets = []
        for i, g in enumerate(games):
            tickets.append(ctx.submit(g))
            if i % 4 == 3:
                time.sleep(0.002)  # later games arrive while earlier ones run
        for g, t, a in zip(games, tickets, alone):
            rc, f, st = ctx.wait(t, g.n)
            assert rc == eg.EG_OK
            pins.expect_equal(f, a, f"{g.name}: mix vs alone")
            pins.expect_equal(f, oracle_mod.solve(g).f, f"{g.name}: mix vs oracle")


def test_admission_by_footprint(oracle_mod):
    games = [synth.gen_uniform(20000, 6, 50, 100 + i) for i in range(8)]
    need = eg.check(games[0])["device_bytes"]
    # room for about two games at a time: the rest wait for memory
    with eg.Context(0, hbm_budget_bytes=int(3.2 * need), max_slots=16) as ctx:
        tickets = [ctx.submit(g) for g in games]
        for g, t in zip(games, tickets):
            rc, f, st = ctx.wait(t, g.n)
            pins.expect_equal(f, oracle_mod.solve(g).f, g.name)


def test_refuses_game_larger_than_budget():
    g = synth.gen_uniform(200000, 8, 10, 1)
    with eg.Context(0, hbm_budget_bytes=1 << 20) as ctx:
        with pytest.raises(eg.EgError) as ei:
            ctx.submit(g)
        assert ei.value.code == eg.EG_ENOMEM


def test_submit_rejects_invalid_game():
    g = synth.make_game(2, [(0, 1, -3), (1, 0, 1)], [0, 1], W=1)  # W below 3
    with eg.Context(0, hbm_budget_bytes=GiB) as ctx:
        with pytest.raises(eg.EgError) as ei:
            ctx.submit(g)
        assert ei.value.code == eg.EG_EINVAL


def test_cancel_running_and_pending(oracle_mod):
    slow = synth.gen_torus(64, seed=4)  # ~1.7e5 rounds
    quick = synth.gen_plain()
    with eg.Context(0, hbm_budget_bytes=GiB, max_slots=1) as ctx:
        t1 = ctx.submit(slow)
        t2 = ctx.submit(quick)  # waits for the only slot
        t3 = ctx.submit(quick)
        time.sleep(0.2)
        assert ctx.cancel(t2) == eg.EG_OK
        assert ctx.cancel(t1) == eg.EG_OK
        with pytest.raises(eg.EgError) as ei:
            ctx.wait(t1, slow.n)
        assert ei.value.code == eg.EG_ECANCELED
        with pytest.raises(eg.EgError) as ei:
            ctx.wait(t2, quick.n)
        assert ei.value.code == eg.EG_ECANCELED
        rc, f, st = ctx.wait(t3, quick.n)
        pins.expect_equal(f, oracle_mod.solve(quick).f, "after cancellations")
        with pytest.raises(eg.EgError) as ei:
            ctx.poll(t3, quick.n)  # retired
        assert ei.value.code == eg.EG_ENOTFOUND


def test_many_small_games_one_at_a_time_vs_batched(oracle_mod):
    games = [synth.gen_stream_game(i, scale_n=0.02) for i in range(40)]
    with eg.Context(0, hbm_budget_bytes=GiB) as ctx:
        res = ctx.solve_batch(games)
    for g, (f, st) in zip(games, res):
        pins.expect_equal(f, oracle_mod.solve(g).f, g.name)


def test_small_mode_in_the_batch_counts_every_lift(oracle_mod):
    """Games whose active sets shrink finish in the batch's small mode (one
    block, many rounds per launch) beside games still in the epochs: CF8's
    climb keeps its exact lift and change counts, and every game matches the
    oracle."""
    climbs = [pins.cf8_game(k) for k in (5, 400, 3000)]
    others = [synth.gen_torus(24, seed=4), synth.gen_uniform(4000, 8, 100, 7), synth.gen_rmat(11, 16, seed=3)]
    games = climbs + others
    with eg.Context(0, hbm_budget_bytes=2 * GiB) as ctx:
        res = ctx.solve_batch(games)
    for k, (f, st) in zip((5, 400, 3000), res[:3]):
        pins.expect_equal(f, [pins.TOP] + [0] * k, f"CF8 k={k}")
        assert st["changes"] == k + 1 and st["lifts"] == k + 2
    for g, (f, st) in zip(others, res[3:]):
        pins.expect_equal(f, oracle_mod.solve(g).f, g.name)
