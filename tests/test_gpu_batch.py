"""Batched iteration and serving (continuous batching) against the oracle and
against one-game solves: every game's credits are the same alone and in the
mix, whatever else shares the device."""
import threading
import time

import numpy as np
import pytest

import pins
from paper_1710_03647_amd import eg, synth

pytestmark = pytest.mark.gpu
GiB = 1 << 30


def window_game(n: int, deg: int, seed: int):
    """A game stored with 64-bit values although the device encoding of TOP
    (B + P + 1, P the largest positive weight) is below 2^31: W just above
    2^31 / n and positive weights at most W / 2 put B + P + 1 below 2^31 and
    B + P + 1 + W above it."""
    W = (1 << 31) // n + 1
    g = synth.gen_uniform(n, deg, W, seed, name=f"window-n{n}-s{seed}")
    w = g.w.astype(np.int64)
    g.w = np.where(w > W // 2, w // 4, w).astype(np.int32)
    return g


def int64_games():
    games = [synth.gen_rmat(16, 16, wlim=40000, seed=5), window_game(3, 2, 1), window_game(100, 4, 2),
             window_game(1000, 4, 3), window_game(5000, 6, 4)]
    for g in games:
        info = eg.check(g)
        assert info["value_bits"] == 64, g.name
    return games


def mix_games():
    games = [synth.gen_stream_game(i, scale_n=0.05) for i in range(10)]
    games += [synth.gen_plain(), synth.gen_torus(16, seed=5), synth.gen_rmat(10, 8, wlim=300, seed=9)]
    games += [synth.gen_random_small(900 + i, n_max=7) for i in range(6)]
    games.append(pins.cf8_game(300))
    games += int64_games()
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


def test_int64_games_in_the_batch_match_oracle(oracle_mod):
    """Games stored with 64-bit values, including ones whose TOP encoding fits
    32 bits, run through the epochs and the small mode with their own width."""
    games = int64_games()
    with eg.Context(0, hbm_budget_bytes=2 * GiB) as ctx:
        res = ctx.solve_batch(games)
    for g, (f, st) in zip(games, res):
        pins.expect_equal(f, oracle_mod.solve(g).f, g.name)


def test_destroy_context_cancels_tickets_and_wakes_waiter():
    """eg_ctx_destroy while a thread is blocked in eg_wait on a running game:
    the waiter returns EG_ECANCELED, the pending ticket is cancelled too, and
    the context's live game is freed with it."""
    slow = synth.gen_torus(128, seed=4)  # many seconds of rounds: still running when the context goes
    ctx = eg.Context(0, hbm_budget_bytes=GiB, max_slots=1)
    live = ctx.create(synth.gen_plain())
    t_run = ctx.submit(slow)
    t_wait = ctx.submit(slow)  # no free slot: stays pending
    got = {}

    def waiter(name, t):
        try:
            ctx_handle_wait = ctx.wait(t, slow.n)
            got[name] = ("returned", ctx_handle_wait[0])
        except eg.EgError as e:
            got[name] = ("error", e.code)

    threads = [threading.Thread(target=waiter, args=("running", t_run)),
               threading.Thread(target=waiter, args=("pending", t_wait))]
    for th in threads:
        th.start()
    time.sleep(0.5)
    assert not got, "the slow game finished before the context was destroyed"
    ctx.close()
    for th in threads:
        th.join(timeout=60)
        assert not th.is_alive()
    assert got == {"running": ("error", eg.EG_ECANCELED), "pending": ("error", eg.EG_ECANCELED)}
    assert live.handle is None
    live.destroy()  # a no-op once the context has freed it


def test_submit_device_pointers(oracle_mod):
    import torch

    dev = torch.device("cuda", 0)
    games = [synth.gen_stream_game(i, scale_n=0.05) for i in range(3)]
    with eg.Context(0, hbm_budget_bytes=GiB) as ctx:
        tickets = []
        for game in games:
            arrs = [torch.from_numpy(a).to(dev) for a in (game.off, game.tgt, game.w, game.owner_bits())]
            torch.cuda.synchronize()
            tickets.append(ctx.submit(n=game.n, offsets=arrs[0], targets=arrs[1], weights=arrs[2],
                                      owner_bits=arrs[3], W=game.W, device=True))
            del arrs  # the call copied them
        for game, t in zip(games, tickets):
            rc, f, st = ctx.wait(t, game.n)
            pins.expect_equal(f, oracle_mod.solve(game).f, f"{game.name}: device-pointer submit")


def test_seeded_serving_matches_oracle(oracle_mod):
    """Serving with top_seeding: each admitted game gets a seeding pass before
    its first round; the credits stay the oracle's."""
    games = mix_games()
    with eg.Context(0, hbm_budget_bytes=2 * GiB, max_slots=6, top_seeding=1) as ctx:
        tickets = [ctx.submit(g) for g in games]
        for g, t in zip(games, tickets):
            rc, f, st = ctx.wait(t, g.n)
            pins.expect_equal(f, oracle_mod.solve(g).f, f"{g.name}: seeded serving")
