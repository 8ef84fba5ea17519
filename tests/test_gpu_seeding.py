"""TOP seeding (negative cycles that player 1 can force, set to TOP between
rounds) changes the work, never the credits: every game below is checked
against the oracle with seeding on."""
import numpy as np
import pytest

import pins
from paper_1710_03647_amd import eg, synth

pytestmark = pytest.mark.gpu
TOP = pins.TOP


@pytest.fixture(scope="module")
def sctx():
    c = eg.Context(0, top_seeding=1)
    yield c
    c.close()


def seeded_solve(ctx, game, **kw):
    with ctx.create(game) as g:
        f, st, rc = g.solve(**kw)
    return f, st


def test_seeded_brute_force(sctx):
    pins.pin_brute(lambda g: seeded_solve(sctx, g)[0], count=300, seed0=81_000)


@pytest.mark.parametrize("pin", pins.CLOSED_FORMS, ids=lambda p: p.__name__)
def test_seeded_closed_forms(sctx, pin):
    pin(lambda g: seeded_solve(sctx, g)[0])


SEEDED = [
    ("plain", synth.gen_plain),
    ("uniform-4k", lambda: synth.gen_uniform(1 << 12, 16, 1000, 2)),
    ("uniform-ragged", lambda: synth.gen_uniform(12345, 5, 300, 21)),
    ("uniform-3000-d4", lambda: synth.gen_uniform(3000, 4, 30, 9)),
    ("rmat-12", lambda: synth.gen_rmat(12, 16, seed=3)),
    ("rmat-14", lambda: synth.gen_rmat(14, 16, seed=3)),
    ("rmat-16-int64", lambda: synth.gen_rmat(16, 16, wlim=40000, seed=5)),
    ("torus-48", lambda: synth.gen_torus(48, seed=4)),
]


@pytest.mark.parametrize("name,make", SEEDED, ids=[s[0] for s in SEEDED])
def test_seeded_matches_oracle(sctx, oracle_mod, name, make):
    game = make()
    f, st = seeded_solve(sctx, game)
    pins.expect_equal(f, oracle_mod.solve(game).f, name)
    assert st["seed_passes"] >= 1


def test_seeding_cuts_rounds(sctx, oracle_mod):
    """A game whose TOP vertices must otherwise climb to the bound: seeding
    proves them TOP early, so the solve needs far fewer rounds."""
    game = synth.gen_rmat(14, 16, seed=3)
    want = oracle_mod.solve(game).f
    with eg.Context(0) as plain:
        f0, st0 = seeded_solve(plain, game)
    f1, st1 = seeded_solve(sctx, game)
    pins.expect_equal(f0, want, "plain")
    pins.expect_equal(f1, want, "seeded")
    assert st1["seeded"] > 0
    assert st1["rounds"] * 4 < st0["rounds"]


def test_seeded_resume_and_repeat(sctx, oracle_mod):
    game = synth.gen_torus(32, seed=4)
    want = oracle_mod.solve(game).f
    noise = synth.to_int(synth.draws(5, 2, 0, game.n), 0, 40)
    with sctx.create(game) as g:
        for _ in range(3):
            f, _, _ = g.solve()
            pins.expect_equal(f, want, "repeat")
        g.set_measure(np.minimum(want, noise))
        f, _, _ = g.solve(resume=True)
        pins.expect_equal(f, want, "resume")


def test_negative_self_loop_of_player1_is_seeded(sctx, oracle_mod):
    """A player-1 vertex with a negative self-loop loses whatever else it can
    reach: the first seeding pass sets it to TOP even though another of its
    edges has a larger term (plainly it would climb for about B / 2 rounds)."""
    game = synth.make_game(3, [(0, 0, -1), (0, 1, -100), (1, 2, 0), (2, 2, 0)], [1, 1, 0], W=100)
    f, st = seeded_solve(sctx, game)
    pins.expect_equal(f, oracle_mod.solve(game).f, "player-1 negative self-loop")
    assert f[0] == TOP and st["seeded"] >= 1 and st["rounds"] <= 4
    with eg.Context(0) as plain:
        f0, st0 = seeded_solve(plain, game)
    pins.expect_equal(f0, f, "plain")
    assert st0["rounds"] > 50


def test_seeding_hub_rows(sctx, oracle_mod):
    """Player-1 hubs whose rows are scanned by a whole wave: rows of 33 to
    several thousand edges, chosen edge late in the row, ties on the term."""
    rows = []
    n = 64
    for v in range(n):
        deg = 1 + (v * 97) % 3000 if v % 3 == 0 else 1 + v % 5
        rows.append([((v * 31 + 7 * k) % n, ((k * 13 + v) % 41) - 20) for k in range(deg)])
    edges = [(v, t, w) for v, row in enumerate(rows) for t, w in row]
    owner = [1 if v % 2 == 0 else 0 for v in range(n)]
    game = synth.make_game(n, edges, owner, W=20, name="hub-rows")
    f, st = seeded_solve(sctx, game)
    pins.expect_equal(f, oracle_mod.solve(game).f, "hub rows")


def choice_game(deg, mode):
    """Player-1 vertex 0 with `deg` out-edges, all into vertices that are not
    forced (player 0 with two edges: they never enter sigma1) except a few
    that pin the candidate order of sigma1 (see the caller).  Rows up to 64
    edges are chosen flattened per tile, longer ones a wave per row, and rows
    above 2048 edges in pieces over several blocks."""
    a, b = 1, 2                  # player 1, one edge each back to vertex 0
    fill0 = 3                    # fillers: player 0, two edges each
    nfill = 64
    n = fill0 + nfill
    pa, pb, ps = int(0.6 * deg), int(0.9 * deg), int(0.8 * deg)
    row = []
    for k in range(deg):
        if k == pa and mode == "tie":
            row.append((a, -7))          # term 7, the first of two equal largest terms
        elif k == pb:
            row.append((b, -7))          # term 7 (in "selfloop": the largest term)
        elif k == ps and mode == "selfloop":
            row.append((0, -1))          # negative self-loop, term 1
        else:
            row.append((fill0 + k % nfill, 0))
    edges = [(0, t, w) for t, w in row]
    edges += [(a, 0, -1), (b, 0, 100)]   # 0 -> a -> 0 sums to -8, 0 -> b -> 0 to 93
    for i in range(nfill):
        v = fill0 + i
        edges += [(v, v, 0), (v, fill0 + (i + 1) % nfill, 1)]
    owner = [1, 1, 1] + [0] * nfill
    return synth.make_game(n, edges, owner, W=100, name=f"choice-{mode}-{deg}")


@pytest.mark.parametrize("deg", [50, 1500, 5000, 40000])
@pytest.mark.parametrize("mode", ["tie", "selfloop"])
def test_seeding_candidate_order_in_every_row_path(sctx, oracle_mod, deg, mode):
    """sigma1's order decides what the first pass proves.  "tie": two edges
    share the largest term and only the first (lower index) closes a
    negative cycle, so exactly {0, a} are seeded.  "selfloop": a negative
    self-loop beats an edge with a larger term whose cycle is positive, so
    exactly {0} is seeded.  Every row length path of the choice is used."""
    game = choice_game(deg, mode)
    f, st = seeded_solve(sctx, game)
    pins.expect_equal(f, oracle_mod.solve(game).f, game.name)
    assert st["seeded"] == (2 if mode == "tie" else 1), (game.name, st["seeded"])


def off_choice_cycle_game(fillers=47):
    """Player-1 vertex 0 has a larger first-pass term towards 1 (a player-1
    vertex with a positive self-loop) than towards 2, and 0 -> 2 -> 0 sums to
    -2: player 1 wins from 0 and 2, but the first choice pass follows 0 -> 1
    and sees no negative cycle.  Isolated fillers raise B = (n - 1) W, so
    the plain climb is long."""
    n = 3 + fillers
    edges = [(0, 1, -10), (0, 2, -1), (1, 1, 100), (2, 0, -1)]
    edges += [(v, v, 0) for v in range(3, n)]
    owner = [1, 1, 1] + [0] * fillers
    return synth.make_game(n, edges, owner, W=100, name="off-choice-cycle")


def test_bellman_ford_seeding_finds_a_cycle_off_the_first_choice(oracle_mod):
    """top_seeding = k > 1 runs k Bellman-Ford passes over the forced subgraph
    before reading the cycles off the choice: the pass values make 0 -> 2
    the better edge, so the first seeding pass proves 0 and 2 TOP (Lemma 1),
    where one choice pass proves nothing until later passes at doubling
    round counts."""
    game = off_choice_cycle_game()
    want = oracle_mod.solve(game).f
    assert want[0] == TOP and want[2] == TOP and want[1] == 0
    with eg.Context(0, top_seeding=1) as c1:
        f1, st1 = seeded_solve(c1, game)
    with eg.Context(0, top_seeding=8) as c8:
        f8, st8 = seeded_solve(c8, game)
    pins.expect_equal(f1, want, "one choice pass")
    pins.expect_equal(f8, want, "8 Bellman-Ford passes")
    assert st8["seeded"] >= 2 and st8["seed_passes"] == 1, st8
    assert st8["rounds"] * 8 < st1["rounds"], (st8["rounds"], st1["rounds"])


def test_bellman_ford_seeding_brute_force():
    with eg.Context(0, top_seeding=4) as ctx:
        pins.pin_brute(lambda g: seeded_solve(ctx, g)[0], count=200, seed0=91_000)


@pytest.mark.parametrize("name,make", SEEDED, ids=[s[0] for s in SEEDED])
def test_bellman_ford_seeding_matches_oracle(oracle_mod, name, make):
    game = make()
    with eg.Context(0, top_seeding=6) as ctx:
        f, st = seeded_solve(ctx, game)
    pins.expect_equal(f, oracle_mod.solve(game).f, f"{name} (6 Bellman-Ford passes)")
