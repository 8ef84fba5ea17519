"""Writes credit_goldens.json: the CPU oracle's least fixpoint of larger seeded
instances, for device tests at sizes where re-running the oracle inside a test
would take minutes to an hour.

Only the oracle (``oracle/``) and the input generator (``synth``, which holds
none of the method's arithmetic) are called here; nothing comes from the
device solver.  Each entry is keyed by instance name and records the SHA-256 of
the instance's arrays (so a test can tell that it regenerated the same game),
the SHA-256 of the credits (int64 little-endian, TOP = INT64_MAX), summary
counts, and 64 sampled (vertex, credit) pairs for diagnostics.

Usage:  python tests/golden/make_credit_goldens.py [-jN] [name ...]   (default: all,
        one process per instance up to the CPU count; entries of other names
        are kept)
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor, as_completed

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
OUT = os.path.join(HERE, "credit_goldens.json")


def instances():
    """name -> (generator call as text, zero-argument generator)."""
    from paper_1710_03647_amd import synth

    d = {
        "rmat18": ("synth.gen_rmat(18, 16, seed=3)", lambda: synth.gen_rmat(18, 16, seed=3)),
        "rmat20": ("synth.gen_rmat(20, 16, seed=3)", lambda: synth.gen_rmat(20, 16, seed=3)),
        "uniform16": ("synth.gen_uniform(1 << 16, 16, 1000, 2)", lambda: synth.gen_uniform(1 << 16, 16, 1000, 2)),
        "torus128": ("synth.gen_torus(128, seed=4)", lambda: synth.gen_torus(128, seed=4)),
        "torus256": ("synth.gen_torus(256, seed=4)", lambda: synth.gen_torus(256, seed=4)),
    }
    for i in range(32):
        d[f"stream{i}"] = (f"synth.gen_stream_game({i})", (lambda i=i: synth.gen_stream_game(i)))
    return d


def credits_sha256(f) -> str:
    import numpy as np

    return hashlib.sha256(np.ascontiguousarray(f, dtype="<i8").tobytes()).hexdigest()


def sample_indices(n: int, k: int = 64):
    from paper_1710_03647_amd import synth

    return sorted(set(int(x) for x in synth.to_int(synth.draws(77, 9, 0, k), 0, n - 1)))


def compute(name: str) -> dict:
    import numpy as np

    from oracle import oracle

    call, make = instances()[name]
    game = make()
    t0 = time.perf_counter()
    r = oracle.solve(game)
    dt = time.perf_counter() - t0
    assert r.status == 0
    f = r.f
    top = np.iinfo(np.int64).max
    fin = f[f != top]
    idx = sample_indices(game.n)
    return {"generator": call, "instance_sha256": game.sha256(), "n": int(game.n), "m": int(game.m),
            "W": int(game.W), "bound": int(r.bound), "credits_sha256": credits_sha256(f),
            "top": int(np.sum(f == top)), "finite_max": int(fin.max()) if len(fin) else None,
            "finite_sum": int(fin.sum()), "oracle_lifts": int(r.lifts), "oracle_seconds": round(dt, 1),
            "samples": [[i, int(f[i])] for i in idx]}


def store(name: str, entry: dict) -> None:
    """Merge one entry into the table on disk (several runs may write at once)."""
    import fcntl

    with open(OUT + ".lock", "w") as lk:
        fcntl.flock(lk, fcntl.LOCK_EX)
        table = json.load(open(OUT)) if os.path.exists(OUT) else {}
        table[name] = entry
        tmp = OUT + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
            fh.write("\n")
        os.replace(tmp, OUT)


def main(names, workers=None):
    from oracle import oracle

    oracle.build()
    names = names or list(instances())
    workers = workers or min(len(names), max(1, (os.cpu_count() or 2) - 1))
    with ProcessPoolExecutor(max_workers=workers) as ex:
        futs = {ex.submit(compute, name): name for name in names}
        for fut in as_completed(futs):
            name, entry = futs[fut], fut.result()
            store(name, entry)
            print(f"{name}: n={entry['n']} m={entry['m']} top={entry['top']} oracle {entry['oracle_seconds']} s",
                  flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    jobs = None
    if args and args[0].startswith("-j"):
        jobs = int(args.pop(0)[2:])
    main(args, jobs)
