"""Writes instance_hashes.json: SHA-256 of generated instances (inputs only).

Run from the repository root: python tests/golden/make_instance_hashes.py
It calls only the seeded generators; no solver result is stored.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from paper_1710_03647_amd import synth  # noqa: E402

CASES = {
    "plain": lambda: synth.gen_plain(),
    "uniform-n4096-d16": lambda: synth.gen_uniform(4096, 16, 1000, 2),
    "rmat-s10": lambda: synth.gen_rmat(10, 16, seed=3),
    "torus-32": lambda: synth.gen_torus(32, seed=4),
    "stream-g0": lambda: synth.gen_stream_game(0),
    "stream-g17": lambda: synth.gen_stream_game(17),
}

if __name__ == "__main__":
    out = {k: f().sha256() for k, f in CASES.items()}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "instance_hashes.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1))
