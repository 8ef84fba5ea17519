"""Sanitizer builds of the host code (CPU only, no GPU needed).

- The CPU oracle (plain C) built with AddressSanitizer and UndefinedBehavior
  Sanitizer, loaded into a child Python process (ASan runtime preloaded), runs
  every worklist order, the bound, the unstable count and the strategy on
  tiny and mid-size games.
- libeg's host validation path (eg_check) built with the host side of its
  sources instrumented (the device code is built as usual), linked into a
  small driver (tests/sanitize/check_host_main.cpp) that covers every
  rejection cause and random valid games.

Any sanitizer report aborts the child, which fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ROCM = "/opt/rocm"


def gcc_runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


CHILD = r"""
import sys
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import numpy as np
from oracle import oracle
from paper_1710_03647_amd import synth
import pins
lib = {lib!r}
games = [synth.gen_random_small(5000 + i, n_max=7) for i in range(200)]
games += [synth.gen_uniform(3000, 4, 30, 9), synth.gen_rmat(10, 16, seed=3), synth.gen_torus(12, seed=4),
          pins.cf8_game(50)]
for g in games:
    ref = None
    for order in ("fifo", "lifo", "random", "jacobi", "rounds", "alg1"):
        r = oracle.solve(g, order=order, lib_path=lib)
        assert r.status == 0
        if ref is None:
            ref = r.f
        assert np.array_equal(r.f, ref), (g.name, order)
    for mode in (oracle.BOUND_NW, oracle.BOUND_MG):
        b = oracle.bound_of(g, bound_mode=mode, lib_path=lib)
        assert oracle.count_unstable(g, ref, b, lib_path=lib) == 0
    choice, missing = oracle.strategy(g, ref, lib_path=lib)
    assert missing == 0
    part = oracle.solve(g, max_lifts=3, lib_path=lib)
    assert part.status in (0, 1)
print("sanitized oracle ok", len(games))
"""


def test_oracle_under_asan_ubsan(tmp_path):
    asan = gcc_runtime("libasan.so")
    if not asan or not shutil.which("gcc"):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-o", lib, os.path.join(ROOT, "oracle", "eg_oracle.c")])
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    code = CHILD.format(root=ROOT, tests=HERE, lib=lib)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitized oracle ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def test_host_validation_under_asan_ubsan(tmp_path):
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    clangxx = os.path.join(ROCM, "llvm", "bin", "clang++")
    if not (os.path.exists(hipcc) and os.path.exists(clangxx)):
        pytest.skip("ROCm toolchain not installed")
    csrc = os.path.join(ROOT, "paper_1710_03647_amd", "csrc")
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-mcode-object-version=5",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include"), "-I", csrc]
    # host side of the API instrumented; each sanitizer flag applies to the host pass only
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    procs = []
    from paper_1710_03647_amd.build import SOURCES

    for src in SOURCES:
        extra = host_san if src in ("eg_api.hip", "eg_serve.hip") else []
        obj = str(tmp_path / src.replace(".hip", ".o"))
        procs.append(subprocess.Popen([hipcc, *common, *extra, "-c", os.path.join(csrc, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
        objs.append(obj)
    for p in procs:
        out, err = p.communicate(timeout=600)
        assert p.returncode == 0, err[-3000:]
    main_o = str(tmp_path / "main.o")
    subprocess.check_call([clangxx, "-O1", "-g", "-fsanitize=address,undefined", "-I", os.path.join(ROOT, "include"),
                           "-c", os.path.join(HERE, "sanitize", "check_host_main.cpp"), "-o", main_o])
    exe = str(tmp_path / "check_host")
    subprocess.check_call([clangxx, "-fsanitize=address,undefined", main_o, *objs, "-L", os.path.join(ROCM, "lib"),
                           "-lamdhip64", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}", "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "ok: 0 failures" in r.stdout
