"""CPU emulation of the device-side dependency protocol of the batched launch
and of the server's host bookkeeping (tests/native/emulate.cpp), compiled
with g++ and the address and undefined-behaviour sanitizers.

  dag    random ticks of the serving workload (orders log-uniform in
         [64, 8192], tuned tiles, FP32 and FP64), edge geometries and the
         batched workload: workspace layout, the merged ticket order (each
         matrix keeps its own ticket order), and dag.h's readiness and
         publish rules under random completion orders with 1 to 512 workers,
         checked against an independent dependency model (blocks read and
         written in the blocked program order) and for deadlock;
  serve  the server core with a fake arena, clock and device results: two
         ticks in flight, corrections and FP64 refactors, resident factors
         with LRU eviction and releases; every live device and pinned region
         is disjoint from every other and accounted for after every step,
         new requests start in arrival order, and the server drains.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_11937_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "native", "emulate.cpp")


@pytest.fixture(scope="module")
def emulator(tmp_path_factory):
    from paper_2606_11937_amd import build
    d = tmp_path_factory.mktemp("emulate")
    gen = build.gen_tuned_tiles(out_dir=str(d))  # the tile tables the library compiles in
    exe = str(d / "emulate")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-Wall", "-I", CSRC, "-I", os.path.dirname(gen), SRC, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def run(exe, *args, timeout=600):
    r = subprocess.run([exe, *map(str, args)], capture_output=True, text=True, timeout=timeout,
                       env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1", "UBSAN_OPTIONS": "print_stacktrace=1"})
    return r.returncode, r.stdout + r.stderr


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_counter_protocol(emulator, seed):
    rc, out = run(emulator, "dag", seed, 30)
    assert rc == 0 and "OK dag" in out, out[-3000:]


@pytest.mark.parametrize("seed", [4, 5])
def test_server_core(emulator, seed):
    rc, out = run(emulator, "serve", seed, 4000)
    assert rc == 0 and out.count("OK serve") == 2, out[-3000:]


# (file, text, replacement, mode): mistakes planted in copies of the headers;
# the emulation must fail on each (early start, deadlock, leak, eviction of a
# factor in use)
MUTANTS = [
    ("dag.h", "ld(pdone + gk) >= need && ld(ver + gi * NRB + gk) >= u.J;",
     "ld(pdone + gk) >= need && ld(ver + gi * NRB + gk) >= u.J - 1;", "dag"),
    ("dag.h", "return ld(pdone + gs) > gs && ld(ver + gi * NRB + gs) >= u.J + u.K;",
     "return ld(pdone + gs) >= gs && ld(ver + gi * NRB + gs) >= u.J + u.K;", "dag"),
    ("dag.h", "ld(ver + gi * NRB + gt) >= u.J + u.K;", "ld(ver + gi * NRB + gt) >= u.J + u.K + 1;", "dag"),
    ("dag.h", "add(pdone + tc_gid(g, u.I, u.a));", "add(pdone + tc_gid(g, u.J, u.K));", "dag"),
    ("serve_core.h", "if (kv.second.alive && kv.second.refs == 0 &&", "if (kv.second.alive && kv.second.refs >= 0 &&",
     "serve"),
    ("serve_core.h", "    dev_.release(t.meta_dev, t.meta_bytes);\n    pin_.release", "    pin_.release", "serve"),
    ("batch_plan.h", "if (sz > 0) {\n          slots.push_back", "if (sz > 1) {\n          slots.push_back", "dag"),
]


@pytest.mark.parametrize("fname,old,new,mode", MUTANTS, ids=[f"{m[0]}:{i}" for i, m in enumerate(MUTANTS)])
def test_emulation_catches_planted_mistakes(tmp_path, fname, old, new, mode):
    import shutil

    from paper_2606_11937_amd import build
    inc = tmp_path / "inc"
    inc.mkdir()
    for f in ("dag.h", "batch_plan.h", "serve_core.h"):
        shutil.copy(os.path.join(CSRC, f), inc / f)
    src = (inc / fname).read_text()
    assert src.count(old) == 1, f"mutation site not found in {fname}"
    (inc / fname).write_text(src.replace(old, new))
    gen = build.gen_tuned_tiles(out_dir=str(tmp_path))
    exe = str(tmp_path / "emulate")
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-I", str(inc), "-I", os.path.dirname(gen), SRC, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    rc, out = run(exe, mode, 1, 30 if mode == "dag" else 3000)
    assert rc != 0, out[-2000:]  # a failed check, or a crash of the mutant
