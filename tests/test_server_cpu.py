"""Admission policy of the serving loop (first-fit arena over the memory
budget, batch formation), exercised on the CPU through a small driver built
from the library's host-only policy header, and checked against a Python
model of the same rules on random traces."""
import os
import random
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_15602_amd", "csrc")
DRIVER_SRC = os.path.join(ROOT, "tests", "serve_policy_driver.cpp")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("policy") / "serve_policy_driver")
    subprocess.check_call([gxx, "-std=c++17", "-O1", "-Wall", "-Werror", "-I", CSRC, DRIVER_SRC, "-o", exe])
    return exe


def run(exe, lines):
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout.strip().splitlines()


def parse_batch(line):
    parts = line.split()
    assert parts[0] == "batch"
    taken = [tuple(int(v) for v in p.split(":")) for p in parts[1:] if ":" in p]
    kv = dict(p.split("=") for p in parts[1:] if "=" in p)
    return taken, int(kv["blocked"]), int(kv["used"]), int(kv["ranges"])


def test_request_bytes(driver):
    out = run(driver, ["bytes 256 512 512", "bytes 3 5 7", "bytes 1 1 1"])
    def a(x):
        return (x + 255) // 256 * 256
    # bins (C bytes per pixel) and the fixed-point channel sum (8 bytes per pixel)
    assert int(out[0]) == a(256 * 512 * 512) + a(8 * 512 * 512)
    assert int(out[1]) == a(105) + a(8 * 35)
    assert int(out[2]) == 2 * 256


def test_fifo_and_batch_cap(driver):
    out = run(driver, ["reset 100000"] + [f"push {t} 0 1000" for t in range(1, 8)] + ["form 3", "form 3", "form 3"])
    b = [parse_batch(l) for l in out]
    assert [t for t, _ in b[0][0]] == [1, 2, 3]
    assert [t for t, _ in b[1][0]] == [4, 5, 6]
    assert [t for t, _ in b[2][0]] == [7]
    assert [o for _, o in b[0][0]] == [0, 1000, 2000]  # first fit packs from the start
    assert b[2][2] == 7000 and b[2][1] == 0


def test_memory_cut_and_no_overtaking(driver):
    # 10 000 bytes: requests of 4000, 4000, 5000 (does not fit), then 100
    out = run(driver, ["reset 10000", "push 1 0 4000", "push 2 0 4000", "push 3 0 5000", "push 4 0 100",
                       "form 8", "state", "free 1", "form 8", "free 2", "form 8", "state"])
    t, blocked, used, _ = parse_batch(out[0])
    assert [x for x, _ in t] == [1, 2] and blocked == 3 and used == 8000
    assert out[1].endswith("pending=3,4")           # 4 did not overtake 3
    t, blocked, _, _ = parse_batch(out[2])          # 4000 free at the front, 2000 at the end
    assert t == [] and blocked == 3                 # still no contiguous 5000
    t, blocked, used, ranges = parse_batch(out[3])  # all free again: one range
    assert [x for x, _ in t] == [3, 4] and blocked == 0 and used == 5100
    assert out[4].startswith("used=5100 peak=8000")


def test_other_groups_keep_their_place(driver):
    out = run(driver, ["reset 100000", "push 1 0 10", "push 2 1 10", "push 3 0 10", "push 4 1 10", "push 5 2 10",
                       "form 8", "state", "form 8", "state", "form 8", "state"])
    assert [x for x, _ in parse_batch(out[0])[0]] == [1, 3]
    assert out[1].endswith("pending=2,4,5")
    assert [x for x, _ in parse_batch(out[2])[0]] == [2, 4]
    assert [x for x, _ in parse_batch(out[4])[0]] == [5]
    assert out[5].endswith("pending=")


def test_oversized_request_never_fits(driver):
    out = run(driver, ["reset 1000", "push 9 0 1001", "form 4", "state"])
    t, blocked, used, _ = parse_batch(out[0])
    assert t == [] and blocked == 9 and used == 0


def test_release_coalesces(driver):
    lines = ["reset 1000"] + [f"push {t} 0 100" for t in range(1, 11)] + ["form 16"]
    lines += [f"free {t}" for t in (2, 4, 6, 8, 10, 1, 3, 5, 7, 9)] + ["state"]
    out = run(driver, lines)
    assert parse_batch(out[0])[2] == 1000
    assert out[-1].startswith("used=0 peak=1000 ranges=1")


class PyPolicy:
    """The same rules written independently: first-fit over a sorted free list."""

    def __init__(self, size):
        self.free = [(0, size)]
        self.size = size
        self.used = 0
        self.pending = []
        self.live = {}

    def alloc(self, n):
        if n == 0 or n > self.size:
            return None
        for i, (o, l) in enumerate(self.free):
            if l >= n:
                if l == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (o + n, l - n)
                self.used += n
                return o
        return None

    def release(self, o, n):
        self.free.append((o, n))
        self.free.sort()
        merged = []
        for a, l in self.free:
            if merged and merged[-1][0] + merged[-1][1] == a:
                merged[-1] = (merged[-1][0], merged[-1][1] + l)
            else:
                merged.append((a, l))
        self.free = merged
        self.used -= n

    def form(self, maxb):
        taken, blocked = [], 0
        if not self.pending:
            return taken, blocked
        g = self.pending[0][1]
        keep = []
        stop = False
        for req in self.pending:
            t, grp, n = req
            if stop or grp != g or len(taken) >= maxb:
                keep.append(req)
                continue
            o = self.alloc(n)
            if o is None:
                blocked = t
                stop = True
                keep.append(req)
                continue
            taken.append((t, o))
            self.live[t] = (o, n)
        self.pending = keep
        return taken, blocked


@pytest.mark.parametrize("seed", range(6))
def test_random_trace_matches_model(driver, seed):
    rng = random.Random(seed)
    size = rng.choice([5000, 20000, 100000])
    model = PyPolicy(size)
    lines = [f"reset {size}"]
    expect = []
    ticket = 1
    for _ in range(300):
        op = rng.random()
        if op < 0.5:
            n = rng.choice([rng.randint(1, size // 4), rng.randint(1, size // 20)])
            g = rng.randint(0, 2)
            lines.append(f"push {ticket} {g} {n}")
            model.pending.append((ticket, g, n))
            ticket += 1
        elif op < 0.75:
            mb = rng.randint(1, 6)
            lines.append(f"form {mb}")
            expect.append(model.form(mb) + (None,))
        elif model.live:
            t = rng.choice(sorted(model.live))
            o, n = model.live.pop(t)
            model.release(o, n)
            lines.append(f"free {t}")
    out = run(driver, lines)
    assert len(out) == len(expect)
    for line, (taken, blocked, _) in zip(out, expect):
        t, b, _, _ = parse_batch(line)
        assert t == taken and b == blocked
