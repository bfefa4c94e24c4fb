"""The request server's range allocator (csrc/arena.h, host-only C++) against a plain
first-fit model: same offsets on random alloc/release scripts, no overlap between live
ranges, and one free range of the whole capacity once everything is released."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2408_09399_amd", "csrc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("arena") / "arena_check")
    # host-only harness, built with AddressSanitizer and UndefinedBehaviorSanitizer: a bad
    # access or undefined behaviour in the allocator ends it with a non-zero status
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-I", CSRC, os.path.join(ROOT, "tests", "arena_check.cpp"),
                    "-o", exe], check=True)
    return exe


class FirstFit:
    """Free ranges as a sorted list of [offset, size]; the lowest fitting range is split."""

    def __init__(self, capacity, align):
        self.align = align
        self.cap = capacity // align * align
        self.free = [[0, self.cap]] if self.cap else []

    def rnd(self, b):
        b = max(b, 1)
        return (b + self.align - 1) // self.align * self.align

    def alloc(self, b):
        need = self.rnd(b)
        for i, (o, s) in enumerate(self.free):
            if s >= need:
                if s == need:
                    self.free.pop(i)
                else:
                    self.free[i] = [o + need, s - need]
                return o
        return -1

    def release(self, o, b):
        self.free.append([o, self.rnd(b)])
        self.free.sort()
        merged = []
        for o2, s2 in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o2:
                merged[-1][1] += s2
            else:
                merged.append([o2, s2])
        self.free = merged


@pytest.mark.parametrize("seed", range(6))
def test_matches_first_fit_model(harness, seed):
    rng = np.random.default_rng(seed)
    cap, align = int(rng.integers(1 << 12, 1 << 20)), int(rng.choice([1, 64, 256]))
    model = FirstFit(cap, align)
    script, expect, live = [f"C {cap} {align}"], [], []
    for _ in range(600):
        if live and rng.random() < 0.45:
            o, b = live.pop(int(rng.integers(len(live))))
            script.append(f"R {o} {b}")
            model.release(o, b)
        else:
            b = int(rng.integers(0, cap // 6))
            o = model.alloc(b)
            script.append(f"A {b}")
            expect.append(o)
            if o >= 0:
                live.append((o, b))
    for o, b in live:
        script.append(f"R {o} {b}")
        model.release(o, b)
    script.append("S")
    out = subprocess.run([harness], input="\n".join(script) + "\n", capture_output=True, text=True,
                         check=True).stdout.split("\n")
    got = [int(x) for x in out[: len(expect)]]
    assert got == expect
    used, ranges, largest = map(int, out[len(expect)].split())
    assert (used, ranges, largest) == (0, 1, model.cap)


def test_live_ranges_never_overlap(harness):
    rng = np.random.default_rng(99)
    cap = 1 << 16
    model = FirstFit(cap, 256)
    live = []
    for _ in range(2000):
        if live and rng.random() < 0.5:
            o, b = live.pop(int(rng.integers(len(live))))
            model.release(o, b)
        else:
            b = int(rng.integers(1, 5000))
            o = model.alloc(b)
            if o >= 0:
                live.append((o, b))
        spans = sorted((o, o + model.rnd(b)) for o, b in live)
        for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
            assert a1 <= b0
        assert all(e <= model.cap for _, e in spans)
