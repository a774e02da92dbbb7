"""The bin-load study behind the default bin capacity (tests/p2c_tail.c).

The C program simulates the load process of long uniform access under the
batched placement rule (rounds of ceil(B/16) keys that choose on the loads
at the round's start) and under one-at-a-time placement.  Here it is pinned
against a plain Python replay of the same rules over the same SplitMix64
stream on small sizes, and a short run checks its output.  The long runs
(10^9 accesses at N = 2^20) are made by hand:

    gcc -O2 -o p2c_tail tests/p2c_tail.c
    ./p2c_tail 1048576 16 4096 1000000000 <seed> rounds|sequential
"""
import json
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
M64 = (1 << 64) - 1


class SplitMix64:
    def __init__(self, seed):
        self.s = seed & M64

    def next(self):
        self.s = (self.s + 0x9E3779B97F4A7C15) & M64
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        return z ^ (z >> 31)

    def below(self, n):
        return (self.next() * n) >> 64


def replay(N, c, q, accesses, seed, sequential, Z):
    r = SplitMix64(seed)
    B = (N + c - 1) // c
    rs = 1 if sequential else (B + 15) // 16

    def pair():
        a = r.below(B)
        return a, (a + 1 + r.below(B - 1)) % B

    load = [0] * B
    binof = [0] * N
    for r0 in range(0, N, rs):
        ch = []
        for i in range(r0, min(N, r0 + rs)):
            a, b = pair()
            ch.append(b if load[b] < load[a] else a)
        for j, i in enumerate(range(r0, min(N, r0 + rs))):
            binof[i] = ch[j]
            load[ch[j]] += 1
    maxever = max(load)
    atleast = [0] * 8
    done = 0
    while done < accesses:
        seen, mv = set(), []
        for _ in range(q):
            k = r.below(N)
            if k not in seen:
                seen.add(k)
                mv.append(k)
        if sequential:
            for k in mv:
                load[binof[k]] -= 1
                a, b = pair()
                binof[k] = b if load[b] < load[a] else a
                load[binof[k]] += 1
                maxever = max(maxever, load[binof[k]])
        else:
            for k in mv:
                load[binof[k]] -= 1
            for r0 in range(0, len(mv), rs):
                chunk = mv[r0:r0 + rs]
                ch = []
                for k in chunk:
                    a, b = pair()
                    ch.append(b if load[b] < load[a] else a)
                for k, b in zip(chunk, ch):
                    binof[k] = b
                    load[b] += 1
                    maxever = max(maxever, load[b])
        mx = max(load)
        for j in range(8):
            if mx >= Z - 2 + j:
                atleast[j] += 1
        done += q
    return maxever, atleast


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("p2c") / "p2c_tail")
    subprocess.run(["gcc", "-O2", "-Wall", "-o", out, os.path.join(HERE, "p2c_tail.c")], check=True)
    return out


def _run(exe, *args):
    r = subprocess.run([exe] + [str(a) for a in args], capture_output=True, text=True, check=True)
    return json.loads(r.stdout)


@pytest.mark.parametrize("N,c,q,rule", [(512, 4, 24, "rounds"), (512, 4, 24, "sequential"), (2048, 8, 100, "rounds"),
                                        (300, 3, 7, "rounds")])
def test_simulator_matches_a_python_replay(exe, N, c, q, rule):
    acc = 40 * q
    got = _run(exe, N, c, q, acc, 12345, rule, 6)
    mx, atleast = replay(N, c, q, acc, 12345, rule == "sequential", 6)
    assert got["max_load"] == mx
    assert [got["batch_ends_at_least"][str(4 + j)] for j in range(8)] == atleast


def test_short_run_stays_within_capacity(exe):
    for rule in ("rounds", "sequential"):
        got = _run(exe, 1 << 16, 8, 4096, 2_000_000, 7, rule)
        assert got["Z"] == 13 and got["max_load"] <= 14
        assert got["batches"] * 4096 == got["accesses"]
