"""CPU: the serving allocators, compiled with g++ and driven with random
sequences.  The device arena (csrc/arena.hpp): every step checks that free
and used blocks tile the range, that neighbouring free blocks are merged,
and that live blocks never overlap.  The pinned request rings
(csrc/ring.hpp): blocks come out in FIFO order and are released in any
order; live blocks never overlap, a refusal happens only when no contiguous
free run of that size exists at the head or after a wrap, and the ring is
whole again at the end."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include "arena.hpp"
int main(int argc, char** argv) {
    unsigned seed = (unsigned)atoi(argv[1]);
    std::mt19937_64 rng(seed);
    const uint64_t cap = 1 << 20;
    rgb::Arena a(cap, 256);
    std::map<uint64_t, uint64_t> live;  // offset -> size asked
    for (int step = 0; step < 20000; ++step) {
        bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            uint64_t n = 1 + rng() % 40000;
            uint64_t largest = a.largest_free();
            uint64_t off = a.alloc(n);
            if (off == UINT64_MAX) {
                if (a.rounded(n) <= largest) { printf("alloc failed though it fits\n"); return 1; }
            } else {
                if (off % 256 || off + n > cap) { printf("bad block\n"); return 1; }
                auto it = live.lower_bound(off);
                if (it != live.end() && it->first < off + a.rounded(n)) { printf("overlap\n"); return 1; }
                if (it != live.begin()) { auto p = std::prev(it); if (p->first + a.rounded(p->second) > off) { printf("overlap\n"); return 1; } }
                live[off] = n;
            }
        } else {
            auto it = live.begin();
            std::advance(it, rng() % live.size());
            if (!a.release(it->first)) { printf("release failed\n"); return 1; }
            live.erase(it);
        }
        if (!a.consistent()) { printf("inconsistent at step %d\n", step); return 1; }
    }
    for (auto& kv : live) a.release(kv.first);
    if (a.in_use() != 0 || a.largest_free() != cap || !a.consistent()) { printf("not whole again\n"); return 1; }
    if (a.release(12345)) { printf("released a non-block\n"); return 1; }
    printf("ok\n");
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver():
    d = tempfile.mkdtemp()
    src = os.path.join(d, "arena_test.cpp")
    exe = os.path.join(d, "arena_test")
    open(src, "w").write(DRIVER)
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_1902_04995_amd", "csrc"),
                           src, "-o", exe])
    return exe


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_arena_random_sequences(driver, seed):
    r = subprocess.run([driver, str(seed)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr


RING_DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include "ring.hpp"
int main(int argc, char** argv) {
    unsigned seed = (unsigned)atoi(argv[1]);
    std::mt19937_64 rng(seed);
    const int64_t cap = 100000;
    rgb::Ring r(cap);
    std::map<uint64_t, std::pair<int64_t, int64_t>> live;  // id -> (pos, n)
    for (int step = 0; step < 30000; ++step) {
        bool do_alloc = live.empty() || (rng() % 100) < 52;
        if (do_alloc) {
            int64_t n = (rng() % 10 == 0) ? 0 : (int64_t)(1 + rng() % 30000);
            int64_t h = r.head(), t = r.tail(), used = r.used();
            bool wrapped = used > 0 && h <= t;
            if (used == 0) { h = 0; t = 0; }
            bool fits = wrapped ? (t - h >= n) : (cap - h >= n || t >= n);
            int64_t pos; uint64_t id;
            bool ok = r.alloc(n, pos, id);
            if (ok != fits) { printf("alloc %d but fits %d (n=%lld h=%lld t=%lld used=%lld)\n", ok, fits,
                                     (long long)n, (long long)h, (long long)t, (long long)used); return 1; }
            if (ok) {
                if (pos < 0 || pos + n > cap) { printf("out of range\n"); return 1; }
                for (auto& kv : live) {
                    int64_t p = kv.second.first, q = kv.second.second;
                    if (n > 0 && q > 0 && pos < p + q && p < pos + n) { printf("overlap\n"); return 1; }
                }
                live[id] = {pos, n};
            }
        } else {
            auto it = live.begin();
            std::advance(it, rng() % live.size());
            if (!r.release(it->first)) { printf("release failed\n"); return 1; }
            if (r.release(it->first)) { printf("double release accepted\n"); return 1; }
            live.erase(it);
        }
        if (!r.consistent()) { printf("inconsistent at step %d\n", step); return 1; }
    }
    for (auto& kv : live) r.release(kv.first);
    if (r.used() != 0 || r.blocks() != 0 || !r.consistent()) { printf("not empty again\n"); return 1; }
    int64_t pos; uint64_t id;
    if (!r.alloc(cap, pos, id) || pos != 0) { printf("whole ring not free\n"); return 1; }
    printf("ok\n");
    return 0;
}
"""


@pytest.fixture(scope="module")
def ring_driver():
    d = tempfile.mkdtemp()
    src = os.path.join(d, "ring_test.cpp")
    exe = os.path.join(d, "ring_test")
    open(src, "w").write(RING_DRIVER)
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_1902_04995_amd", "csrc"),
                           src, "-o", exe])
    return exe


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_ring_random_sequences(ring_driver, seed):
    r = subprocess.run([ring_driver, str(seed)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
