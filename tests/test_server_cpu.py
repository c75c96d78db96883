"""CPU: the serving arena allocator (paper_1902_04995_amd/csrc/arena.hpp),
compiled with g++ and driven with random alloc/free sequences; every step
checks that free and used blocks tile the range, that neighbouring free
blocks are merged, and that live blocks never overlap."""
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
