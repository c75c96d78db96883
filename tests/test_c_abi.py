"""The boundary used from C: include/rgb.h is strict C99, and a plain C
program (tests/c_abi_solve.c: HIP's C runtime API for device memory and a
non-blocking stream, nothing else) solves a batch through rgb_solve_batch and
rgb_solve_batch_noalloc with the results of the FP64 oracle."""
import os
import subprocess
import sys

import numpy as np
import pytest

import lpcheck
from paper_1902_04995_amd import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_1902_04995_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _build(out_dir):
    exe = os.path.join(out_dir, "c_abi_solve")
    cmd = ["gcc", "-std=gnu11", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-isystem", os.path.join(ROCM, "include"),
           os.path.join(ROOT, "tests", "c_abi_solve.c"), "-o", exe, "-L", LIBDIR, "-lrgb",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", f"-Wl,-rpath,{LIBDIR}", f"-Wl,-rpath,{ROCM}/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_header_is_strict_c99(tmp_path):
    src = tmp_path / "h.c"
    src.write_text('#include "rgb.h"\nint main(void) { return rgb_version() == 0; }\n')
    r = subprocess.run(["gcc", "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror", "-fsyntax-only",
                        "-I", os.path.join(ROOT, "include"), str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_c_caller_builds_and_links(tmp_path):
    if not os.path.exists(os.path.join(LIBDIR, "librgb.so")):
        pytest.fail("librgb.so missing: build it with __graft_entry__.build()")
    assert os.path.exists(_build(str(tmp_path)))


def _write_batch(path, bt):
    with open(path, "wb") as f:
        np.array([bt.num_lps, bt.num_constraints], np.int64).tofile(f)
        np.ascontiguousarray(bt.offsets, np.int64).tofile(f)
        for a in (bt.ax, bt.ay, bt.b, bt.cx, bt.cy):
            np.ascontiguousarray(a, np.float32).tofile(f)


@pytest.mark.gpu
@pytest.mark.parametrize("variant", [0, 4])  # AUTO, BINNED
def test_c_caller_matches_oracle(tmp_path, oracle_lib, variant):
    exe = _build(str(tmp_path))
    bt = gen.concat([gen.uniform_batch(1500, 64, seed=90), gen.uneven_batch(800, 8, 3000, seed=91),
                     gen.tiny_integer_batch(1500, m_max=12, K=4, seed=92, boxed=True),
                     gen.tiny_random_batch(800, m_max=40, seed=93)])
    inp, outp = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    _write_batch(inp, bt)
    print(f"[c-abi] variant={variant} lps={bt.num_lps}", flush=True)
    sys.stdout.flush()
    r = subprocess.run([exe, inp, outp, str(variant)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    raw = np.fromfile(outp, dtype=np.uint8)
    B = bt.num_lps
    assert raw.size == 2 * 12 * B
    ref = oracle_lib.solve(bt)
    solves = []
    for k in range(2):
        chunk = raw[k * 12 * B:(k + 1) * 12 * B]
        x = chunk[:4 * B].view(np.float32)
        y = chunk[4 * B:8 * B].view(np.float32)
        st = chunk[8 * B:].view(np.int32)
        bs, bx = lpcheck.compare(st, x, y, ref["status"], ref["x"], ref["y"])
        assert len(bs) == 0 and len(bx) == 0, (k, bs[:5], bx[:5])
        solves.append(chunk)
    assert np.array_equal(solves[0], solves[1])  # with and without allocation: the same bits
