"""The C-ABI library loads and exports every function include/rgb.h declares,
and the Python binding's signatures match the header (CPU only: no compute
calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    """(name, number of parameters) for every function prototype in include/*.h."""
    out = {}
    inc = os.path.join(ROOT, "include")
    for fn in sorted(os.listdir(inc)):
        if not fn.endswith(".h"):
            continue
        src = open(os.path.join(inc, fn)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"\b(rgb_\w+)\s*\(([^;{]*?)\)\s*;", src):
            params = m.group(2).strip()
            n = 0 if params in ("", "void") else params.count(",") + 1
            out[m.group(1)] = n
    return out


def test_header_declares_the_entry_points():
    d = _declared()
    for name in ("rgb_version", "rgb_ctx_create", "rgb_ctx_destroy", "rgb_ctx_last_error", "rgb_solve_batch"):
        assert name in d, name


def test_library_exports_every_declared_symbol():
    import paper_1902_04995_amd as rgb
    path = rgb.LIB_PATH
    if not os.path.exists(path):
        pytest.fail(f"{path} missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    for name in _declared():
        assert hasattr(lib, name), f"{name} declared in include/ but not exported"


def test_binding_signatures_match_header():
    import paper_1902_04995_amd as rgb
    L = rgb.lib()
    for name, n in _declared().items():
        f = getattr(L, name)
        if name == "rgb_version":  # no parameters: ctypes leaves argtypes unset
            continue
        assert f.argtypes is not None, f"{name} has no ctypes signature in the binding"
        assert len(f.argtypes) == n, (name, len(f.argtypes), n)


def test_version_string_without_gpu():
    import paper_1902_04995_amd as rgb
    assert b"gfx950" in rgb.lib().rgb_version()


def test_null_context_errors_without_gpu():
    import paper_1902_04995_amd as rgb
    L = rgb.lib()
    assert L.rgb_solve_batch(None, 0, 0, *([None] * 9), None, None) == -1
    assert L.rgb_ctx_last_error(None) == b"null context"
    assert L.rgb_ctx_destroy(None) == 0
    assert L.rgb_ctx_create(0, None, None) == -1


def test_null_handles_are_rejected_without_gpu():
    """Every entry point checks its handle and arguments before any HIP call."""
    import paper_1902_04995_amd as rgb
    L = rgb.lib()
    ERR, OK = -1, 0
    assert L.rgb_autotune(None, 0, 0, *([None] * 9), 1, 1.0, None, None, None) == ERR
    assert L.rgb_plan_create(None, 0, 0, *([None] * 9), None, None) == ERR
    assert L.rgb_plan_launch(None, None) == ERR
    assert L.rgb_plan_destroy(None) == OK
    assert L.rgb_ctx_get_tuning(None, None) == ERR
    assert L.rgb_server_create(None, None, None) == ERR
    assert L.rgb_server_submit(None, 0, 0, *([None] * 6), None) == ERR
    assert L.rgb_server_poll(None, 0, 0, None, None, None, None, None) == ERR
    assert L.rgb_server_destroy(None) == OK
    assert L.rgb_solve_batch_host(None, 0, 0, *([None] * 9), None, 0, None) == ERR
    assert L.rgb_crowd_create(None, 10, None, None, None, None) == ERR
    assert L.rgb_crowd_step(None, *([None] * 7), 0, None, None) == ERR
    assert L.rgb_crowd_num_rows(None, None) == ERR
    assert L.rgb_crowd_rows(None, None, None, None, None, None) == ERR
    assert L.rgb_crowd_destroy(None) == OK
    # contention 3 is not a power of two: refused before anything is launched
    assert L.rgb_reduce_bench_run(2, 3, 0, None, None, None) == ERR


def test_output_tensors_are_checked():
    """Caller-supplied outputs must be float32/float32/int32, contiguous, on
    the batch's device and hold one entry per LP (the kernels write that many)."""
    import torch

    import paper_1902_04995_amd as rgb
    dev = torch.device("cpu")
    ok = (torch.empty(5), torch.empty(5), torch.empty(5, dtype=torch.int32))
    rgb._check_out(ok, 5, dev)
    for bad in ((torch.empty(4), ok[1], ok[2]),                         # too short
                (ok[0], torch.empty(5, dtype=torch.float64), ok[2]),    # wrong dtype
                (ok[0], ok[1], torch.empty(5)),                         # status not int32
                (torch.empty(10)[::2], ok[1], ok[2]),                   # not contiguous
                (ok[0], ok[1])):                                        # missing one
        with pytest.raises((TypeError, ValueError)):
            rgb._check_out(bad, 5, dev)
