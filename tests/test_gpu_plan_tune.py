"""GPU: autotuning and captured plans, through the C ABI.

Whatever configuration the autotuner picks, results must stay bit-identical
to the plain kernel's; a captured plan must reproduce the eager solve on
every replay, with eager work and host synchronisation between replays, and
must pick up new input values written into the same buffers.
"""
import sys

import numpy as np
import pytest

import lpcheck
from paper_1902_04995_amd import gen

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rgb():
    import torch
    assert torch.cuda.is_available()
    import paper_1902_04995_amd as rgb
    rgb.lib()
    return rgb


def _host(out):
    return [t.cpu().numpy() for t in out]


def test_tuning_roundtrip_and_validation(rgb):
    ctx = rgb.Context(0)
    t = ctx.tuning
    d = t.to_dict()
    assert d["variant"] in ("persistent", "binned", "batched", "pooled")
    d["batched_lanes"] = 32
    d["log2_lanes"][9] = 4
    ctx.tuning = d
    assert ctx.tuning.batched_lanes == 32 and ctx.tuning.log2_lanes[9] == 4
    bad = dict(d, batched_lanes=12)
    with pytest.raises(rgb.RgbError):
        ctx.tuning = bad
    bad = dict(d)
    bad["log2_lanes"] = [7] * 16
    with pytest.raises(rgb.RgbError):
        ctx.tuning = bad
    ctx.close()


@pytest.mark.parametrize("which", ["uneven", "crowd"])
def test_autotune_keeps_results(rgb, oracle_lib, which):
    import torch
    bt = gen.uneven_batch(3000, 8, 2000, seed=5) if which == "uneven" else gen.crowd_batch(8192, seed=5)
    dev = rgb.DeviceBatch(bt, "cuda:0")
    ctx = rgb.Context(0)
    _say(f"[gpu] autotune {which}")
    best = dev.autotune(reps=2, budget_ms=1500.0, ctx=ctx)
    assert best.ms > 0 and best.variant in (2, 3, 4, 5)
    assert ctx.tuning.to_dict() == best.to_dict()
    _say(f"[gpu] tuned: {best.to_dict()}")
    got = _host(dev.solve(variant="auto", ctx=ctx))
    ref = _host(dev.solve(variant="plain", ctx=ctx))
    torch.cuda.synchronize()
    for a, b in zip(got, ref):
        assert np.array_equal(a, b, equal_nan=True)
    o = oracle_lib.solve(bt)
    bs, bx = lpcheck.compare(got[2], got[0], got[1], o["status"], o["x"], o["y"])
    assert len(bs) == 0 and len(bx) == 0
    ctx.close()


@pytest.mark.parametrize("variant", ["persistent", "binned", "batched", "pooled", "plain"])
def test_plan_replays_match_eager(rgb, variant):
    import torch
    bt = gen.uneven_batch(2000, 8, 1500, seed=11)
    dev = rgb.DeviceBatch(bt, "cuda:0")
    eager = _host(dev.solve(variant=variant, want_n_1dlp=True))
    plan = dev.plan(variant=variant, want_n_1dlp=True)
    for rep in range(4):
        _say(f"[gpu] plan {variant} replay {rep}")
        for t in plan.out:
            t.fill_(-7)  # eager work between replays
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        got = _host(plan.out) + [plan.n_1dlp.cpu().numpy()]
        for a, b in zip(got, eager):
            assert np.array_equal(a, b, equal_nan=True), (variant, rep)
    # new values in the same buffers: the replay solves the new LPs
    dev.b.mul_(2.0)
    eager2 = _host(dev.solve(variant=variant))
    plan.launch()
    torch.cuda.synchronize()
    for a, b in zip(_host(plan.out), eager2):
        assert np.array_equal(a, b, equal_nan=True)
    opt = eager[2] == 0
    assert np.allclose(eager2[0][opt], 2 * eager[0][opt], rtol=1e-6, atol=1e-6)
    plan.close()


def test_two_plans_overlap_on_two_streams(rgb):
    """Plans own their workspaces, so two may run at once."""
    import torch
    b1 = rgb.DeviceBatch(gen.uneven_batch(1500, 8, 1500, seed=1), "cuda:0")
    b2 = rgb.DeviceBatch(gen.uniform_batch(1500, 200, seed=2), "cuda:0")
    e1 = _host(b1.solve(variant="persistent"))
    e2 = _host(b2.solve(variant="persistent"))
    p1 = b1.plan(variant="persistent")
    p2 = b2.plan(variant="persistent")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for rep in range(3):
        _say(f"[gpu] two plans rep {rep}")
        p1.launch(s1)
        p2.launch(s2)
        torch.cuda.synchronize()
        for a, b in zip(_host(p1.out), e1):
            assert np.array_equal(a, b, equal_nan=True)
        for a, b in zip(_host(p2.out), e2):
            assert np.array_equal(a, b, equal_nan=True)
    p1.close()
    p2.close()


_CHILD = r"""
import json, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import torch
import paper_1902_04995_amd as rgb
from paper_1902_04995_amd import gen
z = np.load(sys.argv[3])
bt = gen.Batch(z["offsets"], z["ax"], z["ay"], z["b"], z["cx"], z["cy"], z["kind"], "t")
ctx = rgb.Context(0, tuning_table=sys.argv[2])
x, y, st = rgb.DeviceBatch(bt, "cuda:0").solve(variant="auto", ctx=ctx)
torch.cuda.synchronize()
np.savez(sys.argv[4], x=x.cpu().numpy(), y=y.cpu().numpy(), st=st.cpu().numpy())
print(json.dumps(ctx.tuning.to_dict()))
"""


def test_tuning_table_persists_across_processes(rgb, tmp_path):
    """rgb_autotune merges its result into a JSON table keyed by device and
    size class; a fresh process that creates its context from the table
    solves with that configuration (no search) and gets the same bits."""
    import json
    import os
    import subprocess

    import torch
    bt = gen.uneven_batch(4000, 8, 3000, seed=9)
    dev = rgb.DeviceBatch(bt, "cuda:0")
    table = str(tmp_path / "tuning.json")
    ctx = rgb.Context(0)
    _say("[gpu] autotune with a table")
    best = dev.autotune(reps=2, budget_ms=1500.0, ctx=ctx, table_path=table)
    got = _host(dev.solve(variant="auto", ctx=ctx))
    torch.cuda.synchronize()
    doc = json.load(open(table))
    assert doc["format"] == "rgb-tuning-1" and len(doc["devices"]) == 1
    (key, entry), = doc["devices"].items()
    assert "gfx950" in key and entry["variant"] == best.to_dict()["variant"]
    assert entry["classes"], "no size class was tuned"
    np.savez(tmp_path / "batch.npz", offsets=bt.offsets, ax=bt.ax, ay=bt.ay, b=bt.b, cx=bt.cx, cy=bt.cy,
             kind=bt.kind)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    _say("[gpu] fresh process from the table")
    r = subprocess.run([sys.executable, "-c", _CHILD, root, table, str(tmp_path / "batch.npz"),
                        str(tmp_path / "out.npz")], capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    child = json.loads(r.stdout.strip().splitlines()[-1])
    want = best.to_dict()
    assert child["variant"] == want["variant"]
    for c, v in entry["classes"].items():
        assert child["log2_lanes"][int(c)] == v["log2_lanes"]
    for k in ("batched_lanes", "queue_share", "chunk", "pool_lanes", "pool_wait", "pool_rows"):
        assert child[k] == want[k], k
    out = np.load(tmp_path / "out.npz")
    for a, b_ in zip((out["x"], out["y"], out["st"]), got):
        assert np.array_equal(a, b_, equal_nan=True)
    # a second tuning run on another batch keeps the classes it did not measure
    small = rgb.DeviceBatch(gen.uniform_batch(3000, 60, seed=2), "cuda:0")
    small.autotune(reps=2, budget_ms=800.0, ctx=rgb.Context(0), table_path=table)
    doc2 = json.load(open(table))
    (entry2,) = doc2["devices"].values()
    for c in entry["classes"]:
        assert c in entry2["classes"]
    # a missing table leaves the defaults; an unreadable one is refused
    assert rgb.Context(0, tuning_table=str(tmp_path / "missing.json")).tuning.to_dict() == \
        rgb.Context(0).tuning.to_dict()
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    with pytest.raises(rgb.RgbError):
        rgb.Context(0, tuning_table=str(bad))
    ctx.close()
