"""GPU parity: every kernel family against the FP64 oracle, through the C ABI.

Bar (per LP): status bit-exact; for OPTIMAL, ||x - x_oracle|| <=
1e-4 * max(1, ||x_oracle||) (FP32 solver vs FP64 oracle).  Kernel families
must also agree with each other bit for bit (min/max reductions with a
smallest-index tie-break are exact and order free).
"""
import os
import sys

import numpy as np
import pytest

import lpcheck
from lpcheck import OPTIMAL
from paper_1902_04995_amd import gen

pytestmark = pytest.mark.gpu

# (variant, lanes_per_lp, pool_wait) combinations exercised; 0 = library default
SHAPES = [("plain", 0, 0), ("batched", 0, 0), ("batched", 4, 0), ("batched", 8, 0), ("batched", 16, 0),
          ("batched", 32, 0), ("batched", 64, 0), ("persistent", 0, 0), ("pooled", 0, 0), ("pooled", 8, -1),
          ("pooled", 16, 8), ("pooled", 4, 2)]
# pooled kernels by (lanes_per_lp, rows per lane), all at the default wait
POOL_SHAPES = [(g, r) for g in (4, 8, 16) for r in (1, 2, 4)]


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


def _run(rgb, bt, variant, g=0, s=0, n1d=False, rows=0):
    import torch
    dev = rgb.DeviceBatch(bt, "cuda:0")
    out = dev.solve(variant=variant, lanes_per_lp=g, pool_wait=s, pool_rows=rows, want_n_1dlp=n1d)
    torch.cuda.synchronize()
    out = [t.cpu().numpy() for t in out]
    return [out[2], out[0], out[1]] + out[3:]   # status, x, y[, n_1dlp]


def _check(bt, ref, got, label, allow=0):
    """Status bit-exact and x* within the bar against the oracle; when the
    run returned the count of 1D LPs (got[3]), that count must equal the
    oracle's on every LP the oracle decides with a margin of at least
    lpcheck.N1D_MARGIN."""
    st, x, y = got[0], got[1].astype(np.float64), got[2].astype(np.float64)
    bs, bx = lpcheck.compare(st, x, y, ref["status"], ref["x"], ref["y"])
    msg = f"{label}: {len(bs)} status / {len(bx)} x mismatches of {bt.num_lps}"
    bn, skipped = [], 0
    if len(got) > 3:
        bn, skipped = lpcheck.compare_n1d(got[3], ref)
        msg += f"; {len(bn)} 1D-LP count mismatches ({skipped} LPs below the margin left out)"
    if len(bs) or len(bx) or len(bn):
        for k in list(bs[:5]) + list(bx[:5]) + list(bn[:5]):
            msg += (f"\n  lp {k} m={bt.sizes()[k]} got st={st[k]} x=({x[k]:.9g},{y[k]:.9g})"
                    f" ref st={ref['status'][k]} x=({ref['x'][k]:.9g},{ref['y'][k]:.9g}) margin={ref['margin'][k]:.3g}")
            if len(got) > 3:
                msg += f" n1d={got[3][k]} ref n1d={ref['n_1dlp'][k]}"
    _say(msg)
    assert len(bs) + len(bx) + len(bn) <= allow, msg
    return msg


CASES = {
    "golden": lambda: lpcheck.golden_batch(os.path.join(lpcheck.GOLDEN, "hand_lps.txt"))[0],
    "tiny_random": lambda: gen.tiny_random_batch(3000, m_max=70, seed=2),
    "tiny_int_boxed": lambda: gen.tiny_integer_batch(3000, m_max=12, K=6, seed=3, boxed=True),
    "plain_cfg": lambda: gen.make_config("plain", seed=0),
    "uniform_small": lambda: gen.make_config("uniform", seed=0, scale=0.02),
    "uneven_small": lambda: gen.uneven_batch(2500, 8, 1500, seed=0),
    "crowd_small": lambda: gen.make_config("crowd", seed=0, scale=0.02),
}


@pytest.mark.parametrize("case", list(CASES))
def test_parity_vs_oracle(rgb, oracle_lib, case):
    bt = CASES[case]()
    ref = oracle_lib.solve(bt)
    base = None
    for variant, g, s in SHAPES:
        _say(f"[gpu] case={case} variant={variant} G={g} S={s} lps={bt.num_lps} rows={bt.num_constraints}")
        got = _run(rgb, bt, variant, g, s, n1d=True)
        _check(bt, ref, got, f"{case}/{variant}/{g}x{s}")
        if base is None:
            base = got
        else:
            for a, b_, name in zip(got, base, ("status", "x", "y", "n_1dlp")):
                assert np.array_equal(a, b_, equal_nan=True) if a.dtype.kind == "f" else np.array_equal(a, b_), \
                    f"{case}: {variant}/{g}x{s} differs from plain in {name}"


@pytest.mark.parametrize("case", ["tiny_random", "tiny_int_boxed", "uniform_small", "uneven_small", "crowd_small"])
def test_pool_shapes_match_plain(rgb, oracle_lib, case):
    """Every pooled (lanes, rows per lane) instance against the oracle and,
    bit for bit, against the plain kernel."""
    bt = CASES[case]()
    ref = oracle_lib.solve(bt)
    base = _run(rgb, bt, "plain", n1d=True)
    for g, r in POOL_SHAPES:
        for w in (-1, 0, 8):
            _say(f"[gpu] case={case} pooled G={g} R={r} W={w}")
            got = _run(rgb, bt, "pooled", g, w, n1d=True, rows=r)
            _check(bt, ref, got, f"{case}/pooled/{g}x{r}/w{w}")
            for a, b_, name in zip(got, base, ("status", "x", "y", "n_1dlp")):
                assert np.array_equal(a, b_, equal_nan=True) if a.dtype.kind == "f" else np.array_equal(a, b_), \
                    f"{case}: pooled {g}x{r} w{w} differs from plain in {name}"


def test_parity_tiny_integer_degenerate(rgb, oracle_lib):
    """Integer LPs are full of exact ties (concurrent and coincident lines,
    single-point regions); the exact guards must reproduce the exact answer."""
    bt = gen.tiny_integer_batch(4000, m_max=10, K=4, seed=4)
    ref = oracle_lib.solve(bt)
    for variant, g, s in (("plain", 0, 0), ("batched", 4, 0), ("batched", 64, 0), ("pooled", 4, -1), ("pooled", 16, 8)):
        _say(f"[gpu] case=tiny_int variant={variant} G={g} S={s}")
        _check(bt, ref, _run(rgb, bt, variant, g, s), f"tiny_int/{variant}")


def _nonfinite_lps():
    """Non-finite values in every field, before and after the row that
    starts a 1D LP, in corner, ray and vertex states."""
    lps = [([], (1.0, 0.0)),
           ([(1, 0, 1), (0, 1, 1)], (np.inf, 1.0)),
           ([(1, 0, 1), (0, 1, 1)], (1.0, -np.inf)),
           ([(1, 0, 1), (0, 0, -1), (0, 1, 1)], (1.0, 1.0)),
           ([(0, 0, 0), (1, 0, 1), (-1, 0, 1), (0, 1, 1), (0, -1, 1)], (1.0, 1.0))]
    ring = [(np.cos(t), np.sin(t), 2.0) for t in np.linspace(0, 2 * np.pi, 90, endpoint=False)]
    for bad in (np.inf, -np.inf, np.nan):
        for field in range(3):
            row = [0.5, 0.25, 1.0]
            row[field] = bad
            row = tuple(row)
            base = [(1, 0, 1), (0, 1, 1), (1, 1, 1.5)]
            for pos in range(4):  # first row (corner), after a ray, at the vertex, last
                lps.append((base[:pos] + [row] + base[pos:], (1.0, 1.0)))
            # in a long LP: windows with violations before and after it
            lps.append((ring[:40] + [row] + ring[40:], (0.3, 0.7)))
    return lps


def _nextafter32(t, steps):
    t = np.float32(t)
    for _ in range(abs(steps)):
        t = np.nextafter(t, np.float32(np.inf if steps > 0 else -np.inf))
    return float(t)


def _parallel_lps():
    """A row parallel to the line of a later violated row, with offsets at the
    FP32 neighbours of where the line's point lands (the parallel case of
    Sec. 2.1 decided at the rounding of p0): x >= t and lx x <= 1 (empty iff
    t > 1/lx), and a.x >= t with a.x <= 1 along other directions (empty iff
    t > 1), in both orders, and after 100 far rows."""
    lps = []
    far = [(np.cos(t), np.sin(t), 50.0) for t in np.linspace(0, 2 * np.pi, 100, endpoint=False)]
    for lx in range(1, 41):
        for k in range(-2, 3):
            t = _nextafter32(1.0 / lx, k)
            h, l = (-1.0, 0.0, -t), (float(lx), 0.0, 1.0)
            lps.append(([h, l], (1.0, 0.0)))
            lps.append(([l, h], (1.0, 0.0)))
            if lx % 4 == 1:
                lps.append((far + [h, l], (1.0, 0.25)))
    for ax, ay in [(1, 2), (3, -1), (-2, 5), (7, 3), (0, 3), (5, 0), (-4, -9)]:
        for scale in (1.0, 2.0, 0.5, 3.0):
            for k in range(-2, 3):
                t = _nextafter32(1.0, k)
                h = (-scale * ax, -scale * ay, -scale * t)
                l = (float(ax), float(ay), 1.0)
                lps.append(([h, l], (float(ax), float(ay))))
                lps.append(([l, h], (float(ay), -float(ax))))
    return lps


def _range_lps():
    """Positions beyond the FP32 range inside a 1D LP, and vertices beyond it."""
    a, big = 1e-30, 1e10
    lps = [
        # y >= 1e-30 x + 1e10, x <= 5, x >= -5, then y <= 0: on y = 0 the first row
        # bounds at x = -1e40 (an FP32 overflow) and the LP is infeasible
        ([(a, -1, -big), (1, 0, 5), (-1, 0, 5), (0, 1, 0)], (0.0, -1.0)),
        # a vertex at x = 1e40: INVALID; the same vertex on the way: INVALID
        ([(1e-10, 0, 1e30), (0, 1, 1)], (1.0, 1.0)),
        ([(1e-10, 0, 1e30), (0, 1, 1), (1, 0, 5)], (1.0, 1.0)),
        # the far row only bounds a 1D LP from the side that is not chosen
        ([(1, 0, 5), (1e-10, 0, 1e30), (0, 1, 1)], (1.0, 1.0)),
        ([(1, 0, 3e38), (0, 1, 1)], (1.0, 1.0)),
    ]
    rng = np.random.default_rng(17)
    for _ in range(300):  # small integer LPs with one or two rows of tiny slope and huge offset
        m = int(rng.integers(3, 9))
        rows = [tuple(float(v) for v in rng.integers(-4, 5, 3)) for _ in range(m)]
        for _ in range(int(rng.integers(1, 3))):
            s = float(rng.choice([-1, 1]))
            rows.insert(int(rng.integers(0, len(rows) + 1)),
                        (float(rng.integers(1, 5)) * a * s, float(rng.choice([-1, 1])),
                         float(rng.integers(-3, 4)) * big))
        lps.append((rows, tuple(float(v) for v in rng.integers(-3, 4, 2))))
    return lps


EDGE_SETS = {"nonfinite": _nonfinite_lps, "parallel": _parallel_lps, "range": _range_lps}


def test_empty_batch(rgb):
    import torch
    dev = torch.device("cuda:0")
    z64 = torch.zeros(1, dtype=torch.int64, device=dev)
    e32 = torch.empty(0, dtype=torch.float32, device=dev)
    for variant in ("plain", "batched", "persistent", "binned", "pooled"):
        x, y, st = rgb.solve_batch(z64, e32, e32, e32, e32, e32, variant=variant)
        assert x.numel() == 0


@pytest.mark.parametrize("edge", list(EDGE_SETS))
def test_edge_cases(rgb, oracle_lib, edge):
    bt = lpcheck.rows_batch(EDGE_SETS[edge](), edge)
    ref = oracle_lib.solve(bt)
    if edge == "nonfinite":
        assert ref["status"][:5].tolist() == [2, 3, 3, 1, 0]
        assert np.all(ref["status"][5:] == 3)
    if edge == "range":
        assert ref["status"][:5].tolist() == [1, 3, 3, 0, 0]
    base = None
    for variant, g, s in SHAPES:
        _say(f"[gpu] case=edge/{edge} variant={variant} G={g} S={s} lps={bt.num_lps}")
        got = _run(rgb, bt, variant, g, s, n1d=True)
        _check(bt, ref, got, f"edge/{edge}/{variant}/{g}x{s}")
        if base is None:
            base = got
        for a, b_ in zip(got[:3], base[:3]):
            assert np.array_equal(a, b_, equal_nan=True), f"edge/{edge}: {variant}/{g} differs from plain"


def test_malformed_offsets_are_invalid_not_read(rgb):
    import torch
    dev = torch.device("cuda:0")
    N = 8
    ax = torch.ones(N, dtype=torch.float32, device=dev)
    c = torch.ones(4, dtype=torch.float32, device=dev)
    # LP0 fine, LP1 decreasing, LP2 past the end, LP3 decreasing
    offs = torch.tensor([0, 4, 2, 100, 8], dtype=torch.int64, device=dev)
    for variant in ("plain", "batched", "persistent", "binned", "pooled"):
        _say(f"[gpu] case=malformed variant={variant}")
        x, y, st = rgb.solve_batch(offs, ax, ax, ax, c, c, variant=variant)
        torch.cuda.synchronize()
        s = st.cpu().tolist()
        assert s[0] != 3 and s[1] == 3 and s[2] == 3 and s[3] == 3, s


@pytest.mark.parametrize("m", [1, 63, 64, 65, 300, 1200, 5000])
def test_sizes_around_group_widths(rgb, oracle_lib, m):
    """LP sizes around the group widths and well beyond them."""
    bt = gen.uniform_batch(96, m, seed=m)
    ref = oracle_lib.solve(bt)
    for variant, g, s in SHAPES:
        _say(f"[gpu] case=overflow m={m} variant={variant} G={g} S={s}")
        _check(bt, ref, _run(rgb, bt, variant, g, s), f"overflow{m}/{variant}/{g}x{s}")


def test_one_huge_lp(rgb, oracle_lib):
    """One LP of 2^20 rows between small ones: the largest size class, the
    longest 1D LPs (a pooled round then serves one LP with most of the wave)."""
    bt = gen.concat([gen.uniform_batch(3, 40, seed=6), gen.uniform_batch(1, 1 << 20, seed=7),
                     gen.uniform_batch(5, 300, seed=8)])
    ref = oracle_lib.solve(bt)
    base = None
    for variant, g, s in (("plain", 0, 0), ("batched", 64, 0), ("batched", 8, 0), ("persistent", 0, 0),
                          ("binned", 0, 0), ("pooled", 4, -1), ("pooled", 16, 0)):
        _say(f"[gpu] case=huge variant={variant} G={g} S={s}")
        got = _run(rgb, bt, variant, g, s, n1d=True)
        _check(bt, ref, got, f"huge/{variant}/{g}")
        if base is None:
            base = got
        for a, b_ in zip(got, base):
            assert np.array_equal(a, b_, equal_nan=True)


def _tied_large_lps(num_lps=500, seed=11):
    """LPs of 2,100-3,600 rows whose optimum sits among exact ties: 40 rows
    with integer coefficients in [-4, 4] that all hold at an integer point p
    (half of them pass through it) and the box |x|, |y| <= 6 are scattered
    at random positions among far rows that never bind (unit normals,
    offsets 60-70).  Many rows then pass through the optimal vertex, and the
    rows attaining the last 1D LP's bound lie anywhere in the LP: in a
    kernel's LDS cache, in the memory part of its 1D LPs or in the chunk of
    the line's own row."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(2100, 3600, num_lps)
    offsets = np.zeros(num_lps + 1, np.int64)
    np.cumsum(sizes, out=offsets[1:])
    ax, ay, b = (np.empty(int(offsets[-1]), np.float32) for _ in range(3))
    box = np.array([[1, 0, 6], [-1, 0, 6], [0, 1, 6], [0, -1, 6]], np.float32)
    for k, m in enumerate(sizes):
        p = rng.integers(-3, 4, 2)
        a = rng.integers(-4, 5, (40, 2))
        slack = np.where(rng.random(40) < 0.5, 0, rng.integers(1, 5, 40))
        ints = np.concatenate([a, (a @ p + slack)[:, None]], 1).astype(np.float32)
        t = rng.random(m - 44) * 2.0 * np.pi
        far = np.stack([np.cos(t), np.sin(t), 60.0 + 10.0 * rng.random(m - 44)], 1).astype(np.float32)
        rows = np.concatenate([ints, box, far])[rng.permutation(m)]
        s, e = offsets[k], offsets[k + 1]
        ax[s:e], ay[s:e], b[s:e] = rows[:, 0], rows[:, 1], rows[:, 2]
    c = rng.integers(-4, 5, (num_lps, 2)).astype(np.float32)
    return gen.Batch(offsets, ax, ay, b, c[:, 0].copy(), c[:, 1].copy(), np.full(num_lps, gen.KIND_OTHER, np.int8),
                     "tied_large")


def test_large_lps_with_tied_bounds_match_plain(rgb, oracle_lib):
    """The second defining row of a vertex is the smallest row attaining the
    last 1D LP's bound (ties broken by index).  Kernels that find it from
    where their 1D LPs saw the bound (binned, and the group kernel on LPs of
    more than 2,048 rows at 32 or 64 lanes) must give the plain kernel's bits,
    which come from a pass over every earlier row."""
    bt = _tied_large_lps()
    ref = oracle_lib.solve(bt)
    base = _run(rgb, bt, "plain", n1d=True)
    _check(bt, ref, base, "tied_large/plain")
    for variant, g in (("binned", 0), ("batched", 64), ("batched", 32), ("batched", 16), ("persistent", 0),
                       ("pooled", 0)):
        _say(f"[gpu] case=tied_large variant={variant} G={g} lps={bt.num_lps} rows={bt.num_constraints}")
        got = _run(rgb, bt, variant, g, n1d=True)
        _check(bt, ref, got, f"tied_large/{variant}/{g}")
        for a, b_, name in zip(got, base, ("status", "x", "y", "n_1dlp")):
            assert np.array_equal(a, b_, equal_nan=True) if a.dtype.kind == "f" else np.array_equal(a, b_), \
                f"tied_large: {variant}/{g} differs from plain in {name}"


def test_largest_lp_size_every_lp(rgb, oracle_lib):
    """4,096 LPs of 8,196 rows (the largest size of the uneven recipe, where the
    kernels that record their 1D-LP bound steps do most of their work): every
    LP against the oracle, every family bit for bit against the plain kernel."""
    bt = gen.uniform_batch(4096, 8192, seed=12)
    ref = oracle_lib.solve(bt)
    base = None
    for variant, g in (("plain", 0), ("binned", 0), ("batched", 64), ("batched", 32), ("persistent", 0)):
        _say(f"[gpu] case=largest variant={variant} G={g} lps={bt.num_lps} rows={bt.num_constraints}")
        got = _run(rgb, bt, variant, g, n1d=True)
        _check(bt, ref, got, f"largest/{variant}/{g}")
        if base is None:
            base = got
        for a, b_, name in zip(got, base, ("status", "x", "y", "n_1dlp")):
            assert np.array_equal(a, b_, equal_nan=True) if a.dtype.kind == "f" else np.array_equal(a, b_), \
                f"largest: {variant}/{g} differs from plain in {name}"


# the launches the benchmark's autotuner has picked for each workload
# (batched at 16 lanes on uniform, 8 on crowd, binned on uneven), and the
# other families
FULL = [("uniform", "batched", 16), ("crowd", "batched", 8), ("uneven", "binned", 0)] + \
    [(n, v, 0) for n in ("uniform", "uneven", "crowd") for v in ("persistent", "pooled")]
_FULL_CACHE = {}


def _full(name, oracle_lib):
    if name not in _FULL_CACHE:
        _FULL_CACHE.clear()
        bt = gen.make_config(name, seed=0)
        _FULL_CACHE[name] = (bt, oracle_lib.solve(bt))
    return _FULL_CACHE[name]


@pytest.mark.parametrize("name,variant,g", sorted(FULL))
def test_full_size_every_lp(rgb, oracle_lib, name, variant, g):
    """Full-size workloads in the benchmark's launch configurations: status,
    x* and the count of 1D LPs of every LP against the oracle's solve of the
    whole batch."""
    bt, ref = _full(name, oracle_lib)
    _say(f"[gpu] case=full {name} variant={variant} lanes={g} lps={bt.num_lps} rows={bt.num_constraints}")
    got = _run(rgb, bt, variant, g, n1d=True)
    _check(bt, ref, got, f"full/{name}/{variant}/{g}")
    st = got[0]
    if name != "crowd":
        assert np.all(st[bt.kind == gen.KIND_BOXED] == OPTIMAL)
        assert np.all(st[bt.kind == gen.KIND_INFEASIBLE] == 1)
        assert np.all(st[bt.kind == gen.KIND_UNBOUNDED] == 2)
