"""Pins for the n-dimensional oracle (CPU only).  The oracle is FP64 vertex
enumeration for any n (the definition of the optimum written out); each check
here is independent of its arithmetic: exact integer enumeration, hand-solved
fixtures, the separately written 2D and 3D oracles, a closed form, reduction
to a lower dimension, optimality certificates, an LP library and metamorphic
relations."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import lpcheck
from lpcheck import INFEASIBLE, OPTIMAL, UNBOUNDED, INVALID
from paper_1902_04995_amd import gen, gen3, genn


@pytest.fixture(scope="module")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


def _exact_mismatches(oracle_lib, batch, res):
    bad = []
    for k, (st, v) in enumerate(oracle_lib.brute_force_n_batch(batch)):
        if st != res["status"][k]:
            bad.append((k, "status", st, int(res["status"][k])))
        elif v is not None:
            ref = np.array([float(t) for t in v])
            if not np.all(np.abs(res["x"][k] - ref) <= 1e-9 * np.maximum(1.0, np.abs(ref))):
                bad.append((k, "x", ref, res["x"][k]))
    return bad


EXACT_CASES = [
    # (n, kind, LPs, m_max, K, seed)
    (4, "int", 150, 6, 1, 0),
    (4, "int", 120, 5, 2, 1),
    (4, "int_boxed", 50, 4, 2, 2),
    (4, "rand", 100, 8, 2, 3),
    (5, "int", 60, 6, 1, 4),
    (5, "int_boxed", 10, 3, 1, 5),
    (5, "rand", 24, 9, 6, 6),
]


def _exact_batch(n, kind, lps, m_max, K, seed):
    if kind == "rand":  # K is the smallest row count here
        return genn.tiny_random_n_batch(n, lps, m_max=m_max, m_min=K, seed=seed)
    return genn.tiny_integer_n_batch(n, lps, m_max=m_max, K=K, seed=seed, boxed=kind == "int_boxed")


@pytest.mark.parametrize("case", EXACT_CASES, ids=lambda c: f"{c[0]}d_{c[1]}_{c[5]}")
def test_oraclen_matches_exact_enumeration(oracle_lib, case):
    bt = _exact_batch(*case)
    res = oracle_lib.solve_n(bt)
    assert _exact_mismatches(oracle_lib, bt, res) == []
    counts = np.bincount(res["status"], minlength=4)
    assert counts[OPTIMAL] > 0, counts


def test_oraclen_exact_cases_cover_every_status(oracle_lib):
    seen = np.zeros(4, np.int64)
    for case in EXACT_CASES:
        bt = _exact_batch(*case)
        seen += np.bincount(oracle_lib.solve_n(bt)["status"], minlength=4)
    assert seen[OPTIMAL] > 0 and seen[INFEASIBLE] > 0 and seen[UNBOUNDED] > 0, seen


def test_oraclen_hand_solved_golden(oracle_lib):
    lps = lpcheck.parse_golden_n(os.path.join(lpcheck.GOLDEN, "lpn_hand.txt"))
    assert len(lps) >= 18
    assert {lp["dim"] for lp in lps} >= {2, 3, 4, 5}
    for lp in lps:
        res = oracle_lib.solve_n(lpcheck.golden_n_batch(lp), threads=1)
        st, x = lp["expect"]
        assert res["status"][0] == st, lp["name"]
        if x is not None:
            np.testing.assert_allclose(res["x"][0], x, atol=1e-12, err_msg=lp["name"])
        else:
            assert np.isnan(res["x"][0]).all()


def _as_n(bt3):
    return genn.BatchN(bt3.offsets, np.stack([bt3.ax, bt3.ay, bt3.az]), bt3.b, np.stack([bt3.cx, bt3.cy, bt3.cz]),
                       bt3.kind, bt3.box, bt3.name)


def test_oraclen_agrees_with_3d_oracle(oracle_lib):
    """n = 3 against the separately written 3D oracle, on its own pinned
    workloads (degenerate integer, continuous, the sphere recipe)."""
    for bt3 in (gen3.tiny_integer_batch3(400, m_max=7, K=2, seed=21),
                gen3.tiny_integer_batch3(300, m_max=6, K=2, seed=22, boxed=True),
                gen3.tiny_random_batch3(300, m_max=20, seed=23),
                gen3.uniform3_batch(100, 40, seed=24)):
        r3 = oracle_lib.solve3(bt3)
        rn = oracle_lib.solve_n(_as_n(bt3))
        assert np.array_equal(r3["status"], rn["status"]), bt3.name
        ok = np.isfinite(r3["x"]).all(1)
        assert np.array_equal(ok, np.isfinite(rn["x"]).all(1))
        np.testing.assert_allclose(rn["x"][ok], r3["x"][ok], rtol=1e-9, atol=1e-9)


def test_oraclen_agrees_with_2d_oracle(oracle_lib):
    """n = 2 against the 2D Seidel oracle, which uses a symbolic box: LPs it
    finds infeasible or unbounded are infeasible or end on the finite box
    here, and its optimal points strictly inside the box are found here."""
    M = 4096.0
    for bt in (gen.tiny_integer_batch(600, m_max=8, K=3, seed=25), gen.tiny_random_batch(400, m_max=30, seed=26),
               gen.make_config("uniform", seed=27, scale=200 / 131072)):
        r2 = oracle_lib.solve(bt)
        bn = genn.BatchN(bt.offsets, np.stack([bt.ax, bt.ay]), bt.b, np.stack([bt.cx, bt.cy]),
                         np.zeros(bt.num_lps, np.int8), M)
        rn = oracle_lib.solve_n(bn)
        st2 = r2["status"]
        x2 = np.stack([r2["x"], r2["y"]], 1)
        inside = (st2 == OPTIMAL) & (np.abs(x2).max(1) < M * 0.5)
        assert (rn["status"][st2 == INFEASIBLE] == INFEASIBLE).all()
        assert (rn["status"][st2 == UNBOUNDED] == UNBOUNDED).all()
        assert (rn["status"][inside] == OPTIMAL).all()
        np.testing.assert_allclose(rn["x"][inside], x2[inside], rtol=1e-9, atol=1e-9)
        assert inside.sum() > bt.num_lps // 10


def test_oraclen_simplex_closed_form(oracle_lib):
    """Over the simplex x >= 0, sum x <= s the optimum of c.x is s max(0,
    max_k c_k), at s e_k for the unique largest positive c_k, else at 0."""
    rng = np.random.default_rng(28)
    for n in (2, 3, 4, 5, 6):
        rows, cs, want = [], [], []
        for _ in range(40):
            s = float(rng.integers(1, 9))
            r = np.zeros((n + 1, n + 1))
            r[:n, :n] = -np.eye(n)
            r[n, :n] = 1.0
            r[n, n] = s
            rows.append(r[rng.permutation(n + 1)])
            c = rng.standard_normal(n).astype(np.float32).astype(np.float64)
            if rng.random() < 0.2:
                c = -np.abs(c)
            cs.append(c)
            x = np.zeros(n)
            if c.max() > 0:
                x[np.argmax(c)] = s
            want.append(x)
        res = oracle_lib.solve_n(genn.from_rows(rows, cs, 100.0))
        assert (res["status"] == OPTIMAL).all(), n
        np.testing.assert_allclose(res["x"], np.array(want), atol=1e-12)


def test_oraclen_reduces_to_lower_dimension(oracle_lib):
    """An LP in n + 1 dimensions whose rows leave x_{n+1} out, plus the rows
    |x_{n+1}| <= 1 and no objective on it, is the n-dimensional LP with
    x_{n+1} = -1 (the smallest value) appended: checked for n = 3 against the
    3D oracle and for n = 4 against n = 4."""
    bt3 = gen3.concat3([gen3.tiny_random_batch3(150, m_max=15, seed=29), gen3.uniform3_batch(60, 30, seed=30, box=100.0)])
    cases = [(_as_n(bt3), oracle_lib.solve3(bt3))]
    bt4 = genn.tiny_random_n_batch(4, 120, m_max=12, seed=31)
    cases.append((bt4, oracle_lib.solve_n(bt4)))
    for bt, ref in cases:
        n = bt.dim
        rows, cs = [], []
        for k in range(bt.num_lps):
            a, b, c = bt.lp(k)
            r = np.zeros((a.shape[1] + 2, n + 2))
            r[:a.shape[1], :n] = a.T
            r[:a.shape[1], n + 1] = b
            r[-2, n], r[-1, n] = 1.0, -1.0
            r[-2:, n + 1] = 1.0
            rows.append(r)
            cs.append(list(c) + [0.0])
        up = oracle_lib.solve_n(genn.from_rows(rows, cs, bt.box))
        assert np.array_equal(up["status"], ref["status"])
        ok = np.isfinite(ref["x"]).all(1)
        np.testing.assert_allclose(up["x"][ok, :n], ref["x"][ok], rtol=1e-9, atol=1e-9)
        assert (up["x"][ok, n] == -1.0).all()


def test_oraclen_certificates_and_highs(oracle_lib):
    """Status against HiGHS (with the box as bounds), the objective value, and
    a KKT certificate for every OPTIMAL LP: feasibility and multipliers
    lambda >= 0 on the tight rows with sum lambda a = c."""
    from scipy.optimize import linprog
    for n, m in ((4, 30), (5, 20)):
        bt = genn.concat_n([genn.uniform_n_batch(n, 120, m, seed=32 + n, infeasible_frac=0.1, unbounded_frac=0.1),
                            genn.tiny_random_n_batch(n, 60, m_max=14, seed=34 + n, box=1.0e4)])
        res = oracle_lib.solve_n(bt)
        counts = np.bincount(res["status"], minlength=4)
        assert counts[OPTIMAL] > 0 and counts[INFEASIBLE] > 0 and counts[UNBOUNDED] > 0, counts
        for k in range(bt.num_lps):
            a, b, c = bt.lp(k)
            A = a.T.astype(np.float64)
            bb = b.astype(np.float64)
            lp = linprog(-c, A_ub=A, b_ub=bb, bounds=[(-bt.box, bt.box)] * n, method="highs")
            if lp.status == 2:
                assert res["status"][k] == INFEASIBLE, k
                continue
            assert lp.status == 0, lp.message
            assert res["status"][k] in (OPTIMAL, UNBOUNDED), k
            assert float(c @ res["x"][k]) == pytest.approx(-lp.fun, rel=1e-9, abs=1e-9)
            if res["status"][k] == OPTIMAL:
                viol, resid = lpcheck.kkt_residual3(A, bb, c, res["x"][k])
                assert viol <= 1e-9 and resid <= 1e-9, (n, k, viol, resid)
                assert np.max(np.abs(res["x"][k])) < bt.box
            else:
                assert np.max(np.abs(res["x"][k])) == pytest.approx(bt.box, rel=1e-9)


def test_oraclen_metamorphic(oracle_lib):
    """The optimum does not depend on the row order, and scaling a row by a
    power of two (exact in fp32) changes nothing; permuting the coordinates of
    rows and objective permutes a unique optimum."""
    for n in (4, 5):
        bt = genn.uniform_n_batch(n, 150, 24, seed=40 + n)
        base = oracle_lib.solve_n(bt)
        rng = np.random.default_rng(42 + n)
        order = np.concatenate([s + rng.permutation(e - s) for s, e in zip(bt.offsets[:-1], bt.offsets[1:])])
        r = oracle_lib.solve_n(bt.with_rows(a=bt.a[:, order], b=bt.b[order]))
        assert np.array_equal(r["status"], base["status"])
        np.testing.assert_allclose(r["x"], base["x"], rtol=1e-12, atol=1e-12)
        sc = np.where(rng.random(bt.num_constraints) < 0.5, 2.0, 0.25).astype(np.float32)
        r = oracle_lib.solve_n(bt.with_rows(a=bt.a * sc, b=bt.b * sc))
        assert np.array_equal(r["status"], base["status"])
        np.testing.assert_allclose(r["x"], base["x"], rtol=1e-12, atol=1e-12)
        perm = rng.permutation(n)
        r = oracle_lib.solve_n(bt.with_rows(a=bt.a[perm], c=bt.c[perm]))
        assert np.array_equal(r["status"], base["status"])
        np.testing.assert_allclose(r["x"], base["x"][:, perm], rtol=1e-12, atol=1e-12)


def test_oraclen_invalid_inputs(oracle_lib):
    bt = genn.tiny_random_n_batch(4, 6, m_max=5, m_min=3, seed=50)
    a = bt.a.copy()
    a[2, bt.offsets[1]] = np.nan
    b = bt.b.copy()
    b[bt.offsets[2]] = np.inf
    c = bt.c.copy()
    c[3, 3] = -np.inf
    res = oracle_lib.solve_n(bt.with_rows(a=a, b=b, c=c))
    assert list(res["status"][1:4]) == [INVALID] * 3
    assert np.isnan(res["x"][1:4]).all()
    for box in (0.0, -1.0, np.inf, np.nan):
        r = oracle_lib.solve_n(bt.with_rows(box=box))
        assert (r["status"] == INVALID).all()
    bad = genn.BatchN(np.zeros(2, np.int64), np.zeros((7, 0), np.float32), np.zeros(0, np.float32),
                      np.zeros((7, 1), np.float32), np.zeros(1, np.int8), 1.0)
    with pytest.raises(ValueError):
        oracle_lib.solve_n(bad)


# Planted mistakes: each mutant of the oracle source must fail a pin above.
MUTANTSN = [
    ("if (f > bf + tol) return 1;", "if (f < bf - tol) return 1;"),                   # minimises
    ("if (v[k] < bv[k] - tol) return 1;", "if (v[k] > bv[k] + tol) return 1;"),        # largest tie-break
    ("if (lhs - P[j].b > 1e-10", "if (P[j].b - lhs > 1e-10"),                         # row sense flipped
    ("P[np].a[k] = s == 0 ? 1.0 : -1.0;", "P[np].a[k] = 1.0;"),                      # one-sided box
    ("for (int j = 0; j < np && ok; ++j) {", "for (int j = 0; j + 1 < np && ok; ++j) {"),  # dropped row
    ("for (int i = col + 1; i < n; ++i) {\n            double f", "for (int i = col + 2; i < n; ++i) {\n            double f"),  # skipped elimination
    ("if (b[i] < 0.0) { /* 0 <= b fails", "if (b[i] > 0.0) { /* 0 <= b fails"),        # zero-row sense
    ("*status = top >= M * (1.0 - 1e-9) ? UNBOUNDED : OPTIMAL;", "*status = OPTIMAL;"),  # box status
    ("if (intersect(n, H, v)) {", "if (idx[0] != 1 && intersect(n, H, v)) {"),        # subsets skipped
]


@pytest.mark.parametrize("mi", range(len(MUTANTSN)))
def test_pins_catch_planted_mistakes_n(oracle_lib, mi):
    import ctypes
    src = open(os.path.join(os.path.dirname(oracle_lib.__file__), "lpn_oracle.c")).read()
    old, new = MUTANTSN[mi]
    assert src.count(old) == 1, old
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "m.c")
        so = os.path.join(d, "m.so")
        open(c, "w").write(src.replace(old, new))
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-o", so, c, "-lm"])
        lib = ctypes.CDLL(so)
        saved = oracle_lib._loadn()
        lib.rgb_oraclen_solve_range.argtypes = saved.rgb_oraclen_solve_range.argtypes
        lib.rgb_oraclen_solve_range.restype = ctypes.c_int
        oracle_lib._libn = lib
        try:
            caught = False
            for lp in lpcheck.parse_golden_n(os.path.join(lpcheck.GOLDEN, "lpn_hand.txt")):
                r = oracle_lib.solve_n(lpcheck.golden_n_batch(lp), threads=1)
                st, x = lp["expect"]
                if r["status"][0] != st or (x is not None and not np.allclose(r["x"][0], x)):
                    caught = True
                    break
            if not caught:
                for case in EXACT_CASES[:2]:
                    bt = _exact_batch(*case)
                    if _exact_mismatches(oracle_lib, bt, oracle_lib.solve_n(bt, threads=1)):
                        caught = True
                        break
            assert caught, MUTANTSN[mi]
        finally:
            oracle_lib._libn = saved
