"""Pins for the 3D oracle (CPU only).  The oracle is FP64 vertex enumeration
(the definition of the optimum written out); each check here is independent
of its arithmetic: exact rational enumeration, hand-solved fixtures, closed
forms, optimality certificates, metamorphic relations and an LP library."""
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest

import lpcheck
from lpcheck import INFEASIBLE, OPTIMAL, UNBOUNDED, INVALID
from paper_1902_04995_amd import gen3


@pytest.fixture(scope="module")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


def _exact_mismatches(oracle_lib, batch, res):
    bad = []
    for k, (st, v) in enumerate(oracle_lib.brute_force3_batch(batch)):
        if st != res["status"][k]:
            bad.append((k, "status", st, int(res["status"][k])))
        elif v is not None:
            ref = np.array([float(t) for t in v])
            if not np.all(np.abs(res["x"][k] - ref) <= 1e-9 * np.maximum(1.0, np.abs(ref))):
                bad.append((k, "x", ref, res["x"][k]))
    return bad


@pytest.mark.parametrize("K,m_max,boxed,seed", [(1, 5, False, 0), (2, 6, False, 1), (3, 6, True, 2), (2, 8, True, 3)])
def test_oracle3_matches_exact_enumeration_integer(oracle_lib, K, m_max, boxed, seed):
    bt = gen3.tiny_integer_batch3(250, m_max=m_max, K=K, seed=seed, boxed=boxed)
    res = oracle_lib.solve3(bt)
    assert _exact_mismatches(oracle_lib, bt, res) == []
    counts = np.bincount(res["status"], minlength=4)
    assert counts[OPTIMAL] > 0 and counts[INFEASIBLE] > 0, counts
    assert boxed or counts[UNBOUNDED] > 0, counts


def test_oracle3_matches_exact_enumeration_continuous(oracle_lib):
    bt = gen3.tiny_random_batch3(150, m_max=9, seed=4)
    res = oracle_lib.solve3(bt)
    assert _exact_mismatches(oracle_lib, bt, res) == []


def test_oracle3_hand_solved_golden(oracle_lib):
    lps = lpcheck.parse_golden3(os.path.join(lpcheck.GOLDEN, "lp3_hand.txt"))
    assert len(lps) >= 15
    for lp, bt in zip(lps, lpcheck.golden3_batch(lps)):
        res = oracle_lib.solve3(bt, threads=1)
        st, xyz = lp["expect"]
        assert res["status"][0] == st, lp["name"]
        if xyz is not None:
            np.testing.assert_allclose(res["x"][0], xyz, atol=1e-12, err_msg=lp["name"])
        else:
            assert np.isnan(res["x"][0]).all()


def test_oracle3_circumscribed_sphere_closed_form(oracle_lib):
    """Planes tangent to the unit sphere at n Fibonacci-lattice points: the
    polytope contains the ball and lies within the sphere of radius 1/cos(r)
    (r the lattice's covering radius), so max c.x over it is between |c| and
    |c|/cos(r); the optimum lies within that band along c."""
    n = 400
    i = np.arange(n) + 0.5
    phi = np.arccos(1 - 2 * i / n)
    th = math.pi * (1 + 5 ** 0.5) * i
    nrm = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1).astype(np.float32)
    rng = np.random.default_rng(5)
    cs = rng.standard_normal((6, 3)).astype(np.float32)
    parts = []
    for c in cs:
        parts.append(gen3.Batch3(np.array([0, n], np.int64), nrm[:, 0].copy(), nrm[:, 1].copy(), nrm[:, 2].copy(),
                                 np.ones(n, np.float32), c[:1], c[1:2], c[2:], np.zeros(1, np.int8), 100.0))
    bt = gen3.concat3(parts)
    res = oracle_lib.solve3(bt)
    assert (res["status"] == OPTIMAL).all()
    cosr = math.cos(2.0 * math.sqrt(math.pi / n))  # a generous bound on the covering radius
    for k, c in enumerate(cs.astype(np.float64)):
        val = float(c @ res["x"][k])
        cn = float(np.linalg.norm(c))
        assert cn * (1 - 1e-12) <= val <= cn / cosr, (val, cn)
        assert np.linalg.norm(res["x"][k]) <= 1.0 / cosr + 1e-12


def test_oracle3_certificates_and_highs(oracle_lib):
    """Status against HiGHS (with the box as bounds), the objective value, and
    a KKT certificate for every OPTIMAL LP: feasibility and multipliers
    lambda >= 0 on the tight rows with sum lambda a = c."""
    from scipy.optimize import linprog
    bt = gen3.concat3([gen3.make_config3("uniform3", seed=2, scale=300 / 65536), gen3.uniform3_batch(60, 40, seed=3)])
    res = oracle_lib.solve3(bt)
    counts = np.bincount(res["status"], minlength=4)
    assert counts[OPTIMAL] > 0 and counts[INFEASIBLE] > 0 and counts[UNBOUNDED] > 0, counts
    for k in range(bt.num_lps):
        ax, ay, az, b, c = bt.lp(k)
        A = np.stack([ax, ay, az], 1).astype(np.float64)
        bb = b.astype(np.float64)
        cc = np.array(c, np.float64)
        lp = linprog(-cc, A_ub=A, b_ub=bb, bounds=[(-bt.box, bt.box)] * 3, method="highs")
        if lp.status == 2:
            assert res["status"][k] == INFEASIBLE, k
            continue
        assert lp.status == 0, lp.message
        assert res["status"][k] in (OPTIMAL, UNBOUNDED), k
        assert float(cc @ res["x"][k]) == pytest.approx(-lp.fun, rel=1e-9, abs=1e-9)
        if res["status"][k] == OPTIMAL:
            viol, resid = lpcheck.kkt_residual3(A, bb, cc, res["x"][k])
            assert viol <= 1e-9 and resid <= 1e-9, (k, viol, resid)
            assert np.max(np.abs(res["x"][k])) < bt.box
        else:
            assert np.max(np.abs(res["x"][k])) == pytest.approx(bt.box, rel=1e-9)


def test_oracle3_metamorphic(oracle_lib):
    """The optimum does not depend on the row order, and scaling a row by a
    power of two (exact in fp32) changes nothing; permuting the coordinates of
    rows and objective permutes a unique optimum."""
    bt = gen3.make_config3("uniform3", seed=6, scale=200 / 65536)
    base = oracle_lib.solve3(bt)
    rng = np.random.default_rng(7)
    order = np.concatenate([s + rng.permutation(e - s) for s, e in zip(bt.offsets[:-1], bt.offsets[1:])])
    r = oracle_lib.solve3(bt.with_rows(ax=bt.ax[order], ay=bt.ay[order], az=bt.az[order], b=bt.b[order]))
    assert np.array_equal(r["status"], base["status"])
    np.testing.assert_allclose(r["x"], base["x"], rtol=1e-12, atol=1e-12)
    sc = np.where(rng.random(bt.num_constraints) < 0.5, 2.0, 0.25).astype(np.float32)
    r = oracle_lib.solve3(bt.with_rows(ax=bt.ax * sc, ay=bt.ay * sc, az=bt.az * sc, b=bt.b * sc))
    assert np.array_equal(r["status"], base["status"])
    np.testing.assert_allclose(r["x"], base["x"], rtol=1e-12, atol=1e-12)
    sw = gen3.Batch3(bt.offsets, bt.ay, bt.az, bt.ax, bt.b, bt.cy, bt.cz, bt.cx, bt.kind, bt.box)
    r = oracle_lib.solve3(sw)
    assert np.array_equal(r["status"], base["status"])
    np.testing.assert_allclose(r["x"], base["x"][:, [1, 2, 0]], rtol=1e-12, atol=1e-12)


def test_oracle3_invalid_inputs(oracle_lib):
    bt = gen3.tiny_random_batch3(6, m_max=5, m_min=3, seed=9)
    ax = bt.ax.copy()
    ax[bt.offsets[1]] = np.nan
    b = bt.b.copy()
    b[bt.offsets[2]] = np.inf
    cz = bt.cz.copy()
    cz[3] = np.nan
    bad = gen3.Batch3(bt.offsets, ax, bt.ay, bt.az, b, bt.cx, bt.cy, cz, bt.kind, bt.box)
    res = oracle_lib.solve3(bad)
    assert list(res["status"][1:4]) == [INVALID] * 3
    for box in (0.0, -1.0, np.inf, np.nan):
        r = oracle_lib.solve3(bt.with_rows(box=box))
        assert (r["status"] == INVALID).all()
    # an empty LP is the box's own optimal corner
    e = gen3.Batch3(np.zeros(2, np.int64), *[np.zeros(0, np.float32)] * 4, np.float32([1]), np.float32([-2]),
                    np.float32([0]), np.zeros(1, np.int8), 3.0)
    r = oracle_lib.solve3(e)
    assert r["status"][0] == UNBOUNDED and list(r["x"][0]) == [3.0, -3.0, -3.0]


# Planted mistakes: each mutant of the oracle source must fail a pin above.
MUTANTS3 = [
    ("if (f > bf + tol) return 1;", "if (f < bf - tol) return 1;"),                 # minimises
    ("if (v[k] < bv[k] - tol) return 1;", "if (v[k] > bv[k] + tol) return 1;"),      # largest tie-break
    ("if (lhs - P[j].b > 1e-10", "if (P[j].b - lhs > 1e-10"),                       # row sense flipped
    ("P[n].a[k] = s == 0 ? 1.0 : -1.0;", "P[n].a[k] = 1.0;"),                      # one-sided box
    ("for (int j = 0; j < n && ok; ++j) {", "for (int j = 0; j + 1 < n && ok; ++j) {"),  # dropped row
    ("A2[k] = rhs[0];", "A2[k] = rhs[1];"),                                          # Cramer column
    ("if (bi < 0.0) {  /* 0 <= b fails", "if (bi > 0.0) {  /* 0 <= b fails"),        # zero-row sense
    ("*status = top >= M * (1.0 - 1e-9) ? UNBOUNDED : OPTIMAL;", "*status = OPTIMAL;"),  # box status
]


@pytest.mark.parametrize("mi", range(len(MUTANTS3)))
def test_pins_catch_planted_mistakes3(oracle_lib, mi):
    import ctypes
    src = open(os.path.join(os.path.dirname(oracle_lib.__file__), "lp3_oracle.c")).read()
    old, new = MUTANTS3[mi]
    assert src.count(old) == 1, old
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "m.c")
        so = os.path.join(d, "m.so")
        open(c, "w").write(src.replace(old, new))
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-o", so, c, "-lm"])
        lib = ctypes.CDLL(so)
        saved = oracle_lib._load3()
        lib.rgb_oracle3_solve_range.argtypes = saved.rgb_oracle3_solve_range.argtypes
        oracle_lib._lib3 = lib
        try:
            caught = False
            for bt in (gen3.tiny_integer_batch3(300, m_max=6, K=2, seed=11),
                       gen3.tiny_integer_batch3(300, m_max=6, K=2, seed=12, boxed=True),
                       gen3.tiny_random_batch3(100, m_max=8, seed=13)):
                if _exact_mismatches(oracle_lib, bt, oracle_lib.solve3(bt, threads=1)):
                    caught = True
                    break
            if not caught:
                lps = lpcheck.parse_golden3(os.path.join(lpcheck.GOLDEN, "lp3_hand.txt"))
                for lp, bt in zip(lps, lpcheck.golden3_batch(lps)):
                    r = oracle_lib.solve3(bt, threads=1)
                    st, xyz = lp["expect"]
                    if r["status"][0] != st or (xyz is not None and not np.allclose(r["x"][0], xyz)):
                        caught = True
                        break
            assert caught, MUTANTS3[mi]
        finally:
            oracle_lib._lib3 = saved
