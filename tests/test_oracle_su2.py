"""Pins of the oracle's SU(2) group data against the thesis and against
closed forms / an exact library (sympy's Wigner symbols)."""
import itertools
import math

import numpy as np
import pytest

from oracle import su2
from tests.conftest import golden_path


def _read_rows(name):
    rows = []
    for line in open(golden_path(name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(line.split())
    return rows


def test_cg_example6_values():
    # Example 6: CG values of 1/2 (x) 1/2
    for r in _read_rows("cg_example6.txt"):
        tj1, tm1, tj2, tm2, tj, tm, sgn, num, den = map(int, r)
        want = sgn * math.sqrt(num / den)
        assert su2.cg(tj1, tm1, tj2, tm2, tj, tm) == pytest.approx(want, abs=1e-15)


def test_cg_matches_sympy_exact():
    from sympy import Rational as R
    from sympy.physics.wigner import clebsch_gordan
    for tj1, tj2, tj in itertools.product(range(0, 7), repeat=3):
        if not su2.triangle(tj1, tj2, tj):
            continue
        for tm1 in range(-tj1, tj1 + 1, 2):
            for tm2 in range(-tj2, tj2 + 1, 2):
                tm = tm1 + tm2
                if abs(tm) > tj:
                    continue
                ref = float(clebsch_gordan(R(tj1, 2), R(tj2, 2), R(tj, 2), R(tm1, 2), R(tm2, 2), R(tm, 2)))
                assert su2.cg(tj1, tm1, tj2, tm2, tj, tm) == pytest.approx(ref, abs=2e-16)


def test_cg_orthogonality():
    # eq:cgunitary, both identities, for every pair of spins up to 5/2
    for tj1, tj2 in itertools.product(range(0, 6), repeat=2):
        js = [tj for tj in range(abs(tj1 - tj2), tj1 + tj2 + 1, 2)]
        # stack all coupled columns: (m1,m2) x (J,M)
        cols = np.concatenate([su2.cg_tensor(tj1, tj2, tj).reshape((tj1 + 1) * (tj2 + 1), tj + 1)
                               for tj in js], axis=1)
        assert cols.shape[0] == cols.shape[1]
        np.testing.assert_allclose(cols.T @ cols, np.eye(cols.shape[0]), atol=1e-14)
        np.testing.assert_allclose(cols @ cols.T, np.eye(cols.shape[0]), atol=1e-14)


def test_cg_selection_rules():
    assert su2.cg(2, 0, 2, 0, 2, 0) == 0.0          # <1 0;1 0|1 0> = 0
    assert su2.cg(2, 2, 2, 0, 2, 0) == 0.0          # m1+m2 != m
    assert su2.cg(2, 0, 2, 0, 6, 0) == 0.0          # triangle violated
    assert su2.cg(1, 1, 2, 0, 1, 1) != 0.0


def _read_matrices(name):
    mats, cur, label = {}, None, None
    for line in open(golden_path(name)):
        line = line.strip()
        if line.startswith("# matrix"):
            _, _, label, n = line.split()
            cur = []
            mats[label] = cur
            continue
        if not line or line.startswith("#"):
            continue
        row = []
        for tok in line.split():
            a, b = map(int, tok.split("/"))
            row.append(math.copysign(math.sqrt(abs(a) / b), a) if a else 0.0)
        cur.append(row)
    return {k: np.array(v) for k, v in mats.items()}


def test_generators_examples():
    g = _read_matrices("generators_examples.txt")
    jx, jy, jz = su2.generators(2)
    np.testing.assert_allclose(jx, g["Jx"], atol=1e-15)
    np.testing.assert_allclose(jy.imag, g["Jy_imag"], atol=1e-15)
    np.testing.assert_allclose(jy.real, 0, atol=1e-15)
    np.testing.assert_allclose(jz, g["Jz"], atol=1e-15)
    from oracle import invariance as I
    import workloads as W
    jx5, jy5, jz5 = I.leg_generators(W.Leg((0, 2), (2, 1), "out"))
    np.testing.assert_allclose(jx5, g["Jx5"], atol=1e-15)
    np.testing.assert_allclose(jy5.imag, g["Jy5_imag"], atol=1e-15)
    np.testing.assert_allclose(jz5, g["Jz5"], atol=1e-15)
    jx4, jy4, _ = I.leg_generators(W.Leg((1,), (3,), "out"))
    np.testing.assert_allclose(jx4, g["Jx4"], atol=1e-15)
    np.testing.assert_allclose(jy4.imag, g["Jy4_imag"], atol=1e-15)


def test_generators_algebra_and_casimir():
    # eq:algebra and eq:irrepz for spins up to 4
    for tj in range(0, 9):
        jx, jy, jz = su2.generators(tj)
        np.testing.assert_allclose(jx @ jy - jy @ jx, 1j * jz, atol=1e-12)
        np.testing.assert_allclose(jy @ jz - jz @ jy, 1j * jx, atol=1e-12)
        np.testing.assert_allclose(jz @ jx - jx @ jz, 1j * jy, atol=1e-12)
        j = tj / 2
        np.testing.assert_allclose(jx @ jx + jy @ jy + jz @ jz, j * (j + 1) * np.eye(tj + 1), atol=1e-12)


def test_cg_intertwines_generators():
    # C maps the product basis to the coupled one: (J1 + J2) C = C J
    for tj1, tj2 in itertools.product(range(0, 5), repeat=2):
        g1, g2 = su2.generators(tj1), su2.generators(tj2)
        for tj in range(abs(tj1 - tj2), tj1 + tj2 + 1, 2):
            c = su2.cg_tensor(tj1, tj2, tj).reshape(-1, tj + 1)
            g = su2.generators(tj)
            for k in range(3):
                tot = np.kron(g1[k], np.eye(tj2 + 1)) + np.kron(np.eye(tj1 + 1), g2[k])
                np.testing.assert_allclose(tot @ c, c @ g[k], atol=1e-12)


def test_omega_example10_and_formula():
    rows = _read_rows("omega_example10.txt")
    w1 = np.array([[float(x) for x in r] for r in rows[:3]]) / math.sqrt(3)
    w2 = np.array([[float(x) for x in r] for r in rows[3:]]) / math.sqrt(5)
    np.testing.assert_allclose(su2.omega(2), w1, atol=1e-15)
    np.testing.assert_allclose(su2.omega(4), w2, atol=1e-15)
    assert su2.omega(0)[0, 0] == 1.0
    # eq:singletomega: omega_{m,-m} equals the CG coupling (j,m),(j,-m) to spin 0
    for tj in range(0, 7):
        w = su2.omega(tj)
        for a in range(tj + 1):
            tm = -tj + 2 * a
            assert w[a, tj - a] == pytest.approx(su2.cg(tj, tm, tj, -tm, 0, 0), abs=1e-15)


def test_cup_cap_inverse():
    # eq:wiggle
    for tj in range(0, 9):
        np.testing.assert_allclose(su2.cup(tj) @ su2.cap(tj), np.eye(tj + 1), atol=1e-14)
        np.testing.assert_allclose(su2.cap(tj) @ su2.cup(tj), np.eye(tj + 1), atol=1e-14)


def test_sixj_matches_sympy():
    from sympy import Rational as R
    from sympy.physics.wigner import wigner_6j
    n = 0
    for t in itertools.product(range(0, 6), repeat=6):
        ta, tb, tc, td, te, tf = t
        ok = all(su2.triangle(*x) for x in ((ta, tb, tc), (ta, te, tf), (td, tb, tf), (td, te, tc)))
        if not ok:
            assert su2.sixj(*t) == 0.0
            continue
        assert su2.sixj(*t) == pytest.approx(float(wigner_6j(*[R(x, 2) for x in t])), abs=1e-15)
        n += 1
    assert n > 1000


def test_sixj_large_spins_against_sympy():
    from sympy import Rational as R
    from sympy.physics.wigner import wigner_6j
    cases = [(16, 16, 16, 16, 16, 16), (8, 16, 12, 16, 8, 12), (15, 9, 8, 7, 10, 11),
             (16, 8, 8, 8, 16, 8), (13, 11, 8, 9, 12, 15), (16, 15, 9, 16, 13, 8)]
    for t in cases:
        ta, tb, tc, td, te, tf = t
        if not all(su2.triangle(*x) for x in ((ta, tb, tc), (ta, te, tf), (td, tb, tf), (td, te, tc))):
            assert su2.sixj(*t) == 0.0
            continue
        assert su2.sixj(*t) == pytest.approx(float(wigner_6j(*[R(x, 2) for x in t])), abs=1e-15)


def test_fmove_equals_cg_overlap():
    # eq:sixj against eq:f (fourth factor read as C_{A,E->ABC})
    for t in itertools.product(range(0, 5), repeat=6):
        assert su2.fmove(*t) == pytest.approx(su2.fmove_from_cg(*t), abs=1e-14)


def test_fmove_orthogonal_and_trivial_cases():
    for tA, tB, tC, tJ in itertools.product(range(0, 7), repeat=4):
        ds = [d for d in range(0, 13) if su2.triangle(tA, tB, d) and su2.triangle(d, tC, tJ)]
        es = [e for e in range(0, 13) if su2.triangle(tB, tC, e) and su2.triangle(tA, e, tJ)]
        assert len(ds) == len(es)
        if not ds:
            continue
        f = np.array([[su2.fmove(tA, tB, tC, tJ, d, e) for e in es] for d in ds])
        np.testing.assert_allclose(f @ f.T, np.eye(len(ds)), atol=1e-13)
    # a spin-0 leg makes the recoupling trivial
    for tB, tC in itertools.product(range(0, 6), repeat=2):
        for tJ in range(abs(tB - tC), tB + tC + 1, 2):
            assert su2.fmove(0, tB, tC, tJ, tB, tJ) == pytest.approx(1.0, abs=1e-14)


def test_swap_phase_is_cg_symmetry():
    # eq:braid3: C_{b,a->c} = R C_{a,b->c}, and R^2 = 1
    for ta, tb in itertools.product(range(0, 6), repeat=2):
        for tc in range(abs(ta - tb), ta + tb + 1, 2):
            r = su2.swap_phase(ta, tb, tc)
            assert r * r == 1.0
            cab = su2.cg_tensor(ta, tb, tc)
            cba = su2.cg_tensor(tb, ta, tc)
            np.testing.assert_allclose(np.transpose(cba, (1, 0, 2)), r * cab, atol=1e-14)
