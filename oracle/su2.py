"""SU(2) group data from closed formulas (oracle; test infrastructure only).

All spins and projections are passed doubled (``tj = 2j``, ``tm = 2m``) so that
half-integer spins stay integers.  Every coefficient is evaluated exactly in
rational arithmetic and rounded to FP64 only at the final square root.

Conventions follow the thesis' review of SU(2) (section "Representations of
the group SU(2)"): basis vectors of a spin-j irrep are ordered by m ascending;
J_z is diag(m) and the ladder operators act as in the ladder equation
(eq:irrepladder), which fixes the Condon-Shortley phase of the Clebsch-Gordan
coefficients (eq:cg).  (The J_y printed in Example 2 has the opposite sign of
the ladder equation; Examples 3-5 agree with it, and so does this module.)
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache

import numpy as np


def _int(x2: int) -> int:
    """Half of an even doubled quantity."""
    if x2 % 2:
        raise ValueError("half-integer where an integer is required")
    return x2 // 2


@lru_cache(maxsize=None)
def _fact(n: int) -> int:
    if n < 0:
        raise ValueError("negative factorial")
    return math.factorial(n)


def triangle(ta: int, tb: int, tc: int) -> bool:
    """Fusion rule (eq:fusionrules): |a-b| <= c <= a+b with a+b+c an integer."""
    return abs(ta - tb) <= tc <= ta + tb and (ta + tb + tc) % 2 == 0


def _signed_sqrt(sign: int, square: Fraction) -> float:
    if square == 0 or sign == 0:
        return 0.0
    return float(sign) * math.sqrt(float(square))


@lru_cache(maxsize=None)
def cg(tj1: int, tm1: int, tj2: int, tm2: int, tj: int, tm: int) -> float:
    """Clebsch-Gordan coefficient <j1 m1; j2 m2 | j m> of eq:cg (fusing j1, j2
    into j), by Racah's closed formula in exact rationals."""
    if tm1 + tm2 != tm or not triangle(tj1, tj2, tj):
        return 0.0
    for tjx, tmx in ((tj1, tm1), (tj2, tm2), (tj, tm)):
        if abs(tmx) > tjx or (tjx + tmx) % 2:
            return 0.0
    a = _int(tj1 + tj2 - tj)
    b = _int(tj1 - tj2 + tj)
    c = _int(-tj1 + tj2 + tj)
    s = _int(tj1 + tj2 + tj) + 1
    j1pm1, j1mm1 = _int(tj1 + tm1), _int(tj1 - tm1)
    j2pm2, j2mm2 = _int(tj2 + tm2), _int(tj2 - tm2)
    jpm, jmm = _int(tj + tm), _int(tj - tm)
    pref2 = Fraction((tj + 1) * _fact(a) * _fact(b) * _fact(c), _fact(s))
    pref2 *= _fact(j1pm1) * _fact(j1mm1) * _fact(j2pm2) * _fact(j2mm2) * _fact(jpm) * _fact(jmm)
    # sum over k with every factorial argument non-negative
    k_lo = max(0, _int(tj2 - tj - tm1), _int(tj1 - tj + tm2))
    k_hi = min(a, j1mm1, j2pm2)
    total = Fraction(0)
    for k in range(k_lo, k_hi + 1):
        den = (_fact(k) * _fact(a - k) * _fact(j1mm1 - k) * _fact(j2pm2 - k)
               * _fact(_int(tj - tj2 + tm1) + k) * _fact(_int(tj - tj1 - tm2) + k))
        total += Fraction((-1) ** k, den)
    if total == 0:
        return 0.0
    sign = 1 if total > 0 else -1
    return _signed_sqrt(sign, pref2 * total * total)


def cg_tensor(tj1: int, tj2: int, tj: int) -> np.ndarray:
    """C[m1, m2, m] = <j1 m1; j2 m2 | j m> with each m ascending."""
    out = np.zeros((tj1 + 1, tj2 + 1, tj + 1))
    for a in range(tj1 + 1):
        tm1 = -tj1 + 2 * a
        for b in range(tj2 + 1):
            tm2 = -tj2 + 2 * b
            tm = tm1 + tm2
            if abs(tm) <= tj:
                out[a, b, (tm + tj) // 2] = cg(tj1, tm1, tj2, tm2, tj, tm)
    return out


def _delta2(ta: int, tb: int, tc: int) -> Fraction:
    """Square of the triangle coefficient Delta(a,b,c)."""
    return Fraction(_fact(_int(ta + tb - tc)) * _fact(_int(ta - tb + tc)) * _fact(_int(-ta + tb + tc)),
                    _fact(_int(ta + tb + tc) + 1))


@lru_cache(maxsize=None)
def sixj(ta: int, tb: int, tc: int, td: int, te: int, tf: int) -> float:
    """Wigner 6j symbol {a b c; d e f} by Racah's closed formula, exactly."""
    triads = ((ta, tb, tc), (ta, te, tf), (td, tb, tf), (td, te, tc))
    if not all(triangle(*t) for t in triads):
        return 0.0
    abc, aef, dbf, dec = (_int(sum(t)) for t in triads)
    abde, bcef, cafd = _int(ta + tb + td + te), _int(tb + tc + te + tf), _int(tc + ta + tf + td)
    pref2 = Fraction(1)
    for t in triads:
        pref2 *= _delta2(*t)
    total = Fraction(0)
    for t in range(max(abc, aef, dbf, dec), min(abde, bcef, cafd) + 1):
        den = (_fact(t - abc) * _fact(t - aef) * _fact(t - dbf) * _fact(t - dec)
               * _fact(abde - t) * _fact(bcef - t) * _fact(cafd - t))
        total += Fraction((-1) ** t * _fact(t + 1), den)
    if total == 0:
        return 0.0
    sign = 1 if total > 0 else -1
    return _signed_sqrt(sign, pref2 * total * total)


def fmove(tjA: int, tjB: int, tjC: int, tjJ: int, tjD: int, tjE: int) -> float:
    """Recoupling coefficient F^{jD jE}_{jA jB jC jJ} (eq:sixj): it takes the
    coupled basis of tree {A,B->D; D,C->J} to that of {B,C->E; A,E->J}
    (eq:fmove), equal to (-1)^(jA+jB+jC+jJ) sqrt((2jD+1)(2jE+1)) {jA jB jD; jC jJ jE}."""
    s6 = sixj(tjA, tjB, tjD, tjC, tjJ, tjE)
    if s6 == 0.0:
        return 0.0
    phase = -1.0 if _int(tjA + tjB + tjC + tjJ) % 2 else 1.0
    return phase * math.sqrt((tjD + 1) * (tjE + 1)) * s6


def fmove_from_cg(tjA: int, tjB: int, tjC: int, tjJ: int, tjD: int, tjE: int) -> float:
    """The same coefficient as the overlap of the two structural tensors
    (eq:f with its last factor read as C_{A,E->J}):
    F = 1/(2J+1) sum_m C_{AB->D} C_{DC->J} C_{BC->E} C_{AE->J}."""
    if not (triangle(tjA, tjB, tjD) and triangle(tjD, tjC, tjJ)
            and triangle(tjB, tjC, tjE) and triangle(tjA, tjE, tjJ)):
        return 0.0
    qd = np.einsum("abd,dcj->abcj", cg_tensor(tjA, tjB, tjD), cg_tensor(tjD, tjC, tjJ))
    qe = np.einsum("bce,aej->abcj", cg_tensor(tjB, tjC, tjE), cg_tensor(tjA, tjE, tjJ))
    return float(np.sum(qd * qe)) / (tjJ + 1)


def swap_phase(tja: int, tjb: int, tjc: int) -> float:
    """Swap factor R = (-1)^(ja+jb-jc) of eq:braid3: C_{b,a->c} = R C_{a,b->c}."""
    return -1.0 if _int(tja + tjb - tjc) % 2 else 1.0


def omega(tj: int) -> np.ndarray:
    """omega_j of eq:singletomega: (omega)_{m,-m} = (-1)^(j-m)/sqrt(2j+1), m ascending."""
    n = tj + 1
    w = np.zeros((n, n))
    for a in range(n):
        tm = -tj + 2 * a
        w[a, n - 1 - a] = (-1.0) ** _int(tj - tm) / math.sqrt(n)
    return w


def cup(tj: int) -> np.ndarray:
    """cup_j = sqrt(2j+1) omega_j (eq:cupj)."""
    return math.sqrt(tj + 1) * omega(tj)


def cap(tj: int) -> np.ndarray:
    """cap_j = (-1)^(2j) sqrt(2j+1) omega_j (eq:capj)."""
    return ((-1.0) ** tj) * math.sqrt(tj + 1) * omega(tj)


def generators(tj: int):
    """(J_x, J_y, J_z) of the spin-j irrep from eq:irrepz and eq:irrepladder."""
    n = tj + 1
    j = tj / 2.0
    ms = [(-tj + 2 * a) / 2.0 for a in range(n)]
    jz = np.diag(ms).astype(complex)
    jp = np.zeros((n, n), dtype=complex)
    for a in range(n - 1):
        m = ms[a]
        jp[a + 1, a] = math.sqrt(j * (j + 1) - m * (m + 1))
    jm = jp.conj().T
    jx = (jp + jm) / 2.0
    jy = (jp - jm) / 2.0j
    return jx, jy, jz


def irrep_element(tj: int, r) -> np.ndarray:
    """W_r = exp(i r.J) on the spin-j irrep (eq:exp)."""
    from scipy.linalg import expm
    jx, jy, jz = generators(tj)
    return expm(1j * (r[0] * jx + r[1] * jy + r[2] * jz))
