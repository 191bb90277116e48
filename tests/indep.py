"""Test-side helpers that restate the paper's basis and mode orderings in a
notation of their own, so that the oracle's tables are checked against an
independent transcription.

* P_a(x) of eq. (9) is the Legendre polynomial L_a(2x) divided by its leading
  coefficient (numpy.polynomial.legendre), i.e. the monic Legendre polynomial
  on [-1/2, 1/2].
* Modes are written as letter strings: each 'x', 'y', 'z' raises the degree
  of P in that coordinate, each 't' the power of tau.  The lists below follow
  eq. (10)-(12), (14)-(16) and the face expansions (D.2), (D.7), (D.12).
"""

import numpy as np
from numpy.polynomial import legendre as npleg

_LEAD = {0: 1.0, 1: 2.0, 2: 6.0, 3: 20.0}


def P(a, x):
    c = np.zeros(a + 1)
    c[a] = 1.0
    return npleg.legval(2.0 * np.asarray(x, dtype=np.float64), c) / _LEAD[a]


SPACE_TIME_WORDS = {
    2: "1 x y z t",
    3: "1 x y z xx yy zz xy yz xz t tt xt yt zt",
    4: ("1 x y z xx yy zz xy yz xz xxx yyy zzz xxy xxz xyy yyz xzz yzz xyz "
        "t tt ttt xt yt zt xtt ytt ztt xxt yyt zzt xyt yzt xzt"),
}

# (D.2), (D.7), (D.12) in face coordinates: 'a' = first transverse, 'b' = second.
FACE_WORDS = {
    2: "1 a b t",
    3: "1 a b aa bb ab t tt at bt",
    4: "1 a b aa bb ab aaa bbb aab abb t tt ttt at bt att btt aat bbt abt",
}


def exps(word, letters):
    if word == "1":
        return tuple(0 for _ in letters)
    return tuple(word.count(ch) for ch in letters)


def st_modes(order):
    return [exps(w, "xyzt") for w in SPACE_TIME_WORDS[order].split()]


def face_modes(order):
    return [exps(w, "abt") for w in FACE_WORDS[order].split()]


def st_value(coeffs, order, point):
    """sum_m coeffs[m] phi_m(point) with phi_m = P_a P_b P_c tau^d."""
    x, y, z, t = point
    out = 0.0
    for c, (a, b, cc, d) in zip(coeffs, st_modes(order)):
        out = out + c * P(a, x) * P(b, y) * P(cc, z) * t ** d
    return out


def face_value(coeffs, order, point):
    s1, s2, t = point
    out = 0.0
    for c, (a, b, d) in zip(coeffs, face_modes(order)):
        out = out + c * P(a, s1) * P(b, s2) * t ** d
    return out


def gauss(n, lo, hi):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (hi - lo) * x + 0.5 * (hi + lo), 0.5 * (hi - lo) * w
