"""Pins the numeric constants the device exponential is built from.

The table-driven e^{-r} in the kernels uses 2^(j/64) as hi + lo pairs and a
head/tail split of ln2/64; they are checked here against high-precision
decimal arithmetic, independent of the code that wrote them.
"""
import math
import os
import re
from decimal import Decimal, getcontext
from fractions import Fraction

import pytest

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2403_07412_amd", "csrc")
HEX = r"[-+]?0x[0-9a-fA-F.]+p[-+]?\d+"

getcontext().prec = 80


def _read(name):
    with open(os.path.join(CSRC, name)) as f:
        return f.read()


def _fma(a: float, b: float, c: float) -> float:
    """a * b + c rounded once (exact rational arithmetic, correctly rounded division)."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _nearest(v: Decimal) -> float:
    """The double nearest to v (ties cannot occur for these irrational values)."""
    f = float(v)
    for cand in (math.nextafter(f, math.inf), math.nextafter(f, -math.inf)):
        if abs(Decimal(cand) - v) < abs(Decimal(f) - v):
            f = cand
    return f


def test_exp_table_is_two_to_the_j_over_64_in_two_parts():
    body = _read("exp_table.h")
    pairs = re.findall(r"\{(%s),\s*(%s)\}" % (HEX, HEX), body)
    assert len(pairs) == 64
    for j, (hi_s, lo_s) in enumerate(pairs):
        exact = Decimal(2) ** (Decimal(j) / 64)
        hi, lo = float.fromhex(hi_s), float.fromhex(lo_s)
        assert hi == _nearest(exact), j
        assert lo == _nearest(exact - Decimal(hi)), j
        # hi + lo carries about 107 bits
        assert abs(Decimal(hi) + Decimal(lo) - exact) <= exact * Decimal(2) ** -104, j


def test_exp_reduction_constants():
    body = _read("device_common.h")
    fn = body[body.index("double exp_neg_tab("):]
    fn = fn[:fn.index("\n}\n")]
    consts = [float.fromhex(c) for c in re.findall(HEX, fn)]
    inv, head, tail = consts[0], -consts[1], -consts[2]
    ln2_64 = Decimal(2).ln() / 64
    assert inv == _nearest(1 / ln2_64)
    # the head has at most 36 significant bits, so n * head is exact for |n| < 2^17
    m, e = math.frexp(head)
    assert (m * 2 ** 36).is_integer()
    assert tail == _nearest(ln2_64 - Decimal(head))
    # n (head + tail) then misses n ln2/64 by under 2^17 * 2^-90 ln2/64, far below an ulp of f
    assert abs(Decimal(head) + Decimal(tail) - ln2_64) < ln2_64 * Decimal(2) ** -90
    # largest reduced index: r up to 746 -> |n| <= 746 * 64 / ln2 < 2^17
    assert 746 * 64 / math.log(2) < 2 ** 17


@pytest.mark.parametrize("r", [0.0, 1e-300, 0.01, 0.5, 1.0, 7.25, 30.0, 300.0, 700.0, 745.0])
def test_exp_algorithm_on_host(r):
    """The same steps in Python doubles agree with math.exp to about half an ulp."""
    body = _read("exp_table.h")
    pairs = [(float.fromhex(a), float.fromhex(b)) for a, b in re.findall(r"\{(%s),\s*(%s)\}" % (HEX, HEX), body)]
    x = max(-r, -746.0)
    nf = float(round(x * float.fromhex("0x1.71547652b82fep+6")))
    n = int(nf)
    f = _fma(nf, -float.fromhex("0x1.62e42fefa0000p-7"), x)
    f = _fma(nf, -float.fromhex("0x1.cf79abc9e3b3ap-46"), f)
    q = _fma(f, 1.0 / 720.0, 1.0 / 120.0)
    for c in (1.0 / 24.0, 1.0 / 6.0, 0.5, 1.0):
        q = _fma(q, f, c)
    q *= f
    th, tl = pairs[n & 63]
    got = math.ldexp(th + _fma(th, q, tl), n >> 6)
    exact = (-Decimal(r)).exp()
    ulp = math.ulp(float(exact))
    assert abs(Decimal(got) - exact) <= Decimal(0.52) * Decimal(ulp)
