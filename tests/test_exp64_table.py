"""Host check of the FP64 walk's exponential (k_walk.hip, exp_nonpos): the
Taylor coefficients are 1/k! rounded to double, the two-part ln2 sums to ln2
and its first part has at most 29 significant bits (so k ln2_hi is exact for
the k the walk reaches), and the reduction plus Horner's rule in FP64 stays
within 4 ulps of exp (40-digit mpmath) on -20 <= x <= 0."""
import math
import os
import re
from fractions import Fraction

import numpy as np
import pytest

mp = pytest.importorskip("mpmath")

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2609_17658_amd", "csrc", "k_walk.hip")


def _consts():
    src = open(SRC).read()
    body = re.search(r"kExpTaylor\[14\] = \{(.*?)\};", src, re.S).group(1)
    table = [float(x) for x in body.replace("\n", " ").split(",") if x.strip()]
    m = re.search(r"kLn2Hi = (\S+), kLn2Lo = (\S+), kLog2e = ([^;]+);", src)
    return table, float.fromhex(m.group(1)), float.fromhex(m.group(2)), float(m.group(3))


def test_taylor_coefficients_are_inverse_factorials():
    table, _, _, _ = _consts()
    assert table == [float(Fraction(1, math.factorial(k))) for k in range(13, -1, -1)]


def test_ln2_split():
    _, hi, lo, log2e = _consts()
    mp.mp.dps = 40
    assert abs(mp.mpf(hi) + mp.mpf(lo) - mp.log(2)) < mp.mpf(2) ** -86  # lo rounded to double
    m, _ = math.frexp(hi)
    assert (m * 2 ** 29) == int(m * 2 ** 29)  # 29 significant bits
    assert abs(log2e - float(1 / mp.log(2))) == 0.0


def test_exp_accuracy():
    table, hi, lo, log2e = _consts()
    mp.mp.dps = 40
    worst = 0.0
    for x in np.concatenate([np.linspace(-20.0, 0.0, 2001), [-1e-300, -0.0, -0.34657, -0.34658]]):
        x = max(float(x), -1100.0)
        kd = float(np.rint(x * log2e))
        r = math.fma(-kd, hi, x) if hasattr(math, "fma") else float(mp.mpf(-kd) * hi + x)
        r = math.fma(-kd, lo, r) if hasattr(math, "fma") else float(mp.mpf(-kd) * lo + r)
        y = table[0]
        for c in table[1:]:
            y = float(mp.mpf(y) * r + c)  # one rounding per step, as the device's FMA
        got = math.ldexp(y, int(kd))
        ref = mp.exp(mp.mpf(x))
        ulp = math.ulp(float(ref))
        worst = max(worst, float(abs(mp.mpf(got) - ref)) / ulp)
    assert worst <= 4.0, worst
