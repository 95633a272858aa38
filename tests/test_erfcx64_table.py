"""Host check of the FP64 walk's erfcx polynomial (k_walk.hip): the table in
the source is the one its generator prints, and Horner's rule in FP64 over
it stays within 2e-15 of exp(u^2) erfc(u) (40-digit mpmath) on 0 <= u <= 3."""
import os
import re
import subprocess
import sys

import numpy as np
import pytest

mp = pytest.importorskip("mpmath")

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2609_17658_amd", "csrc")


def _table():
    src = open(os.path.join(CSRC, "k_walk.hip")).read()
    body = re.search(r"kErfcx64\[26\] = \{(.*?)\};", src, re.S).group(1)
    return [float(x) for x in body.replace("\n", " ").split(",") if x.strip()]


def test_table_matches_generator():
    out = subprocess.run([sys.executable, os.path.join(CSRC, "gen_erfcx64.py")], capture_output=True,
                         text=True, check=True).stdout
    body = re.search(r"\{(.*?)\};", out, re.S).group(1)
    gen = [float(x) for x in body.replace("\n", " ").split(",") if x.strip()]
    assert gen == _table()


def test_polynomial_accuracy():
    c = _table()
    assert len(c) == 26
    mp.mp.dps = 40
    worst = 0.0
    for u in np.linspace(0.0, 3.0, 301):
        t = u * (2.0 / 3.0) - 1.0  # the device fuses this; the difference is below 1e-16
        y = c[0]
        for a in c[1:]:
            y = y * t + a
        ref = mp.erfc(mp.mpf(u)) * mp.exp(mp.mpf(u) ** 2)
        worst = max(worst, abs(y / float(ref) - 1.0))
    assert worst <= 2e-15
