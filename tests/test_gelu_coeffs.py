"""The GELU epilogue's constants in surrogate.hip are the ones the fitting
script produces, and the fits meet their stated accuracy (the polynomial
and rational pieces against scipy's erf / erfcx in float64)."""
import os
import re
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2501_09398_amd", "csrc")


def parse(text, name):
    m = re.search(r"constexpr float " + name + r"\[\d+\] = \{(.*?)\};", text)
    assert m, name
    return np.array([float(v.strip().rstrip("f")) for v in m.group(1).split(",")], np.float32)


def test_gelu_constants_match_the_fit():
    out = subprocess.run([sys.executable, os.path.join(CSRC, "gelu_coeffs.py")], capture_output=True, text=True,
                         check=True).stdout
    src = open(os.path.join(CSRC, "surrogate.hip")).read()
    for name in ("kPhiS", "kErfcxP", "kErfcxQ"):
        assert np.array_equal(parse(out, name), parse(src, name)), name
    errs = [float(v) for v in re.findall(r"([0-9.]+e-[0-9]+)", out.splitlines()[0])]
    assert errs[0] < 1e-8 and errs[1] < 1e-8


def test_gelu_pieces_in_float64():
    from scipy.special import erf, erfcx
    src = open(os.path.join(CSRC, "surrogate.hip")).read()
    S = parse(src, "kPhiS").astype(np.float64)
    P = parse(src, "kErfcxP").astype(np.float64)
    Q = parse(src, "kErfcxQ").astype(np.float64)
    x = np.linspace(-1.0, 1.0, 20001)
    phi = 0.5 + x * np.polyval(S[::-1], x * x)
    assert np.max(np.abs(phi / (0.5 * (1.0 + erf(x / np.sqrt(2.0)))) - 1.0)) < 2e-7
    v = np.linspace(0.0, 10.0, 20001)
    R = np.polyval(P[::-1], v) / np.polyval(Q[::-1], v)
    assert np.max(np.abs(R / erfcx(v) - 1.0)) < 1e-7
