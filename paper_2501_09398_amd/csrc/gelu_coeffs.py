"""Coefficients of the normal distribution function Phi used by the GELU
epilogues of surrogate.hip (run by hand; prints the C constants).

Phi(x) = erfc(-x / sqrt 2) / 2 in two pieces:
  |x| <= 1 : Phi(x) = 1/2 + x S(x^2), S a degree-5 polynomial (the Taylor
             series of erf is odd, so Phi - 1/2 is x times a series in x^2);
  |x| >  1 : erfc(v) = exp(-v^2) R(v), v = |x| / sqrt 2, with R = erfcx the
             scaled complementary error function, approximated on [0, 10] by
             a rational function P(v) / Q(v) of degrees (4, 5); Phi = erfc/2
             for x < 0 and 1 - erfc/2 for x > 0.
Both fits minimise the maximum relative error on a dense grid by least
squares with Lawson reweighting (Q is normalised to Q(0) = 1; the rational
fit is linearised as in Sanathanan and Koerner, 1963, with the previous
iterate's denominator as weight).  The reference values come from scipy's
erf / erfcx.
"""
import numpy as np
from scipy.special import erf, erfcx


def fit_small(deg=5, iters=60):
    x = np.linspace(1e-6, 1.0001, 40001)
    f = (0.5 * erf(x / np.sqrt(2.0))) / x            # S(x^2)
    A = np.vander(x * x, deg + 1, increasing=True)
    wgt, best = np.ones_like(x), None
    for _ in range(iters):
        c, *_ = np.linalg.lstsq(A * (wgt / f)[:, None], f * (wgt / f), rcond=None)
        r = A @ c / f - 1.0
        e = float(np.max(np.abs(r)))
        if best is None or e < best[0]:
            best = (e, c)
        wgt = wgt * np.sqrt(np.abs(r)) + 1e-30
        wgt /= wgt.max()
    return best


def fit_tail(m=4, n=5, vmax=10.0, iters=60):
    v = np.linspace(0.0, vmax, 40001)
    f = erfcx(v)
    Vp = np.vander(v, m + 1, increasing=True)
    Vq = np.vander(v, n + 1, increasing=True)[:, 1:]
    q, wgt, best = np.ones_like(v), np.ones_like(v), None
    for _ in range(iters):
        A = np.hstack([Vp, -f[:, None] * Vq])
        w = wgt / (np.abs(q) * f)
        sol, *_ = np.linalg.lstsq(A * w[:, None], f * w, rcond=None)
        a, b = sol[:m + 1], np.concatenate([[1.0], sol[m + 1:]])
        q = np.polyval(b[::-1], v)
        r = np.polyval(a[::-1], v) / q / f - 1.0
        e = float(np.max(np.abs(r)))
        if best is None or e < best[0]:
            best = (e, a, b)
        wgt = wgt * np.sqrt(np.abs(r)) + 1e-30
        wgt /= wgt.max()
    return best


def c_floats(name, v):
    body = ", ".join(f"{np.float32(c).item():.9e}f" for c in v)
    return f"constexpr float {name}[{len(v)}] = {{{body}}};"


if __name__ == "__main__":
    es, s = fit_small()
    et, a, b = fit_tail()
    print(f"// |x| <= 1: max relative error of S {es:.2e}; erfcx on [0, 10]: {et:.2e}")
    print(c_floats("kPhiS", s))
    print(c_floats("kErfcxP", a))
    print(c_floats("kErfcxQ", b))
