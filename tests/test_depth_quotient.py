"""CPU check of the arithmetic the GPU raster uses for a fragment's depth key.

The key's high word is float(area2 / s) with the quotient first rounded to
double, exactly as the oracle computes it with an IEEE division.  The kernel
(quotient_f32 in vs_common.h) forms that quotient from the hardware reciprocal
estimate with two Newton steps, the quotient and one residual step, i.e. the
FP64 division's own steps without its operand scaling and special-value
fix-up.  This test runs the same steps on the host with every multiply-add
rounded once (exact rational arithmetic, then one correctly rounded
conversion) and a reciprocal estimate anywhere within the hardware's
documented 2^-23 relative error, on operands of the depth-key form and on
quotients placed next to a double rounding midpoint (the hard cases of
correct rounding), and requires the correctly rounded double quotient every
time.  No GPU is needed; the GPU parity tests compare the keys themselves.
"""
import random
from fractions import Fraction

import numpy as np

EPS_RCP = 2.0 ** -23   # relative error bound of the hardware FP64 reciprocal estimate


def rn(x: Fraction) -> float:
    """Round an exact rational to the nearest double (ties to even)."""
    return float(x)   # int / int true division: correctly rounded


def fma(a: float, b: float, c: float) -> float:
    return rn(Fraction(a) * Fraction(b) + Fraction(c))


def rcp_estimate(s: float, delta: float) -> float:
    """A reciprocal estimate with relative error delta (|delta| <= EPS_RCP), rounded to double."""
    return rn(Fraction(1) / Fraction(s) * (1 + Fraction(delta)))


def quotient(a: float, s: float, delta: float) -> float:
    """The kernel's steps: r = rcp(s); two Newton steps; q0 = a r; q = q0 + (a - s q0) r."""
    r = rcp_estimate(s, delta)
    r = fma(r, fma(-s, r, 1.0), r)
    r = fma(r, fma(-s, r, 1.0), r)
    q0 = a * r   # one rounding, as v_mul_f64
    return fma(fma(-s, q0, a), r, q0)


def check(a: float, s: float, delta: float):
    want = rn(Fraction(a) / Fraction(s))
    got = quotient(a, s, delta)
    assert got == want, (a, s, delta, got, want)
    assert np.float32(got) == np.float32(want)


def _deltas(rng):
    return (EPS_RCP, -EPS_RCP, 0.0, rng.uniform(-EPS_RCP, EPS_RCP))


def test_depth_key_operands():
    # a = area2: a positive integer (twice a triangle's area in 1/256 px units);
    # s = E0 wa + E1 wb + E2 wc: integer edge values times reciprocal depths
    rng = random.Random(20241202)
    for _ in range(1500):
        a = float(rng.randint(1, 2 ** 40))
        w = [1.0 / rng.uniform(0.05, 500.0) for _ in range(3)]
        e = [rng.random() for _ in range(3)]
        tot = sum(e)
        E = [float(int(a * x / tot)) for x in e]
        s = (E[0] * w[0] + E[1] * w[1]) + E[2] * w[2]
        if s <= 0.0:
            continue
        for d in _deltas(rng):
            check(a, s, d)


def test_quotients_next_to_rounding_midpoints():
    # a / s within a few double ulps of a midpoint between two doubles, where
    # one rounding error too many would change the correctly rounded result
    rng = random.Random(7)
    n = 0
    for _ in range(1500):
        x = rng.uniform(0.01, 1000.0)                 # a depth
        m = Fraction(x) + Fraction(np.spacing(x)) / 2  # midpoint above x
        s = rng.uniform(1e-3, 2.0 ** 40)
        a = rn(m * Fraction(s))
        if a < 1.0:
            continue
        for d in _deltas(rng):
            check(a, s, d)
        n += 1
    assert n > 1000


def test_float_key_of_exact_midpoint_cases():
    # quotients that are exactly a double which is a float rounding midpoint
    # (ties to even at the float conversion): q = f + ulp_f / 2 exactly
    rng = random.Random(11)
    for _ in range(800):
        f = np.float32(rng.uniform(0.01, 1000.0))
        mid = Fraction(float(f)) + Fraction(float(np.spacing(f))) / 2   # exact in double
        s = float(rng.randint(1, 2 ** 20))
        a = rn(mid * Fraction(s))
        if Fraction(a) != mid * Fraction(s):
            continue   # keep only exact products, so a / s is the midpoint itself
        for d in _deltas(rng):
            check(a, s, d)
