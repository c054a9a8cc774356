"""The double-precision exp/expm1 kernel polynomial of the device code: its
ten coefficients are the Remez fit that gen_exp_minimax.py computes (the
degree-9 minimax polynomial of (e^r - 1 - r)/r^2 on [-ln2/2, ln2/2]), the
fit equioscillates at its stated level, and the double-precision evaluation
of e^r - 1 as the kernel performs it (every fused multiply-add rounded once,
simulated exactly) stays within one ulp of e^r and of e^r - 1."""
import importlib.util
import math
import os
import random
import re
from decimal import Decimal
from fractions import Fraction

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2401_01745_amd", "csrc")


def _gen():
    spec = importlib.util.spec_from_file_location("gen_exp_minimax", os.path.join(CSRC, "gen_exp_minimax.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _device_coefficients():
    """c0..c9 of the double expm1_reduced, read from the device header."""
    src = open(os.path.join(CSRC, "emrkc_device.h")).read()
    body = src[src.index("__device__ __forceinline__ double expm1_reduced"):]
    body = body[:body.index("\n}\n")]
    lits = re.findall(r"(0x1\.[0-9a-f]+p-?\d+)", body)
    assert len(lits) == 10, lits
    return [float.fromhex(x) for x in reversed(lits)]  # listed from c9 down to c0


def test_device_coefficients_are_the_remez_fit():
    gen = _gen()
    c, level, maxerr = gen.remez()
    # converged: the error equioscillates at the level of the last reference
    assert float(level) < 1.1e-16 and abs(float(maxerr - level)) <= 1e-3 * float(level)
    dev = _device_coefficients()
    assert dev == [float(cj) for cj in c]
    # the rounded coefficients keep the fit's error (Decimal evaluation)
    A = gen.A
    worst = Decimal(0)
    for i in range(801):
        r = -A + 2 * A * Decimal(i) / 800
        p = Decimal(0)
        for cj in reversed(dev):
            p = p * r + Decimal(cj)
        worst = max(worst, abs(p - gen.f(r)))
    assert float(worst) <= 1.2e-16, float(worst)


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))  # one rounding (correctly rounded division)


def test_double_evaluation_within_one_ulp():
    dev = _device_coefficients()

    def q_of(r):  # the kernel's operations for e^r - 1 on the reduced argument
        p = dev[-1]
        for cj in reversed(dev[:-1]):
            p = _fma(p, r, cj)
        return _fma(float(Fraction(p) * Fraction(r)), r, r)

    def ref(r):  # e^r - 1 to 40 digits
        d, s, t, j = Decimal(r), Decimal(0), Decimal(r), 1
        while abs(t) > Decimal(10) ** -38:
            s += t
            j += 1
            t = t * d / j
        return s

    random.seed(3)
    a = math.log(2) / 2
    rs = [random.uniform(-a, a) for _ in range(1500)] + [a, -a, 1e-3, -1e-3, 1e-8, 0.25, -0.25]
    for r in rs:
        q, R = q_of(r), ref(r)
        assert abs(Decimal(q) - R) <= Decimal(math.ulp(float(R))), r            # expm1 (k = 0)
        assert abs(Decimal(q + 1.0) - (R + 1)) <= Decimal(math.ulp(float(R + 1))), r  # exp
