"""The series constants of the device sine and cosine, checked on the CPU.

The walk directions and the manufactured sources evaluate sin(pi y) and
cos(pi y) by an exact reduction to |f| <= 1/4 and the Maclaurin series of
sin(pi f), cos(pi f); the nonlinearity's sine uses the plain Maclaurin series
for |u| <= 2.  These tests read the coefficients from the device header and
pin them to the mathematics: each one against (-1)^k pi^(2k+1)/(2k+1)! (or
the factorial) computed to 60 digits, and the truncated series, evaluated in
double precision in the same Horner order, against the correctly rounded
sine and cosine over the whole reduced range.  A mistyped digit, a dropped
term or a wrong sign fails one of them.
"""
import math
import os
import re
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "paper_2608_22190_amd", "csrc", "hpsmc_device.h")
getcontext().prec = 60


def _pi():
    """pi to 60 digits by Machin's formula."""
    def atan_inv(x):
        x = Decimal(x)
        s, t, n, k = Decimal(0), 1 / x, 1, 0
        while True:
            term = t / n
            if term < Decimal(10) ** -58:
                return s
            s += term if k % 2 == 0 else -term
            t /= x * x
            n += 2
            k += 1
    return 16 * atan_inv(5) - 4 * atan_inv(239)


PI = _pi()


def _body(signature):
    text = open(HEADER).read()
    i = text.index(signature)
    j = text.index("\n}\n", i)
    return text[i:j]


def _hex_floats(body):
    return [float.fromhex(h) for h in re.findall(r"-?0x1\.[0-9a-f]+p[+-]\d+", body)]


def _coefficients_fp64():
    """(sine coefficients highest first, cosine coefficients highest first) of the FP64 routine."""
    vals = _hex_floats(_body("__device__ __forceinline__ void sincospi_series(double y"))
    assert len(vals) == 17, len(vals)
    return vals[:9], vals[9:]


def test_pi_reference():
    assert abs(float(PI) - math.pi) == 0.0
    assert str(PI).startswith("3.14159265358979323846264338327950288419716939937510")


def test_fp64_sincospi_coefficients_are_the_maclaurin_coefficients():
    sc, cc = _coefficients_fp64()
    for idx, v in enumerate(reversed(sc)):      # k = 0 .. 8: (-1)^k pi^(2k+1) / (2k+1)!
        exact = (-1) ** idx * PI ** (2 * idx + 1) / math.factorial(2 * idx + 1)
        assert v == float(exact), (idx, v, exact)
    for idx, v in enumerate(reversed(cc)):      # k = 1 .. 8 (the constant term 1 is a literal)
        k = idx + 1
        exact = (-1) ** k * PI ** (2 * k) / math.factorial(2 * k)
        assert v == float(exact), (k, v, exact)


def test_fp32_sincospi_coefficients_are_the_fp64_ones_rounded():
    sc, cc = _coefficients_fp64()
    vals = _hex_floats(_body("__device__ __forceinline__ void sincospi_series(float y"))
    # FP32 keeps the lowest five sine and five (non-constant) cosine coefficients
    assert vals[:5] == sc[-5:]
    assert vals[5:] == cc[-5:]


def _sincospi_fp64(y, coefficients=None):
    """The device routine's steps in double precision: exact reduction, Horner, quarter turns."""
    sc, cc = coefficients or _coefficients_fp64()
    n = float(np.rint(2.0 * y))
    f = y - 0.5 * n                              # exact for the arguments used
    z = f * f
    ps = sc[0]
    for c in sc[1:]:
        ps = ps * z + c
    pc = cc[0]
    for c in cc[1:]:
        pc = pc * z + c
    sn, cs = ps * f, pc * z + 1.0
    q = int(n)
    a, b = (cs, sn) if q & 1 else (sn, cs)
    return (-a if q & 2 else a), (-b if (q + 1) & 2 else b)


def _sin_cos_pi_ref(y):
    """sin(pi y), cos(pi y) from the 60-digit pi by their Taylor series in Decimal."""
    fr = Fraction(float(y))
    x = Decimal(fr.numerator) / Decimal(fr.denominator) * PI
    rs, rc, t_s, t_c = Decimal(0), Decimal(0), x, Decimal(1)
    for m in range(40):
        rs += t_s
        rc += t_c
        t_s *= -x * x / ((2 * m + 2) * (2 * m + 3))
        t_c *= -x * x / ((2 * m + 1) * (2 * m + 2))
    return float(rs), float(rc)


def test_fp64_sincospi_accuracy_over_the_reduced_range():
    """Within 3e-16 of sin(pi y), cos(pi y) for y in [-2, 2] (the walk uses (0, 2), sources [-1, 1])."""
    worst = 0.0
    for y in np.linspace(-2.0, 2.0, 4001):
        s, c = _sincospi_fp64(float(y))
        rs, rc = _sin_cos_pi_ref(y)
        worst = max(worst, abs(s - rs), abs(c - rc))
    print(f"max |error| = {worst:.3e}")
    assert worst < 3e-16


def test_fp64_sine_of_u_series():
    """The nonlinearity's FP64 series: the literals are 1/(2k+1)!, and the series is within
    two units in the last place of 1 (4.44e-16) of sin u for |u| <= 2.  The host rounds the
    final multiply-add twice where the device fuses it, hence the second unit."""
    body = _body("__device__ __forceinline__ double sin_of_u(double u)")
    dens = [int(d) for d in re.findall(r"1\.0 / (\d+)\.0", body)]
    assert dens == [math.factorial(n) for n in range(27, 2, -2)], dens
    signs = re.findall(r"(-?)1\.0 / \d+\.0", body)
    assert signs == ["" if k % 2 == 0 else "-" for k in range(len(signs))], signs
    worst = 0.0
    for u in np.linspace(-2.0, 2.0, 8001):
        z = u * u
        p = 0.0
        for k, d in enumerate(dens):
            c = 1.0 / d if k % 2 == 0 else -1.0 / d
            p = c if k == 0 else p * z + c
        val = -p * z * u + u
        worst = max(worst, abs(val - math.sin(u)))
    assert worst <= 2 * 2.0 ** -52, worst


def _worst_sine_error(coefficients):
    worst = 0.0
    for y in np.linspace(-0.25, 0.25, 2001):
        s, _ = _sincospi_fp64(float(y), coefficients)
        worst = max(worst, abs(s - math.sin(math.pi * y)))
    return worst


@pytest.mark.parametrize("bad", [None, "drop_term", "flip_sign", "perturb"])
def test_the_pins_reject_plausible_mistakes(bad):
    """A series with a dropped term, a flipped sign or a perturbed digit fails the accuracy
    bar that the header's series meets (the case None is that control)."""
    sc, cc = _coefficients_fp64()
    sc2 = list(sc)
    if bad == "drop_term":
        sc2[1] = 0.0            # the f^15 term
    elif bad == "flip_sign":
        sc2[-2] = -sc2[-2]
    elif bad == "perturb":
        sc2[-3] = sc2[-3] * (1 + 1e-12)
    worst = _worst_sine_error((sc2, cc))
    if bad is None:
        assert worst <= 3e-16, worst
    else:
        assert worst > 3e-16, worst
