"""Accuracy of the assembly kernel's sin/cos of the Green's function phase
(sincos_phase in csrc/assemble.hip): Cody-Waite reduction by pi/2 with a
three-part constant, then Taylor series on the reduced argument.

The constants and coefficients are read from the kernel source, and the
device arithmetic is reproduced exactly on the host: each fused multiply-add
is evaluated in rational arithmetic and rounded once (IEEE round to nearest
even), plain products and rint likewise.  The result is compared with the
host's libm sin/cos (accurate to within an ulp) over the documented argument
range, including the quadrant boundaries."""

import math
import os
import re
from fractions import Fraction

import numpy as np

SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", "paper_2308_01457_amd", "csrc",
                   "assemble.hip")


def _kernel_constants():
    s = open(SRC).read()
    body = s[s.index("void sincos_phase("):]
    body = body[:body.index("\n}\n")]
    hexes = dict(re.findall(r"(kTwoOverPi|P1|P2|P3) = (-?0x[0-9a-fA-Fp.+-]+)", body))
    c = {k: float.fromhex(v) for k, v in hexes.items()}
    ps = re.findall(r"double ps = ([-0-9.e]+);", body) + re.findall(r"ps = fma\(ps, r2, ([-0-9.e]+)\);", body)
    pc = re.findall(r"double pc = ([-0-9.e]+);", body) + re.findall(r"pc = fma\(pc, r2, ([-0-9.e]+)\);", body)
    vmax = float(re.search(r"kTrigPhaseMax = ([0-9.e]+);", s).group(1))
    return c, [float(v) for v in ps], [float(v) for v in pc], vmax


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _sincos_phase(x, c, ps, pc):
    n = float(np.rint(x * c["kTwoOverPi"]))
    r = _fma(-n, c["P1"], x)
    r = _fma(-n, c["P2"], r)
    r = _fma(-n, c["P3"], r)
    r2 = r * r
    s = ps[0]
    for a in ps[1:]:
        s = _fma(s, r2, a)
    s = _fma(s * r2, r, r)
    co = pc[0]
    for a in pc[1:]:
        co = _fma(co, r2, a)
    q = int(n) & 3
    s0, c0 = (co, s) if q & 1 else (s, co)
    return (-s0 if q & 2 else s0), (-c0 if (q + 1) & 2 else c0)


def test_constants_are_the_series_and_pi_over_two():
    c, ps, pc, vmax = _kernel_constants()
    assert len(ps) == 8 and len(pc) == 9
    # Taylor coefficients (-1)^j / (2j+1)! and (-1)^j / (2j)!, highest degree first
    for a, j in zip(ps, range(8, 0, -1)):
        assert a == (-1) ** j / math.factorial(2 * j + 1)
    for a, j in zip(pc, range(8, -1, -1)):
        assert a == (-1) ** j / math.factorial(2 * j)
    # P1 + P2 + P3 is pi/2 to ~2^-160; compare with 60 digits of pi
    pi60 = Fraction("3.14159265358979323846264338327950288419716939937510582097494")
    err = Fraction(c["P1"]) + Fraction(c["P2"]) + Fraction(c["P3"]) - pi60 / 2
    assert abs(float(err)) < 2.0 ** -160
    assert c["P1"] == float(pi60 / 2) and abs(c["kTwoOverPi"] - float(2 / pi60)) == 0.0
    assert vmax == 1e5


def test_accuracy_over_the_phase_range():
    c, ps, pc, vmax = _kernel_constants()
    rng = np.random.default_rng(5)
    xs = list(rng.uniform(-40.0, 40.0, 1500)) + list(rng.uniform(-vmax, vmax, 300))
    # quadrant boundaries and their neighbours, tiny and zero arguments
    for m in range(-60, 61):
        b = m * math.pi / 4
        xs += [b, math.nextafter(b, math.inf), math.nextafter(b, -math.inf)]
    xs += [0.0, -0.0, 1e-300, -1e-20, 5e-9]
    worst = 0.0
    for x in xs:
        s, co = _sincos_phase(float(x), c, ps, pc)
        worst = max(worst, abs(s - math.sin(x)), abs(co - math.cos(x)))
    # about an ulp of a result of magnitude <= 1 (2^-53 = 1.1e-16), plus the
    # reduction error that grows with |x| (|n| ulp(P3)-level terms)
    assert worst < 4e-16, worst
