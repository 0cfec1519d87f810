"""CPU check of the numerical method behind the mixed path's FP64 log and exp
(the zeta -> b power of Eq. 2): the same steps -- range reduction, the atanh
series of ln m through s^9, the Taylor series of e^r through r^8, ln 2 split
into a 21-bit head and a tail, reciprocals from an estimate good to a float
ulp plus one Newton step -- evaluated here with exactly rounded IEEE
arithmetic (fma emulated through rationals) and compared with 50-digit
references.  The series are cut for the accuracy the mixed path can use: zeta
itself is an FP32 sum, so b is only known to ~1e-8 relative there.  The GPU
parity tests check the kernel itself."""
import decimal
import math
import random
from fractions import Fraction

decimal.getcontext().prec = 50
LN2_HI = float.fromhex("0x1.62e42p-1")
LN2_LO = float.fromhex("0x1.fdf473de6af28p-22")
LOG2E = 1.4426950408889634


def fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def recip(d):
    # the hardware estimate, modelled as 1/d to within a float ulp (the
    # largest error that one Newton step still takes below 2^-46)
    r = 1.0 / d
    r *= 1.0 + 2.0 ** -23
    return fma(fma(-d, r, 1.0), r, r)


def ln_steps(y):
    m, e = math.frexp(y)
    if m < 0.7071067811865476:
        m += m
        e -= 1
    f = m - 1.0
    s = f * recip(2.0 + f)
    s2 = s * s
    p = 1.0 / 9.0
    for k in (7, 5, 3):
        p = fma(p, s2, 1.0 / k)
    t = s + s
    lnm = fma(t, s2 * p, t)
    return fma(float(e), LN2_HI, fma(float(e), LN2_LO, lnm))


def exp_steps(t):
    t = min(max(t, -760.0), 760.0)
    kf = float(round(t * LOG2E))
    r = fma(-kf, LN2_HI, t)
    r = fma(-kf, LN2_LO, r)
    p = 1.0 / math.factorial(8)
    for n in range(7, -1, -1):
        p = fma(p, r, 1.0 / math.factorial(n))
    return math.ldexp(p, int(kf))


def test_ln2_split_is_exact_to_the_head():
    # the head has at most 21 significant bits, so k * head is exact for |k| < 2^11
    assert Fraction(LN2_HI).denominator.bit_length() - 1 <= 21
    ref = decimal.Decimal(2).ln()
    assert abs(decimal.Decimal(LN2_HI) + decimal.Decimal(LN2_LO) - ref) < decimal.Decimal("1e-21")


def test_log_and_exp_relative_error():
    rng = random.Random(7)
    worst_ln = worst_exp = 0.0
    for _ in range(3000):
        y = math.exp(rng.uniform(-80.0, 80.0))
        ref = decimal.Decimal(y).ln()
        if ref != 0:
            worst_ln = max(worst_ln, float(abs((decimal.Decimal(ln_steps(y)) - ref) / ref)))
        t = rng.uniform(-700.0, 700.0)
        ref = decimal.Decimal(t).exp()
        worst_exp = max(worst_exp, float(abs((decimal.Decimal(exp_steps(t)) - ref) / ref)))
    # truncation: 2 s^11 / 11 against ln m (|s| < 0.172) and r^9 / 9!
    assert worst_ln < 3e-9
    assert worst_exp < 4e-10


def test_log_near_one_absolute_error():
    rng = random.Random(8)
    for _ in range(2000):
        y = 1.0 + rng.uniform(-0.3, 0.3)
        assert abs(float(decimal.Decimal(ln_steps(y)) - decimal.Decimal(y).ln())) < 1e-9


def test_bond_order_power():
    # b = exp(-ln(1 + x) / (2 eta)), x = exp(eta (ln beta + ln zeta)) for the Si entry
    beta, eta = 1.1e-6, 0.78734
    rng = random.Random(9)
    for _ in range(500):
        zeta = math.exp(rng.uniform(-5.0, 12.0))
        x = exp_steps(eta * (math.log(beta) + ln_steps(zeta)))
        b = exp_steps(-ln_steps(1.0 + x) / (2.0 * eta))
        ref = (1 + (decimal.Decimal(beta) * decimal.Decimal(zeta)) ** decimal.Decimal(eta)) ** (
            -1 / (2 * decimal.Decimal(eta)))
        assert abs(decimal.Decimal(b) - ref) / ref < decimal.Decimal("5e-9")
