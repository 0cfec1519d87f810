"""CPU check of the numerical method behind the float paths' pair functions
f_R = A exp(-lambda1 r) and f_A = -B exp(-lambda2 r) (Eq. 1).  The FP32
steps are evaluated here in exactly rounded IEEE single precision (numpy
float32, fma emulated through rationals) and compared with 50-digit
references:
  mixed path (exp_decay_f32): k = rint(-lambda r / ln 2), the reduced
    argument kept as th + tl with th exact (17-bit head of ln 2) and tl the
    small rest (rounding error of lambda r, the lo parts of lambda and of the
    FP64 distance r + r_lo, k times the tail of ln 2); e^th (1 + tl) with
    e^th = 1 + th + th^2 q(th), q through its th^6 term and 1 + th an exact
    pair; the result scaled by 2^k and A in FP64;
  all-FP32 path: the argument ln A - lambda r formed as a float pair
    (two-product, two-sum), the same reduction and series, rounded once.
The GPU parity tests check the kernels themselves; this test fixes the
accuracy the method reaches, which is what lets a lone bond meet the force
bound (its force is the difference of two terms ~25 times larger)."""
import decimal
import math
from fractions import Fraction

import numpy as np

decimal.getcontext().prec = 50
f32 = np.float32
LN2_HI = f32(float.fromhex("0x1.62e4p-1"))
LN2_LO = f32(0.69314718055994530942 - float(LN2_HI))
LOG2E = f32(1.44269504)


def fmaf(a, b, c):
    return f32(float(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c))))


def exp_pair_steps(a, a_lo):
    a, a_lo = f32(a), f32(a_lo)
    kf = f32(np.rint(f32(a * LOG2E)))
    t1 = fmaf(-kf, LN2_HI, a)
    p = f32(kf * LN2_LO)
    pe = fmaf(kf, LN2_LO, -p)
    th = f32(t1 - p)
    bb = f32(th - t1)
    e1 = f32(f32(t1 - f32(th - bb)) + f32(-p - bb))
    tl = f32(f32(e1 - pe) + a_lo)
    sq = f32(th * th)
    sqe = fmaf(th, th, -sq)
    q = f32(1.0 / math.factorial(8))
    for n in (7, 6, 5, 4, 3):
        q = fmaf(q, th, f32(1.0 / math.factorial(n)))
    q = fmaf(q, th, f32(0.5))
    eth = f32(f32(1.0) + fmaf(sq, q, th))
    tail = fmaf(tl, eth, fmaf(sq, q, f32(sqe * q)))
    hi = f32(f32(1.0) + th)
    lo = f32(f32(f32(f32(1.0) - hi) + th) + tail)
    return math.ldexp(float(hi) + float(lo), int(kf))


def exp_scaled_steps(lnA, lnA_lo, lam, lam_lo, r, r_lo):
    p = f32(lam * r)
    pe = fmaf(lam, r, -p)
    s = f32(lnA - p)
    bb = f32(s - lnA)
    e = f32(f32(lnA - f32(s - bb)) + f32(-p - bb))
    lo = f32(f32(f32(f32(e + lnA_lo) - pe) - f32(lam_lo * r)) - f32(lam * r_lo))
    return exp_pair_steps(s, lo)


def exp_decay_steps(A, lam, lam_lo, r, r_lo):
    p = f32(lam * r)
    pe = fmaf(lam, r, -p)
    kf = f32(np.rint(f32(-p * LOG2E)))
    th = fmaf(kf, -LN2_HI, -p)
    tl = f32(f32(f32(f32(-pe) - f32(lam_lo * r)) - f32(lam * r_lo)) - f32(kf * LN2_LO))
    sq = f32(th * th)
    sqe = fmaf(th, th, -sq)
    q = f32(1.0 / math.factorial(8))
    for n in (7, 6, 5, 4, 3):
        q = fmaf(q, th, f32(1.0 / math.factorial(n)))
    q = fmaf(q, th, f32(0.5))
    eth = f32(f32(1.0) + fmaf(sq, q, th))
    tail = fmaf(tl, eth, fmaf(sq, q, f32(sqe * q)))
    hi = f32(f32(1.0) + th)
    lo = f32(f32(f32(f32(1.0) - hi) + th) + tail)
    return math.ldexp(float(hi) + float(lo), int(kf)) * A


def split(x):
    hi = f32(x)
    return hi, f32(x - float(hi))


def rel_err(v, ref):
    return abs((decimal.Decimal(v) - ref) / ref)


def test_ln2_split():
    # 17 significant bits in the head: k * head is exact for |k| < 2^7
    assert Fraction(float(LN2_HI)).denominator.bit_length() - 1 <= 17
    ref = decimal.Decimal(2).ln()
    assert abs(decimal.Decimal(float(LN2_HI)) + decimal.Decimal(float(LN2_LO)) - ref) < decimal.Decimal("1e-12")


def test_exp_pair_accuracy():
    rng = np.random.default_rng(3)
    worst = decimal.Decimal(0)
    args = list(rng.uniform(-12.0, 12.0, 1500)) + list(rng.uniform(-0.4, 0.4, 300)) + [0.0, 0.3465, -0.3466, 11.5]
    for x in args:
        a, a_lo = split(x)
        ref = (decimal.Decimal(float(a)) + decimal.Decimal(float(a_lo))).exp()
        worst = max(worst, rel_err(exp_pair_steps(a, a_lo), ref))
    # a float ulp is 2^-24 = 6.0e-8 relative: the method stays below a quarter of it
    assert worst < decimal.Decimal("1.5e-8"), worst


def test_mixed_pair_terms_of_silicon():
    """The mixed path's f_R and f_A of the silicon set over the pair range, r
    carried as a float plus its FP64 rounding error, to a fraction of a
    float ulp."""
    A, B, l1, l2 = 1830.8, 471.18, 2.4799, 1.7322
    L1, L1_lo = split(l1)
    L2, L2_lo = split(l2)
    worst = decimal.Decimal(0)
    for r in np.linspace(1.5, 3.2, 400):
        r += 1e-9 * math.sin(1e3 * r)
        rh, rl = split(r)
        rd = decimal.Decimal(float(rh)) + decimal.Decimal(float(rl))
        ref_r = decimal.Decimal(A) * (-decimal.Decimal(l1) * rd).exp()
        ref_a = decimal.Decimal(B) * (-decimal.Decimal(l2) * rd).exp()
        worst = max(worst, rel_err(exp_decay_steps(A, L1, L1_lo, rh, rl), ref_r),
                    rel_err(exp_decay_steps(B, L2, L2_lo, rh, rl), ref_a))
    assert worst < decimal.Decimal("1.5e-8"), worst


def test_single_pair_terms_of_silicon():
    """The all-FP32 path's argument formation and exponential (before its
    final rounding to float) over the pair range."""
    A, B, l1, l2 = 1830.8, 471.18, 2.4799, 1.7322
    lnA, lnA_lo = split(math.log(A))
    lnB, lnB_lo = split(math.log(B))
    L1, L1_lo = split(l1)
    L2, L2_lo = split(l2)
    worst = decimal.Decimal(0)
    for r in np.linspace(1.5, 3.2, 400):
        r += 1e-9 * math.sin(1e3 * r)          # not on a float grid point
        rh, rl = split(r)
        rd = decimal.Decimal(float(rh)) + decimal.Decimal(float(rl))
        ref_r = decimal.Decimal(A) * (-decimal.Decimal(l1) * rd).exp()
        ref_a = decimal.Decimal(B) * (-decimal.Decimal(l2) * rd).exp()
        worst = max(worst, rel_err(exp_scaled_steps(lnA, lnA_lo, L1, L1_lo, rh, rl), ref_r),
                    rel_err(exp_scaled_steps(lnB, lnB_lo, L2, L2_lo, rh, rl), ref_a))
    assert worst < decimal.Decimal("2e-8"), worst
    # so a lone bond's force, the difference f_R' + f_A' ~ 0.56 of two terms
    # of ~13.5 eV/A at 2.35 A, carries at most 2 * 13.5 * 2e-8 = 5.4e-7 eV/A
    # (1e-6 relative) from these functions
