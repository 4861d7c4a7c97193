"""Coefficients of the device exponential's polynomial (exp_nonpos in sa_device.h).

e^r on [-ln2/2, ln2/2] is approximated by the degree-11 polynomial that interpolates it at the 12
Chebyshev nodes of the interval (a near-minimax fit), solved in 200-bit arithmetic and rounded to
double.  The script prints the coefficients, the largest relative error of the rounded polynomial
on a fine grid, and the ulp error of the whole device routine (argument reduction by a two-part
ln 2, Horner evaluation with one rounding per fused multiply-add, scaling by 2^n) against the
correctly rounded exponential on a seeded sample, emulated here in exact arithmetic.

    python gen_exp_poly.py
"""
import math
import random

import mpmath as mp

mp.mp.prec = 200
HALF_LN2 = mp.log(2) / 2
DEGREE = 11


def chebyshev_interpolant(deg):
    n = deg + 1
    xs = [HALF_LN2 * mp.cos(mp.pi * (k + mp.mpf(1) / 2) / n) for k in range(n)]
    A = mp.matrix([[x ** j for j in range(n)] for x in xs])
    c = mp.lu_solve(A, mp.matrix([mp.exp(x) for x in xs]))
    return [float(mp.nstr(c[j], 40)) for j in range(n)]


def fma(x, y, z):
    return float(mp.mpf(x) * mp.mpf(y) + mp.mpf(z))


def device_exp(x, coefs):
    xc = x if x > -746.0 else -746.0
    n = float(round(xc * 1.4426950408889634))
    r = fma(-n, 0.6931471803691238, xc)
    r = fma(-n, 1.9082149292705877e-10, r)
    p = coefs[-1]
    for c in reversed(coefs[:-1]):
        p = fma(p, r, c)
    return math.ldexp(p, int(n))


def main():
    coefs = chebyshev_interpolant(DEGREE)
    grid = [HALF_LN2 * (2 * i / 4000 - 1) for i in range(4001)]
    rel = max(abs(sum(mp.mpf(coefs[j]) * r ** j for j in range(DEGREE + 1)) / mp.exp(r) - 1) for r in grid)
    print("coefficients c0..c%d:" % DEGREE)
    for j, c in enumerate(coefs):
        print("  c%-2d = %r" % (j, c))
    print("largest relative error of the rounded polynomial: 2^%.2f" % float(mp.log(rel, 2)))
    rng = random.Random(1)
    xs = [-rng.uniform(0, 1) for _ in range(3000)] + [-rng.uniform(0, 40) for _ in range(3000)] + \
         [-rng.uniform(600, 745) for _ in range(500)]
    errs = []
    for x in xs:
        y = device_exp(x, coefs)
        errs.append(float(abs(mp.mpf(y) - mp.exp(mp.mpf(x))) / math.ulp(y)))
    print("device routine on %d arguments: max %.3f ulp, not correctly rounded %.1f %%"
          % (len(xs), max(errs), 100.0 * sum(e > 0.5 for e in errs) / len(errs)))


if __name__ == "__main__":
    main()
