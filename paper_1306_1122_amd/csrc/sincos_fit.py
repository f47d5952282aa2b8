"""Provenance of the constants of the FP64 sin/cos in dbie_internal.h: the polynomial coefficients of
sincos_halfturn, and (`python sincos_fit.py table`) the table, reduction constants and sine
coefficients of sincos_table16 (its cosine is the Taylor series to r^8, coefficients +-1/n! rounded
to double).

Discrete least squares on 500 Chebyshev nodes of z = r^2 in [0, (pi/2)^2], in 50-digit arithmetic:
    sin r = r + r^3 P(z),  weight z   (P of degree 7)
    cos r = 1 - z/2 + z^2 Q(z),  weight z^2   (Q of degree 6)
then rounded to double. Prints the coefficients (P, then Q, lowest degree first), the largest
absolute errors of the rounded polynomials on [0, pi/2], and the two-part pi of the Cody-Waite
reduction. Run: python sincos_fit.py (needs mpmath).
"""
import mpmath as mp


def fit(target, weight, deg, nodes):
    A = mp.matrix(len(nodes), deg + 1)
    b = mp.matrix(len(nodes), 1)
    for i, z in enumerate(nodes):
        w = weight(z)
        for j in range(deg + 1):
            A[i, j] = w * z ** j
        b[i] = w * target(z)
    return [float(x) for x in mp.lu_solve(A.T * A, A.T * b)]


def main():
    mp.mp.dps = 50
    Z = (mp.pi / 2) ** 2
    nodes = [Z * (1 - mp.cos(mp.pi * (k + mp.mpf(1) / 2) / 500)) / 2 for k in range(500)]
    P = fit(lambda z: (mp.sin(mp.sqrt(z)) - mp.sqrt(z)) / mp.sqrt(z) ** 3, lambda z: z, 7, nodes)
    Q = fit(lambda z: (mp.cos(mp.sqrt(z)) - 1 + z / 2) / z ** 2, lambda z: z * z, 6, nodes)
    print("P", [repr(x) for x in P])
    print("Q", [repr(x) for x in Q])
    es = ec = mp.mpf(0)
    for k in range(1, 3001):
        r = mp.pi / 2 * k / 3000
        z = r * r
        es = max(es, abs(r + r ** 3 * sum(mp.mpf(P[j]) * z ** j for j in range(len(P))) - mp.sin(r)))
        ec = max(ec, abs(1 - z / 2 + z * z * sum(mp.mpf(Q[j]) * z ** j for j in range(len(Q))) - mp.cos(r)))
    print("largest absolute error of sin %.2e, of cos %.2e" % (float(es), float(ec)))
    hi = float(mp.pi)
    print("pi =", repr(hi), "+", repr(float(mp.pi - hi)), "; 1/pi =", repr(float(1 / mp.pi)))


if __name__ == "__main__" and len(__import__("sys").argv) == 1:
    main()


def table16_sin():
    """Sine of sincos_table16 on |r| <= pi/32: sin r = r + r^3 P(z), z = r^2, P of degree 2, by
    discrete least squares on 500 Chebyshev nodes of z in [0, (pi/32)^2] with weight z^(3/2) (the
    absolute error of sin r is r^3 times that of P), in 50-digit arithmetic, then rounded to double.
    Returns P (lowest degree first)."""
    mp.mp.dps = 50
    Z = (mp.pi / 32) ** 2
    nodes = [Z * (1 - mp.cos(mp.pi * (k + mp.mpf(1) / 2) / 500)) / 2 for k in range(500)]
    return fit(lambda z: (mp.sin(mp.sqrt(z)) - mp.sqrt(z)) / mp.sqrt(z) ** 3, lambda z: z ** mp.mpf(1.5), 2,
               nodes)


def table16():
    """The table of sincos_table16 (dbie_internal.h): (sin, cos)(j pi / 16), j = 0..31, each rounded
    to the nearest double from 50-digit values, the two-part pi / 16 and 16 / pi of its reduction,
    the sine coefficients (`table16_sin`) and the largest absolute errors on [0, pi/32] of its sine
    and of the cosine 1 - z/2 + z^2 (1/4! - z/6! + z^2/8!). Run: python sincos_fit.py table"""
    mp.mp.dps = 50
    for j in range(32):
        a = mp.mpf(j) / 16   # sinpi and cospi are exact at the multiples of 1/2
        print("    {%s, %s}," % (repr(float(mp.sinpi(a))), repr(float(mp.cospi(a)))))
    hi = float(mp.pi / 16)
    print("pi/16 =", repr(hi), "+", repr(float(mp.pi / 16 - hi)), "; 16/pi =", repr(float(16 / mp.pi)))
    P = table16_sin()
    print("sin P", [repr(x) for x in P])
    Q = [1 / 24.0, -1 / 720.0, 1 / 40320.0]
    es = ec = mp.mpf(0)
    for k in range(1, 3001):
        r = mp.pi / 32 * k / 3000
        z = r * r
        es = max(es, abs(r + r ** 3 * sum(mp.mpf(P[j]) * z ** j for j in range(3)) - mp.sin(r)))
        ec = max(ec, abs(1 - z / 2 + z * z * sum(mp.mpf(Q[j]) * z ** j for j in range(3)) - mp.cos(r)))
    print("largest absolute error of sin %.2e, of cos %.2e" % (float(es), float(ec)))


if __name__ == "__main__" and len(__import__("sys").argv) > 1 and __import__("sys").argv[1] == "table":
    table16()
