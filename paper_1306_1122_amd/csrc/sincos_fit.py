"""Provenance of the polynomial coefficients of sincos_reduced (dbie_internal.h).

Discrete least squares on 400 Chebyshev nodes of z = r^2 in [0, (pi/4)^2], in 50-digit arithmetic:
    sin r = r + r^3 P(z),  weight z   (relative error of sin)
    cos r = 1 - z/2 + z^2 Q(z),  weight z^2   (absolute error of cos)
with P, Q of degree 5, then rounded to double. Prints the coefficients (P, then Q, lowest degree
first), the largest error of the rounded polynomials on [0, pi/4], and the two-part pi/2 of the
Cody-Waite reduction. Run: python sincos_fit.py (needs mpmath).
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
    Z = (mp.pi / 4) ** 2
    nodes = [Z * (1 - mp.cos(mp.pi * (k + mp.mpf(1) / 2) / 400)) / 2 for k in range(400)]
    P = fit(lambda z: (mp.sin(mp.sqrt(z)) - mp.sqrt(z)) / mp.sqrt(z) ** 3, lambda z: z, 5, nodes)
    Q = fit(lambda z: (mp.cos(mp.sqrt(z)) - 1 + z / 2) / z ** 2, lambda z: z * z, 5, nodes)
    print("P", [repr(x) for x in P])
    print("Q", [repr(x) for x in Q])
    es = ec = mp.mpf(0)
    for k in range(1, 2001):
        r = mp.pi / 4 * k / 2000
        z = r * r
        es = max(es, abs((r + r ** 3 * sum(mp.mpf(P[j]) * z ** j for j in range(6)) - mp.sin(r)) / mp.sin(r)))
        ec = max(ec, abs(1 - z / 2 + z * z * sum(mp.mpf(Q[j]) * z ** j for j in range(6)) - mp.cos(r)))
    print("largest relative error of sin %.2e, absolute error of cos %.2e" % (float(es), float(ec)))
    hi = float(mp.pi / 2)
    print("pi/2 =", repr(hi), "+", repr(float(mp.pi / 2 - hi)), "; 2/pi =", repr(float(2 / mp.pi)))


if __name__ == "__main__":
    main()
