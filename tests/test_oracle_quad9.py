"""Pins of the Eq. (15) quadratic-element oracle (no GPU)."""
import math

import numpy as np
import pytest
from scipy.integrate import dblquad

import oracle
from test_oracle_pins import gaussian_axis, solid_angle_fraction


def test_unit_boundary_converges_to_the_node_rectangle_solid_angle():
    # B0 = 1: the shape functions sum to one, so Eq. 15 integrates the kernel over the rectangle
    # spanned by the nodes; 4x4 Gauss points per element converge at high order
    p = np.array([[0.13], [0.27], [0.4]])
    exact = solid_angle_fraction(-1 - 0.13, 1 - 0.13, -1 - 0.27, 1 - 0.27, 0.4)
    errs = []
    for n in (9, 17, 33):
        h = 2.0 / (n - 1)
        B, _ = oracle.field_quad9(np.ones((3, n, n)), -1.0, -1.0, h, p, np.zeros((3, 1)), G=4)
        errs.append(abs(B[0, 0] - exact))
    assert errs[2] < 1e-10
    assert math.log2(errs[0] / errs[1]) > 6 and math.log2(errs[1] / errs[2]) > 6


def test_quadratic_boundary_against_adaptive_quadrature():
    # a quadratic B0 is reproduced exactly by the 9-node interpolation, so Eq. 15 with many Gauss
    # points equals the exact integral of K * B0 over the node rectangle (independent 2-D quadrature)
    n, h, x0, y0 = 7, 0.5, -1.2, 0.3
    xs, ys = x0 + h * np.arange(n), y0 + h * np.arange(n)
    X, Y = np.meshgrid(xs, ys)
    c = [0.7, -0.4, 0.25, 0.3, -0.2, 0.15]

    def poly(x, y):
        return c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y

    B0 = np.stack([poly(X, Y), 2.0 * poly(X, Y), -poly(X, Y)])
    pt = np.array([[0.41], [1.37], [0.9]])
    lam = np.array([[0.0], [0.8], [1.9]])
    B, _ = oracle.field_quad9(B0, x0, y0, h, pt, lam, G=10)
    for p, scale in ((0, 1.0), (1, 2.0), (2, -1.0)):
        def f(y, x):
            return scale * poly(x, y) * oracle.kernel(lam[p, 0], x - pt[0, 0], y - pt[1, 0], pt[2, 0])
        ref = dblquad(f, xs[0], xs[-1], ys[0], ys[-1], epsabs=1e-13, epsrel=1e-12)[0]
        assert abs(B[p, 0] - ref) < 1e-10 * max(1.0, abs(ref))


def test_gradient_and_tangents_match_differences():
    rng = np.random.default_rng(71)
    n, h = 9, 0.5
    B0 = rng.normal(size=(3, n, n))
    xyz = np.stack([rng.uniform(0, 4, 4), rng.uniform(0, 4, 4), rng.uniform(0.3, 2.0, 4)])
    lam = rng.uniform(0.2, 1.2, size=(3, 4))
    B, dB, tan = oracle.field_quad9(B0, 0.0, 0.0, h, xyz, lam, tangents=True)
    step = 1e-6
    for q in range(3):
        e = np.zeros((3, 1))
        e[q] = step
        fd = (oracle.field_quad9(B0, 0.0, 0.0, h, xyz + e, lam)[0]
              - oracle.field_quad9(B0, 0.0, 0.0, h, xyz - e, lam)[0]) / (2 * step)
        for p in range(3):
            np.testing.assert_allclose(dB[3 * p + q], fd[p], atol=1e-7 * np.abs(dB).max())
    mu = lam * lam
    for p in range(3):
        mp, mm = mu.copy(), mu.copy()
        mp[p] += 1e-6
        mm[p] -= 1e-6
        op = oracle.field_quad9(B0, 0.0, 0.0, h, xyz, np.sqrt(mp))
        om = oracle.field_quad9(B0, 0.0, 0.0, h, xyz, np.sqrt(mm))
        np.testing.assert_allclose(tan[p], (op[0][p] - om[0][p]) / 2e-6, atol=1e-6 * np.abs(tan).max())
        for q in range(3):
            np.testing.assert_allclose(tan[3 + 3 * p + q], (op[1][3 * p + q] - om[1][3 * p + q]) / 2e-6,
                                       atol=1e-6 * np.abs(tan).max())


@pytest.mark.parametrize("z_over_h", [0.5, 1.0])
def test_near_boundary_accuracy_beats_the_nodal_rule(z_over_h):
    # Gaussian boundary, point on the axis close to the boundary: the quadratic elements with 4x4
    # Gauss points are far closer to the closed form than the one-point-per-pixel nodal rule
    s, h, lam = 3.0, 0.5, 0.6
    half = int(11 * s / h)
    n = 2 * half + 1
    x0 = -half * h
    X, Y = np.meshgrid(x0 + h * np.arange(n), x0 + h * np.arange(n))
    G0 = np.exp(-(X * X + Y * Y) / (2 * s * s))
    B0 = np.stack([G0, G0, G0])
    z = z_over_h * h
    ref = gaussian_axis(lam, z, s)[0]
    pt = np.array([[0.0], [0.0], [z]])
    Bq, _ = oracle.field_quad9(B0, x0, x0, h, pt, np.full((3, 1), lam), G=4)
    Bn = oracle.field_only(B0, x0, x0, h, pt, np.full((3, 1), lam))
    eq, en = abs(Bq[0, 0] - ref), abs(Bn[0, 0] - ref)
    assert eq < 0.1 * en, (eq, en)


def test_even_node_counts_are_rejected():
    with pytest.raises(ValueError):
        oracle.field_quad9(np.ones((3, 4, 5)), 0.0, 0.0, 1.0, np.array([[0.0], [0.0], [1.0]]), np.zeros((3, 1)))
