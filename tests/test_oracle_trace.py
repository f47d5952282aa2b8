"""Pins of the oracle's field-line tracer (CPU): straight lines in a uniform field, the dipole
field-line invariant r / sin^2(theta) with fourth-order convergence in the step, the stop rule at
the box, trilinear interpolation exact on trilinear functions, and current lines of a field whose
J is known in closed form."""
import math

import numpy as np

import oracle


def test_uniform_field_gives_straight_lines_and_stops_at_the_box():
    d = np.array([1.0, 2.0, 2.0]) / 3.0
    direction = lambda xyz: np.repeat(d[:, None], xyz.shape[1], axis=1)
    seeds = np.array([[0.1, 0.2], [0.0, 0.1], [0.05, 0.3]])
    pts, cnt = oracle.rk4_trace(direction, seeds, 0.01, 200, [-1, -1, 0], [1, 1, 1])
    for j in range(2):
        line = pts[: cnt[j], :, j]
        s = 0.01 * np.arange(cnt[j])
        np.testing.assert_allclose(line, seeds[:, j][None, :] + s[:, None] * d[None, :], atol=1e-13)
        # the last point is inside and one more step would leave the box (z > 1 first here)
        assert np.all(line[-1] <= 1.0) and line[-1][2] + 0.01 * d[2] > 1.0
        assert np.all(np.isnan(pts[cnt[j]:, :, j]))
    back, cb = oracle.rk4_trace(direction, seeds, 0.01, 5, [-1, -1, 0], [1, 1, 1], sense=-1.0)
    np.testing.assert_allclose(back[cb[0] - 1, :, 0], seeds[:, 0] - 0.01 * (cb[0] - 1) * d, atol=1e-13)


def _dipole_direction(xyz):
    # point dipole m = z-hat at the origin: B = (3 (m.r) r - m r^2) / r^5
    r2 = np.sum(xyz * xyz, axis=0)
    B = 3 * xyz[2] * xyz - np.array([0.0, 0.0, 1.0])[:, None] * r2
    return B / np.sqrt(np.sum(B * B, axis=0))


def test_dipole_lines_keep_their_invariant_to_fourth_order():
    seed = np.array([[0.3], [0.0], [0.4]])
    inv0 = 0.5 / (0.3 / 0.5) ** 2          # r / sin^2(theta)
    errs = []
    for ds in (0.04, 0.02):
        n = int(round(0.8 / ds))
        pts, cnt = oracle.rk4_trace(_dipole_direction, seed, ds, n, [-5, -5, -5], [5, 5, 5])
        p = pts[cnt[0] - 1, :, 0]
        r = np.linalg.norm(p)
        st2 = (p[0] ** 2 + p[1] ** 2) / r ** 2
        errs.append(abs(r / st2 - inv0))
        assert abs(p[1]) < 1e-15   # stays in its meridian plane
    assert errs[0] < 1e-5
    assert 10.0 < errs[0] / errs[1] < 24.0   # 2^4 = 16


def test_trilinear_is_exact_on_trilinear_functions_and_clamps():
    rng = np.random.default_rng(3)
    a = rng.normal(size=8)
    f = lambda x, y, z: a[0] + a[1] * x + a[2] * y + a[3] * z + a[4] * x * y + a[5] * y * z + a[6] * x * z + a[7] * x * y * z
    xs, ys, zs = np.arange(5) * 0.5, np.arange(4) * 0.25 + 1.0, np.arange(3) * 2.0
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    grid = np.stack([f(X, Y, Z), 2 * f(X, Y, Z)])
    p = np.stack([rng.uniform(0, 2, 50), rng.uniform(1, 1.75, 50), rng.uniform(0, 4, 50)])
    v = oracle.trilinear(grid, (0.0, 1.0, 0.0), (0.5, 0.25, 2.0), p)
    np.testing.assert_allclose(v[0], f(*p), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(v[1], 2 * f(*p), rtol=1e-12, atol=1e-12)
    out = oracle.trilinear(grid, (0.0, 1.0, 0.0), (0.5, 0.25, 2.0), np.array([[9.0], [-3.0], [1.0]]))
    np.testing.assert_allclose(out[0], f(2.0, 1.0, 1.0), rtol=1e-12)


def test_dbie_direction_is_the_unit_field_and_current():
    """On a small magnetogram the direction is B/|B| of `field` at the interpolated lambda and the
    current direction is curl B / |curl B| (checked by central differences of B)."""
    rng = np.random.default_rng(4)
    B0 = rng.normal(size=(3, 9, 11))
    lam_grid = rng.uniform(-0.3, 0.3, size=(3, 2, 2, 2))
    d = oracle.dbie_direction(B0, 0.0, 0.0, 1.0, lam_grid, (0.0, 0.0, 1.0), (10.0, 8.0, 4.0))
    dj = oracle.dbie_direction(B0, 0.0, 0.0, 1.0, lam_grid, (0.0, 0.0, 1.0), (10.0, 8.0, 4.0), current=True)
    p = np.array([[4.3], [3.7], [2.2]])
    lam = oracle.trilinear(lam_grid, (0.0, 0.0, 1.0), (10.0, 8.0, 4.0), p)
    B, dB = oracle.field(B0, 0.0, 0.0, 1.0, p, lam)
    np.testing.assert_allclose(d(p), B / np.linalg.norm(B), rtol=1e-14)
    e = 1e-5
    G = np.zeros((3, 3))
    for q in range(3):
        dp = np.zeros((3, 1))
        dp[q] = e
        G[:, q] = ((oracle.field(B0, 0.0, 0.0, 1.0, p + dp, lam)[0] - oracle.field(B0, 0.0, 0.0, 1.0, p - dp, lam)[0])
                   / (2 * e))[:, 0]
    J = np.array([G[2, 1] - G[1, 2], G[0, 2] - G[2, 0], G[1, 0] - G[0, 1]])
    np.testing.assert_allclose(dj(p)[:, 0], J / np.linalg.norm(J), atol=1e-7)
