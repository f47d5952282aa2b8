"""Pins of the FP64 CPU oracle against facts fixed by the paper and by the mathematics (no GPU).

Each test names what it pins. The closed forms are derived independently of the oracle's sums:
  * lambda = 0, B0 = 1 on a rectangle: the half-space Poisson kernel integrates to the solid-angle
    fraction sum_corners +-atan(XY / (z sqrt(X^2+Y^2+z^2))) / (2 pi);
  * B0 = exp(-rho^2 / 2 s^2), point on the axis: B = cos(lambda z) - (z/s^2) E I with
    E I = e^{z^2/2s^2} int_z^inf cos(lambda r) e^{-r^2/2s^2} dr = s sqrt(pi/2) Re[e^{i lambda z} w((lambda s^2 + i z)/(s sqrt 2))]
    (w = Faddeeva function), dB/dz = -lambda sin(lambda z) - (1 + z^2/s^2) E I / s^2 + (z/s^2) cos(lambda z),
    dB/dmu = (z/2) E I and d(dB/dz)/dmu = (1 + z^2/s^2) E I / 2 - (z/2) cos(lambda z).
"""
import math

import numpy as np
import pytest
from scipy.integrate import dblquad
from scipy.special import wofz

import oracle


# ------------------------------------------------------------------------------------------------
# helpers (closed forms; none of them calls the oracle)
# ------------------------------------------------------------------------------------------------
def solid_angle_fraction(X1, X2, Y1, Y2, z):
    def F(X, Y):
        return math.atan(X * Y / (z * math.sqrt(X * X + Y * Y + z * z)))
    return (F(X2, Y2) - F(X1, Y2) - F(X2, Y1) + F(X1, Y1)) / (2.0 * math.pi)


def gaussian_EI(lam, z, s):
    return s * math.sqrt(math.pi / 2.0) * np.real(
        np.exp(1j * lam * z) * wofz((lam * s * s + 1j * z) / (s * math.sqrt(2.0))))


def gaussian_axis(lam, z, s):
    EI = gaussian_EI(lam, z, s)
    B = math.cos(lam * z) - z / (s * s) * EI
    dBdz = -lam * math.sin(lam * z) - (1.0 + z * z / (s * s)) * EI / (s * s) + z / (s * s) * math.cos(lam * z)
    dBdmu = 0.5 * z * EI
    dBdz_dmu = 0.5 * (1.0 + z * z / (s * s)) * EI - 0.5 * z * math.cos(lam * z)
    return B, dBdz, dBdmu, dBdz_dmu


def centred_grid(half_px, h):
    n = 2 * half_px + 1
    x0 = -half_px * h
    return n, x0


def random_case(rng, nx=9, ny=7, npts=6, h=0.5, zmin=0.3, zmax=3.0, lam_scale=1.5):
    B0 = rng.normal(size=(3, ny, nx))
    x0, y0 = -0.3, 0.2
    xyz = np.stack([rng.uniform(x0, x0 + nx * h, npts), rng.uniform(y0, y0 + ny * h, npts),
                    rng.uniform(zmin, zmax, npts)])
    lam = rng.uniform(-lam_scale, lam_scale, size=(3, npts))
    return B0, x0, y0, h, xyz, lam


# ------------------------------------------------------------------------------------------------
# P1: lambda = 0 normalisation (2 pi, h^2 weights, z / r^3)
# ------------------------------------------------------------------------------------------------
def test_solid_angle_formula_matches_quadrature():
    # the helper itself against adaptive 2-D quadrature of z / (2 pi r^3)
    X1, X2, Y1, Y2, z = -0.7, 1.3, -0.4, 0.9, 0.6
    q = dblquad(lambda y, x: z / (2 * math.pi * (x * x + y * y + z * z) ** 1.5), X1, X2, Y1, Y2,
                epsabs=1e-14, epsrel=1e-13)[0]
    assert abs(q - solid_angle_fraction(X1, X2, Y1, Y2, z)) < 1e-12


def test_lambda0_unit_boundary_converges_to_solid_angle_at_second_order():
    # rectangle [-1, 1.5] x [-0.5, 1] covered by cells of side h; point above it
    xi, yi, z = 0.17, 0.31, 0.45
    exact = solid_angle_fraction(-1.0 - xi, 1.5 - xi, -0.5 - yi, 1.0 - yi, z)
    errs = []
    for k in (40, 80, 160):
        h = 0.5 / k * 1.0
        nx, ny = int(round(2.5 / h)), int(round(1.5 / h))
        B0 = np.stack([np.full((ny, nx), 1.0), np.full((ny, nx), 2.0), np.full((ny, nx), -3.0)])
        x0, y0 = -1.0 + 0.5 * h, -0.5 + 0.5 * h
        B = oracle.field_only(B0, x0, y0, h, np.array([[xi], [yi], [z]]), np.zeros((3, 1)))
        np.testing.assert_allclose(B[:, 0] / np.array([1.0, 2.0, -3.0]), B[0, 0], rtol=1e-13)
        errs.append(abs(B[0, 0] - exact))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    for o in orders:
        assert 1.8 <= o <= 2.2, (errs, orders)


# ------------------------------------------------------------------------------------------------
# P2 / P3: lambda != 0 closed forms on the axis of a Gaussian boundary
# ------------------------------------------------------------------------------------------------
@pytest.mark.parametrize("z", [4.0, 6.5])
def test_gaussian_axis_closed_form(z):
    h, s = 0.5, 3.0
    n, x0 = centred_grid(int(11 * s / h), h)
    X, Y = oracle.pixel_centres(n, n, x0, x0, h)
    G = np.exp(-(X * X + Y * Y) / (2 * s * s)).reshape(n, n)
    lam = np.array([0.0, 0.35, 0.8])
    B, dB, tan = oracle.field(np.stack([G, G, G]), x0, x0, h, np.array([[0.0], [0.0], [z]]),
                              lam[:, None], tangents=True)
    for p in range(3):
        Bc, dz, dmu, dzdmu = gaussian_axis(lam[p], z, s)
        assert abs(B[p, 0] - Bc) < 1e-12
        assert abs(dB[3 * p + 2, 0] - dz) < 1e-12
        assert abs(tan[p, 0] - dmu) < 1e-11
        assert abs(tan[3 + 3 * p + 2, 0] - dzdmu) < 1e-11
        # horizontal derivatives vanish on the axis of a symmetric grid
        assert abs(dB[3 * p + 0, 0]) < 1e-13 and abs(dB[3 * p + 1, 0]) < 1e-13


def test_gaussian_axis_quadrature_error_decays_exponentially():
    # the midpoint rule on a smooth, decaying integrand: error ~ exp(-2 pi z / h)
    s, lam = 3.0, 0.5
    errs = []
    for z in (1.0, 1.5, 2.0):
        h = 1.0
        n, x0 = centred_grid(int(11 * s / h), h)
        X, Y = oracle.pixel_centres(n, n, x0, x0, h)
        G = np.exp(-(X * X + Y * Y) / (2 * s * s)).reshape(n, n)
        B = oracle.field_only(np.stack([G, G, G]), x0, x0, h, np.array([[0.0], [0.0], [z]]),
                              np.full((3, 1), lam))
        errs.append(abs(B[0, 0] - gaussian_axis(lam, z, s)[0]))
    rates = [math.log(errs[i] / errs[i + 1]) / 0.5 for i in range(2)]
    for r in rates:
        assert 0.7 * 2 * math.pi < r < 1.3 * 2 * math.pi, (errs, rates)


# ------------------------------------------------------------------------------------------------
# P3 / P5: derivatives against finite differences of the field
# ------------------------------------------------------------------------------------------------
def test_gradient_matches_central_differences():
    rng = np.random.default_rng(7)
    B0, x0, y0, h, xyz, lam = random_case(rng)
    B, dB = oracle.field(B0, x0, y0, h, xyz, lam)
    step = 1e-5 * h
    scale = np.abs(dB).max()
    for q in range(3):
        e = np.zeros((3, 1))
        e[q] = step
        Bp = oracle.field_only(B0, x0, y0, h, xyz + e, lam)
        Bm = oracle.field_only(B0, x0, y0, h, xyz - e, lam)
        fd = (Bp - Bm) / (2 * step)
        for p in range(3):
            np.testing.assert_allclose(dB[3 * p + q], fd[p], rtol=0, atol=1e-8 * scale)


def test_tangents_match_central_differences_in_mu():
    rng = np.random.default_rng(8)
    B0, x0, y0, h, xyz, lam = random_case(rng)
    lam = np.abs(lam) + 0.2
    _, _, tan = oracle.field(B0, x0, y0, h, xyz, lam, tangents=True)
    mu = lam * lam
    dmu = 1e-6
    for p in range(3):
        mp = mu.copy()
        mp[p] += dmu
        mm = mu.copy()
        mm[p] -= dmu
        Bp, dBp = oracle.field(B0, x0, y0, h, xyz, np.sqrt(mp))
        Bm, dBm = oracle.field(B0, x0, y0, h, xyz, np.sqrt(mm))
        scale = np.abs(tan).max()
        np.testing.assert_allclose(tan[p], (Bp[p] - Bm[p]) / (2 * dmu), atol=1e-7 * scale)
        for q in range(3):
            np.testing.assert_allclose(tan[3 + 3 * p + q], (dBp[3 * p + q] - dBm[3 * p + q]) / (2 * dmu),
                                       atol=1e-7 * scale)
        # the other components do not depend on mu_p
        for o in range(3):
            if o != p:
                assert np.all(Bp[o] == Bm[o])


def test_paper_forward_difference_error_is_first_order_in_delta():
    rng = np.random.default_rng(9)
    B0, x0, y0, h, xyz, lam = random_case(rng, zmin=1.0)
    _, dB = oracle.field(B0, x0, y0, h, xyz, lam)
    e1 = np.abs(oracle.field_fd(B0, x0, y0, h, xyz, lam, 1e-3)[1] - dB).max()
    e2 = np.abs(oracle.field_fd(B0, x0, y0, h, xyz, lam, 0.5e-3)[1] - dB).max()
    assert 1.8 < e1 / e2 < 2.2
    assert e1 < 1e-2 * np.abs(dB).max()


# ------------------------------------------------------------------------------------------------
# P4: rounding of the oracle against a 40-digit brute force (4x4 grid, 5 points, 3 lambda triples)
# ------------------------------------------------------------------------------------------------
def test_rounding_against_mpmath_bruteforce():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    rng = np.random.default_rng(10)
    B0, x0, y0, h, xyz, _ = random_case(rng, nx=4, ny=4, npts=5)
    for trial in range(3):
        lam = rng.uniform(-2, 2, size=(3, 5))
        B, dB, tan = oracle.field(B0, x0, y0, h, xyz, lam, tangents=True)
        ref = np.zeros((24, 5))
        for i in range(5):
            xi, yi, zi = (mp.mpf(float(v)) for v in xyz[:, i])
            for p in range(3):
                lp = mp.mpf(float(lam[p, i]))
                acc = [mp.mpf(0)] * 8
                for b in range(4):
                    for a in range(4):
                        dx = mp.mpf(x0) + a * mp.mpf(h) - xi
                        dy = mp.mpf(y0) + b * mp.mpf(h) - yi
                        r = mp.sqrt(dx * dx + dy * dy + zi * zi)
                        t = lp * r
                        Nn = t * mp.sin(t) + mp.cos(t)
                        F = Nn / r ** 3
                        G = (t * t * mp.cos(t) - 3 * Nn) / r ** 5
                        dF = mp.cos(t) / (2 * r)
                        dG = -Nn / (2 * r ** 3)
                        bv = mp.mpf(float(B0[p, b, a]))
                        acc[0] += zi * F * bv
                        acc[1] += -zi * G * dx * bv
                        acc[2] += -zi * G * dy * bv
                        acc[3] += (F + zi * zi * G) * bv
                        acc[4] += zi * dF * bv
                        acc[5] += -zi * dG * dx * bv
                        acc[6] += -zi * dG * dy * bv
                        acc[7] += (dF + zi * zi * dG) * bv
                w = mp.mpf(h) ** 2 / (2 * mp.pi)
                ref[p, i] = float(w * acc[0])
                for q in range(3):
                    ref[3 + 3 * p + q, i] = float(w * acc[1 + q])
                ref[12 + p, i] = float(w * acc[4])
                for q in range(3):
                    ref[15 + 3 * p + q, i] = float(w * acc[5 + q])
        got = np.vstack([B, dB, tan])
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())


# ------------------------------------------------------------------------------------------------
# P6: invariances
# ------------------------------------------------------------------------------------------------
def test_linearity_in_B0():
    rng = np.random.default_rng(11)
    B0, x0, y0, h, xyz, lam = random_case(rng)
    B1 = rng.normal(size=B0.shape)
    a, b = 0.7, -1.9
    o0 = np.vstack(oracle.field(B0, x0, y0, h, xyz, lam, tangents=True))
    o1 = np.vstack(oracle.field(B1, x0, y0, h, xyz, lam, tangents=True))
    o2 = np.vstack(oracle.field(a * B0 + b * B1, x0, y0, h, xyz, lam, tangents=True))
    np.testing.assert_allclose(o2, a * o0 + b * o1, atol=1e-13 * np.abs(o2).max())


def test_mirror_in_x():
    rng = np.random.default_rng(12)
    nx, ny, h = 9, 6, 0.5
    B0 = rng.normal(size=(3, ny, nx))
    x0 = -(nx - 1) / 2 * h
    y0 = 0.1
    xyz = np.stack([rng.uniform(-2, 2, 5), rng.uniform(0, 3, 5), rng.uniform(0.3, 2, 5)])
    lam = rng.uniform(-1, 1, (3, 5))
    B, dB = oracle.field(B0, x0, y0, h, xyz, lam)
    Bm, dBm = oracle.field(B0[:, :, ::-1], x0, y0, h, xyz * np.array([[-1.0], [1.0], [1.0]]), lam)
    sc = np.abs(dB).max()
    np.testing.assert_allclose(Bm, B, atol=1e-13 * np.abs(B).max())
    for p in range(3):
        np.testing.assert_allclose(dBm[3 * p + 0], -dB[3 * p + 0], atol=1e-13 * sc)
        np.testing.assert_allclose(dBm[3 * p + 1], dB[3 * p + 1], atol=1e-13 * sc)
        np.testing.assert_allclose(dBm[3 * p + 2], dB[3 * p + 2], atol=1e-13 * sc)


def test_transpose_x_y_on_a_non_square_grid():
    rng = np.random.default_rng(13)
    nx, ny, h = 8, 5, 0.4
    B0 = rng.normal(size=(3, ny, nx))
    x0, y0 = -0.7, 0.3
    xyz = np.stack([rng.uniform(-1, 2, 5), rng.uniform(0, 2, 5), rng.uniform(0.3, 2, 5)])
    lam = rng.uniform(-1, 1, (3, 5))
    B, dB = oracle.field(B0, x0, y0, h, xyz, lam)
    # swap the roles of x and y everywhere: grid, components, points and lambda
    perm = [1, 0, 2]
    B0t = np.stack([B0[1].T, B0[0].T, B0[2].T])
    Bt, dBt = oracle.field(B0t, y0, x0, h, xyz[perm], lam[perm])
    sc = np.abs(dB).max()
    for p in range(3):
        for q in range(3):
            np.testing.assert_allclose(dBt[3 * perm[p] + perm[q]], dB[3 * p + q], atol=1e-13 * sc)
        np.testing.assert_allclose(Bt[perm[p]], B[p], atol=1e-13 * np.abs(B).max())


def test_even_in_lambda_and_scale_invariant_residuals():
    rng = np.random.default_rng(14)
    B0, x0, y0, h, xyz, lam = random_case(rng)
    o = np.vstack(oracle.field(B0, x0, y0, h, xyz, lam))
    om = np.vstack(oracle.field(B0, x0, y0, h, xyz, -lam))
    np.testing.assert_allclose(om, o, atol=1e-14 * np.abs(o).max())
    r1 = oracle.residuals(*oracle.field(B0, x0, y0, h, xyz, lam), h)
    r2 = oracle.residuals(*oracle.field(37.0 * B0, x0, y0, h, xyz, lam), h)
    np.testing.assert_allclose(r2["f"], r1["f"], rtol=1e-12)
    np.testing.assert_allclose(r2["g"], r1["g"], rtol=1e-12)


# ------------------------------------------------------------------------------------------------
# P7: lambda = 0 on a potential boundary (buried monopole): DBIE -> exact potential field
# ------------------------------------------------------------------------------------------------
def test_potential_limit_buried_monopole():
    d = 1.0
    pts = np.array([[0.3, -0.5, 0.8], [0.2, 0.6, -0.4], [0.7, 1.1, 1.6]])

    def exact(x, y, z):
        R = np.stack([x, y, z + d])
        return R / np.sum(R * R, axis=0) ** 1.5

    Bex = exact(*pts)
    errs, jrel = [], []
    for L in (4.0, 8.0, 16.0):
        h = 0.125
        n = int(round(2 * L / h))
        x0 = -L + 0.5 * h
        X, Y = oracle.pixel_centres(n, n, x0, x0, h)
        B0 = exact(X, Y, np.zeros_like(X)).reshape(3, n, n)
        B, dB = oracle.field(B0, x0, x0, h, pts, np.zeros((3, 3)))
        errs.append(np.abs(B - Bex).max() / np.abs(Bex).max())
        res = oracle.residuals(B, dB, h)
        J = res["J"]
        jrel.append(np.max(np.sqrt(np.sum(J * J, 0)) / np.sqrt(np.sum(dB * dB, 0))))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 2e-3
    assert jrel[0] > jrel[2] and jrel[2] < 2e-3


# ------------------------------------------------------------------------------------------------
# residual definitions on hand-built fields
# ------------------------------------------------------------------------------------------------
def test_residuals_on_linear_fields():
    # B(r) = omega x r has curl 2 omega and zero divergence; dB[3p+q] = dB_p/dx_q
    om = np.array([0.3, -1.2, 0.7])
    M = np.array([[0, -om[2], om[1]], [om[2], 0, -om[0]], [-om[1], om[0], 0]])
    dB = M.reshape(9, 1)
    J, D = oracle.curl_div(dB)
    np.testing.assert_allclose(J[:, 0], 2 * om, atol=1e-15)
    assert abs(D[0]) < 1e-15
    # B parallel to J: f = 0; B perpendicular to J: f = 1
    r = oracle.residuals(om.reshape(3, 1) * 2.5, dB, 1.0)
    assert r["f"][0] < 1e-15 and r["g"][0] < 1e-15
    perp = np.cross(om, [1.0, 0, 0]).reshape(3, 1)
    assert abs(oracle.residuals(perp, dB, 1.0)["f"][0] - 1.0) < 1e-14
    # at 30 degrees f = sin 30
    e1 = om / np.linalg.norm(om)
    e2 = perp[:, 0] / np.linalg.norm(perp)
    B = (np.cos(np.pi / 6) * e1 + np.sin(np.pi / 6) * e2).reshape(3, 1)
    assert abs(oracle.residuals(B, dB, 1.0)["f"][0] - 0.5) < 1e-14
    # pure expansion: div = 3c, g = |3c| (h/6) / |B|
    dBe = (0.4 * np.eye(3)).reshape(9, 1)
    Bv = np.array([[1.0], [2.0], [2.0]])
    r = oracle.residuals(Bv, dBe, 0.5)
    assert abs(r["g"][0] - 1.2 * (0.5 / 6) / 3.0) < 1e-15
    assert r["status"][0] == oracle.ST_J_ZERO and r["f"][0] == 0.0
    rz = oracle.residuals(np.zeros((3, 1)), dBe, 1.0)
    assert rz["status"][0] == oracle.ST_DEGENERATE and np.isinf(rz["Phi"][0])


def test_residual_jacobian_matches_differences_in_mu():
    rng = np.random.default_rng(15)
    B0, x0, y0, h, xyz, lam = random_case(rng, npts=4)
    lam = np.abs(lam) + 0.3
    B, dB, tan = oracle.field(B0, x0, y0, h, xyz, lam, tangents=True)
    Jac = oracle.residual_jacobian(B, dB, tan, h)
    mu = lam * lam
    dmu = 1e-6
    for p in range(3):
        mp, mm = mu.copy(), mu.copy()
        mp[p] += dmu
        mm[p] -= dmu
        up = oracle.residuals(*oracle.field(B0, x0, y0, h, xyz, np.sqrt(mp)), h)["u"]
        um = oracle.residuals(*oracle.field(B0, x0, y0, h, xyz, np.sqrt(mm)), h)["u"]
        np.testing.assert_allclose(Jac[:, p], (up - um) / (2 * dmu), atol=1e-6 * np.abs(Jac).max())


# ------------------------------------------------------------------------------------------------
# P9: the VJP is the transpose of the forward map, and g_lambda its lambda derivative
# ------------------------------------------------------------------------------------------------
def test_vjp_dot_product():
    rng = np.random.default_rng(16)
    B0, x0, y0, h, xyz, lam = random_case(rng, npts=8)
    x = rng.normal(size=B0.shape)
    gB = rng.normal(size=(3, 8))
    gdB = rng.normal(size=(9, 8))
    B, dB = oracle.field(x, x0, y0, h, xyz, lam)
    lhs = np.sum(gB * B) + np.sum(gdB * dB)
    gB0, _, _ = oracle.vjp(B0, x0, y0, h, xyz, lam, gB, gdB)
    rhs = np.sum(gB0 * x)
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + np.abs(gB0).max())


def test_vjp_selected_pixels_are_forward_maps_of_unit_fields():
    """gB0 at a chosen pixel k and component p equals <g, A(lambda) e_pk>: the forward map applied to
    a magnetogram that is 1 at that pixel and component and 0 elsewhere (the restricted output path,
    with its own point chunking, pinned to the forward sum)."""
    rng = np.random.default_rng(18)
    B0, x0, y0, h, xyz, lam = random_case(rng, npts=300)
    gB = rng.normal(size=(3, 300))
    gdB = rng.normal(size=(9, 300))
    ny, nx = B0.shape[1:]
    pix = np.array([0, nx * ny - 1, nx + 2, rng.integers(nx * ny)])
    sel, none1, none2 = oracle.vjp(B0, x0, y0, h, xyz, lam, gB, gdB, pixels=pix)
    assert sel.shape == (3, pix.size) and none1 is None and none2 is None
    for j, k in enumerate(pix):
        for p in range(3):
            e = np.zeros_like(B0)
            e[p].flat[k] = 1.0
            B, dB = oracle.field(e, x0, y0, h, xyz, lam)
            ref = np.sum(gB * B) + np.sum(gdB * dB)
            assert abs(sel[p, j] - ref) <= 1e-12 * max(abs(ref), 1.0), (k, p)


def test_vjp_lambda_gradient_matches_differences():
    rng = np.random.default_rng(17)
    B0, x0, y0, h, xyz, lam = random_case(rng, npts=5)
    gB = rng.normal(size=(3, 5))
    gdB = rng.normal(size=(9, 5))
    _, glam, _ = oracle.vjp(B0, x0, y0, h, xyz, lam, gB, gdB)

    def L(lm):
        B, dB = oracle.field(B0, x0, y0, h, xyz, lm)
        return np.sum(gB * B, axis=0) + np.sum(gdB * dB, axis=0)

    step = 1e-6
    for p in range(3):
        lp, lmn = lam.copy(), lam.copy()
        lp[p] += step
        lmn[p] -= step
        np.testing.assert_allclose(glam[p], (L(lp) - L(lmn)) / (2 * step), atol=1e-6 * np.abs(glam).max())


def test_absolute_term_sums():
    """field(..., absolute=True): with one pixel every row is a single term, so each absolute sum is
    the row's own magnitude (pins each row's terms and prefactors); with B0 >= 0 at lambda = 0 the
    terms of B and of the mu-tangent rows tan[p] are all positive, so those sums equal the rows; and
    in general every absolute sum bounds its row."""
    rng = np.random.default_rng(41)
    xyz = np.stack([rng.uniform(-3, 3, 9), rng.uniform(-3, 3, 9), rng.uniform(0.2, 4, 9)])
    lam = rng.uniform(-1.5, 1.5, size=(3, 9))
    one = rng.normal(size=(3, 1, 1))
    B, dB, tan, aB, adB, atan = oracle.field(one, 0.3, -0.2, 0.7, xyz, lam, tangents=True, absolute=True)
    for a, r in ((aB, B), (adB, dB), (atan, tan)):
        np.testing.assert_allclose(a, np.abs(r), rtol=1e-13, atol=0)
    B0 = np.abs(rng.normal(size=(3, 6, 7)))
    B, dB, tan, aB, adB, atan = oracle.field(B0, 0.0, 0.0, 0.5, xyz, np.zeros((3, 9)), tangents=True, absolute=True)
    np.testing.assert_allclose(aB, B, rtol=1e-13)
    np.testing.assert_allclose(atan[:3], tan[:3], rtol=1e-13)
    B, dB, tan, aB, adB, atan = oracle.field(rng.normal(size=(3, 6, 7)), 0.0, 0.0, 0.5, xyz, lam, tangents=True,
                                             absolute=True)
    for a, r in ((aB, B), (adB, dB), (atan, tan)):
        assert np.all(a >= np.abs(r) * (1 - 1e-13))
    two = oracle.field(B0, 0.0, 0.0, 0.5, xyz, lam, absolute=True)
    assert len(two) == 4
