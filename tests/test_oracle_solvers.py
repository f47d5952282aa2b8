"""Pins of the oracle's lambda solvers and of the Low & Lou exact field (no GPU)."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle
from workloads import LowLou, config1


# ------------------------------------------------------------------------------------------------
# Downhill simplex: the same trial sequence as SciPy's Nelder-Mead (same coefficients, same
# initial simplex) on functions without ties
# ------------------------------------------------------------------------------------------------
def _scipy_trials(fun, x0, delta, k):
    pts = []

    def f(x):
        pts.append(np.array(x, dtype=np.float64))
        return fun(x)

    sim = np.array([x0] + [x0 + delta * np.eye(3)[j] for j in range(3)])
    minimize(f, x0, method="Nelder-Mead",
             options=dict(initial_simplex=sim, maxfev=k + 10, maxiter=10 * k, xatol=0.0, fatol=0.0,
                          adaptive=False))
    return pts


@pytest.mark.parametrize("name", ["rosenbrock", "quadratic", "wavy"])
def test_nelder_mead_matches_scipy_trial_sequence(name):
    A = np.array([[3.0, 0.4, -0.2], [0.4, 1.5, 0.3], [-0.2, 0.3, 0.7]])
    funs = {
        "rosenbrock": lambda x: float(sum(100 * (x[1:] - x[:-1] ** 2) ** 2 + (1 - x[:-1]) ** 2)),
        "quadratic": lambda x: float((x - 0.3) @ A @ (x - 0.3)),
        "wavy": lambda x: float(np.sum(np.sin(3 * x) ** 2) + 0.1 * np.sum(x * x) + 0.01 * x[0]),
    }
    fun = funs[name]
    x0 = np.array([-0.4, 0.9, 0.2])
    k = 150
    ref = _scipy_trials(fun, x0, 0.25, k)
    r = oracle.nelder_mead(lambda x: (fun(x), False), x0, 0.25, k)
    ours = [h[0] for h in r.history]
    m = min(len(ref), len(ours)) - 4
    assert m > 100
    for a, b in zip(ours[:m], ref[:m]):
        np.testing.assert_array_equal(a, b)


def test_nelder_mead_stops_on_done_and_budget():
    calls = []

    def fun(x):
        calls.append(x)
        v = float(np.sum((x - 1.0) ** 2))
        return v, v < 1e-3

    r = oracle.nelder_mead(fun, np.zeros(3), 0.5, 500)
    assert r.converged and r.fx < 1e-3 and r.trials == len(calls)
    np.testing.assert_array_equal(r.x, calls[-1])
    r2 = oracle.nelder_mead(lambda x: (float(np.sum(x * x)) + 1.0, False), np.ones(3), 0.5, 17)
    assert not r2.converged and r2.trials == 17
    assert r2.fx == min(h[1] for h in r2.history)


# ------------------------------------------------------------------------------------------------
# Levenberg-Marquardt: on a linear residual it reaches the least-squares minimum
# ------------------------------------------------------------------------------------------------
def test_lm_reaches_linear_least_squares_minimum():
    rng = np.random.default_rng(3)
    A = rng.normal(size=(4, 3))
    x_star = np.array([0.8, 1.7, 0.4])
    b = A @ x_star + 0.05 * rng.normal(size=4)
    sol = np.linalg.lstsq(A, b, rcond=None)[0]
    assert np.all(sol > 0)
    phi_min = float(np.sum((A @ sol - b) ** 2))

    def evalfun(mu):
        u = A @ mu - b
        return u, A, float(u @ u), float(np.max(np.abs(u))), oracle.ST_BUDGET

    mu, st, trials, rho, Phi = oracle.levenberg_marquardt(evalfun, np.zeros(3), 20, 0.0, 1e6)
    assert trials == 20
    np.testing.assert_allclose(mu, sol, rtol=1e-9)
    assert abs(Phi - phi_min) < 1e-12 * max(1.0, phi_min)


def test_lm_phi_is_monotone_on_a_dbie_point():
    w = config1()
    b = w.boundaries[0]
    prob = oracle.PointProblem(b.B0, b.x0, b.y0, b.h, w.xyz[:, 37])
    seen = []

    def evalfun(mu):
        (B, dB, tan), res = prob.eval(np.sqrt(mu), tangents=True)
        seen.append(float(res["Phi"][0]))
        Jac = oracle.residual_jacobian(B, dB, tan, prob.h)[:, :, 0]
        return res["u"][:, 0], Jac, float(res["Phi"][0]), float(res["rho"][0]), int(res["status"][0])

    mu, st, trials, rho, Phi = oracle.levenberg_marquardt(evalfun, np.zeros(3), 20, 1e-4,
                                                           (np.pi / b.h) ** 2)
    best = np.minimum.accumulate(seen)
    assert Phi == best[-1] and Phi <= seen[0]
    assert np.all(mu >= 0)


# ------------------------------------------------------------------------------------------------
# the DBIE per-point solvers
# ------------------------------------------------------------------------------------------------
def test_point_solvers_are_deterministic_and_consistent():
    w = config1()
    b = w.boundaries[0]
    cap = math.pi / b.h
    delta = oracle.default_nm_step(b.nx, b.ny, b.h)
    for i in (5, 130, 333):
        prob = oracle.PointProblem(b.B0, b.x0, b.y0, b.h, w.xyz[:, i])
        r1 = oracle.solve_point_nm(prob, np.zeros(3), 30, 1e-4, delta, cap)
        r2 = oracle.solve_point_nm(prob, np.zeros(3), 30, 1e-4, delta, cap)
        np.testing.assert_array_equal(r1[0], r2[0])
        assert r1[1:] == r2[1:]
        # the returned rho is the residual at the returned lambda
        _, res = prob.eval(r1[0])
        assert abs(float(res["rho"][0]) - r1[3]) <= 1e-15 * max(1.0, r1[3])
        # it is no worse than the start
        _, res0 = prob.eval(np.zeros(3))
        assert float(res["Phi"][0]) <= float(res0["Phi"][0])


# ------------------------------------------------------------------------------------------------
# Low & Lou exact field (the input of the first workload)
# ------------------------------------------------------------------------------------------------
def test_lowlou_m0_is_the_closed_form_dipole_profile():
    ll = LowLou(n=1, m=0)
    assert ll.a2 == 0.0
    mu = np.linspace(-0.99, 0.99, 41)
    P, dP = ll.P(mu)
    np.testing.assert_allclose(P, 5.0 * (1 - mu * mu), rtol=1e-10)
    np.testing.assert_allclose(dP, -10.0 * mu, atol=1e-9)


def test_lowlou_n1_m1_eigenfunction():
    ll = LowLou(n=1, m=1)
    mu = np.linspace(-1 + 1e-9, 1 - 1e-9, 20001)
    P, dP = ll.P(mu)
    assert abs(P[0]) < 1e-7 and abs(P[-1]) < 1e-7
    assert abs(dP[0] - 10.0) < 1e-6
    # one interior zero; for n = 1 the nonlinearity is odd, so the m = 1 profile is odd
    assert int(np.sum(np.sign(P[1:-1]) != np.sign(P[:-2]))) == 1
    np.testing.assert_allclose(P, -P[::-1], atol=1e-9)
    # the residual of the ODE on the profile
    h = 1e-4
    m = np.linspace(-0.9, 0.9, 19)
    Pp = (ll.P(m + h)[0] - 2 * ll.P(m)[0] + ll.P(m - h)[0]) / h ** 2
    Pm = ll.P(m)[0]
    res = (1 - m * m) * Pp + 2 * Pm + ll.a2 * 2 * Pm ** 3
    assert np.max(np.abs(res)) < 1e-5 * np.max(np.abs(2 * Pm))


def test_lowlou_field_is_force_free_and_solenoidal():
    ll = LowLou(n=1, m=1, l=0.3, Phi=math.pi / 4)
    rng = np.random.default_rng(0)
    p = rng.uniform([-1, -1, 0.1], [1, 1, 1], size=(25, 3)).T
    e = 1e-5
    G = np.zeros((3, 3, p.shape[1]))
    for k in range(3):
        d = np.zeros((3, 1))
        d[k] = e
        G[:, k] = (ll.field(*(p + d)) - ll.field(*(p - d))) / (2 * e)
    B = ll.field(*p)
    nB = np.linalg.norm(B, axis=0)
    div = G[0, 0] + G[1, 1] + G[2, 2]
    J = np.array([G[2, 1] - G[1, 2], G[0, 2] - G[2, 0], G[1, 0] - G[0, 1]])
    f = np.linalg.norm(np.cross(J.T, B.T), axis=1) / (np.linalg.norm(J, axis=0) * nB)
    gradscale = np.sqrt(np.sum(G * G, axis=(0, 1)))
    assert np.max(np.abs(div) / gradscale) < 1e-7
    assert np.max(f) < 1e-6


def test_lowlou_n3_m1_eigenfunction_and_field():
    """n = 3, m = 1 (the Table 1 case): the first eigenvalue above a = 0. The a = 0 profile for n = 3
    is (1 - mu^2) dP_3/dmu (2 interior zeros); this one has 3, satisfies the ODE, vanishes at both
    ends with P'(-1) = 10, and its field is force-free and solenoidal."""
    ll = LowLou(n=3, m=1, l=0.3, Phi=4 * math.pi / 5)
    assert 0.0 < ll.a2 < 40.0
    mu = np.linspace(-1 + 1e-9, 1 - 1e-9, 20001)
    P, dP = ll.P(mu)
    assert abs(P[0]) < 1e-7 and abs(P[-1]) < 1e-7 and abs(dP[0] - 10.0) < 1e-6
    assert int(np.sum(np.sign(P[1:-1]) != np.sign(P[:-2]))) == 3
    h = 1e-4
    m = np.linspace(-0.9, 0.9, 19)
    Pm = ll.P(m)[0]
    Pp = (ll.P(m + h)[0] - 2 * Pm + ll.P(m - h)[0]) / h ** 2
    res = (1 - m * m) * Pp + 12 * Pm + ll.a2 * (4.0 / 3.0) * np.sign(Pm) * np.abs(Pm) ** (5.0 / 3.0)
    assert np.max(np.abs(res)) < 1e-5 * np.max(np.abs(12 * Pm))
    rng = np.random.default_rng(1)
    p = rng.uniform([-1, -1, 0.05], [1, 1, 2], size=(25, 3)).T
    e = 1e-5
    G = np.zeros((3, 3, p.shape[1]))
    for k in range(3):
        d = np.zeros((3, 1))
        d[k] = e
        G[:, k] = (ll.field(*(p + d)) - ll.field(*(p - d))) / (2 * e)
    B = ll.field(*p)
    div = G[0, 0] + G[1, 1] + G[2, 2]
    J = np.array([G[2, 1] - G[1, 2], G[0, 2] - G[2, 0], G[1, 0] - G[0, 1]])
    f = np.linalg.norm(np.cross(J.T, B.T), axis=1) / (np.linalg.norm(J, axis=0) * np.linalg.norm(B, axis=0))
    assert np.max(np.abs(div) / np.sqrt(np.sum(G * G, axis=(0, 1)))) < 1e-7
    assert np.max(f) < 1e-6


def test_table1_workload_layout():
    from workloads import lowlou_table1
    w = lowlou_table1()
    bd = w.boundaries[0]
    assert bd.B0.shape == (3, 192, 192) and w.n_points == 63 * 64 * 64
    h = bd.h
    # the region's columns are the central 64 boundary nodes; the bottom layer is boundary data
    jj, ii = w.meta["bottom_idx"]
    np.testing.assert_allclose(bd.x0 + ii[:64] * h, w.xyz[0, :64], atol=1e-15)
    exact0 = w.meta["ll"].field(bd.x0 + ii * h, bd.y0 + jj * h, np.zeros(ii.size))
    np.testing.assert_array_equal(exact0, bd.B0[:, jj, ii])
    assert abs(w.xyz[2].min() - h) < 1e-15 and abs(w.xyz[2].max() - 63 * h) < 1e-12
