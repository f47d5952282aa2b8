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
class _LinearMuProblem:
    """A stand-in for PointProblem in the gradient form: the residual vector is linear in mu,
    u(mu) = A mu - b, with orthogonal columns of A, so that the least-squares minimum over the box
    0 <= mu <= cap^2 is the unconstrained minimum clipped per component. Records every mu it sees."""

    def __init__(self, mu_star, status=oracle.ST_BUDGET, h=1.0):
        q, _ = np.linalg.qr(np.random.default_rng(5).normal(size=(4, 4)))
        self.A = q[:, :3] * np.array([2.0, 0.7, 1.3])
        self.b = self.A @ np.asarray(mu_star, np.float64) + 0.3 * q[:, 3]   # residual 0.3 at the minimum
        self.status, self.h, self.seen = status, h, []

    def lm_eval(self, mu):
        self.seen.append(np.array(mu, np.float64))
        u = self.A @ mu - self.b
        return u, self.A, float(u @ u), float(np.max(np.abs(u))), self.status


def test_solve_point_lm_returns_lambda_of_the_box_constrained_minimum():
    """Least squares in mu with one component beyond cap^2: the wrapper starts at mu = lambda0^2 and
    returns sqrt of the minimum clipped to [0, cap^2] (cap = 1.2 tells cap^2 = 1.44 from cap, and
    lambda from mu), with status BUDGET after exactly `budget` trials when eps = 0."""
    mu_star = np.array([0.25, 2.0, 0.5])
    cap = 1.2
    prob = _LinearMuProblem(mu_star)
    lam, st, trials, rho = oracle.solve_point_lm(prob, np.array([-0.3, 0.0, 0.1]), 60, 0.0, cap, radius0=0.1)
    np.testing.assert_array_equal(prob.seen[0], np.array([-0.3, 0.0, 0.1]) ** 2)
    np.testing.assert_allclose(lam, np.sqrt([0.25, cap * cap, 0.5]), rtol=1e-9)
    assert st == oracle.ST_BUDGET and trials == 60 == len(prob.seen)
    # every proposal stayed in the box
    assert all(np.all(m >= 0.0) and np.all(m <= cap * cap) for m in prob.seen)
    # rho is the residual at the returned point
    assert abs(rho - np.max(np.abs(prob.A @ lam ** 2 - prob.b))) < 1e-12


def test_solve_point_lm_trust_radius_is_in_lambda():
    """From lambda = 0 with a full Gauss-Newton step beyond the radius Delta0 in every component, the
    first proposal is sqrt(mu) = Delta0 in each (a radius applied to mu would give sqrt(Delta0));
    after that acceptance the radius doubles, so the second proposal moves sqrt(mu) by at most
    2 Delta0; with radius0 = inf the first proposal is the damped step itself, damped by nu0 (1 by
    default)."""
    prob = _LinearMuProblem([0.25, 0.9, 0.5])
    oracle.solve_point_lm(prob, np.zeros(3), 3, 0.0, 1.2, radius0=0.1)
    np.testing.assert_allclose(np.sqrt(prob.seen[1]), [0.1, 0.1, 0.1], rtol=1e-15)
    step2 = np.sqrt(prob.seen[2]) - np.sqrt(prob.seen[1])
    assert np.all(step2 <= 0.2 * (1 + 1e-12)) and np.any(step2 >= 0.2 * (1 - 1e-12))
    for nu0 in (None, 1e-3):
        free = _LinearMuProblem([0.25, 0.9, 0.5])
        kw = {} if nu0 is None else dict(nu0=nu0)
        oracle.solve_point_lm(free, np.zeros(3), 2, 0.0, 1.2, **kw)
        d = oracle.lm_direction(free.A, -free.b, 1.0 if nu0 is None else nu0)
        np.testing.assert_allclose(free.seen[1], np.clip(d, 0.0, 1.44), rtol=1e-15)
    # the two dampings give different first steps (the pin would not see a swapped default otherwise)
    assert not np.allclose(oracle.lm_direction(free.A, -free.b, 1.0), oracle.lm_direction(free.A, -free.b, 1e-3))


class _ScriptedLM:
    """A stand-in whose first calls return scripted (u, Phi): call 1 has u = 0 (so the next proposal
    repeats mu), call 2 is accepted and points at a far target, call 3 is rejected."""

    def __init__(self, target, cap):
        self.A = np.diag([2.0, 0.7, 1.3, 0.0])[:, :3] + 0.0
        self.t = np.asarray(target, np.float64)
        self.cap, self.seen = cap, []

    def lm_eval(self, mu):
        self.seen.append(np.array(mu, np.float64))
        k = len(self.seen)
        u = np.zeros(4) if k == 1 else self.A @ (np.asarray(mu) - self.t)
        phi = {1: 10.0, 2: 5.0, 3: 100.0}.get(k, float(u @ u))
        return u, self.A, phi, 1.0, oracle.ST_BUDGET


def test_solve_point_lm_infinite_radius_never_shrinks():
    """radius0 = inf is no trust region at all: after an acceptance and a rejection the next proposal
    still reaches the damped step's far target (a radius that became the cap on acceptance and was
    halved on rejection would stop it at cap / 2); a finite radius0 does stop it. A small initial
    damping (1e-3) keeps the damped steps close to the Gauss-Newton ones, so the target is reached."""
    cap = 1.2
    target = [0.81 * cap * cap, 0.01, 0.01]
    free = _ScriptedLM(target, cap)
    oracle.solve_point_lm(free, np.zeros(3), 4, 0.0, cap, nu0=1e-3)
    assert np.array_equal(free.seen[1], np.zeros(3))            # u = 0: no step
    assert math.sqrt(free.seen[3][0]) > 0.85 * cap               # not limited after the rejection
    boxed = _ScriptedLM(target, cap)
    oracle.solve_point_lm(boxed, np.zeros(3), 4, 0.0, cap, nu0=1e-3, radius0=0.25)
    # 0.25 doubled on acceptance (0.5), halved on rejection (0.25): the fourth proposal moves 0.25
    np.testing.assert_allclose(math.sqrt(boxed.seen[2][0]), 0.5, rtol=1e-15)
    np.testing.assert_allclose(math.sqrt(boxed.seen[3][0]), 0.25, rtol=1e-15)


def test_solve_point_lm_status_mapping():
    # converged at the start: one trial, |lambda0| returned
    prob = _LinearMuProblem([0.25, 0.9, 0.5])
    lam, st, tr, rho = oracle.solve_point_lm(prob, np.array([-0.5, 0.3, 0.0]), 20, 1e3, 2.0)
    assert st == oracle.ST_CONVERGED and tr == 1
    np.testing.assert_array_equal(lam, [0.5, 0.3, 0.0])
    # J = 0 at every trial is not a failure of the point: BUDGET
    prob = _LinearMuProblem([0.25, 0.9, 0.5], status=oracle.ST_J_ZERO)
    assert oracle.solve_point_lm(prob, np.zeros(3), 7, 0.0, 2.0)[1:3] == (oracle.ST_BUDGET, 7)

    class Degenerate:
        def __init__(self, st):
            self.st = st

        def lm_eval(self, mu):
            return np.zeros(4), np.zeros((4, 3)), math.inf, math.inf, self.st

    for code in (oracle.ST_DEGENERATE, oracle.ST_NONFINITE):
        lam, st, tr, rho = oracle.solve_point_lm(Degenerate(code), np.array([0.2, 0.0, 0.0]), 9, 1e-4, 2.0)
        assert st == code and tr == 1 and rho == math.inf


def test_lm_eval_jacobian_is_the_mu_derivative():
    """PointProblem.lm_eval takes mu = lambda^2: its Jacobian (from the tangents, pinned separately)
    equals central differences of its own residual vector in that argument (had it taken lambda, the
    differences would be 2 lambda times larger)."""
    w = config1()
    b = w.boundaries[0]
    prob = oracle.PointProblem(b.B0, b.x0, b.y0, b.h, w.xyz[:, 200])
    mu = np.array([1.7, 0.6, 2.3])
    u, Jac, Phi, rho, st = prob.lm_eval(mu)
    assert abs(Phi - u @ u) < 1e-14 and st == oracle.ST_BUDGET
    e = 1e-6
    for p in range(3):
        d = np.zeros(3)
        d[p] = e
        fd = (prob.lm_eval(mu + d)[0] - prob.lm_eval(mu - d)[0]) / (2 * e)
        np.testing.assert_allclose(Jac[:, p], fd, rtol=1e-6, atol=1e-9 * np.max(np.abs(Jac)))


class _QuadraticLambdaProblem:
    """A stand-in for PointProblem in the derivative-free form: Phi(lambda) = |lambda - c|^2 + phi0,
    rho = sqrt(Phi); records every lambda it evaluates."""

    def __init__(self, c, phi0=0.01, status=oracle.ST_BUDGET, conv_at=None):
        self.c, self.phi0, self.status, self.conv_at, self.seen = np.asarray(c, np.float64), phi0, status, conv_at, []

    def eval(self, lam):
        self.seen.append(np.array(lam, np.float64))
        phi = float(np.sum((lam - self.c) ** 2) + self.phi0)
        rho = math.sqrt(phi)
        if self.conv_at is not None and len(self.seen) == self.conv_at:
            rho = 0.0
        return None, dict(Phi=np.array([phi]), rho=np.array([rho]), status=np.array([self.status]))


def test_solve_point_nm_cap_counts_trials_without_evaluating():
    """The optimum lies beyond the cap in x: proposals outside |lambda_p| <= cap cost a trial but are
    never evaluated (Phi = +inf), the result is the best evaluated (hence feasible) vertex, and the
    status is BUDGET after exactly `budget` trials."""
    cap = 1.0
    prob = _QuadraticLambdaProblem([3.0, 0.2, -0.1])
    lam, st, trials, rho = oracle.solve_point_nm(prob, np.zeros(3), 80, 1e-6, 0.25, cap)
    assert st == oracle.ST_BUDGET and trials == 80
    assert all(np.all(np.abs(x) <= cap) for x in prob.seen)
    assert len(prob.seen) < trials                      # some trials were infeasible proposals
    phis = [float(np.sum((x - prob.c) ** 2) + 0.01) for x in prob.seen]
    k = int(np.argmin(phis))
    np.testing.assert_array_equal(lam, prob.seen[k])
    assert rho == math.sqrt(phis[k])
    # it moved to the face x = cap of the box, near the best feasible value (2^2 + 0.01)
    assert lam[0] > 0.9 and phis[k] < 4.01 + 0.05 < phis[0]


def test_solve_point_nm_status_mapping():
    # a trial with rho <= eps ends the search with that trial's lambda
    prob = _QuadraticLambdaProblem([0.3, 0.2, 0.1], conv_at=6)
    lam, st, tr, rho = oracle.solve_point_nm(prob, np.zeros(3), 50, 1e-4, 0.25, 5.0)
    assert st == oracle.ST_CONVERGED and tr == 6 and rho == 0.0
    np.testing.assert_array_equal(lam, prob.seen[5])
    # J = 0 at the best point: BUDGET
    prob = _QuadraticLambdaProblem([0.3, 0.2, 0.1], status=oracle.ST_J_ZERO)
    assert oracle.solve_point_nm(prob, np.zeros(3), 12, 1e-4, 0.25, 5.0)[1:3] == (oracle.ST_BUDGET, 12)

    class Degenerate:
        def eval(self, lam):
            return None, dict(Phi=np.array([math.inf]), rho=np.array([math.inf]),
                              status=np.array([oracle.ST_DEGENERATE]))

    lam, st, tr, rho = oracle.solve_point_nm(Degenerate(), np.zeros(3), 9, 1e-4, 0.25, 5.0)
    assert st == oracle.ST_DEGENERATE and tr == 9


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
