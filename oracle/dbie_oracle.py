"""Plain, slow FP64 CPU oracle for the DBIE hot path (Wang, Yan & Tan, arXiv:1306.1122).

TEST INFRASTRUCTURE. Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py may
import or run anything in this package. It shares no code with the GPU library and imports nothing
from it; its inputs come from the `workloads` generators or from the caller.

Everything is float64 NumPy, written to be checked against the paper by eye:

* `kernel`          - the DBIE half-space kernel of Eq. (6).
* `field`           - the nodal sum of Eq. (16) with a_ik = h^2 K (pixel centres, weight h^2), plus
                      the first derivatives at frozen lambda (zeroth-order lambda expansion, Eq. 13)
                      and the derivatives with respect to mu = lambda^2 ("tangents").
* `field_fd`        - the paper's own first-order finite difference at frozen lambda, delta = 1e-3 h
                      (Section 2.1 after Eq. 12), kept as a cross-check of the analytic derivatives.
* `residuals`       - J = curl B (Eq. 14), f_i (Eq. 8), g_i (Eq. 9), Phi = f^2 + g^2.
* `residual_jacobian` - d(residual vector)/d mu by the chain rule through the tangents.
* `nelder_mead`, `solve_point_nm` - the derivative-free lambda search (downhill simplex,
                      Section 2.1; Lagarias et al. 1998 formulation).
* `solve_point_lm`  - Levenberg-Marquardt in mu = lambda^2 using the tangents (gradient form).
* `vjp`             - the transpose of the nodal sum (gradient with respect to B0) and the lambda
                      gradient from the tangents.

Sums over pixels use numpy's pairwise summation along a contiguous axis (error ~log2(N_pix) ulp
of the sum of absolute terms).

Readings where the paper is silent:
  * nodes are pixel centres with weight h^2; the field outside the magnetogram is zero (Eq. 3 text);
  * one lambda per field component and point;
  * derivatives are the exact delta -> 0 limit at frozen lambda;
  * Delta V / Delta sigma in g_i = h/6 (cube of side h);
  * Phi = f^2 + g^2 combines Eqs. (10)-(11); convergence is max(f, g) <= eps (Eq. 12);
  * |J| = 0 gives f = 0 (status J_ZERO); |B| = 0 is DEGENERATE.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Callable, List, Optional, Tuple

import numpy as np

TWO_PI = 2.0 * math.pi

# per-point status codes (same meaning as the library's)
ST_CONVERGED, ST_BUDGET, ST_DEGENERATE, ST_J_ZERO, ST_NONFINITE = 0, 1, 2, 3, 4


# ------------------------------------------------------------------------------------------------
# Eq. (6): the kernel
# ------------------------------------------------------------------------------------------------
def kernel(lam, dx, dy, z):
    """K(lambda; dx, dy, z) = z [lambda r sin(lambda r) + cos(lambda r)] / (2 pi r^3),
    r^2 = dx^2 + dy^2 + z^2, with (dx, dy) = (x - x_i, y - y_i) and z = z_i (Eq. 6)."""
    r = np.sqrt(dx * dx + dy * dy + z * z)
    t = lam * r
    return z * (t * np.sin(t) + np.cos(t)) / (TWO_PI * r ** 3)


def pixel_centres(nx: int, ny: int, x0: float, y0: float, h: float):
    """Flattened (x, y) of the pixel centres, x fastest (row-major [ny][nx])."""
    X, Y = np.meshgrid(x0 + h * np.arange(nx), y0 + h * np.arange(ny))
    return X.ravel(), Y.ravel()


# ------------------------------------------------------------------------------------------------
# Eq. (16) nodal sum + frozen-lambda derivatives (Eq. 13) + mu-tangents
# ------------------------------------------------------------------------------------------------
def field(B0, x0, y0, h, xyz, lam, tangents: bool = False, chunk: int = 64, absolute: bool = False):
    """Field, frozen-lambda gradient and (optionally) mu-tangents at every point.

    B0: [3, ny, nx]; xyz: [3, N]; lam: [3, N] (lambda_p for p = x, y, z).
    Returns B [3, N], dB [9, N] with dB[3p+q] = d B_p / d x_q at frozen lambda, and if requested
    tan [12, N] = d/d mu_p of the rows (B_0..2, dB_0..8) that belong to component p
    (tan[p] = dB_p/dmu_p, tan[3+3p+q] = d(dB_p/dx_q)/dmu_p).

    With F(r) = N(lambda r)/r^3, N(t) = t sin t + cos t, and F'(r) = (t^2 cos t - 3N)/r^4:
      B_p      = (z h^2 / 2pi) sum_k F B0_pk
      dB_p/dx  = (z h^2 / 2pi) sum_k F'(r) (x_i - x_k)/r B0_pk      (and likewise y)
      dB_p/dz  = (h^2 / 2pi)   sum_k [F + z^2 F'(r)/r] B0_pk
    and dF/dmu = cos(t)/(2r), d(F'/r)/dmu = -N/(2 r^3).

    absolute=True also returns, after the others, the same rows summed over the absolute values of
    their terms (sum_k |term_k|, with the same prefactors): the scale that bounds the rounding error
    of any summation order of each row.
    """
    B0 = np.asarray(B0, np.float64)
    xyz = np.asarray(xyz, np.float64)
    lam = np.asarray(lam, np.float64)
    ny, nx = B0.shape[1:]
    X, Y = pixel_centres(nx, ny, x0, y0, h)
    Bk = B0.reshape(3, -1)
    npts = xyz.shape[1]
    B = np.zeros((3, npts))
    dB = np.zeros((9, npts))
    tan = np.zeros((12, npts)) if tangents else None
    if absolute:
        aB, adB = np.zeros((3, npts)), np.zeros((9, npts))
        atan = np.zeros((12, npts)) if tangents else None
    w = h * h / TWO_PI
    for s in range(0, npts, chunk):
        e = min(npts, s + chunk)
        xi = xyz[0, s:e, None]
        yi = xyz[1, s:e, None]
        zi = xyz[2, s:e, None]
        dx = X[None, :] - xi          # x_k - x_i
        dy = Y[None, :] - yi
        r2 = dx * dx + dy * dy + zi * zi
        r = np.sqrt(r2)
        z = zi[:, 0]
        for p in range(3):
            t = lam[p, s:e, None] * r
            sn, cs = np.sin(t), np.cos(t)
            N = t * sn + cs
            F = N / (r2 * r)                              # N / r^3
            G = (t * t * cs - 3.0 * N) / (r2 * r2 * r)    # F'(r) / r
            b = Bk[p][None, :]
            B[p, s:e] = w * z * np.sum(F * b, axis=1)
            dB[3 * p + 0, s:e] = -w * z * np.sum(G * dx * b, axis=1)
            dB[3 * p + 1, s:e] = -w * z * np.sum(G * dy * b, axis=1)
            dB[3 * p + 2, s:e] = w * np.sum((F + z[:, None] ** 2 * G) * b, axis=1)
            if absolute:
                aB[p, s:e] = w * z * np.sum(np.abs(F * b), axis=1)
                adB[3 * p + 0, s:e] = w * z * np.sum(np.abs(G * dx * b), axis=1)
                adB[3 * p + 1, s:e] = w * z * np.sum(np.abs(G * dy * b), axis=1)
                adB[3 * p + 2, s:e] = w * np.sum(np.abs((F + z[:, None] ** 2 * G) * b), axis=1)
            if tangents:
                dF = cs / (2.0 * r)                       # dF/dmu
                dG = -N / (2.0 * r2 * r)                  # d(F'/r)/dmu
                tan[p, s:e] = w * z * np.sum(dF * b, axis=1)
                tan[3 + 3 * p + 0, s:e] = -w * z * np.sum(dG * dx * b, axis=1)
                tan[3 + 3 * p + 1, s:e] = -w * z * np.sum(dG * dy * b, axis=1)
                tan[3 + 3 * p + 2, s:e] = w * np.sum((dF + z[:, None] ** 2 * dG) * b, axis=1)
                if absolute:
                    atan[p, s:e] = w * z * np.sum(np.abs(dF * b), axis=1)
                    atan[3 + 3 * p + 0, s:e] = w * z * np.sum(np.abs(dG * dx * b), axis=1)
                    atan[3 + 3 * p + 1, s:e] = w * z * np.sum(np.abs(dG * dy * b), axis=1)
                    atan[3 + 3 * p + 2, s:e] = w * np.sum(np.abs((dF + z[:, None] ** 2 * dG) * b), axis=1)
    out = (B, dB, tan) if tangents else (B, dB)
    if absolute:
        out = out + ((aB, adB, atan) if tangents else (aB, adB))
    return out


def field_only(B0, x0, y0, h, xyz, lam, chunk: int = 64):
    """B alone: the Eq. (16) nodal sum, B_p(i) = sum_k h^2 K(lambda_pi; x_k - x_i, y_k - y_i, z_i) B0_pk."""
    B0 = np.asarray(B0, np.float64)
    ny, nx = B0.shape[1:]
    X, Y = pixel_centres(nx, ny, x0, y0, h)
    Bk = B0.reshape(3, -1)
    npts = xyz.shape[1]
    B = np.zeros((3, npts))
    for s in range(0, npts, chunk):
        e = min(npts, s + chunk)
        dx = X[None, :] - xyz[0, s:e, None]
        dy = Y[None, :] - xyz[1, s:e, None]
        for p in range(3):
            K = kernel(lam[p, s:e, None], dx, dy, xyz[2, s:e, None])
            B[p, s:e] = h * h * np.sum(K * Bk[p][None, :], axis=1)
    return B


def field_fd(B0, x0, y0, h, xyz, lam, delta_px: float = 1e-3):
    """The paper's forward first-order difference at frozen lambda with delta = delta_px * h."""
    xyz = np.asarray(xyz, np.float64)
    d = delta_px * h
    B = field_only(B0, x0, y0, h, xyz, lam)
    dB = np.zeros((9, xyz.shape[1]))
    for q in range(3):
        sh = xyz.copy()
        sh[q] += d
        Bq = field_only(B0, x0, y0, h, sh, lam)
        for p in range(3):
            dB[3 * p + q] = (Bq[p] - B[p]) / d
    return B, dB


# ------------------------------------------------------------------------------------------------
# Eqs. (8), (9), (14): residuals
# ------------------------------------------------------------------------------------------------
def curl_div(dB):
    """J = curl B (Eq. 14) and div B from dB[3p+q] = dB_p/dx_q."""
    J = np.stack([dB[7] - dB[5], dB[2] - dB[6], dB[3] - dB[1]])
    D = dB[0] + dB[4] + dB[8]
    return J, D


def residuals(B, dB, h, dv_over_dsigma_h: float = 1.0 / 6.0):
    """f_i = |J x B| / (|J||B|) (Eq. 8) and g_i = |div B| dV / (|B| dSigma) (Eq. 9).

    Returns f, g, Phi = f^2 + g^2, rho = max(f, g), status, and the signed residual vector
    u = (J x B / (|J||B|), sign(div B) g) of length 4 with |u|^2 = Phi.
    """
    J, D = curl_div(dB)
    nB = np.sqrt(np.sum(B * B, axis=0))
    nJ = np.sqrt(np.sum(J * J, axis=0))
    c = dv_over_dsigma_h * h
    JxB = np.cross(J.T, B.T).T
    with np.errstate(divide="ignore", invalid="ignore"):
        u3 = JxB / (nJ * nB)
        s = c * D / nB
    status = np.full(B.shape[1], ST_BUDGET, np.int32)
    jzero = nJ == 0.0
    u3[:, jzero] = 0.0
    status[jzero] = ST_J_ZERO
    degen = nB == 0.0
    status[degen] = ST_DEGENERATE
    u3[:, degen] = 0.0
    s = np.where(degen, 0.0, s)
    f = np.sqrt(np.sum(u3 * u3, axis=0))
    g = np.abs(s)
    u = np.vstack([u3, s[None, :]])
    bad = ~(np.all(np.isfinite(B), axis=0) & np.all(np.isfinite(dB), axis=0))
    status[bad] = ST_NONFINITE
    Phi = f * f + g * g
    rho = np.maximum(f, g)
    Phi = np.where(bad | degen, np.inf, Phi)
    rho = np.where(bad | degen, np.inf, rho)
    return dict(f=f, g=g, Phi=Phi, rho=rho, status=status, u=u, J=J, D=D)


def residual_jacobian(B, dB, tan, h, dv_over_dsigma_h: float = 1.0 / 6.0):
    """d u / d mu_p (shape [4, 3, N]) for the residual vector u of `residuals`, by the chain rule.

    Only B_p and the row dB_p/dx_q depend on mu_p; their mu-derivatives are the tangents."""
    J, D = curl_div(dB)
    nB = np.sqrt(np.sum(B * B, axis=0))
    nJ = np.sqrt(np.sum(J * J, axis=0))
    c = dv_over_dsigma_h * h
    w = np.cross(J.T, B.T).T
    out = np.zeros((4, 3, B.shape[1]))
    for p in range(3):
        Bd = np.zeros_like(B)
        Bd[p] = tan[p]
        dBd = np.zeros_like(dB)
        for q in range(3):
            dBd[3 * p + q] = tan[3 + 3 * p + q]
        Jd, Dd = curl_div(dBd)
        wd = np.cross(Jd.T, B.T).T + np.cross(J.T, Bd.T).T
        with np.errstate(divide="ignore", invalid="ignore"):
            da = np.sum(J * Jd, axis=0) / nJ
            db = np.sum(B * Bd, axis=0) / nB
            du3 = wd / (nJ * nB) - w * (da / nJ + db / nB) / (nJ * nB)
            ds = c * Dd / nB - c * D * db / (nB * nB)
        du3[:, nJ == 0.0] = 0.0
        out[:3, p] = du3
        out[3, p] = ds
    return out


# ------------------------------------------------------------------------------------------------
# VJP: transpose of Eq. (16) with its frozen-lambda derivative rows
# ------------------------------------------------------------------------------------------------
def vjp(B0, x0, y0, h, xyz, lam, gB=None, gdB=None, chunk: int = 64, pixels=None):
    """g_B0[p, k] = sum_i h^2 [K_p gB_p + dK_p/dx_i gdB_{p,x} + dK_p/dy_i gdB_{p,y} + dK_p/dz_i gdB_{p,z}]
    and g_lambda from the tangents: g_mu_p = gB_p . tan_p + sum_q gdB_pq . tan_pq, g_lambda = 2 lambda g_mu.

    pixels (flat indices b * nx + a): only those outputs, as g_B0 [3, len(pixels)], with g_lambda
    and g_mu returned as None (the same sum over every point, for a few pixels of a large problem)."""
    B0 = np.asarray(B0, np.float64)
    ny, nx = B0.shape[1:]
    npts = xyz.shape[1]
    if gB is None:
        gB = np.zeros((3, npts))
    if gdB is None:
        gdB = np.zeros((9, npts))
    X, Y = pixel_centres(nx, ny, x0, y0, h)
    if pixels is not None:
        pixels = np.asarray(pixels, np.int64)
        X, Y = X[pixels], Y[pixels]
        chunk = max(chunk, (1 << 18) // max(len(pixels), 1))
    gB0 = np.zeros((3, X.size))
    w = h * h / TWO_PI
    for s in range(0, npts, chunk):
        e = min(npts, s + chunk)
        dx = X[None, :] - xyz[0, s:e, None]
        dy = Y[None, :] - xyz[1, s:e, None]
        zi = xyz[2, s:e, None]
        r2 = dx * dx + dy * dy + zi * zi
        r = np.sqrt(r2)
        for p in range(3):
            t = lam[p, s:e, None] * r
            sn, cs = np.sin(t), np.cos(t)
            N = t * sn + cs
            F = N / (r2 * r)
            G = (t * t * cs - 3.0 * N) / (r2 * r2 * r)
            coef = (zi * F * gB[p, s:e, None]
                    - zi * G * dx * gdB[3 * p + 0, s:e, None]
                    - zi * G * dy * gdB[3 * p + 1, s:e, None]
                    + (F + zi * zi * G) * gdB[3 * p + 2, s:e, None])
            gB0[p] += w * np.sum(np.ascontiguousarray(coef.T), axis=1)
    if pixels is not None:
        return gB0, None, None
    _, _, tan = field(B0, x0, y0, h, xyz, lam, tangents=True)
    gmu = np.zeros((3, npts))
    for p in range(3):
        gmu[p] = gB[p] * tan[p] + sum(gdB[3 * p + q] * tan[3 + 3 * p + q] for q in range(3))
    glam = 2.0 * lam * gmu
    return gB0.reshape(3, ny, nx), glam, gmu


# ------------------------------------------------------------------------------------------------
# Derivative-free lambda search: downhill simplex (Section 2.1; Lagarias, Reeds, Wright & Wright 1998)
# ------------------------------------------------------------------------------------------------
@dataclass
class NMResult:
    x: np.ndarray
    fx: float
    trials: int
    converged: bool
    history: List[Tuple[np.ndarray, float]]


def nelder_mead(fun: Callable[[np.ndarray], Tuple[float, bool]], x0, delta: float, budget: int,
                rho: float = 1.0, chi: float = 2.0, gamma: float = 0.5, sigma: float = 0.5) -> NMResult:
    """Downhill simplex on fun(x) -> (value, done).

    One call of `fun` is one trial. The search stops as soon as a trial reports done (that trial's x
    is returned) or after `budget` trials (the best trial is returned; ties keep the earlier one).
    Initial simplex: x0 and x0 + delta e_j. Vertices keep fixed slots; the order is by
    (value, slot). Reflection, expansion, outside/inside contraction and shrink follow Lagarias et al.
    """
    x0 = np.asarray(x0, np.float64)
    n = x0.size
    hist: List[Tuple[np.ndarray, float]] = []
    best = [None, np.inf]

    class _Stop(Exception):
        pass

    def trial(x):
        v, done = fun(x)
        hist.append((x.copy(), v))
        if v < best[1] or best[0] is None:
            best[0], best[1] = x.copy(), v
        if done:
            best[0], best[1] = x.copy(), v
            raise _Stop(True)
        if len(hist) >= budget:
            raise _Stop(False)
        return v

    sim = [x0.copy()] + [x0 + delta * np.eye(n)[j] for j in range(n)]
    val = [np.inf] * (n + 1)
    try:
        for j in range(n + 1):
            val[j] = trial(sim[j])
        while True:
            order = sorted(range(n + 1), key=lambda j: (val[j], j))
            lo, hi, sh = order[0], order[-1], order[-2]
            xbar = sim[order[0]].copy()
            for j in order[1:-1]:
                xbar = xbar + sim[j]
            xbar = xbar / n
            xr = (1.0 + rho) * xbar - rho * sim[hi]
            fr = trial(xr)
            if fr < val[lo]:
                xe = (1.0 + rho * chi) * xbar - rho * chi * sim[hi]
                fe = trial(xe)
                if fe < fr:
                    sim[hi], val[hi] = xe, fe
                else:
                    sim[hi], val[hi] = xr, fr
                continue
            if fr < val[sh]:
                sim[hi], val[hi] = xr, fr
                continue
            if fr < val[hi]:
                xc = (1.0 + gamma * rho) * xbar - gamma * rho * sim[hi]
                fc = trial(xc)
                if fc <= fr:
                    sim[hi], val[hi] = xc, fc
                    continue
            else:
                xcc = (1.0 - gamma) * xbar + gamma * sim[hi]
                fcc = trial(xcc)
                if fcc < val[hi]:
                    sim[hi], val[hi] = xcc, fcc
                    continue
            # shrink towards the best vertex, in the current order
            for j in order[1:]:
                sim[j] = sim[lo] + sigma * (sim[j] - sim[lo])
                val[j] = trial(sim[j])
    except _Stop as st:
        return NMResult(best[0], best[1], len(hist), bool(st.args[0]), hist)


class PointProblem:
    """Evaluation of one point's residual at a lambda triple (one trial = one (B, grad B) evaluation)."""

    def __init__(self, B0, x0, y0, h, xyz_i, dv_over_dsigma_h=1.0 / 6.0):
        self.B0, self.x0, self.y0, self.h = B0, x0, y0, h
        self.p = np.asarray(xyz_i, np.float64).reshape(3, 1)
        self.c = dv_over_dsigma_h

    def eval(self, lam3, tangents=False):
        lam = np.asarray(lam3, np.float64).reshape(3, 1)
        out = field(self.B0, self.x0, self.y0, self.h, self.p, lam, tangents=tangents)
        res = residuals(out[0], out[1], self.h, self.c)
        return out, res

    def lm_eval(self, mu3):
        """One trial of the gradient form at mu = lambda^2: the residual vector u (`residuals`), its
        Jacobian du/dmu (`residual_jacobian`, from the tangents at lambda = sqrt(mu)), Phi, rho and
        the status."""
        (B, dB, tan), res = self.eval(np.sqrt(np.asarray(mu3, np.float64)), tangents=True)
        Jac = residual_jacobian(B, dB, tan, self.h, self.c)[:, :, 0]
        return res["u"][:, 0], Jac, float(res["Phi"][0]), float(res["rho"][0]), int(res["status"][0])


def default_nm_step(boundary_nx: int, boundary_ny: int, h: float) -> float:
    """Initial simplex edge 1/L, L = the magnetogram's longer side in length units."""
    return 1.0 / (max(boundary_nx, boundary_ny) * h)


def solve_point_nm(prob: PointProblem, lam0, budget: int, eps: float, delta: float,
                   lam_cap: float) -> Tuple[np.ndarray, int, int, float]:
    """Nelder-Mead on Phi(lambda) for one point; returns (lambda*, status, trials, rho*)."""
    info = {}

    def fun(lam):
        if np.any(np.abs(lam) > lam_cap):
            return np.inf, False
        _, res = prob.eval(lam)
        rho = float(res["rho"][0])
        info[tuple(lam)] = (rho, int(res["status"][0]))
        return float(res["Phi"][0]), bool(rho <= eps)

    r = nelder_mead(fun, lam0, delta, budget)
    rho, st = info.get(tuple(r.x), (np.inf, ST_NONFINITE))
    if r.converged:
        st = ST_CONVERGED
    elif st in (ST_J_ZERO, ST_BUDGET):
        st = ST_BUDGET
    return r.x, st, r.trials, rho


# ------------------------------------------------------------------------------------------------
# Gradient form: Levenberg-Marquardt in mu = lambda^2 (Marquardt 1963 scaling)
# ------------------------------------------------------------------------------------------------
def lm_direction(Jac, u, nu):
    """Solve (A + nu diag(A)) d = -J^T u, A = J^T J, with diag(A) floored at 1e-12 max diag(A)."""
    A = Jac.T @ Jac
    gvec = Jac.T @ u
    dg = np.diag(A).copy()
    m = dg.max()
    if not np.isfinite(m) or m <= 0.0:
        return np.zeros(3)
    dg = np.maximum(dg, 1e-12 * m)
    return np.linalg.solve(A + nu * np.diag(dg), -gvec)


def levenberg_marquardt(evalfun, mu0, budget: int, eps: float, mu_cap: float, nu0: float = 1.0,
                        radius0: float = math.inf):
    """Projected Levenberg-Marquardt on Phi(mu) = |u(mu)|^2, mu in [0, mu_cap]^3, with a trust region
    in lambda = sqrt(mu).

    evalfun(mu) -> (u [4], Jac [4, 3] = du/dmu, Phi, rho, status); one call is one trial.
    Start at mu0 with damping nu0; each iteration solves the damped normal equations
    (J^T J + nu diag(J^T J)) d = -J^T u (`lm_direction`) for a step d, and the proposal
    mu + d is clipped, per component, into the box where sqrt(mu) lies within the radius Delta of the
    accepted point's sqrt(mu) and inside [0, sqrt(mu_cap)]. The proposal is evaluated and accepted if
    Phi falls (nu /= 10, Delta doubled up to sqrt(mu_cap)) or rejected (nu *= 10, Delta halved).
    Delta starts at radius0; radius0 = inf means no trust region: every proposal is mu + d clipped to
    the box [0, mu_cap] and Delta never changes. Stops when rho <= eps or after `budget` trials.
    Returns (mu, status, trials, rho, Phi)."""
    mu = np.asarray(mu0, np.float64).copy()
    u, Jac, Phi, rho, st = evalfun(mu)
    trials = 1
    if not np.isfinite(Phi):
        return mu, st, trials, rho, Phi
    if rho <= eps:
        return mu, ST_CONVERGED, trials, rho, Phi
    nu = nu0
    cap = math.sqrt(mu_cap)
    radius = radius0
    while trials < budget:
        d = lm_direction(Jac, u, nu)
        if math.isinf(radius):
            mu_new = np.clip(mu + d, 0.0, mu_cap)
        else:
            lam = np.sqrt(mu)
            lo = np.maximum(lam - radius, 0.0)
            hi = np.minimum(lam + radius, cap)
            mu_new = np.minimum(np.maximum(mu + d, lo * lo), hi * hi)
        u2, Jac2, Phi2, rho2, st2 = evalfun(mu_new)
        trials += 1
        if rho2 <= eps:
            return mu_new, ST_CONVERGED, trials, rho2, Phi2
        if Phi2 < Phi:
            mu, u, Jac, Phi, rho = mu_new, u2, Jac2, Phi2, rho2
            nu = nu / 10.0
            if not math.isinf(radius):
                radius = min(2.0 * radius, cap)
        else:
            nu = nu * 10.0
            if not math.isinf(radius):
                radius = 0.5 * radius
    return mu, ST_BUDGET, trials, rho, Phi


def solve_point_lm(prob, lam0, budget: int, eps: float, lam_cap: float, nu0: float = 1.0,
                   radius0: float = math.inf) -> Tuple[np.ndarray, int, int, float]:
    """Gradient form for one point: LM in mu = lambda^2 >= 0 (`levenberg_marquardt`, box [0, cap^2],
    trust radius radius0 in lambda); one trial = one call of prob.lm_eval(mu), which for a DBIE point
    is one evaluation of (B, grad B, tangents) at lambda = sqrt(mu). Returns (|lambda*|, status,
    trials, rho*); the status is CONVERGED, BUDGET (J_ZERO points included: f = 0 is a finite
    residual), or the residual status of a start with non-finite Phi (DEGENERATE, NONFINITE)."""
    mu, st, trials, rho, _ = levenberg_marquardt(prob.lm_eval, np.asarray(lam0, np.float64) ** 2, budget,
                                                 eps, lam_cap * lam_cap, nu0, radius0)
    return np.sqrt(mu), st, trials, rho


# ------------------------------------------------------------------------------------------------
# Eq. (15): 9-node quadratic boundary elements with Gauss-Legendre quadrature
# ------------------------------------------------------------------------------------------------
def _lagrange3(xi):
    """Quadratic Lagrange shape functions on the nodes -1, 0, 1 (rows) at the abscissae xi."""
    xi = np.asarray(xi, np.float64)
    return np.stack([0.5 * xi * (xi - 1.0), 1.0 - xi * xi, 0.5 * xi * (xi + 1.0)])


def field_quad9(B0, x0, y0, h, xyz, lam, G: int = 4, tangents: bool = False, chunk: int = 16):
    """Eq. (15): B_p(i) = sum_e sum_j [int int K N_j J dxi deta] B0_p(node j of e).

    The magnetogram's nodes (pixel centres) are grouped into 9-node elements: element (m, n) holds
    the nodes a = 2m..2m+2, b = 2n..2n+2 (so nx and ny must be odd); on it x = x0 + (2m+1+xi) h,
    y = y0 + (2n+1+eta) h, J = h^2 and N_j(xi, eta) = L_alpha(xi) L_beta(eta) with the quadratic Lagrange
    polynomials. Each element integral uses G x G Gauss-Legendre points. The frozen-lambda gradient
    rows and mu-tangents follow as in `field` (derivatives of K with respect to the point)."""
    B0 = np.asarray(B0, np.float64)
    ny, nx = B0.shape[1:]
    if nx % 2 == 0 or ny % 2 == 0 or nx < 3 or ny < 3:
        raise ValueError("9-node elements need odd nx, ny >= 3")
    ex, ey = (nx - 1) // 2, (ny - 1) // 2
    xg, wg = np.polynomial.legendre.leggauss(G)
    Lg = _lagrange3(xg)                                  # [3 nodes, G points]
    npts = xyz.shape[1]
    B = np.zeros((3, npts))
    dB = np.zeros((9, npts))
    tan = np.zeros((12, npts)) if tangents else None
    # every element-node-Gauss contribution as one list of (position, weight x B0 of the node)
    # m, n: element; alpha, beta: node in the element; g, q: Gauss point
    m = np.arange(ex)[:, None, None, None, None, None]
    n = np.arange(ey)[None, :, None, None, None, None]
    al = np.arange(3)[None, None, :, None, None, None]
    be = np.arange(3)[None, None, None, :, None, None]
    g = np.arange(G)[None, None, None, None, :, None]
    q = np.arange(G)[None, None, None, None, None, :]
    shp = (ex, ey, 3, 3, G, G)
    gx = np.broadcast_to(x0 + (2 * m + 1 + xg[g]) * h, shp).ravel()
    gy = np.broadcast_to(y0 + (2 * n + 1 + xg[q]) * h, shp).ravel()
    wN = np.broadcast_to(wg[g] * wg[q] * Lg[al, g] * Lg[be, q] * h * h, shp).ravel()
    na = np.broadcast_to(2 * m + al, shp).ravel()
    nb = np.broadcast_to(2 * n + be, shp).ravel()
    bw = [wN * B0[p][nb, na] for p in range(3)]          # weight of each term times the node value
    for s in range(0, npts, chunk):
        e = min(npts, s + chunk)
        xi = xyz[0, s:e, None]
        yi = xyz[1, s:e, None]
        zi = xyz[2, s:e, None]
        dx = gx[None, :] - xi
        dy = gy[None, :] - yi
        r2 = dx * dx + dy * dy + zi * zi
        r = np.sqrt(r2)
        z = zi[:, 0]
        for p in range(3):
            t = lam[p, s:e, None] * r
            sn, cs = np.sin(t), np.cos(t)
            N = t * sn + cs
            F = N / (r2 * r)
            Gd = (t * t * cs - 3.0 * N) / (r2 * r2 * r)
            b = bw[p][None, :] / TWO_PI
            B[p, s:e] = z * np.sum(F * b, axis=1)
            dB[3 * p + 0, s:e] = -z * np.sum(Gd * dx * b, axis=1)
            dB[3 * p + 1, s:e] = -z * np.sum(Gd * dy * b, axis=1)
            dB[3 * p + 2, s:e] = np.sum((F + z[:, None] ** 2 * Gd) * b, axis=1)
            if tangents:
                dF = cs / (2.0 * r)
                dG = -N / (2.0 * r2 * r)
                tan[p, s:e] = z * np.sum(dF * b, axis=1)
                tan[3 + 3 * p + 0, s:e] = -z * np.sum(dG * dx * b, axis=1)
                tan[3 + 3 * p + 1, s:e] = -z * np.sum(dG * dy * b, axis=1)
                tan[3 + 3 * p + 2, s:e] = np.sum((dF + z[:, None] ** 2 * dG) * b, axis=1)
    if tangents:
        return B, dB, tan
    return B, dB
