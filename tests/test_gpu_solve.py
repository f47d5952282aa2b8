"""GPU lambda search (dbie_solve_lambda) against the oracle's solvers and re-evaluation.

lambda* is not unique (the paper notes several lambda satisfy the conditions at a point), so the
parity is on what is fixed: every point the GPU marks CONVERGED must satisfy max(f, g) <= eps when the
FP64 oracle re-evaluates it at the returned lambda; the GPU's (B, f, g) at lambda* match the oracle
there; and with FP64 evaluations the simplex trajectories coincide with the oracle's except where
rounding flips a near-tie decision.
"""
import ctypes
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1306_1122_amd as D
from _ties import Recording, has_near_tie
from workloads import config1

pytestmark = pytest.mark.gpu


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def lowlou_ctx(precision):
    w = config1()
    bd = w.boundaries[0]
    return w, bd, D.dbie_init([dict(B0=T(bd.B0), x0=bd.x0, y0=bd.y0, h=bd.h)], T(w.xyz), precision=precision)


def oracle_solve(bd, xyz, method, budget, eps, idx, radius0=None, nu0=None):
    """The oracle's search at the points idx (LM trust radius radius0 and initial damping nu0; None =
    the library's defaults, the simplex edge and 1). Returns {i: ((lambda, status, trials, rho),
    recorded trial values)}."""
    cap = math.pi / bd.h
    delta = oracle.default_nm_step(bd.nx, bd.ny, bd.h)
    out = {}
    for i in idx:
        prob = Recording(oracle.PointProblem(bd.B0, bd.x0, bd.y0, bd.h, xyz[:, i]))
        if method == "nm":
            r = oracle.solve_point_nm(prob, np.zeros(3), budget, eps, delta, cap)
        else:
            r = oracle.solve_point_lm(prob, np.zeros(3), budget, eps, cap,
                                      radius0=delta if radius0 is None else radius0,
                                      nu0=1.0 if nu0 is None else nu0)
        out[i] = (r, prob.vals)
    return out


def check_trajectories(lg, st, tr, ref, eps, what):
    """Every point's (|lambda*|, status, trials) equals the oracle's, except a point whose oracle
    trajectory holds a near-tie (tests/_ties.py), where FP64 rounding may flip a decision."""
    same, ties, bad = 0, 0, []
    for i, ((lo, so, to, _), vals) in ref.items():
        if np.allclose(lg[:, i], np.abs(lo), rtol=1e-9, atol=1e-12) and tr[i] == to and st[i] == so:
            same += 1
        elif has_near_tie(vals, eps):
            ties += 1
        else:
            bad.append(i)
    print(f"{what}: identical trajectories {same}/{len(ref)}, near-ties {ties}", flush=True)
    assert not bad, f"{what}: trajectories differ without a near-tie at points {bad}"


@pytest.mark.parametrize("method,budget,radius,damping", [("nm", 50, None, None), ("lm", 20, None, None),
                                                          ("lm", 20, math.inf, None), ("lm", 20, None, 1e-3)])
def test_fp64_solve_matches_oracle_trajectories(method, budget, radius, damping):
    """FP64 searches on the Low & Lou workload: Nelder-Mead, LM with the default trust region (the
    simplex edge) and damping (1), LM without a trust region, and LM damped by 1e-3 at the start,
    every trajectory identical to the oracle's but for near-ties."""
    w, bd, ctx = lowlou_ctx("fp64")
    N = w.n_points
    lam = torch.zeros(3, N, dtype=torch.float64, device="cuda:0")
    kw = {} if radius is None else dict(lm_radius=radius)
    if damping is not None:
        kw["lm_damping"] = damping
    r = D.dbie_solve_lambda(ctx, lam, method=method, max_trials=budget, eps=1e-4, **kw)
    torch.cuda.synchronize()
    lg = r["lam"].cpu().numpy()
    st = r["status"].cpu().numpy()
    tr = r["trials"].cpu().numpy()
    assert np.all(tr >= 1) and np.all(tr <= budget)
    idx = list(range(0, N, 4))
    ref = oracle_solve(bd, w.xyz, method, budget, 1e-4, idx, radius0=radius, nu0=damping)
    check_trajectories(lg, st, tr, ref, 1e-4, f"{method} radius {radius} damping {damping}")
    # field and residuals at lambda*: the GPU's outputs equal the oracle's re-evaluation
    Bo, dBo = oracle.field(bd.B0, bd.x0, bd.y0, bd.h, w.xyz, lg)
    res = oracle.residuals(Bo, dBo, bd.h)
    assert rel(r["B"].cpu(), Bo) <= 1e-10
    fg = r["fg"].cpu().numpy()
    ok = np.isfinite(res["f"])
    assert rel(fg[0][ok], res["f"][ok]) <= 1e-9 and rel(fg[1][ok], res["g"][ok]) <= 1e-9
    conv = st == oracle.ST_CONVERGED
    assert np.all(res["rho"][conv] <= 1e-4 * (1 + 1e-6))
    # the search never ends worse than its start (lambda = 0)
    B0_, dB0_ = oracle.field(bd.B0, bd.x0, bd.y0, bd.h, w.xyz, np.zeros((3, N)))
    phi0 = oracle.residuals(B0_, dB0_, bd.h)["Phi"]
    assert np.all(res["Phi"] <= phi0 * (1 + 1e-12))


def test_fp32c_lm_with_fp64_acceptance():
    w, bd, ctx = lowlou_ctx("fp32c")
    N = w.n_points
    lam = torch.zeros(3, N, dtype=torch.float64, device="cuda:0")
    r = D.dbie_solve_lambda(ctx, lam, method="lm", max_trials=20, eps=1e-4, fp64_accept=True)
    torch.cuda.synchronize()
    lg = r["lam"].cpu().numpy()
    st = r["status"].cpu().numpy()
    Bo, dBo = oracle.field(bd.B0, bd.x0, bd.y0, bd.h, w.xyz, lg)
    res = oracle.residuals(Bo, dBo, bd.h)
    # the acceptance pass is FP64: its field, residuals and statuses are the oracle's
    assert rel(r["B"].cpu(), Bo) <= 1e-10
    conv = st == oracle.ST_CONVERGED
    assert np.array_equal(conv, res["rho"] <= 1e-4)
    B0_, dB0_ = oracle.field(bd.B0, bd.x0, bd.y0, bd.h, w.xyz, np.zeros((3, N)))
    phi0 = oracle.residuals(B0_, dB0_, bd.h)["Phi"]
    # LM accepts only decreases of Phi (in FP32C): allow the FP32C-vs-FP64 difference
    assert np.mean(res["Phi"] <= phi0 * (1 + 1e-4)) >= 0.99


@pytest.mark.parametrize("method", ["nm", "lm"])
def test_fp64_confirmation_of_converged_points_only(method):
    """With no B or fg requested, the FP64 acceptance re-evaluates only the points that converged in
    FP32C: the same lambda and trials as the full acceptance, CONVERGED exactly where the full pass
    has a point that converged in FP32C and passes in FP64, and every CONVERGED point passes the
    oracle's FP64 test."""
    w, bd, ctx = lowlou_ctx("fp32c")
    N = w.n_points
    z = lambda: torch.zeros(3, N, dtype=torch.float64, device="cuda:0")  # noqa: E731
    eps = 0.05
    full = D.dbie_solve_lambda(ctx, z(), method=method, max_trials=30, eps=eps, fp64_accept=True)
    part = D.dbie_solve_lambda(ctx, z(), method=method, max_trials=30, eps=eps, fp64_accept=True,
                               want_B=False, want_fg=False)
    raw = D.dbie_solve_lambda(ctx, z(), method=method, max_trials=30, eps=eps, fp64_accept=False,
                              want_B=False, want_fg=False)
    torch.cuda.synchronize()
    assert torch.equal(full["lam"], part["lam"]) and torch.equal(full["trials"], part["trials"])
    st_full, st_part, st_raw = (r["status"].cpu().numpy() for r in (full, part, raw))
    expect = (st_raw == oracle.ST_CONVERGED) & (st_full == oracle.ST_CONVERGED)
    assert np.array_equal(st_part == oracle.ST_CONVERGED, expect)
    lg = part["lam"].cpu().numpy()
    conv = np.nonzero(st_part == oracle.ST_CONVERGED)[0]
    assert conv.size > 0
    Bo, dBo = oracle.field(bd.B0, bd.x0, bd.y0, bd.h, w.xyz[:, conv], lg[:, conv])
    assert np.all(oracle.residuals(Bo, dBo, bd.h)["rho"] <= eps * (1 + 1e-6))


@pytest.mark.parametrize("method", ["nm", "lm"])
def test_solve_is_deterministic_and_batched_equals_single(method):
    rng = np.random.default_rng(21)
    bds, xyzs, seg = [], [], [0]
    for nx, ny, n in ((20, 16, 300), (12, 30, 257)):
        B0 = rng.normal(size=(3, ny, nx)).astype(np.float32).astype(np.float64)
        bds.append(dict(B0=T(B0), x0=0.0, y0=0.0, h=1.0))
        xyzs.append(np.stack([rng.uniform(0, nx, n), rng.uniform(0, ny, n), rng.uniform(0.5, 8, n)]))
        seg.append(seg[-1] + n)
    xyz = np.concatenate(xyzs, axis=1)
    lam0 = rng.uniform(0, 0.2, size=xyz.shape)
    outs = []
    for prec in ("fp64", "fp32c"):
        ctx = D.dbie_init(bds, T(xyz), seg=seg, precision=prec)
        a = D.dbie_solve_lambda(ctx, T(lam0), method=method, max_trials=12, fp64_accept=False)
        b = D.dbie_solve_lambda(ctx, T(lam0), method=method, max_trials=12, fp64_accept=False)
        for k in ("lam", "status", "trials", "B", "fg"):
            assert torch.equal(a[k], b[k]), (prec, k)
        for bi in range(2):
            c1 = D.dbie_init([bds[bi]], T(xyz[:, seg[bi]:seg[bi + 1]]), precision=prec)
            s1 = D.dbie_solve_lambda(c1, T(lam0[:, seg[bi]:seg[bi + 1]]), method=method, max_trials=12,
                                     fp64_accept=False)
            for k in ("lam", "status", "trials"):
                assert torch.equal(s1[k], a[k][..., seg[bi]:seg[bi + 1]]), (prec, bi, k)
        outs.append(a)


def test_solver_edge_cases():
    rng = np.random.default_rng(22)
    B0 = rng.normal(size=(3, 10, 10))
    xyz = np.stack([rng.uniform(0, 9, 6), rng.uniform(0, 9, 6), rng.uniform(1, 5, 6)])
    ctx = D.dbie_init([dict(B0=T(B0), x0=0.0, y0=0.0, h=1.0)], T(xyz), precision="fp64")
    lam0 = np.zeros((3, 6))
    lam0[0, 1] = np.nan           # non-finite start
    lam0[1, 2] = 10.0             # beyond the cap pi/h: every vertex of the simplex is infeasible
    r = D.dbie_solve_lambda(ctx, T(lam0), method="nm", max_trials=5)
    st = r["status"].cpu().numpy()
    tr = r["trials"].cpu().numpy()
    assert st[1] == D._lib.DBIE_ST_NONFINITE and tr[1] == 0
    assert st[2] == D._lib.DBIE_ST_NONFINITE and tr[2] == 5
    # budget of one trial: exactly one evaluation
    r1 = D.dbie_solve_lambda(ctx, T(np.zeros((3, 6))), method="lm", max_trials=1)
    assert torch.all(r1["trials"] == 1)
    # zero boundary field: |B| = 0 everywhere
    ctx0 = D.dbie_init([dict(B0=T(np.zeros((3, 10, 10))), x0=0.0, y0=0.0, h=1.0)], T(xyz), precision="fp64")
    for m in ("nm", "lm"):
        r0 = D.dbie_solve_lambda(ctx0, T(np.zeros((3, 6))), method=m, max_trials=6)
        assert torch.all(r0["status"] == D._lib.DBIE_ST_DEGENERATE), m
    with pytest.raises(D.DbieError, match="max_trials"):
        D.dbie_solve_lambda(ctx, T(np.zeros((3, 6))), method="nm", max_trials=0)
    for bad in (-1.0, math.nan):
        with pytest.raises(D.DbieError, match="lm_radius"):
            D.dbie_solve_lambda(ctx, T(np.zeros((3, 6))), method="lm", lm_radius=bad)
    for bad in (-1.0, math.nan, math.inf):
        with pytest.raises(D.DbieError, match="lm_damping"):
            D.dbie_solve_lambda(ctx, T(np.zeros((3, 6))), method="lm", lm_damping=bad)


@pytest.mark.parametrize("method,prec", [("nm", "fp64"), ("lm", "fp32c")])
def test_graph_replay_equals_eager_rounds(method, prec):
    """The rounds replayed from a captured HIP graph give bitwise the eager results, on every replay,
    with eager solves and synchronisations in between."""
    w, bd, ctx = lowlou_ctx(prec)
    N = w.n_points
    rng = np.random.default_rng(51)
    for rep in range(3):
        lam0 = T(rng.uniform(0.0, 0.5, size=(3, N)))
        eager = D.dbie_solve_lambda(ctx, lam0.clone(), method=method, max_trials=18, use_graph=False)
        torch.cuda.synchronize()
        graph = D.dbie_solve_lambda(ctx, lam0.clone(), method=method, max_trials=18, use_graph=True)
        torch.cuda.synchronize()
        for k in ("lam", "status", "trials", "B", "fg"):
            assert torch.equal(eager[k], graph[k]), (rep, k)


def test_lowlou_comparison_metrics_are_reported():
    """DBIE on the Low & Lou boundary against the exact field at the 512 interior points, with the
    comparison metrics of Schrijver et al. (2006): C_vec, C_cs, E'_n, E'_m, eps. Reported, not gated
    (boundary truncation, quadrature and lambda non-uniqueness): parity unpinned. Sanity only: the
    field points the right way on average and the searches improve on lambda = 0."""
    w = config1()
    ll = w.meta["ll"]
    exact = ll.field(*w.xyz)
    rows = {}
    for name, prec, meth, bud in (("lambda=0", "fp64", None, 0), ("FP64 Nelder-Mead", "fp64", "nm", 50),
                                  ("FP32C Levenberg-Marquardt", "fp32c", "lm", 20)):
        _, bd, ctx = lowlou_ctx(prec)
        lam = torch.zeros(3, w.n_points, dtype=torch.float64, device="cuda:0")
        if meth is None:
            B = D.dbie_eval_field(ctx, lam)["B"]
        else:
            B = D.dbie_solve_lambda(ctx, lam, method=meth, max_trials=bud)["B"]
        torch.cuda.synchronize()
        rows[name] = oracle.schrijver_metrics(exact, B.cpu().numpy())
    for name, m in rows.items():
        print(name, {k: round(v, 3) for k, v in m.items()}, flush=True)
    for m in rows.values():
        assert m["C_vec"] > 0.5 and m["C_cs"] > 0.0


def test_residual_statistics_on_the_device():
    """dbie_residual_stats against NumPy on the same (f, g): means over finite points, counts; a NaN
    lambda point is left out; repeated calls agree bitwise."""
    w, bd, ctx = lowlou_ctx("fp32c")
    n = w.n_points
    lam = torch.zeros(3, n, dtype=torch.float64, device="cuda:0")
    r = D.dbie_solve_lambda(ctx, lam, method="lm", max_trials=10, eps=1e-3)
    fg = r["fg"]
    st = D.dbie_residual_stats(ctx, fg, eps=1e-3)
    a = fg.cpu().numpy()
    ok = np.isfinite(a[0]) & np.isfinite(a[1])
    assert st["finite"] == int(ok.sum())
    assert st["converged"] == int(np.sum(np.maximum(a[0], a[1])[ok] <= 1e-3))
    assert abs(st["mean_f"] - a[0][ok].mean()) <= 1e-13 * max(1.0, abs(a[0][ok].mean()))
    assert abs(st["mean_g"] - a[1][ok].mean()) <= 1e-13 * max(1.0, abs(a[1][ok].mean()))
    assert st == D.dbie_residual_stats(ctx, fg, eps=1e-3)
    bad = T(np.where(np.arange(n) == 5, np.nan, 0.2) * np.ones((3, 1)))
    e = D.dbie_eval_field(ctx, bad)
    s2 = D.dbie_residual_stats(ctx, e["fg"], eps=1e-4)
    assert s2["finite"] == n - 1


def test_solve_trace_reports_rounds_and_the_end():
    """Solve tracing: round times increase, the per-round convergence counts add up to the points
    that converged in the search, the end of the call comes after the last round, and a traced
    solve returns what an untraced one does."""
    w, bd, ctx = lowlou_ctx("fp32c")
    N = w.n_points
    z = lambda: torch.zeros(3, N, dtype=torch.float64, device="cuda:0")  # noqa: E731
    ref = D.dbie_solve_lambda(ctx, z(), method="lm", max_trials=12, eps=0.05, fp64_accept=False)
    D.dbie_solve_trace(ctx, True)
    r = D.dbie_solve_lambda(ctx, z(), method="lm", max_trials=12, eps=0.05, fp64_accept=False)
    t, cv, t_end = D.dbie_solve_trace_read(ctx, with_end=True)
    D.dbie_solve_trace(ctx, False)
    for k in ("lam", "status", "trials"):
        assert torch.equal(r[k], ref[k]), k
    st = r["status"].cpu().numpy()
    assert 1 <= len(t) <= 12 and np.all(np.diff(t) >= 0) and t_end >= t[-1] > 0
    assert int(cv.sum()) == int(np.sum(st == oracle.ST_CONVERGED))


def test_trace_is_dropped_when_the_workspace_changes():
    """The per-round counts of a traced solve live in the solver's block: handing the context a
    workspace frees that block, so the trace is dropped (0 rounds) rather than read from freed
    memory; a negative round count is refused; a traced solve in the workspace reads back as before."""
    w, bd, ctx = lowlou_ctx("fp32c")
    N = w.n_points
    z = lambda: torch.zeros(3, N, dtype=torch.float64, device="cuda:0")  # noqa: E731
    D.dbie_solve_trace(ctx, True)
    D.dbie_solve_lambda(ctx, z(), method="lm", max_trials=8, eps=0.05, fp64_accept=False)
    t0, cv0 = D.dbie_solve_trace_read(ctx)
    assert len(t0) >= 1
    from paper_1306_1122_amd import _lib
    n = ctypes.c_int32()
    assert _lib.load().dbie_solve_trace_read(ctx.handle, None, None, -1, ctypes.byref(n), None) != 0
    ws = torch.empty(D.dbie_workspace_bytes(ctx), dtype=torch.uint8, device="cuda:0")
    D.dbie_set_workspace(ctx, ws)
    t1, cv1 = D.dbie_solve_trace_read(ctx)
    assert len(t1) == 0 and len(cv1) == 0
    D.dbie_solve_lambda(ctx, z(), method="lm", max_trials=8, eps=0.05, fp64_accept=False)
    t2, cv2 = D.dbie_solve_trace_read(ctx)
    D.dbie_solve_trace(ctx, False)
    assert len(t2) == len(t0) and np.array_equal(cv2, cv0)
