"""GPU parity of the 9-node quadratic element discretisation (Eq. 15) against the oracle's
`field_quad9`, through the C ABI: evaluation (FP64, and FP32C with the elements near a point summed
in FP64), several magnetograms, trials, the adjoint (by the dot-product identity against the oracle's
forward map) and the per-point lambda search."""
import numpy as np
import pytest
import torch

import oracle
from _parity import well_conditioned_fg
from _ties import Recording, has_near_tie
import paper_1306_1122_amd as D

pytestmark = pytest.mark.gpu

TOLS = {"fp64": 1e-10, "fp32c": 1e-5}


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


class Bd:
    def __init__(self, B0, x0, y0, h):
        self.B0, self.x0, self.y0, self.h = B0, x0, y0, h


def magnetogram(rng, nx, ny, x0=0.0, y0=0.0, h=1.0):
    return Bd(rng.normal(size=(3, ny, nx)), x0, y0, h)


def points_over(rng, bd, n, zmin=0.25, zmax=30.0):
    ny, nx = bd.B0.shape[1:]
    return np.stack([rng.uniform(bd.x0 - 2 * bd.h, bd.x0 + (nx + 1) * bd.h, n),
                     rng.uniform(bd.y0 - 2 * bd.h, bd.y0 + (ny + 1) * bd.h, n),
                     bd.h * np.exp(rng.uniform(np.log(zmin), np.log(zmax), n))])


def ctx_for(bds, xyz, G, seg=None, precision="fp64"):
    bl = [dict(B0=T(b.B0), x0=b.x0, y0=b.y0, h=b.h) for b in bds]
    return D.dbie_init(bl, T(xyz), seg=seg, precision=precision, quad_points=G)


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
@pytest.mark.parametrize("G", [2, 3, 4])
@pytest.mark.parametrize("n", [1, 255, 257, 700])
def test_eval_matches_oracle(precision, G, n):
    """Ragged point counts, points above, beside and outside a 33 x 25 magnetogram, z from h/4
    (FP32C: many points with near elements)."""
    TOL = TOLS[precision]
    rng = np.random.default_rng(900 + 10 * G + n)
    bd = magnetogram(rng, 33, 25, x0=-3.0, y0=1.5, h=0.5)
    xyz = points_over(rng, bd, n)
    lam = rng.uniform(-1.5, 1.5, size=(3, n))
    ctx = ctx_for([bd], xyz, G, precision=precision)
    out = D.dbie_eval_field(ctx, T(lam), want_tan=True)
    torch.cuda.synchronize()
    B, dB, tan = oracle.field_quad9(bd.B0, bd.x0, bd.y0, bd.h, xyz, lam, G=G, tangents=True)
    errs = dict(B=rel(out["B"].cpu(), B), dB=rel(out["dB"].cpu(), dB), tan=rel(out["tan"].cpu(), tan))
    print("quad9", precision, G, n, {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= TOL, (k, v)
    res = oracle.residuals(B, dB, bd.h)
    fg = out["fg"].cpu().numpy()
    assert rel(fg[0], res["f"]) <= 10 * TOL and rel(fg[1], res["g"]) <= 10 * TOL


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_smallest_magnetogram_and_several_boundaries(precision):
    rng = np.random.default_rng(920)
    bds = [magnetogram(rng, 3, 3, 0.0, 0.0, 1.0), magnetogram(rng, 41, 17, -2.0, 4.0, 0.25),
           magnetogram(rng, 9, 31, 5.0, -1.0, 2.0)]
    npts = [40, 333, 0]
    xyz = np.concatenate([points_over(rng, b, n) for b, n in zip(bds, npts)], axis=1)
    lam = rng.uniform(-1, 1, size=(3, xyz.shape[1]))
    seg = np.concatenate([[0], np.cumsum(npts)])
    ctx = ctx_for(bds, xyz, 4, seg=seg, precision=precision)
    out = D.dbie_eval_field(ctx, T(lam), want_tan=True)
    torch.cuda.synchronize()
    for b, bd in enumerate(bds):
        s, e = seg[b], seg[b + 1]
        if e == s:
            continue
        B, dB, tan = oracle.field_quad9(bd.B0, bd.x0, bd.y0, bd.h, xyz[:, s:e], lam[:, s:e], G=4, tangents=True)
        for name, ref in (("B", B), ("dB", dB), ("tan", tan)):
            assert rel(out[name][:, s:e].cpu(), ref) <= TOLS[precision], (b, name)


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_trials_and_scalar_lambda_equal_single_calls(precision):
    rng = np.random.default_rng(921)
    bd = magnetogram(rng, 21, 19)
    xyz = points_over(rng, bd, 300)
    ctx = ctx_for([bd], xyz, 3, precision=precision)
    lams = rng.uniform(-1, 1, size=(2, 3, 300))
    multi = D.dbie_eval_field(ctx, T(lams), want_tan=True)
    for k in range(2):
        one = D.dbie_eval_field(ctx, T(lams[k]), want_tan=True)
        for name in ("B", "dB", "tan", "fg"):
            assert torch.equal(multi[name][k], one[name]), name
    lam1 = rng.uniform(-1, 1, size=(1, 300))
    sc = D.dbie_eval_field_scalar(ctx, T(lam1), want_tan=True)
    gen = D.dbie_eval_field(ctx, T(np.repeat(lam1[:, None, :], 3, axis=1)), want_tan=True)
    for name in ("B", "dB", "tan", "fg"):
        if precision == "fp64":
            assert torch.equal(sc[name], gen[name]), name
        else:   # the scalar form shares one sin/cos per pair: a different FP32 rounding order
            assert rel(sc[name].cpu(), gen[name].cpu()) <= 1e-6, name


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_adjoint_dot_product_against_the_oracle_forward_map(precision):
    """B and grad B are linear in B0: <gB, B(dB0)> + <gdB, dB(dB0)> = <gB0, dB0> with the forward map
    computed by the oracle and gB0 by the library's transpose (Gauss-point transpose, then the
    interpolation transpose to the nodes)."""
    rng = np.random.default_rng(922)
    bd = magnetogram(rng, 19, 15, 1.0, -2.0, 0.5)
    n = 400
    xyz = points_over(rng, bd, n)
    lam = rng.uniform(-1, 1, size=(3, n))
    gB, gdB = rng.normal(size=(3, n)), rng.normal(size=(9, n))
    ctx = ctx_for([bd], xyz, 4, precision=precision)
    out = D.dbie_grad(ctx, T(lam), gB=T(gB), gdB=T(gdB), want_gB0=True)
    torch.cuda.synchronize()
    gB0 = D.split_gB0(ctx, out["gB0"])[0].cpu().numpy()
    for trial in range(2):
        dB0 = rng.normal(size=bd.B0.shape)
        Bf, dBf = oracle.field_quad9(dB0, bd.x0, bd.y0, bd.h, xyz, lam, G=4)
        lhs = np.sum(gB * Bf) + np.sum(gdB * dBf)
        rhs = np.sum(gB0 * dB0)
        tol = TOLS[precision]
        assert abs(lhs - rhs) <= tol * np.sqrt(np.sum(gB0 ** 2) * np.sum(dB0 ** 2)), (trial, lhs, rhs)
    # single nodes against the oracle's column of the (linear) forward map: corners, edges, a node
    # inside one element, one shared by two elements and one shared by four
    ny, nx = bd.B0.shape[1:]
    scale = np.abs(gB0).max()
    for p, j, i in ((0, 0, 0), (1, 0, nx - 1), (2, ny - 1, 0), (0, ny - 1, nx - 1), (1, 0, 7), (2, 5, 0),
                    (0, 5, 7), (1, 4, 7), (2, 6, 8)):
        e = np.zeros_like(bd.B0)
        e[p, j, i] = 1.0
        Bf, dBf = oracle.field_quad9(e, bd.x0, bd.y0, bd.h, xyz, lam, G=4)
        ref = np.sum(gB * Bf) + np.sum(gdB * dBf)
        assert abs(gB0[p, j, i] - ref) <= TOLS[precision] * scale, (p, j, i, gB0[p, j, i], ref)


class QuadProblem(oracle.PointProblem):
    """The oracle's per-point problem with the field of Eq. (15) in place of the nodal sum."""

    def __init__(self, *a, G=4, **k):
        super().__init__(*a, **k)
        self.G = G

    def eval(self, lam3, tangents=False):
        lam = np.asarray(lam3, np.float64).reshape(3, 1)
        out = oracle.field_quad9(self.B0, self.x0, self.y0, self.h, self.p, lam, G=self.G, tangents=tangents)
        return out, oracle.residuals(out[0], out[1], self.h, self.c)


def test_fp32c_solve_with_fp64_acceptance():
    """FP32C Levenberg-Marquardt on the element field, accepted by an FP64 re-evaluation: every point
    marked converged meets the tolerance when the oracle re-evaluates it at the returned lambda."""
    rng = np.random.default_rng(924)
    bd = magnetogram(rng, 25, 21)
    n = 400
    xyz = np.stack([rng.uniform(2, 22, n), rng.uniform(2, 18, n), rng.uniform(0.3, 8.0, n)])
    ctx = ctx_for([bd], xyz, 4, precision="fp32c")
    lam0 = torch.zeros(3, n, dtype=torch.float64, device="cuda:0")
    out = D.dbie_solve_lambda(ctx, lam0, method="lm", max_trials=20, eps=1e-3, fp64_accept=True)
    torch.cuda.synchronize()
    conv = np.nonzero(out["status"].cpu().numpy() == 0)[0]
    print("quad9 fp32c LM converged", conv.size, "of", n, flush=True)
    lam = out["lam"].cpu().numpy()
    for i in conv[:40]:
        B, dB = oracle.field_quad9(bd.B0, bd.x0, bd.y0, bd.h, xyz[:, i:i + 1], lam[:, i:i + 1], G=4)
        res = oracle.residuals(B, dB, bd.h)
        assert max(res["f"][0], res["g"][0]) <= 1e-3 * (1 + 1e-9), i


def test_lm_search_follows_the_oracle():
    """Levenberg-Marquardt on the element field (the library's default trust radius, the simplex
    edge): every trajectory (trials, status, lambda*) equals the oracle's LM on the same field, but
    for points whose oracle trajectory holds a near-tie (tests/_ties.py)."""
    rng = np.random.default_rng(923)
    bd = magnetogram(rng, 17, 17)
    n = 48
    xyz = np.stack([rng.uniform(2, 14, n), rng.uniform(2, 14, n), rng.uniform(1.0, 8.0, n)])
    lam0 = rng.uniform(0.01, 0.3, size=(3, n))
    ctx = ctx_for([bd], xyz, 4)
    out = D.dbie_solve_lambda(ctx, T(lam0), method="lm", max_trials=12, eps=1e-4, fp64_accept=False)
    torch.cuda.synchronize()
    lam_g = out["lam"].cpu().numpy()
    st_g = out["status"].cpu().numpy()
    tr_g = out["trials"].cpu().numpy()
    cap = np.pi / bd.h
    radius0 = oracle.default_nm_step(bd.B0.shape[2], bd.B0.shape[1], bd.h)
    same, ties, bad = 0, 0, []
    for i in range(n):
        prob = Recording(QuadProblem(bd.B0, bd.x0, bd.y0, bd.h, xyz[:, i], G=4))
        lam, st, tr, _ = oracle.solve_point_lm(prob, lam0[:, i], 12, 1e-4, cap, radius0=radius0)
        if st == st_g[i] and tr == tr_g[i] and np.allclose(lam, lam_g[:, i], rtol=1e-8, atol=1e-12):
            same += 1
        elif has_near_tie(prob.vals, 1e-4):
            ties += 1
        else:
            bad.append(i)
    print("quad9 LM identical trajectories", same, "of", n, "near-ties", ties, flush=True)
    assert not bad, bad


@pytest.mark.parametrize("G", [2, 4])
def test_full_size_elements_sampled(G):
    """The benchmark's element run: the 128x128 bipole magnetogram cropped to 127x127, all 2^20
    points of the 128x128x64 grid, FP32C in its default launch shape; z-stratified points (48 for
    G = 2, 24 for G = 4) against the oracle's element sum, and their (f, g) against the oracle's
    residuals."""
    from workloads import config2, z_stratified_subsample
    w = config2()
    B0 = np.ascontiguousarray(w.boundaries[0].B0[:, :127, :127])
    ctx = D.dbie_init([dict(B0=T(B0), x0=0.0, y0=0.0, h=1.0)], T(w.xyz), precision="fp32c", quad_points=G)
    out = D.dbie_eval_field(ctx, T(w.lam), want_tan=True)
    torch.cuda.synchronize()
    idx = z_stratified_subsample(w.xyz, 48 if G == 2 else 24, seed=31 + G)
    B, dB, tan = oracle.field_quad9(B0, 0.0, 0.0, 1.0, w.xyz[:, idx], w.lam[:, idx], G=G, tangents=True)
    errs = dict(B=rel(out["B"][:, idx].cpu(), B), dB=rel(out["dB"][:, idx].cpu(), dB),
                tan=rel(out["tan"][:, idx].cpu(), tan))
    print("quad9 full size", G, {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= TOLS["fp32c"], (k, v)
    res = oracle.residuals(B, dB, 1.0)
    fg = out["fg"][:, idx].cpu().numpy()
    # f and g at the path's bar where they are well conditioned (tests/_parity.py)
    okf, okg = well_conditioned_fg(B, dB, res)
    ef, eg = rel(fg[0][okf], res["f"][okf]), rel(fg[1][okg], res["g"][okg])
    print("quad9 full size", G, "f %.1e g %.1e over %d / %d points" % (ef, eg, okf.sum(), okg.sum()), flush=True)
    assert ef <= TOLS["fp32c"] and eg <= TOLS["fp32c"]
