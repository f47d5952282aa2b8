"""GPU parity of dbie_eval_field (through the C ABI) against the FP64 CPU oracle.

Bars: relative L2 <= 1e-10 for the FP64 path and <= 1e-5 for the FP32C path, separately for B,
grad B, the mu-tangents and (f, g) where stated.
"""
import numpy as np
import pytest
import torch

import oracle
from _parity import check_sampled, max_phase
import paper_1306_1122_amd as D
from workloads import config1, config2, z_stratified_subsample

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32c": 1e-5}


def dev():
    return torch.device("cuda:0")


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev())


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def ctx_for(boundaries, xyz, precision, seg=None, **kw):
    bl = [dict(B0=T(b.B0), x0=b.x0, y0=b.y0, h=b.h) for b in boundaries]
    return D.dbie_init(bl, T(xyz), seg=seg, precision=precision, **kw)


def check_against_oracle(ctx, bd, xyz, lam, tol, tangents=True, fg=True, label=""):
    out = D.dbie_eval_field(ctx, T(lam), want_tan=tangents)
    torch.cuda.synchronize()
    prec = "fp64" if tol <= 1e-10 else "fp32c"
    got = {k: out[k].cpu().numpy() for k in (("B", "dB", "tan") if tangents else ("B", "dB"))}
    return check_sampled(got, bd, xyz, lam, prec, label, fg=out["fg"].cpu().numpy() if fg else None, tol=tol)


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_lowlou_full_workload(precision):
    w = config1()
    bd = w.boundaries[0]
    ctx = ctx_for(w.boundaries, w.xyz, precision)
    check_against_oracle(ctx, bd, w.xyz, w.lam, TOL[precision], label=f"lowlou {precision}")


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_bipoles_full_size_sampled(precision):
    """The 128x128 magnetogram with all 128x128x64 points on the GPU, as the benchmark launches it;
    the oracle checks a z-stratified sample of the outputs."""
    w = config2()
    bd = w.boundaries[0]
    ctx = ctx_for(w.boundaries, w.xyz, precision)
    out = D.dbie_eval_field(ctx, T(w.lam), want_tan=True)
    torch.cuda.synchronize()
    idx = z_stratified_subsample(w.xyz, 512, seed=5)
    got = {k: out[k][:, idx].cpu().numpy() for k in ("B", "dB", "tan")}
    check_sampled(got, bd, w.xyz[:, idx], w.lam[:, idx], precision, f"bipoles {precision}",
                  fg=out["fg"][:, idx].cpu().numpy())
    assert torch.isfinite(out["B"]).all() and torch.isfinite(out["dB"]).all()


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
@pytest.mark.parametrize("n", [1, 7, 255, 256, 257, 1030])
def test_ragged_point_counts_and_off_grid_points(precision, n):
    rng = np.random.default_rng(100 + n)
    nx, ny, h, x0, y0 = 37, 29, 0.25, -2.0, 3.0
    B0 = rng.normal(size=(3, ny, nx)).astype(np.float32).astype(np.float64)
    # points inside, beside and far outside the magnetogram; z from 0.3 h to 40 h
    xyz = np.stack([rng.uniform(x0 - 3, x0 + nx * h + 3, n), rng.uniform(y0 - 3, y0 + ny * h + 3, n),
                    h * np.exp(rng.uniform(np.log(0.3), np.log(40.0), n))])
    lam = rng.uniform(-2.0, 2.0, size=(3, n))

    class Bd:
        pass

    bd = Bd()
    bd.B0, bd.x0, bd.y0, bd.h = B0, x0, y0, h
    ctx = ctx_for([bd], xyz, precision)
    check_against_oracle(ctx, bd, xyz, lam, TOL[precision], label=f"ragged n={n} {precision}")


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_points_on_pixel_centres_in_the_lowest_layers(precision):
    """z = 0.5h .. 2h directly above and between pixel centres: the near-field pairs (r < 2h) are
    summed in FP64 on the FP32C path."""
    rng = np.random.default_rng(3)
    nx, ny = 24, 20
    B0 = rng.normal(size=(3, ny, nx)).astype(np.float32).astype(np.float64)
    gx, gy = np.meshgrid(np.arange(2, 22, 0.5), np.arange(2, 18, 0.5))
    pts = []
    for z in (0.5, 1.0, 1.5, 1.999, 2.0):
        pts.append(np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, z)]))
    xyz = np.concatenate(pts, axis=1)
    lam = rng.uniform(-0.5, 0.5, size=xyz.shape)

    class Bd:
        pass

    bd = Bd()
    bd.B0, bd.x0, bd.y0, bd.h = B0, 0.0, 0.0, 1.0
    ctx = ctx_for([bd], xyz, precision)
    check_against_oracle(ctx, bd, xyz, lam, TOL[precision], label=f"near-field {precision}")


def test_nearfield_radius_zero_is_plain_fp32():
    """With the near-field pass switched off every pair is FP32; the error then stays small only
    away from the boundary."""
    rng = np.random.default_rng(4)
    B0 = rng.normal(size=(3, 16, 16)).astype(np.float32).astype(np.float64)
    xyz = np.stack([rng.uniform(0, 15, 200), rng.uniform(0, 15, 200), rng.uniform(3.0, 10.0, 200)])
    lam = rng.uniform(-0.3, 0.3, size=(3, 200))

    class Bd:
        pass

    bd = Bd()
    bd.B0, bd.x0, bd.y0, bd.h = B0, 0.0, 0.0, 1.0
    ctx = ctx_for([bd], xyz, "fp32c", nearfield_radius_h=0.0)
    check_against_oracle(ctx, bd, xyz, lam, 1e-5, fg=False, label="radius 0")


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_several_boundaries_of_uneven_size(precision):
    rng = np.random.default_rng(5)
    # including the degenerate magnetograms: one pixel, one column, one row
    shapes = [(17, 23, 1.0, 0.0, 0.0), (64, 40, 0.5, -3.0, 2.0), (5, 9, 2.0, 1.0, -1.0), (1, 1, 1.0, 4.0, 4.0),
              (1, 13, 0.5, 0.0, 0.0), (11, 1, 1.0, -2.0, 0.0)]
    npts = [300, 1, 700, 5, 40, 33]

    class Bd:
        pass

    bds, xyzs, lams = [], [], []
    for (nx, ny, h, x0, y0), n in zip(shapes, npts):
        bd = Bd()
        bd.B0 = rng.normal(size=(3, ny, nx)).astype(np.float32).astype(np.float64)
        bd.x0, bd.y0, bd.h = x0, y0, h
        bds.append(bd)
        xyzs.append(np.stack([rng.uniform(x0, x0 + nx * h, n), rng.uniform(y0, y0 + ny * h, n),
                              rng.uniform(0.5 * h, 20 * h, n)]))
        lams.append(rng.uniform(-1, 1, size=(3, n)))
    xyz = np.concatenate(xyzs, axis=1)
    lam = np.concatenate(lams, axis=1)
    seg = np.concatenate([[0], np.cumsum(npts)])
    ctx = ctx_for(bds, xyz, precision, seg=seg)
    out = D.dbie_eval_field(ctx, T(lam), want_tan=True)
    torch.cuda.synchronize()
    for b, bd in enumerate(bds):
        s, e = seg[b], seg[b + 1]
        B, dB, tan = oracle.field(bd.B0, bd.x0, bd.y0, bd.h, xyz[:, s:e], lam[:, s:e], tangents=True)
        for name, ref in (("B", B), ("dB", dB), ("tan", tan)):
            err = rel(out[name][:, s:e].cpu(), ref)
            assert err <= TOL[precision], (b, name, err)


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_multi_trial_equals_single_calls_and_is_deterministic(precision):
    w = config1()
    ctx = ctx_for(w.boundaries, w.xyz, precision)
    rng = np.random.default_rng(6)
    lams = rng.uniform(-2, 2, size=(3, 3, w.n_points))
    multi = D.dbie_eval_field(ctx, T(lams), want_tan=True)
    for k in range(3):
        single = D.dbie_eval_field(ctx, T(lams[k]), want_tan=True)
        again = D.dbie_eval_field(ctx, T(lams[k]), want_tan=True)
        for name in ("B", "dB", "tan", "fg"):
            assert torch.equal(multi[name][k], single[name]), name
            assert torch.equal(again[name], single[name]), name


def test_zero_points_and_invalid_points():
    B0 = T(np.ones((3, 4, 4)))
    ctx = D.dbie_init([dict(B0=B0, x0=0.0, y0=0.0, h=1.0)], torch.zeros(3, 0, dtype=torch.float64,
                                                                         device=dev()))
    out = D.dbie_eval_field(ctx, torch.zeros(3, 0, dtype=torch.float64, device=dev()))
    assert out["B"].shape == (3, 0)
    bad = T(np.array([[0.0, 1.0], [0.0, 1.0], [1.0, 0.0]]))
    with pytest.raises(D.DbieError, match="z <= 0"):
        D.dbie_init([dict(B0=B0, x0=0.0, y0=0.0, h=1.0)], bad)
    nanp = T(np.array([[np.nan], [0.0], [1.0]]))
    with pytest.raises(D.DbieError, match="non-finite"):
        D.dbie_init([dict(B0=B0, x0=0.0, y0=0.0, h=1.0)], nanp)
    # the binding rejects what the library could not check: a short offset list, and a caller's
    # output buffer too small for the trials
    pts = T(np.array([[0.5, 1.5], [0.5, 1.5], [1.0, 2.0]]))
    with pytest.raises(ValueError, match="seg must hold"):
        D.dbie_init([dict(B0=B0), dict(B0=B0)], pts, seg=[0, 2])
    ctx2 = D.dbie_init([dict(B0=B0, x0=0.0, y0=0.0, h=1.0)], pts)
    lam2 = torch.zeros(2, 3, 2, dtype=torch.float64, device=dev())
    with pytest.raises(ValueError, match="shape"):
        D.dbie_eval_field(ctx2, lam2, B=torch.empty(3, 2, dtype=torch.float64, device=dev()))
    with pytest.raises(ValueError, match="shape"):
        D.dbie_grad(ctx2, lam2[0], gB=torch.ones(3, 2, dtype=torch.float64, device=dev()),
                    gB0=torch.empty(3, dtype=torch.float64, device=dev()))


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_scalar_lambda_fast_path(precision):
    """One lambda shared by the three components: the fast path against the oracle and against the
    general path with the lambda repeated."""
    w = config2(nz=8)
    bd = w.boundaries[0]
    ctx = ctx_for(w.boundaries, w.xyz, precision)
    rng = np.random.default_rng(61)
    lam1 = rng.uniform(-0.1, 0.1, size=(2, w.n_points))
    out = D.dbie_eval_field_scalar(ctx, T(lam1), want_tan=True)
    gen = D.dbie_eval_field(ctx, T(np.repeat(lam1[:, None, :], 3, axis=1)), want_tan=True)
    torch.cuda.synchronize()
    for k in ("B", "dB", "tan", "fg"):
        if precision == "fp64":
            assert torch.equal(out[k], gen[k]), k
        else:
            assert rel(out[k].cpu(), gen[k].cpu()) <= 1e-6, k
    idx = z_stratified_subsample(w.xyz, 128, seed=9)
    for t in range(2):
        lam3 = np.repeat(lam1[t][None, idx], 3, axis=0)
        B, dB, tan = oracle.field(bd.B0, bd.x0, bd.y0, bd.h, w.xyz[:, idx], lam3, tangents=True)
        for name, ref in (("B", B), ("dB", dB), ("tan", tan)):
            assert rel(out[name][t][:, idx].cpu(), ref) <= TOL[precision], (t, name)


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_large_lambda_needs_range_reduction_and_nan_lambda_stays_local(precision):
    """A 600 x 40 magnetogram with |lambda| h up to 2.9 (near the cap pi/h): lambda r / 2 pi reaches
    ~277 revolutions, beyond the hardware sin/cos range, so the FP32C kernel takes its range-reduced
    form (where the FP32 rounding of r, ~ulp(600) = 6e-5 pixel, is the phase error that remains).
    A NaN lambda at one point gives NaN there only (its wavefront neighbours stay exact)."""
    rng = np.random.default_rng(8)
    nx, ny, n = 600, 40, 130
    B0 = rng.normal(size=(3, ny, nx)).astype(np.float32).astype(np.float64)
    xyz = np.stack([rng.uniform(0, nx, n), rng.uniform(0, ny, n), rng.uniform(0.5, 20, n)])
    lam = rng.uniform(2.5, 2.9, size=(3, n)) * rng.choice([-1.0, 1.0], size=(3, n))

    class Bd:
        pass

    bd = Bd()
    bd.B0, bd.x0, bd.y0, bd.h = B0, 0.0, 0.0, 1.0
    ctx = ctx_for([bd], xyz, precision)
    check_against_oracle(ctx, bd, xyz, lam, TOL[precision], fg=False, label=f"large lambda {precision}")
    check_against_oracle(ctx, bd, xyz, lam, TOL[precision], tangents=False, fg=False,
                         label=f"large lambda, no tangents {precision}")
    bad = lam.copy()
    bad[1, 17] = np.nan
    out = D.dbie_eval_field(ctx, T(bad), want_tan=True)
    ref = D.dbie_eval_field(ctx, T(lam), want_tan=True)
    torch.cuda.synchronize()
    keep = np.ones(n, bool)
    keep[17] = False
    assert torch.isnan(out["B"][1, 17])
    for k in ("B", "dB", "tan"):
        a, b = out[k].cpu().numpy()[:, keep], ref[k].cpu().numpy()[:, keep]
        assert rel(a, b) <= (0.0 if precision == "fp64" else 1e-6), k
    # the single-lambda form on the same points
    sc = D.dbie_eval_field_scalar(ctx, T(lam[:1]), want_tan=True)
    Bs, dBs, tans = oracle.field(B0, 0.0, 0.0, 1.0, xyz, np.repeat(lam[:1], 3, axis=0), tangents=True)
    for k, r in (("B", Bs), ("dB", dBs), ("tan", tans)):
        assert rel(sc[k][0].cpu(), r) <= TOL[precision], k


@pytest.mark.parametrize("G", [0, 2])
def test_fp32c_phase_bound_recomputes_those_points_in_fp64(G):
    """The FP32C accuracy envelope: a point whose largest phase max_p |lambda_p| r_max exceeds 2 pi 128
    radians (with the mu-tangents) or 2 pi 512 (without) has its sums recomputed in FP64 after the
    FP32 pass, near-field pairs (elements, with G = 2) counted once. On a 601 x 41 magnetogram half of
    the points sit near the cap (phases of ~850-1900 radians) and half at |lambda| < 0.4 (< 250
    radians): with tangents the first half equals the FP64 context's result to FP64 regrouping and the
    second half keeps its FP32 rounding; without tangents every point keeps the FP32 pass
    (range-reduced beyond 256 revolutions), within the 1e-5 bar of the oracle."""
    rng = np.random.default_rng(81)
    nx, ny, n = 601, 41, 260
    B0 = rng.normal(size=(3, ny, nx)).astype(np.float32).astype(np.float64)
    xyz = np.stack([rng.uniform(0, nx, n), rng.uniform(0, ny, n), rng.uniform(0.4, 20, n)])
    big = np.arange(n) % 2 == 0
    mag = np.where(big, rng.uniform(2.8, 3.1, size=n), rng.uniform(0.0, 0.4, size=n))
    f = rng.uniform(0.8, 1.0, size=(3, n))
    f[0] = 1.0   # max_p |lambda_p| = mag; r_max >= 300 pixels on this strip, so 2.8 r_max > 2 pi 128
    lam = mag[None, :] * f * rng.choice([-1.0, 1.0], size=(3, n))

    class Bd:
        pass

    bd = Bd()
    bd.B0, bd.x0, bd.y0, bd.h = B0, 0.0, 0.0, 1.0
    tmax = max_phase(bd, xyz, lam)
    hi_tan, hi_field = tmax > 2 * np.pi * 128, tmax > 2 * np.pi * 512
    assert np.array_equal(hi_tan, big) and not hi_field.any()
    c32 = ctx_for([bd], xyz, "fp32c", quad_points=G)
    c64 = ctx_for([bd], xyz, "fp64", quad_points=G)
    a = D.dbie_eval_field(c32, T(lam), want_tan=True)
    b = D.dbie_eval_field(c64, T(lam), want_tan=True)
    p = D.dbie_eval_field(c32, T(lam), want_tan=False)
    torch.cuda.synchronize()
    for k in ("B", "dB", "tan"):
        x, y = a[k].cpu().numpy(), b[k].cpu().numpy()
        e_hi, e_lo = rel(x[:, big], y[:, big]), rel(x[:, ~big], y[:, ~big])
        print(f"phase bound G={G}, with tangents", k, "beyond %.2e, below %.2e" % (e_hi, e_lo), flush=True)
        assert e_hi <= 1e-12 and 1e-10 < e_lo <= 1e-5, k
    for k in ("B", "dB"):
        x, y = p[k].cpu().numpy(), b[k].cpu().numpy()
        e = rel(x, y)
        print(f"phase bound G={G}, without tangents", k, "%.2e" % e, flush=True)
        assert 1e-10 < e <= 1e-5, k
    if G == 0:
        check_against_oracle(c32, bd, xyz, lam, TOL["fp32c"], label="phase bound fp32c")
    else:
        # the element sum of the oracle at a sample (it is slow at this size)
        idx = np.arange(0, n, 13)
        Bq, dBq, tq = oracle.field_quad9(B0, 0.0, 0.0, 1.0, xyz[:, idx], lam[:, idx], G=G, tangents=True)
        for k, r in (("B", Bq), ("dB", dBq), ("tan", tq)):
            e = rel(a[k][:, idx].cpu(), r)
            print(f"phase bound G={G} against the oracle", k, "%.2e" % e, flush=True)
            assert e <= TOL["fp32c"], k


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fp32c_just_below_the_phase_bound_stays_within_the_bar(seed):
    """The bounds that decide the FP64 recompute, checked where the FP32 pass is kept: points whose
    largest phase lies at 0.8-1.0 of the bound (2 pi 128 rad with tangents, 2 pi 512 without) on a
    long magnetogram (701 to 1001 pixels) stay within the FP32C bar of the oracle (relative L2)."""
    rng = np.random.default_rng(500 + seed)
    nx, ny, n = int(rng.integers(701, 1002)), int(rng.integers(15, 45)), 96
    B0 = rng.normal(size=(3, ny, nx)).astype(np.float32).astype(np.float64)
    xyz = np.stack([rng.uniform(-5, nx + 5, n), rng.uniform(-3, ny + 3, n), rng.uniform(0.4, 30, n)])

    class Bd:
        pass

    bd = Bd()
    bd.B0, bd.x0, bd.y0, bd.h = B0, 0.0, 0.0, 1.0
    unit = max_phase(bd, xyz, np.ones((3, n)))   # r_max of each point
    for tan, bound in ((True, 2 * np.pi * 128), (False, 2 * np.pi * 512)):
        t = bound * rng.uniform(0.8, 1.0, size=n)
        f = rng.uniform(0.5, 1.0, size=(3, n))
        f[int(rng.integers(3))] = 1.0
        lam = (t / unit)[None, :] * f * rng.choice([-1.0, 1.0], size=(3, n))
        assert np.all(max_phase(bd, xyz, lam) <= bound)
        ctx = ctx_for([bd], xyz, "fp32c")
        check_against_oracle(ctx, bd, xyz, lam, TOL["fp32c"], tangents=tan, fg=False,
                             label=f"below the phase bound, {nx}x{ny}, tangents {tan}")


@pytest.mark.parametrize("G", [0, 2])
@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_magnetograms_without_points(precision, G):
    """seg may give a magnetogram no points (equal offsets): evaluation, adjoint and search over the
    others are unchanged, and dL/dB0 of a magnetogram without points is zero (nodal rule and 9-node
    elements; the adjoint of the others against the oracle's nodal VJP)."""
    rng = np.random.default_rng(77)

    class Bd:
        pass

    shapes = [(19, 15), (13, 31), (25, 7), (9, 9)]
    npts = [0, 210, 0, 95]
    bds, xyzs = [], []
    for (nx, ny), n in zip(shapes, npts):
        bd = Bd()
        bd.B0 = rng.normal(size=(3, ny, nx))
        bd.x0, bd.y0, bd.h = 0.0, 0.0, 1.0
        bds.append(bd)
        xyzs.append(np.stack([rng.uniform(0, nx, n), rng.uniform(0, ny, n), rng.uniform(0.4, 15, n)]))
    xyz = np.concatenate(xyzs, axis=1)
    n = xyz.shape[1]
    lam = rng.uniform(-0.4, 0.4, size=(3, n))
    seg = np.concatenate([[0], np.cumsum(npts)])
    ctx = ctx_for(bds, xyz, precision, seg=seg, quad_points=G)
    out = D.dbie_eval_field(ctx, T(lam), want_tan=True)
    gB, gdB = rng.normal(size=(3, n)), rng.normal(size=(9, n))
    g = D.dbie_grad(ctx, T(lam), gB=T(gB), gdB=T(gdB))
    parts = D.split_gB0(ctx, g["gB0"])
    torch.cuda.synchronize()
    glam = g["glambda"].cpu().numpy()
    for b, bd in enumerate(bds):
        s, e = seg[b], seg[b + 1]
        if s == e:
            assert torch.count_nonzero(parts[b]).item() == 0, b
            continue
        if G:
            B, dB, tan = oracle.field_quad9(bd.B0, 0.0, 0.0, 1.0, xyz[:, s:e], lam[:, s:e], G=G, tangents=True)
        else:
            B, dB, tan = oracle.field(bd.B0, 0.0, 0.0, 1.0, xyz[:, s:e], lam[:, s:e], tangents=True)
        for name, ref in (("B", B), ("dB", dB), ("tan", tan)):
            assert rel(out[name][:, s:e].cpu(), ref) <= TOL[precision], (b, name)
        assert torch.count_nonzero(parts[b]).item() > 0, b
        if G:
            continue
        gB0, gl, _ = oracle.vjp(bd.B0, 0.0, 0.0, 1.0, xyz[:, s:e], lam[:, s:e], gB[:, s:e], gdB[:, s:e])
        assert rel(parts[b].cpu(), gB0) <= TOL[precision], b
        assert rel(glam[:, s:e], gl) <= TOL[precision], b
    r = D.dbie_solve_lambda(ctx, T(np.abs(lam)), method="lm", max_trials=4, eps=1e-3)
    torch.cuda.synchronize()
    tr = r["trials"].cpu().numpy()
    assert tr.min() >= 1 and tr.max() <= 4
