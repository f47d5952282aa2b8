"""GPU tests at the full sizes of the batched and active-region workloads, and of the shape tuner.

Full-size outputs are checked on sampled points against the oracle (which computes them one by one)
and by properties that hold at any size (bitwise equality of one batched launch with separate
launches, determinism, finiteness).
"""
import os
import tempfile

import numpy as np
import pytest
import torch

import oracle
from _parity import check_sampled
import paper_1306_1122_amd as D
from workloads import config2, config3, config4, config5

pytestmark = pytest.mark.gpu


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def batched():
    return config4()


def test_batched_one_launch_equals_separate_launches(batched):
    """Bitwise, with the same pixel slicing on both sides (one slice: the automatic choice would give
    the small separate contexts several, which regroups the FP64 sums)."""
    w = batched
    bds = [dict(B0=T(b.B0), x0=b.x0, y0=b.y0, h=b.h) for b in w.boundaries]
    ctx = D.dbie_init(bds, T(w.xyz), seg=w.seg, precision="fp32c", pixel_split=1)
    lam = T(w.lam)
    out = D.dbie_eval_field(ctx, lam, want_tan=True)
    again = D.dbie_eval_field(ctx, lam, want_tan=True)
    for k in ("B", "dB", "tan", "fg"):
        assert torch.equal(out[k], again[k]), k
    assert torch.isfinite(out["B"]).all()
    rng = np.random.default_rng(41)
    for b in rng.choice(len(w.boundaries), 6, replace=False):
        s0, s1 = int(w.seg[b]), int(w.seg[b + 1])
        c1 = D.dbie_init([bds[b]], T(w.xyz[:, s0:s1]), precision="fp32c", pixel_split=1)
        one = D.dbie_eval_field(c1, T(w.lam[:, s0:s1]), want_tan=True)
        for k in ("B", "dB", "tan", "fg"):
            assert torch.equal(one[k], out[k][:, s0:s1]), (b, k)


def test_batched_sampled_parity(batched):
    w = batched
    bds = [dict(B0=T(b.B0), x0=b.x0, y0=b.y0, h=b.h) for b in w.boundaries]
    ctx = D.dbie_init(bds, T(w.xyz), seg=w.seg, precision="fp32c")
    out = D.dbie_eval_field(ctx, T(w.lam), want_tan=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(42)
    for b in rng.choice(len(w.boundaries), 4, replace=False):
        s0, s1 = int(w.seg[b]), int(w.seg[b + 1])
        idx = np.sort(rng.choice(np.arange(s0, s1), 64, replace=False))
        got = {k: out[k][:, idx].cpu().numpy() for k in ("B", "dB", "tan")}
        check_sampled(got, w.boundaries[b], w.xyz[:, idx], w.lam[:, idx], "fp32c", f"batched magnetogram {b}",
                      fg=out["fg"][:, idx].cpu().numpy())


def test_active_region_clustered_points_sampled_parity():
    """2^20 points on 4096 arcs over the 512x256 magnetogram (z down to 0.5 pixel: heavy near field)."""
    w = config5()
    bd = w.boundaries[0]
    for prec, tol in (("fp32c", 1e-5), ("fp64", 1e-10)):
        ctx = D.dbie_init([dict(B0=T(bd.B0), x0=0.0, y0=0.0, h=1.0)], T(w.xyz), precision=prec)
        out = D.dbie_eval_field(ctx, T(w.lam), want_tan=(prec == "fp32c"))
        torch.cuda.synchronize()
        rng = np.random.default_rng(43)
        low = np.nonzero(w.xyz[2] < 2.0)[0]
        idx = np.sort(np.concatenate([rng.choice(w.n_points, 96, replace=False), rng.choice(low, 64, replace=False)]))
        rows = ("B", "dB", "tan") if prec == "fp32c" else ("B", "dB")
        got = {k: out[k][:, idx].cpu().numpy() for k in rows}
        check_sampled(got, bd, w.xyz[:, idx], w.lam[:, idx], prec, f"active region {prec}",
                      fg=out["fg"][:, idx].cpu().numpy(), tol=tol)
        # the lowest points alone (near-field pairs summed in FP64)
        lo = np.isin(idx, low)
        check_sampled({k: v[:, lo] for k, v in got.items()}, bd, w.xyz[:, idx[lo]], w.lam[:, idx[lo]], prec,
                      f"active region, points below 2 pixels, {prec}", tol=tol)


def test_tuner_picks_an_instantiated_shape_and_results_do_not_change():
    w = config2(nz=4)
    bd = w.boundaries[0]
    B0 = T(bd.B0)
    xyz = T(w.xyz)
    lam = T(w.lam)
    ref = D.dbie_init([dict(B0=B0, x0=0.0, y0=0.0, h=1.0)], xyz, precision="fp32c")
    r0 = D.dbie_eval_field(ref, lam, want_tan=True)
    with tempfile.TemporaryDirectory() as td:
        cache = os.path.join(td, "tune.txt")
        ctx = D.dbie_init([dict(B0=B0, x0=0.0, y0=0.0, h=1.0)], xyz, precision="fp32c", tune=True,
                          tune_cache=cache)
        q, qt = D.dbie_query(ctx), D.dbie_query_tan(ctx)
        # timed here, or reused from an earlier context of this process with the same key
        assert D.dbie_query_tuned(ctx) in (1, 2)
        lines = [l.split() for l in open(cache).read().split("\n") if l.strip()]
        assert len(lines) == 2 and [l[4] for l in lines] == ["0", "1"]   # the plain pass, then tangents
        assert lines[0][0].startswith("gfx") and lines[0][2:4] == ["16", "14"]   # 2^16 points, 2^14 pixels
        # a second context reads the file and gets the same shapes and split
        ctx2 = D.dbie_init([dict(B0=B0, x0=0.0, y0=0.0, h=1.0)], xyz, precision="fp32c", tune=True,
                           tune_cache=cache)
        assert D.dbie_query_tuned(ctx2) == 3
        assert D.dbie_query(ctx2) == q and D.dbie_query_tan(ctx2) == qt
        assert D.dbie_query_split(ctx2) == D.dbie_query_split(ctx)
    r1 = D.dbie_eval_field(ctx, lam, want_tan=True)
    torch.cuda.synchronize()
    # a different tile shape changes only the FP32 rounding: the lane that sums a point and, with
    # another LDS block height, which pixels share an FP32 block partial; each run is within ~1e-6 of
    # the FP64 sums here, so the two agree to a few 1e-6
    for k in ("B", "dB", "tan"):
        assert rel(r1[k].cpu(), r0[k].cpu()) <= 5e-6, k
    # an explicit shape is honoured, an unknown one is rejected
    D.dbie_set_tile_shape(ctx, 1, 8, 256)
    assert D.dbie_query(ctx)["ppl"] == 1 and D.dbie_query(ctx)["waves"] == 8
    with pytest.raises(D.DbieError, match="not instantiated"):
        D.dbie_set_tile_shape(ctx, 3, 4, 256)


def test_tuner_reuses_its_choice_within_a_size_bucket():
    """A context whose key (architecture, quadrature, pass, floor(log2) of the point count and of the
    pixels per magnetogram) matches an earlier one reuses that choice without timing; its results
    agree with an untuned context's set to the same tile shape (grid or persistent form, split: FP64
    regrouping at most)."""
    w4, w6 = config2(nz=4), config2(nz=6)     # 65,536 and 98,304 points: both 2^16 <= N < 2^17
    B0 = T(w4.boundaries[0].B0)
    a = D.dbie_init([dict(B0=B0, x0=0.0, y0=0.0, h=1.0)], T(w4.xyz), precision="fp32c", tune=True)
    assert D.dbie_query_tuned(a) in (1, 2)
    b = D.dbie_init([dict(B0=B0, x0=0.0, y0=0.0, h=1.0)], T(w6.xyz), precision="fp32c", tune=True)
    assert D.dbie_query_tuned(b) == 2
    shape = lambda c: {k: D.dbie_query(c)[k] for k in ("ppl", "waves", "tile_pixels")}  # noqa: E731
    assert shape(b) == shape(a) and D.dbie_query_tan(b) == D.dbie_query_tan(a)
    assert D.dbie_query_persistent(b) == D.dbie_query_persistent(a)
    assert D.dbie_query_split(b) == D.dbie_query_split(a)
    ref = D.dbie_init([dict(B0=B0, x0=0.0, y0=0.0, h=1.0)], T(w6.xyz), precision="fp32c")
    assert D.dbie_query_tuned(ref) == 0
    qt = D.dbie_query_tan(b)
    D.dbie_set_tile_shape(ref, qt["ppl"], qt["waves"], qt["tile_pixels"])
    lam = T(w6.lam)
    r0 = D.dbie_eval_field(ref, lam, want_tan=True)
    r1 = D.dbie_eval_field(b, lam, want_tan=True)
    torch.cuda.synchronize()
    for k in ("B", "dB", "tan"):
        assert rel(r1[k].cpu(), r0[k].cpu()) <= 1e-12, k


def test_tuner_with_few_points_picks_a_split():
    """With few points (a 2,000-point evaluation over the 256x256 magnetogram: 8 point tiles) the tuner
    also times the pixel split; the result agrees to FP64 regrouping with an untuned one-slice
    context's set to the same tile shape."""
    w = config3(nz=1)
    bd = w.boundaries[0]
    idx = np.random.default_rng(3).choice(w.n_points, 2000, replace=False)
    xyz, lam = T(w.xyz[:, idx]), T(w.lam[:, idx])
    B0 = T(bd.B0)
    ctx = D.dbie_init([dict(B0=B0, x0=0.0, y0=0.0, h=1.0)], xyz, precision="fp32c", tune=True)
    ref = D.dbie_init([dict(B0=B0, x0=0.0, y0=0.0, h=1.0)], xyz, precision="fp32c", pixel_split=1)
    qt = D.dbie_query_tan(ctx)
    D.dbie_set_tile_shape(ref, qt["ppl"], qt["waves"], qt["tile_pixels"])
    S = D.dbie_query_split(ctx)
    print("tuned split for 2000 points:", S, "shape", D.dbie_query(ctx), flush=True)
    assert 1 <= S <= 32 and D.dbie_query_tuned(ctx) in (1, 2)
    r0 = D.dbie_eval_field(ref, lam, want_tan=True)
    r1 = D.dbie_eval_field(ctx, lam, want_tan=True)
    torch.cuda.synchronize()
    for k in ("B", "dB", "tan"):
        assert rel(r1[k].cpu(), r0[k].cpu()) <= 1e-12, k


def test_persistent_form_equals_grid_launch(batched):
    """The persistent grid (tiles pulled from a device counter) and one workgroup per tile compute
    every tile identically: bitwise equal outputs, for evaluation and for a solve."""
    w = batched
    keep = 12
    seg = w.seg[: keep + 1]
    bds = [dict(B0=T(b.B0), x0=b.x0, y0=b.y0, h=b.h) for b in w.boundaries[:keep]]
    xyz, lam = w.xyz[:, : seg[-1]], w.lam[:, : seg[-1]]
    ctx = D.dbie_init(bds, T(xyz), seg=seg, precision="fp32c")
    outs = []
    for persistent in (False, True, False):
        D.dbie_set_tile_shape(ctx, 1, 4, 256, persistent)
        assert D.dbie_query_persistent(ctx)["plain"] == persistent
        outs.append(D.dbie_eval_field(ctx, T(lam), want_tan=True))
        outs.append(D.dbie_solve_lambda(ctx, T(np.abs(lam)), method="lm", max_trials=6, fp64_accept=False))
    for k in ("B", "dB", "tan", "fg"):
        assert torch.equal(outs[0][k], outs[2][k]) and torch.equal(outs[0][k], outs[4][k]), k
    for k in ("lam", "status", "trials", "B", "fg"):
        assert torch.equal(outs[1][k], outs[3][k]) and torch.equal(outs[1][k], outs[5][k]), k


@pytest.mark.parametrize("G", [0, 2])
@pytest.mark.parametrize("precision", ["fp32c", "fp64"])
def test_pixel_slices_match_one_slice_and_the_oracle(G, precision):
    """Few points (the slices fill the chip): every slicing agrees with one slice to FP64 rounding of
    the regrouped sums, and with the oracle to the path's bar; each is deterministic."""
    rng = np.random.default_rng(51)
    nx, ny = 77, 45
    B0 = rng.normal(size=(3, ny, nx)).astype(np.float32).astype(np.float64)
    n = 1500
    xyz = np.stack([rng.uniform(-2, nx + 1, n), rng.uniform(-2, ny + 1, n), rng.uniform(0.4, 30, n)])
    lam = rng.uniform(-0.5, 0.5, size=(3, n))
    outs = {}
    for S in (1, 2, 7, 32, 0):
        ctx = D.dbie_init([dict(B0=T(B0), x0=0.0, y0=0.0, h=1.0)], T(xyz), precision=precision, pixel_split=S,
                          quad_points=G)
        assert D.dbie_query_split(ctx) == S or (S == 0 and D.dbie_query_split(ctx) >= 1)
        a = D.dbie_eval_field(ctx, T(lam), want_tan=True)
        b = D.dbie_eval_field(ctx, T(lam), want_tan=True)
        for k in ("B", "dB", "tan", "fg"):
            assert torch.equal(a[k], b[k]), (S, k)
        outs[S] = a
    print("automatic slices:", D.dbie_query_split(ctx), flush=True)
    for S, o in outs.items():
        for k in ("B", "dB", "tan"):
            assert rel(o[k].cpu(), outs[1][k].cpu()) <= 1e-13, (S, k)
    if G == 0:
        B, dB, tan = oracle.field(B0, 0.0, 0.0, 1.0, xyz, lam, tangents=True)
    else:
        B, dB, tan = oracle.field_quad9(B0, 0.0, 0.0, 1.0, xyz, lam, G=G, tangents=True)
    for k, ref in (("B", B), ("dB", dB), ("tan", tan)):
        assert rel(outs[0][k].cpu(), ref) <= (1e-5 if precision == "fp32c" else 1e-10), k


@pytest.mark.parametrize("G,nx", [(0, 77), (0, 71), (2, 77)])
@pytest.mark.parametrize("tile_pixels", [128, 256, 512])
def test_every_pixel_block_height_matches_the_oracle(tile_pixels, G, nx):
    """LDS pixel blocks of 16, 32 and 64 rows (16 columns wide on the nodal grid, staged from two
    8-column HBM strips; 8 on the element grid) on an nx x 45 magnetogram, whose 45 rows (44 grid rows
    with elements) leave a ragged last block for every height; 71 columns make an odd number of
    8-column strips, so the last nodal block holds one strip and zeros. Points below 2 pixels (masked
    near field) and beyond the magnetogram; one and three pixel slices and the persistent form; the
    passes with and without tangents and the single-lambda pass. Every run equals the oracle (nodal
    rule: relative L2 and the pointwise bound at every point; elements: relative L2) and the 32-row
    blocks up to the FP32 rounding of the regrouped block sums."""
    from workloads import Boundary
    rng = np.random.default_rng(53)
    ny = 45
    B0 = rng.normal(size=(3, ny, nx)).astype(np.float32).astype(np.float64)
    n = 1500
    xyz = np.stack([rng.uniform(-2, nx + 1, n), rng.uniform(-2, ny + 1, n), rng.uniform(0.4, 30, n)])
    lam = rng.uniform(-0.5, 0.5, size=(3, n))
    lam1 = lam[0]
    field = (lambda l: oracle.field(B0, 0.0, 0.0, 1.0, xyz, l, tangents=True)) if G == 0 else \
        (lambda l: oracle.field_quad9(B0, 0.0, 0.0, 1.0, xyz, l, G=G, tangents=True))
    B, dB, tan = field(lam)
    B1, dB1, _ = field(np.stack([lam1] * 3))
    base = None
    for S, persistent in ((1, False), (3, False), (1, True)):
        ctx = D.dbie_init([dict(B0=T(B0), x0=0.0, y0=0.0, h=1.0)], T(xyz), precision="fp32c", pixel_split=S,
                          quad_points=G)
        if base is None:
            base = D.dbie_eval_field(ctx, T(lam), want_tan=True)
        D.dbie_set_tile_shape(ctx, 1, 4, tile_pixels, persistent)
        assert D.dbie_query(ctx)["tile_pixels"] == tile_pixels and D.dbie_query_tan(ctx)["tile_pixels"] == tile_pixels
        out = D.dbie_eval_field(ctx, T(lam), want_tan=True)
        torch.cuda.synchronize()
        label = f"{tile_pixels // 8} rows, G {G}, {S} slices, persistent {persistent}"
        for k, ref in (("B", B), ("dB", dB), ("tan", tan)):
            assert rel(out[k].cpu(), ref) <= 1e-5, (label, k)
            assert rel(out[k].cpu(), base[k].cpu()) <= 5e-6, (label, k)
        if G == 0:
            got = {k: out[k].cpu().numpy() for k in ("B", "dB", "tan")}
            check_sampled(got, Boundary(B0), xyz, lam, "fp32c", label, fg=out["fg"].cpu().numpy())
        plain = D.dbie_eval_field(ctx, T(lam))                 # the pass without tangents
        one = D.dbie_eval_field_scalar(ctx, T(lam1))           # one lambda for the three components
        torch.cuda.synchronize()
        for k, ref in (("B", B), ("dB", dB)):
            assert rel(plain[k].cpu(), ref) <= 1e-5, (label, "plain", k)
        for k, ref in (("B", B1), ("dB", dB1)):
            assert rel(one[k].cpu(), ref) <= 1e-5, (label, "single lambda", k)
        ctx.close()


def test_captured_solve_survives_a_reallocated_accumulator():
    """A solve replays its captured rounds; an evaluation with more trials in between reallocates the
    accumulator, so the next solve must capture again (same results, bitwise)."""
    rng = np.random.default_rng(52)
    B0 = rng.normal(size=(3, 40, 40)).astype(np.float32).astype(np.float64)
    n = 3000
    xyz = np.stack([rng.uniform(0, 39, n), rng.uniform(0, 39, n), rng.uniform(0.5, 20, n)])
    ctx = D.dbie_init([dict(B0=T(B0), x0=0.0, y0=0.0, h=1.0)], T(xyz), precision="fp32c")
    lam0 = rng.uniform(0, 0.2, size=(3, n))
    a = D.dbie_solve_lambda(ctx, T(lam0), method="lm", max_trials=10, fp64_accept=False)
    D.dbie_eval_field(ctx, T(rng.uniform(-1, 1, size=(6, 3, n))))
    b = D.dbie_solve_lambda(ctx, T(lam0), method="lm", max_trials=10, fp64_accept=False)
    c = D.dbie_solve_lambda(ctx, T(lam0), method="lm", max_trials=10, fp64_accept=False, use_graph=False)
    for k in ("lam", "status", "trials", "B", "fg"):
        assert torch.equal(a[k], b[k]) and torch.equal(a[k], c[k]), k


@pytest.mark.parametrize("precision,tol", [("fp32c", 1e-5), ("fp64", 1e-10)])
def test_largest_grid_workload_sampled(precision, tol):
    """The 256x256 magnetogram with all 256x256x128 = 8,388,608 points in one launch (the largest
    single-GPU configuration, the benchmark's workload), with the mu-tangents in FP32C; the oracle
    checks a z-stratified sample (relative L2, every output of every sampled point, f and g)."""
    from workloads import z_stratified_subsample
    w = config3()
    bd = w.boundaries[0]
    ctx = D.dbie_init([dict(B0=T(bd.B0), x0=bd.x0, y0=bd.y0, h=bd.h)], T(w.xyz), precision=precision)
    out = D.dbie_eval_field(ctx, T(w.lam), want_tan=(precision == "fp32c"))
    torch.cuda.synchronize()
    idx = z_stratified_subsample(w.xyz, 256, seed=13)
    rows = ("B", "dB", "tan") if precision == "fp32c" else ("B", "dB")
    got = {k: out[k][:, idx].cpu().numpy() for k in rows}
    check_sampled(got, bd, w.xyz[:, idx], w.lam[:, idx], precision, f"256x256 x 8.4M {precision}",
                  fg=out["fg"][:, idx].cpu().numpy(), tol=tol)
    assert torch.isfinite(out["B"]).all() and torch.isfinite(out["fg"]).all()
    ctx.close()


@pytest.mark.parametrize("which", ["bipoles_128", "active_region_512x256"])
def test_fp32c_matches_fp64_on_every_point(which):
    """Every point of the full workload: the FP32C result against the library's FP64 result (itself
    pinned to the oracle on samples), relative L2 over all points and per magnetogram row."""
    w = config2() if which == "bipoles_128" else config5()
    bd = w.boundaries[0]
    res = {}
    for prec in ("fp64", "fp32c"):
        ctx = D.dbie_init([dict(B0=T(bd.B0), x0=bd.x0, y0=bd.y0, h=bd.h)], T(w.xyz), precision=prec)
        out = D.dbie_eval_field(ctx, T(w.lam), want_tan=True)
        torch.cuda.synchronize()
        res[prec] = {k: out[k].cpu().numpy() for k in ("B", "dB", "tan")}
        ctx.close()
    for k in ("B", "dB", "tan"):
        e = rel(res["fp32c"][k], res["fp64"][k])
        # the worst single point, relative to that point's own magnitude
        a, b = res["fp32c"][k], res["fp64"][k]
        per = np.linalg.norm(a - b, axis=0) / np.maximum(np.linalg.norm(b, axis=0), 1e-300)
        print(which, k, "rel L2 %.2e, worst point %.2e, 99.9%% of points below %.2e" % (
            e, per.max(), np.quantile(per, 0.999)), flush=True)
        assert e <= 1e-5, (k, e)


@pytest.mark.parametrize("workload", ["config3", "config2"])
def test_benchmark_step_at_full_size(workload):
    """The benchmark's step as it runs there (tuned shapes, Levenberg-Marquardt with tangents, three
    trials from the workload's lambda, no FP64 acceptance) on all points of the 256x256 workload (the
    headline, 8.4M points) and of the 128x128 one (2^20): repeated calls give the same trajectory
    bitwise, with and without B and (f, g) requested; at a z-stratified sample the field and residuals
    at the returned lambda match the oracle's to the FP32C bar (every output of every sampled point
    bounded), and LM never ends above its start by more than the FP32C-vs-FP64 difference."""
    from workloads import z_stratified_subsample
    w = config3() if workload == "config3" else config2()
    bd = w.boundaries[0]
    ctx = D.dbie_init([dict(B0=T(bd.B0), x0=bd.x0, y0=bd.y0, h=bd.h)], T(w.xyz), precision="fp32c", tune=True)
    lam0 = T(w.lam)
    a = D.dbie_solve_lambda(ctx, lam0.clone(), method="lm", max_trials=3, eps=1e-4, fp64_accept=False,
                            want_B=False, want_fg=False)
    b = D.dbie_solve_lambda(ctx, lam0.clone(), method="lm", max_trials=3, eps=1e-4, fp64_accept=False)
    torch.cuda.synchronize()
    for k in ("lam", "status", "trials"):
        assert torch.equal(a[k], b[k]), k
    tr = b["trials"].cpu().numpy()
    assert tr.min() >= 1 and tr.max() <= 3
    idx = z_stratified_subsample(w.xyz, 256, seed=61)
    lg = b["lam"].cpu().numpy()[:, idx]
    Bo, dBo = oracle.field(bd.B0, bd.x0, bd.y0, bd.h, w.xyz[:, idx], lg)
    res = oracle.residuals(Bo, dBo, bd.h)
    # B and (f, g) at lambda* in FP32C (no acceptance pass): the path's bar, pointwise, conditioned f, g
    ev = D.dbie_eval_field(ctx, T(np.ascontiguousarray(b["lam"].cpu().numpy())))
    torch.cuda.synchronize()
    assert torch.equal(ev["B"], b["B"]) and torch.equal(ev["fg"], b["fg"])
    got = {k: ev[k][:, idx].cpu().numpy() for k in ("B", "dB")}
    check_sampled(got, bd, w.xyz[:, idx], lg, "fp32c", f"benchmark step {workload}",
                  fg=b["fg"][:, idx].cpu().numpy())
    B0_, dB0_ = oracle.field(bd.B0, bd.x0, bd.y0, bd.h, w.xyz[:, idx], np.abs(w.lam[:, idx]))
    phi0 = oracle.residuals(B0_, dB0_, bd.h)["Phi"]
    assert np.mean(res["Phi"] <= phi0 * (1 + 1e-4) + 1e-12) >= 0.99
