"""Benchmark of the DBIE hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the 256x256 FP32 bipole magnetogram (10 Gaussian bipoles, per-bipole shear alpha in
[0.5, 2], 20 G noise) with all 256x256x128 = 8,388,608 evaluation points (5.5e11 kernel pairs per
trial); synthetic, seeded. The 128x128 workload with 2^20 points runs the same step as an extra.
One step = one call of dbie_solve_lambda in its gradient form (Levenberg-Marquardt in mu = lambda^2)
with a budget of TRIALS_PER_STEP trials over every point: per trial the FP32C bulk sum of B, grad B
and the mu-tangents, the FP64 near-field pairs and residuals, the LM update and the active-set
compaction. The metric is kernel-pair evaluations per second (pixels x points x trials / time).

Printed: one JSON line with the metric, a roofline object for the dominant kernel (the FP32C bulk
sum; its launch time is measured with HIP events on the launch stream by the library), and the FP64
CPU oracle timed on a bounded sample of the same workload on the host cores (cpu_baseline).
"""
import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# algorithmic FP32 flops per kernel pair (point, pixel, trial; all three components): the formulas
# of the field, its frozen-lambda gradient and the mu-tangents counted with FMA = 2, add/mul = 1 and
# each sin, cos, rsqrt = 1
FLOPS_FIELD_GRAD = 68
FLOPS_FIELD_GRAD_TAN = 89
PEAK_FP32_VECTOR_TFLOPS = 157.3
# with packed FP32 switched off, one wave64 VALU instruction per SIMD per 4 cycles: 256 CUs x 4 SIMDs
# x 2.4 GHz / 4 x 64 lanes = 3.93e13 lane-instructions/s; divided by the VALU instructions the kernel
# executes per pair (rocprofv3 SQ_INSTS_VALU, committed with the traffic counters) and times the
# algorithmic flops per pair, this is the kernel's issue ceiling
VALU_LANE_INSTS_PER_S = 256 * 4 * 2.4e9 / 4 * 64
TRIALS_PER_STEP = 3


def _oracle_chunk(args):
    B0, x0, y0, h, xyz, lam = args
    import oracle
    B, dB, tan = oracle.field(B0, x0, y0, h, xyz, lam, tangents=True)
    oracle.residuals(B, dB, h)
    return xyz.shape[1]


def cpu_baseline(w, n_sample, seed=7):
    """The FP64 oracle (as it stands) on a z-stratified sample of the workload's points, one
    process per host core; returns pairs/s of field + grad + tangents + residuals."""
    from workloads import z_stratified_subsample
    bd = w.boundaries[0]
    idx = z_stratified_subsample(w.xyz, n_sample, seed)
    # one worker per host core, at most 16 (the host CPUs one GPU is allotted)
    cores = min(os.cpu_count() or 1, 16)
    chunks = np.array_split(idx, cores * 4)
    jobs = [(bd.B0, bd.x0, bd.y0, bd.h, w.xyz[:, c], w.lam[:, c]) for c in chunks if c.size]
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_chunk, jobs[:cores])          # warm the workers
        t0 = time.perf_counter()
        n = sum(pool.map(_oracle_chunk, jobs))
        dt = time.perf_counter() - t0
    pairs = n * bd.nx * bd.ny
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=pairs / dt, unit="pairs/s", cores=cores, host_cpus=os.cpu_count(), kind="oracle", cpu=model,
                sample=f"{n} z-stratified points of the {w.name} workload x all {bd.nx * bd.ny} pixels "
                       f"(FP64 field + grad + mu-tangents + residuals), {dt:.2f} s wall")


def measured_counters():
    """The committed rocprofv3 counter summary of the dominant kernel (HBM bytes per launch, VALU
    instructions per pair), or None when the kernel source has changed since it was taken."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "traffic_k_field32c.json")) as fh:
            t = json.load(fh)
        with open(os.path.join(ROOT, "paper_1306_1122_amd", "csrc", "k_field32c.hip"), "rb") as fh:
            sha = hashlib.sha256(fh.read()).hexdigest()
    except (OSError, ValueError):
        return None
    return t if t.get("source_sha256") == sha else None


def _timed(f, reps):
    import torch
    f()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        f()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def per_trial_rates(D, ctx, B0, xyz, lam, bd, pairs, s):
    """One evaluation of B and grad B (no tangents: one Nelder-Mead trial) in FP32C and in FP64."""
    out = {}
    for name, prec, reps in (("fp32c_field_grad", "fp32c", 5), ("fp64_field_grad", "fp64", 2)):
        c2 = ctx if prec == "fp32c" else D.dbie_init([dict(B0=B0, x0=bd.x0, y0=bd.y0, h=bd.h)], xyz,
                                                    precision=prec)
        D.dbie_timing(c2, True)
        ms = _timed(lambda: D.dbie_eval_field(c2, lam), reps)
        km, kl = D.dbie_timing_read(c2)
        D.dbie_timing(c2, False)
        k = km / max(kl, 1)
        out[name] = dict(pairs_per_s=pairs / (ms * 1e-3), ms_per_trial=ms, bulk_kernel_ms=k,
                         algorithmic_tflops=FLOPS_FIELD_GRAD * pairs / (k * 1e-3) / 1e12)
        if c2 is not ctx:
            c2.close()
    return out


def error_vs_fp64(D, ctx, ctx64, lam):
    """Error of the FP32C evaluation against the FP64 path on the same points and lambda: relative
    L2 over all points of B, grad B and the mu-tangents, the largest per-point |dB| / |B|, and the
    largest change of f and g (computed in FP64 from either field)."""
    import torch
    a = D.dbie_eval_field(ctx, lam, want_tan=True)
    b = D.dbie_eval_field(ctx64, lam, want_tan=True)
    nrm = torch.linalg.vector_norm
    out = {k + "_rel_l2": float(nrm(a[k] - b[k]) / nrm(b[k])) for k in ("B", "dB", "tan")}
    pt = nrm(a["B"] - b["B"], dim=0) / nrm(b["B"], dim=0)
    out["B_max_point_rel"] = float(pt[torch.isfinite(pt)].max())
    d = (a["fg"] - b["fg"]).abs()
    out["fg_max_abs"] = float(d[torch.isfinite(d)].max())
    out["reference"] = "FP64 path (dbie_eval_field in an FP64 context), same workload, all points"
    return out


def adjoint_and_scalar(D, ctx, lam, pairs, B0, xyz, bd):
    """dbie_grad (B0 adjoint, FP32C and FP64 contexts) and the single-lambda evaluation on the
    benchmark workload."""
    import torch
    N = ctx.n_points
    g = torch.ones(3, N, dtype=torch.float64, device=lam.device)
    gd = torch.ones(9, N, dtype=torch.float64, device=lam.device)
    ms_adj = _timed(lambda: D.dbie_grad(ctx, lam, gB=g, gdB=gd, want_glambda=False), 2)
    c64 = D.dbie_init([dict(B0=B0, x0=bd.x0, y0=bd.y0, h=bd.h)], xyz, precision="fp64")
    ms_adj64 = _timed(lambda: D.dbie_grad(c64, lam, gB=g, gdB=gd, want_glambda=False), 1)
    c64.close()
    lam1 = lam[0].contiguous()
    ms_sc = _timed(lambda: D.dbie_eval_field_scalar(ctx, lam1), 3)
    return dict(adjoint_gB0_ms=ms_adj, adjoint_pairs_per_s=pairs / (ms_adj * 1e-3),
                adjoint_gB0_fp64_ms=ms_adj64, adjoint_fp64_pairs_per_s=pairs / (ms_adj64 * 1e-3),
                scalar_lambda_field_grad_ms=ms_sc, scalar_lambda_pairs_per_s=pairs / (ms_sc * 1e-3))


def schrijver_metrics(B, b):
    """Field-comparison metrics of Schrijver et al. (2006) used by the paper's Table 1: B the exact
    field, b the model, both [3, N]."""
    nB = np.sqrt(np.sum(B * B, axis=0))
    nb = np.sqrt(np.sum(b * b, axis=0))
    dot = np.sum(B * b, axis=0)
    diff = np.sqrt(np.sum((b - B) ** 2, axis=0))
    return dict(C_vec=float(np.sum(dot) / np.sqrt(np.sum(nB ** 2) * np.sum(nb ** 2))),
                C_cs=float(np.mean(dot / (nB * nb))), E_n=float(1.0 - np.sum(diff) / np.sum(nB)),
                E_m=float(1.0 - np.mean(diff / nB)), eps=float(np.sum(nb ** 2) / np.sum(nB ** 2)))


def time_to_solution(D, dev, n_sample=65536, eps=1e-4, workload="config3", nm_budget=200, lm_budget=20,
                     forms=("plain", "fp32c_nm", "fast")):
    """Plain form (FP64 Nelder-Mead, nm_budget trials) vs fast form (FP32C Levenberg-Marquardt with
    the default trust region, lm_budget trials, FP64 acceptance), from lambda = 0, on the workload's
    points (a z-stratified sample of n_sample of them, or all with n_sample=None); the FP32C
    Nelder-Mead (nm_budget trials, FP64 acceptance) separates the precision from the method.
    q* = the solved fraction (max(f, g) <= eps in FP64) the plain form reaches within its budget;
    TTS(form) = solve time until that form's solved fraction reaches q* (round-end HIP events), where
    a point counts from the round of its last trial only if its final status is CONVERGED (for the
    FP32C forms: confirmed by the FP64 acceptance pass, which re-evaluates the points that converged),
    and the FP32C forms add the duration of that pass (the solve's end minus the end of its last
    round). For a workload with an exact field (Low & Lou) each form also reports the comparison
    metrics of its FP64 field at lambda* against the exact field, next to those at lambda = 0."""
    import torch
    import workloads
    from workloads import z_stratified_subsample
    w = getattr(workloads, workload)()
    bd = w.boundaries[0]
    idx = np.arange(w.n_points) if n_sample is None else z_stratified_subsample(w.xyz, n_sample, 3)
    pts = np.ascontiguousarray(w.xyz[:, idx])
    xyz = torch.tensor(pts, dtype=torch.float64, device=dev)
    B0 = torch.tensor(bd.B0, dtype=torch.float64, device=dev)
    n = xyz.shape[1]
    ll = w.meta.get("ll") if w.meta else None
    exact = ll.field(*pts) if ll is not None else None
    ctx64 = D.dbie_init([dict(B0=B0, x0=bd.x0, y0=bd.y0, h=bd.h)], xyz, precision="fp64")
    res = {"workload": (f"all {n} points of {w.name}" if n_sample is None else
                        f"{n} z-stratified points of {w.name}"), "eps": eps}
    if exact is not None:
        b = D.dbie_eval_field(ctx64, torch.zeros(3, n, dtype=torch.float64, device=dev))["B"].cpu().numpy()
        res["metrics_lambda0"] = schrijver_metrics(exact, b)
    table = {"plain": ("plain_fp64_nelder_mead", "fp64", "nm", nm_budget),
             "fp32c_nm": ("fp32c_nelder_mead", "fp32c", "nm", nm_budget),
             "fast": ("fast_fp32c_levenberg_marquardt", "fp32c", "lm", lm_budget)}
    run = [table[f] for f in forms]
    for form, prec, meth, budget in run:
        print(f"time to solution: {form} on {res['workload']}", file=sys.stderr, flush=True)
        ctx = ctx64 if prec == "fp64" else D.dbie_init([dict(B0=B0, x0=bd.x0, y0=bd.y0, h=bd.h)], xyz,
                                                        precision=prec)
        lam = torch.zeros(3, n, dtype=torch.float64, device=dev)
        D.dbie_solve_trace(ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = D.dbie_solve_lambda(ctx, lam, method=meth, max_trials=budget, eps=eps, fp64_accept=True,
                                want_B=False, want_fg=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        t, cv, t_end = D.dbie_solve_trace_read(ctx, with_end=True)
        D.dbie_solve_trace(ctx, False)
        st = r["status"].cpu().numpy()
        tr = r["trials"].cpu().numpy()
        # field, f and g at lambda* in FP64 for the summary (after the timed solve)
        ev = D.dbie_eval_field(ctx64, r["lam"], want_dB=False)
        fg = ev["fg"].cpu().numpy()
        if ctx is not ctx64:
            ctx.close()
        # FP64-confirmed solved fraction at the end of each round (one trial per round)
        ok = tr[st == 0]
        frac = np.array([np.count_nonzero(ok <= k + 1) for k in range(len(t))]) / n
        accept_ms = max(0.0, t_end - float(t[-1])) if (prec == "fp32c" and len(t)) else 0.0
        res[form] = dict(budget=budget, wall_s=wall, rounds=int(len(t)), accept_ms=accept_ms,
                         converged_in_rounds=int(np.sum(cv)),
                         solved_fraction=float(np.mean(st == 0)),
                         mean_f=float(np.nanmean(fg[0])), mean_g=float(np.nanmean(fg[1])),
                         median_rho=float(np.nanmedian(np.maximum(fg[0], fg[1]))),
                         curve_ms=[float(v) for v in t], curve_fraction=[float(v) for v in frac])
        if exact is not None:
            res[form]["metrics"] = schrijver_metrics(exact, ev["B"].cpu().numpy())
    ctx64.close()
    q = res["plain_fp64_nelder_mead"]["solved_fraction"]
    res["q_star"] = q
    res["q_star_points"] = int(round(q * n))
    for form, _, _, _ in run:
        f = np.array(res[form]["curve_fraction"])
        tms = np.array(res[form]["curve_ms"])
        hit = np.nonzero(f >= q)[0] if q > 0 else np.array([], dtype=int)
        res[form]["tts_ms"] = float(tms[hit[0]]) + res[form]["accept_ms"] if hit.size else None
        # keep the JSON line short: curves at 8 sample rounds
        k = np.unique(np.linspace(0, len(tms) - 1, 8).astype(int)) if len(tms) else []
        res[form]["curve_ms"] = [res[form]["curve_ms"][i] for i in k]
        res[form]["curve_fraction"] = [res[form]["curve_fraction"][i] for i in k]
    a = res["plain_fp64_nelder_mead"]["tts_ms"]
    b = res.get("fast_fp32c_levenberg_marquardt", {}).get("tts_ms")
    res["tts_speedup"] = (a / b) if (a and b) else None
    # the precision alone (same derivative-free search in FP32C)
    c = res.get("fp32c_nelder_mead", {}).get("tts_ms")
    if "fp32c_nelder_mead" in res:
        res["tts_speedup_fp32c_nelder_mead"] = (a / c) if (a and c) else None
    return res


def table1_metrics(D, dev, mapping):
    """The paper's Table 1 case (Low & Lou n = 3, m = 1, l = 0.3, Phi = 4 pi / 5; 192^2 boundary, 64^3
    region; one of two readings of its grid mapping): the comparison metrics over the 64^3 region
    nodes against the exact field, for lambda = 0, the plain form (FP64 Nelder-Mead, 50 trials) and
    the fast form (FP32C Levenberg-Marquardt with the default trust region, 20 trials, FP64
    acceptance), each with its solve time."""
    import torch
    from workloads import lowlou_table1
    w = lowlou_table1(mapping=mapping)
    bd = w.boundaries[0]
    jj, ii = w.meta["bottom_idx"]
    bottom = bd.B0[:, jj, ii]
    exact = np.concatenate([bottom, w.meta["ll"].field(*w.xyz)], axis=1)
    T = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)  # noqa: E731
    xyz = T(w.xyz)
    out = {"workload": w.name}
    for name, prec, meth, budget in (("lambda0", "fp64", None, 0), ("plain_fp64_nelder_mead", "fp64", "nm", 50),
                                     ("fast_fp32c_levenberg_marquardt", "fp32c", "lm", 20)):
        ctx = D.dbie_init([dict(B0=T(bd.B0), x0=bd.x0, y0=bd.y0, h=bd.h)], xyz, precision=prec)
        lam = torch.zeros(3, w.n_points, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if meth is None:
            o = D.dbie_eval_field(ctx, lam)
            B, fg, conv = o["B"], o["fg"], float("nan")
        else:
            r = D.dbie_solve_lambda(ctx, lam, method=meth, max_trials=budget, eps=1e-4, fp64_accept=True)
            B, fg = r["B"], r["fg"]
            conv = float((r["status"] == 0).double().mean())
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        ctx.close()
        m = schrijver_metrics(exact, np.concatenate([bottom, B.cpu().numpy()], axis=1))
        fgn = fg.cpu().numpy()
        m.update(solved_fraction=conv, mean_phi=float(np.nanmean(fgn[0] ** 2 + fgn[1] ** 2)), ms=ms)
        out[name] = m
    out["paper_present_dbie"] = dict(C_vec=0.99, C_cs=0.52, E_n=0.83, E_m=-0.53, eps=1.08)
    return out


def batched(D, dev):
    """64 magnetograms of uneven size in one launch (tuned shape) vs one launch per magnetogram (FP32C,
    B + grad B); the tuned shape also in the persistent and the grid form."""
    import torch
    from workloads import config4
    w = config4()
    T = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)  # noqa: E731
    bds = [dict(B0=T(b.B0), x0=b.x0, y0=b.y0, h=b.h) for b in w.boundaries]
    ctx = D.dbie_init(bds, T(w.xyz), seg=w.seg, precision="fp32c", tune=True)
    lam = T(w.lam)
    pairs = w.pairs_per_trial()
    tuned = dict(shape=D.dbie_query(ctx), persistent=D.dbie_query_persistent(ctx), source=D.dbie_query_tuned(ctx))
    one = _timed(lambda: D.dbie_eval_field(ctx, lam), 2)
    # Levenberg-Marquardt rounds over all 64 magnetograms, replayed from the captured graph
    lam_io = torch.empty_like(lam)

    def solve():
        lam_io.copy_(lam.abs())
        D.dbie_solve_lambda(ctx, lam_io, method="lm", max_trials=4, fp64_accept=False, want_B=False,
                            want_fg=False)

    ms_solve = _timed(solve, 1)
    # the tuned shape in the persistent form (tiles pulled from a device counter) and in the grid form
    q = D.dbie_query(ctx)
    D.dbie_set_tile_shape(ctx, q["ppl"], q["waves"], q["tile_pixels"], True)
    pers = _timed(lambda: D.dbie_eval_field(ctx, lam), 2)
    D.dbie_set_tile_shape(ctx, q["ppl"], q["waves"], q["tile_pixels"], False)
    grid = _timed(lambda: D.dbie_eval_field(ctx, lam), 2)
    ctx.close()
    parts = []
    for b in range(len(bds)):
        s0, s1 = int(w.seg[b]), int(w.seg[b + 1])
        parts.append((D.dbie_init([bds[b]], T(w.xyz[:, s0:s1]), precision="fp32c"), T(w.lam[:, s0:s1])))

    def each():
        for c, l in parts:
            D.dbie_eval_field(c, l)

    sep = _timed(each, 1)
    return dict(points=w.n_points, pairs=pairs, one_launch_ms=one, one_launch_pairs_per_s=pairs / (one * 1e-3),
                persistent_launch_ms=pers, persistent_pairs_per_s=pairs / (pers * 1e-3),
                grid_launch_ms=grid, grid_pairs_per_s=pairs / (grid * 1e-3), separate_launches_ms=sep, separate_pairs_per_s=pairs / (sep * 1e-3),
                lm_solve_4_trials_graph_ms=ms_solve, tuned=tuned)


def active_region(D, dev):
    """512x256 active-region-like magnetogram with 2^20 points on 4096 arcs (FP32C + FP64 near field)."""
    import torch
    from workloads import config5
    w = config5()
    bd = w.boundaries[0]
    T = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)  # noqa: E731
    ctx = D.dbie_init([dict(B0=T(bd.B0), x0=0.0, y0=0.0, h=1.0)], T(w.xyz), precision="fp32c")
    lam = T(w.lam)
    pairs = w.pairs_per_trial()
    ms = _timed(lambda: D.dbie_eval_field(ctx, lam), 2)
    mst = _timed(lambda: D.dbie_eval_field(ctx, lam, want_tan=True), 2)
    c64 = D.dbie_init([dict(B0=T(bd.B0), x0=0.0, y0=0.0, h=1.0)], T(w.xyz), precision="fp64")
    err = error_vs_fp64(D, ctx, c64, lam)
    c64.close()
    ctx.close()
    return dict(points=w.n_points, pairs=pairs, field_grad_ms=ms, field_grad_pairs_per_s=pairs / (ms * 1e-3),
                with_tangents_ms=mst, with_tangents_pairs_per_s=pairs / (mst * 1e-3), fp32c_error_vs_fp64=err)


def quad9_elements(D, dev):
    """Eq. (15) 9-node elements on the benchmark magnetogram cropped to 127x127 (odd sides), all
    1,048,576 points: one evaluation of B and grad B per quadrature order, FP32C with the elements
    near a point in FP64, against the nodal rule on the same crop."""
    import torch
    from workloads import config2
    w = config2()
    B0 = np.ascontiguousarray(w.boundaries[0].B0[:, :127, :127])
    T = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)  # noqa: E731
    xyz, lam = T(w.xyz), T(w.lam)
    out = {}
    for G in (0, 2, 4):
        ctx = D.dbie_init([dict(B0=T(B0), x0=0.0, y0=0.0, h=1.0)], xyz, precision="fp32c", quad_points=G)
        ms = _timed(lambda: D.dbie_eval_field(ctx, lam), 2)
        ctx.close()
        npts = 127 * 127 if G == 0 else (G * 63) ** 2
        pairs = w.n_points * npts
        out["nodal" if G == 0 else "G%d" % G] = dict(quadrature_points=npts, field_grad_ms=ms,
                                                      pairs_per_s=pairs / (ms * 1e-3))
    return out


def field_lines(D, dev, n_lines=4096, n_steps=100):
    """RK4 field lines through the FP32C DBIE field of the benchmark magnetogram: 4096 seeds at
    z = 2..10 pixels, step 0.5 pixel, 100 steps, constant lambda 0.02 per pixel (4 evaluations of
    4096 points x 16384 pixels per step)."""
    import torch
    from workloads import config2
    w = config2()
    bd = w.boundaries[0]
    rng = np.random.default_rng(11)
    seeds = np.stack([rng.uniform(16, 112, n_lines), rng.uniform(16, 112, n_lines), rng.uniform(2, 10, n_lines)])
    T = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)  # noqa: E731
    ctx = D.dbie_init([dict(B0=T(bd.B0), x0=0.0, y0=0.0, h=1.0)], T(seeds), precision="fp32c")
    lam = T(np.full((3, 1, 1, 1), 0.02))
    box = (0.0, 0.0, 0.5, 127.0, 127.0, 64.0)
    run = lambda: D.dbie_trace_lines(ctx, lam, (0, 0, 0), (1, 1, 1), box, 0.5, n_steps)  # noqa: E731
    ms = _timed(run, 1)
    cnt = run()["count"]
    ctx.close()
    steps = int(cnt.sum().item()) - n_lines
    return dict(lines=n_lines, steps_taken=steps, ms=ms, line_steps_per_s=steps / (ms * 1e-3),
                pairs_per_s=4 * n_steps * n_lines * bd.nx * bd.ny / (ms * 1e-3))


def lm_step_rate(D, dev, workload, steps=5, warmup=2):
    """The headline step (Levenberg-Marquardt, TRIALS_PER_STEP trials, tuned shapes) on another
    workload: pairs/s and the bulk kernel's mean launch time."""
    import torch
    import workloads
    w = getattr(workloads, workload)()
    bd = w.boundaries[0]
    T = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)  # noqa: E731
    ctx = D.dbie_init([dict(B0=T(bd.B0), x0=bd.x0, y0=bd.y0, h=bd.h)], T(w.xyz), precision="fp32c", tune=True)
    lam = T(w.lam)
    lam_io = torch.empty_like(lam)
    trials = torch.empty(w.n_points, dtype=torch.int32, device=dev)

    def step():
        lam_io.copy_(lam)
        D.dbie_solve_lambda(ctx, lam_io, method="lm", max_trials=TRIALS_PER_STEP, eps=1e-4, fp64_accept=False,
                            trials=trials, want_B=False, want_fg=False)

    for _ in range(warmup):
        step()
    D.dbie_timing(ctx, True)
    D.dbie_timing_read(ctx)
    ms = _timed(step, steps)
    km, kl = D.dbie_timing_read(ctx)
    D.dbie_timing(ctx, False)
    pairs = int(trials.sum().item()) * bd.nx * bd.ny
    ctx.close()
    return dict(workload=w.name, ms_per_step=ms, pairs_per_step=pairs, pairs_per_s=pairs / (ms * 1e-3),
                bulk_kernel_ms=km / max(kl, 1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=24576)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras", default="", help="comma-separated names of the extras to run (default: all)")
    ap.add_argument("--tts-full", default="",
                    help="instead of the benchmark: time to solution over all points of the named workloads "
                         "(comma-separated: config3 = the 256x256 headline workload, ~8 minutes; config5 = the "
                         "active region, ~2 minutes): plain FP64 Nelder-Mead, 200 trials, against the fast form")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed steps, copy 1 GiB once (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--shape", default="", help="FP32C tile shape ppl,waves,tile_pixels")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this library has no multi-GPU path "
              "(points would be sharded across GPUs with the magnetogram replicated).", file=sys.stderr)
        sys.exit(2)

    from workloads import config3
    w = config3()
    # the CPU oracle's worker processes are forked before anything touches the GPU
    cpu = None
    if not args.no_cpu_baseline and not args.tts_full:
        cpu = cpu_baseline(w, args.cpu_sample)

    import torch
    import paper_1306_1122_amd as D
    from paper_1306_1122_amd import _lib

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    _lib.load()   # fails loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    if args.tts_full:
        out = {}
        for name in args.tts_full.split(","):
            print(f"time to solution over all points of {name}", file=sys.stderr, flush=True)
            out[name] = time_to_solution(D, dev, n_sample=None, workload=name, forms=("fast", "plain"))
        print(json.dumps({"time_to_solution_full": out}), flush=True)
        return
    bd = w.boundaries[0]
    N = w.n_points
    pairs = w.pairs_per_trial()
    T = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)  # noqa: E731
    B0 = T(bd.B0)
    xyz = T(w.xyz)
    ctx = D.dbie_init([dict(B0=B0, x0=bd.x0, y0=bd.y0, h=bd.h)], xyz, precision="fp32c", tune=not args.shape)
    if args.shape:
        ppl, waves, tp = (int(v) for v in args.shape.split(","))
        D.dbie_set_tile_shape(ctx, ppl, waves, tp)
    q = D.dbie_query(ctx)
    qt = D.dbie_query_tan(ctx)
    lam = T(w.lam)
    lam_io = torch.empty_like(lam)
    status = torch.empty(N, dtype=torch.int32, device=dev)
    trials = torch.empty(N, dtype=torch.int32, device=dev)

    def step():
        lam_io.copy_(lam)
        D.dbie_solve_lambda(ctx, lam_io, method="lm", max_trials=TRIALS_PER_STEP, eps=1e-4,
                            fp64_accept=False, status=status, trials=trials, want_B=False, want_fg=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    D.dbie_timing(ctx, True)
    D.dbie_timing_read(ctx)
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(s)
    for k in range(args.steps):
        step()
        if k % 5 == 4:
            torch.cuda.synchronize()
            print(f"step {k + 1}/{args.steps}", file=sys.stderr, flush=True)
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    D.dbie_timing(ctx, False)
    kern_ms, launches = D.dbie_timing_read(ctx)
    step_ms = e0.elapsed_time(e1) / args.steps
    kern_avg_ms = kern_ms / max(launches, 1)
    # every point is active in every trial unless it converged earlier: count the evaluations made
    evals_per_step = int(trials.sum().item())
    pairs_per_step = evals_per_step * bd.nx * bd.ny
    value = pairs_per_step / (step_ms * 1e-3)
    # a launch covers the points still active in its round: use the mean pairs per launch
    pairs_per_launch = pairs_per_step * args.steps / max(launches, 1)
    achieved = FLOPS_FIELD_GRAD_TAN * pairs_per_launch / (kern_avg_ms * 1e-3) / 1e12
    counters = measured_counters()
    ceiling = (FLOPS_FIELD_GRAD_TAN * VALU_LANE_INSTS_PER_S / float(counters["valu_per_pair"]) / 1e12
               if counters else None)

    extras = {}
    if not args.no_extras:
        for name, fn in (("per_trial_rates", lambda: per_trial_rates(D, ctx, B0, xyz, lam, bd, pairs, s)),
                         ("adjoint_and_scalar_lambda", lambda: adjoint_and_scalar(D, ctx, lam, pairs, B0, xyz, bd)),
                         ("lm_step_bipoles_128x128_1M_points", lambda: lm_step_rate(D, dev, "config2")),
                         ("time_to_solution_lowlou_all_points",
                          lambda: time_to_solution(D, dev, n_sample=None, workload="config1", nm_budget=50)),
                         ("table1_region", lambda: table1_metrics(D, dev, "region")),
                         ("table1_boundary", lambda: table1_metrics(D, dev, "boundary")),
                         ("time_to_solution", lambda: time_to_solution(D, dev)),
                         ("time_to_solution_eps_0.1", lambda: time_to_solution(D, dev, eps=0.1)),
                         ("time_to_solution_active_region",
                          lambda: time_to_solution(D, dev, workload="config5")),
                         ("batched_64_magnetograms", lambda: batched(D, dev)),
                         ("active_region_512x256_arcs", lambda: active_region(D, dev)),
                         ("quad9_elements_127x127", lambda: quad9_elements(D, dev)),
                         ("field_lines_4096", lambda: field_lines(D, dev))):
            if args.extras and name not in args.extras.split(","):
                continue
            print(f"extra {name}", file=sys.stderr, flush=True)
            try:
                extras[name] = fn()
            except Exception as exc:  # an extra must not hide the headline line
                extras[name] = {"error": repr(exc)}

    # the error of the timed FP32C arithmetic against the FP64 path on the benchmark workload
    # (outside the timed region)
    accuracy = None
    if not args.no_extras:
        c64 = D.dbie_init([dict(B0=B0, x0=bd.x0, y0=bd.y0, h=bd.h)], xyz, precision="fp64")
        accuracy = error_vs_fp64(D, ctx, c64, lam)
        c64.close()

    if args.calib_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()

    line = {
        "metric": "boundary x volume kernel-pair evals/s per lambda trial",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "magnetogram": [bd.nx, bd.ny], "points": N,
                   "pairs_per_trial": pairs, "trials_per_step": TRIALS_PER_STEP,
                   "evals_per_step": evals_per_step,
                   "step": "dbie_solve_lambda, Levenberg-Marquardt, 3-trial budget: per trial FP32C B, "
                           "grad B, mu-tangents + FP64 near field + FP64 residuals + LM update",
                   "tile_shape": [q["ppl"], q["waves"], q["tile_pixels"]],
                   "tile_shape_tangents": [qt["ppl"], qt["waves"], qt["tile_pixels"]],
                   "persistent": D.dbie_query_persistent(ctx), "tuned": D.dbie_query_tuned(ctx)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
                     "traffic": float(counters["hbm_bytes_per_launch"]) if counters else None,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)",
                     "kernel": "k_field32c (FP32C bulk sum with mu-tangents)",
                     "issue_ceiling": ceiling, "frac_of_issue_ceiling": achieved / ceiling if ceiling else None,
                     "flops_per_pair": FLOPS_FIELD_GRAD_TAN, "pairs_per_launch": pairs_per_launch,
                     "avg_launch_ms": kern_avg_ms, "launches": launches},
        "cpu_baseline": cpu,
        "fp32c_error_vs_fp64": accuracy,
        "wall_s": wall,
        "extras": extras,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
