"""Seeded random contexts with several magnetograms (random sizes, some without points):
  * evaluation with two lambda trials per launch and the single-lambda form, nodal rule or 9-node
    elements, both paths, against the oracle;
  * the lambda search (Nelder-Mead and LM; FP64, and FP32C with the FP64 acceptance): every point
    marked CONVERGED satisfies max(f, g) <= eps when the oracle re-evaluates it at the returned lambda,
    the returned B and (f, g) match the oracle there, statuses and trial counts stay in range.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1306_1122_amd as D

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32c": 1e-5}


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def eval_case(seed):
    rng = np.random.default_rng(9000 + seed)
    G = int(rng.choice([0, 0, 2, 3]))
    bds, xyzs, npts = [], [], []
    for _ in range(int(rng.integers(1, 5))):
        if G:
            nx, ny = (2 * int(rng.integers(1, 20)) + 1 for _ in range(2))
        else:
            nx, ny = (int(rng.integers(1, 40)) for _ in range(2))
        h = float(np.exp(rng.uniform(np.log(0.3), np.log(2.0))))
        x0, y0 = (float(v) for v in rng.uniform(-5, 5, 2))
        n = int(rng.choice([0, int(rng.integers(1, 300))]))
        B0 = rng.normal(size=(3, ny, nx))
        xyzs.append(np.stack([rng.uniform(x0 - 2 * h, x0 + (nx + 1) * h, n),
                              rng.uniform(y0 - 2 * h, y0 + (ny + 1) * h, n),
                              h * np.exp(rng.uniform(np.log(0.3), np.log(20.0), n))]))
        bds.append((B0, x0, y0, h))
        npts.append(n)
    return G, bds, npts, xyzs


@pytest.mark.parametrize("seed", [s for s in range(24) if sum(eval_case(s)[2]) > 0])
def test_random_context_evaluation(seed):
    G, bds, npts, xyzs = eval_case(seed)
    rng = np.random.default_rng(9500 + seed)
    xyz = np.concatenate(xyzs, axis=1)
    N = xyz.shape[1]
    seg = np.concatenate([[0], np.cumsum(npts)])
    hs = np.concatenate([np.full(n, bd[3]) for bd, n in zip(bds, npts)])
    lam2 = np.stack([rng.uniform(-1.0, 1.0, size=(3, N)) / hs for _ in range(2)])
    lsc = lam2[0, 0]
    for prec in ("fp64", "fp32c"):
        ctx = D.dbie_init([dict(B0=T(B0), x0=x0, y0=y0, h=h) for (B0, x0, y0, h) in bds], T(xyz), seg=list(seg),
                          precision=prec, quad_points=G)
        out = D.dbie_eval_field(ctx, T(lam2), want_tan=True)
        sc = D.dbie_eval_field_scalar(ctx, T(lsc), want_tan=True)
        torch.cuda.synchronize()
        for b, (B0, x0, y0, h) in enumerate(bds):
            s, e = seg[b], seg[b + 1]
            if s == e:
                continue

            def ref(lam):
                if G:
                    return oracle.field_quad9(B0, x0, y0, h, xyz[:, s:e], lam, G=G, tangents=True)
                return oracle.field(B0, x0, y0, h, xyz[:, s:e], lam, tangents=True)

            for t in range(2):
                for k, r in zip(("B", "dB", "tan"), ref(lam2[t][:, s:e])):
                    assert rel(out[k][t][:, s:e].cpu(), r) <= TOL[prec], (prec, b, t, k)
            for k, r in zip(("B", "dB", "tan"), ref(np.repeat(lsc[None, s:e], 3, axis=0))):
                assert rel(sc[k][:, s:e].cpu(), r) <= TOL[prec], (prec, b, "scalar", k)
        ctx.close()


def solve_case(seed):
    rng = np.random.default_rng(11000 + seed)
    bds, xyzs, npts = [], [], []
    for _ in range(int(rng.integers(1, 4))):
        nx, ny = (int(rng.integers(4, 36)) for _ in range(2))
        h = float(np.exp(rng.uniform(np.log(0.5), np.log(2.0))))
        n = int(rng.integers(0, 200))
        # one sheared bipole and a little noise, so that some points can converge
        yy, xx = np.mgrid[0:ny, 0:nx]
        cx, cy, sg = rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(2, 8)
        Bz = (np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2 * sg ** 2))
              - np.exp(-((xx - cx - 3) ** 2 + (yy - cy) ** 2) / (2 * sg ** 2)))
        B0 = np.stack([0.3 * np.gradient(Bz, axis=0), -0.3 * np.gradient(Bz, axis=1), Bz]) + 0.01 * rng.normal(size=(3, ny, nx))
        xyzs.append(np.stack([rng.uniform(0, nx * h, n), rng.uniform(0, ny * h, n), h * rng.uniform(0.5, 8.0, n)]))
        bds.append((B0, 0.0, 0.0, h))
        npts.append(n)
    return bds, npts, xyzs, float(rng.choice([1e-2, 5e-2, 0.2]))


@pytest.mark.parametrize("seed", [s for s in range(12) if sum(solve_case(s)[1]) > 0])
def test_random_context_search(seed):
    bds, npts, xyzs, eps = solve_case(seed)
    xyz = np.concatenate(xyzs, axis=1)
    N = xyz.shape[1]
    seg = np.concatenate([[0], np.cumsum(npts)])
    for prec in ("fp64", "fp32c"):
        ctx = D.dbie_init([dict(B0=T(B0), x0=x0, y0=y0, h=h) for (B0, x0, y0, h) in bds], T(xyz), seg=list(seg),
                          precision=prec)
        for meth, budget in (("nm", 30), ("lm", 10)):
            r = D.dbie_solve_lambda(ctx, T(np.zeros((3, N))), method=meth, max_trials=budget, eps=eps, fp64_accept=True)
            torch.cuda.synchronize()
            lam, st, tr = r["lam"].cpu().numpy(), r["status"].cpu().numpy(), r["trials"].cpu().numpy()
            Bg, fgg = r["B"].cpu().numpy(), r["fg"].cpu().numpy()
            assert np.all((st >= 0) & (st <= 4)) and tr.min() >= 1 and tr.max() <= budget
            for b, (B0, x0, y0, h) in enumerate(bds):
                s, e = seg[b], seg[b + 1]
                if s == e:
                    continue
                B, dB = oracle.field(B0, x0, y0, h, xyz[:, s:e], lam[:, s:e])[:2]
                res = oracle.residuals(B, dB, h)
                conv = st[s:e] == oracle.ST_CONVERGED
                assert np.all(np.maximum(res["f"], res["g"])[conv] <= eps * (1 + 1e-9)), (prec, meth, b)
                # B and (f, g) at lambda* come from an FP64 evaluation in both contexts
                assert rel(Bg[:, s:e], B) <= TOL["fp64"], (prec, meth, b)
                ok = np.isfinite(res["f"]) & np.isfinite(res["g"])
                assert np.abs(fgg[0, s:e][ok] - res["f"][ok]).max(initial=0.0) <= 1e-6, (prec, meth, b)
                assert np.abs(fgg[1, s:e][ok] - res["g"][ok]).max(initial=0.0) <= 1e-6, (prec, meth, b)
        ctx.close()
