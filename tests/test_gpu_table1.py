"""The Table 1 comparison experiment on the GPU: Low & Lou n=3, m=1, l=0.3, Phi=4pi/5, 192x192 lower
boundary, 64x64x64 test region, the five metrics of Schrijver et al. (2006) against the exact field.

The paper's own numbers come from its implementation (Nelder-Mead from start values it does not
state, its Eq. 15 quadrature); this one solves per point with the library's searches from
lambda = 0 on the nodal rule. The metrics against the paper's row are reported, not gated (parity
unpinned: the case's grid mapping and the search's start are readings). Gated: what the search
itself guarantees (the residual Phi = f^2 + g^2 at lambda* does not exceed its value at the start,
beyond FP32 rounding, and falls on average), finite metrics, and the field direction recovered
almost everywhere (C_vec >= 0.95) by the derivative-free search and by the field at lambda = 0.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1306_1122_amd as D
from workloads import lowlou_table1

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(__file__)


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


@pytest.fixture(scope="module", params=["region", "boundary"])
def case(request):
    w = lowlou_table1(mapping=request.param)
    bd = w.boundaries[0]
    jj, ii = w.meta["bottom_idx"]
    bottom = bd.B0[:, jj, ii]
    exact = np.concatenate([bottom, w.meta["ll"].field(*w.xyz)], axis=1)
    return w, bd, bottom, exact


def test_table1_metrics(case):
    w, bd, bottom, exact = case
    paper = json.load(open(os.path.join(HERE, "golden", "paper_table1_present_dbie.json")))
    rows, phis = {}, {}
    runs = (("no lambda search (lambda = 0)", None, 0),
            ("FP32C Levenberg-Marquardt, 20 trials", "lm", 20),
            ("FP32C Nelder-Mead, 50 trials", "nm", 50))
    ctx = D.dbie_init([dict(B0=T(bd.B0), x0=bd.x0, y0=bd.y0, h=bd.h)], T(w.xyz), precision="fp32c")
    for name, meth, bud in runs:
        lam = torch.zeros(3, w.n_points, dtype=torch.float64, device="cuda:0")
        if meth is None:
            # the start, evaluated in FP64 like the searches' accepted results
            c64 = D.dbie_init([dict(B0=T(bd.B0), x0=bd.x0, y0=bd.y0, h=bd.h)], T(w.xyz), precision="fp64")
            out = D.dbie_eval_field(c64, lam)
            B, fg = out["B"], out["fg"]
            conv = float("nan")
        else:
            r = D.dbie_solve_lambda(ctx, lam, method=meth, max_trials=bud, eps=1e-4)
            B, fg = r["B"], r["fg"]
            conv = float((r["status"] == 0).double().mean())
        torch.cuda.synchronize()
        model = np.concatenate([bottom, B.cpu().numpy()], axis=1)
        rows[name] = oracle.schrijver_metrics(exact, model)
        rows[name]["converged"] = conv
        fgn = fg.cpu().numpy()
        phis[name] = fgn[0] ** 2 + fgn[1] ** 2
        print(w.name, name, {k: round(v, 3) for k, v in rows[name].items()},
              "mean Phi %.4f" % float(np.nanmean(phis[name])), flush=True)
    print("paper, present DBIE", {k: paper[k] for k in ("C_vec", "C_cs", "E_n", "E_m", "eps")}, flush=True)
    phi0 = phis[runs[0][0]]
    for name, meth, _ in runs[1:]:
        m = rows[name]
        assert all(np.isfinite(v) for k, v in m.items() if k != "converged"), (name, m)
        ok = np.isfinite(phi0)
        # the search keeps its best trial and starts at lambda = 0 (FP32C decisions, FP64 result)
        assert np.mean(phis[name][ok] <= phi0[ok] * (1 + 1e-3) + 1e-9) >= 0.999, name
        assert np.nanmean(phis[name]) < np.nanmean(phi0), name
    assert rows[runs[0][0]]["C_vec"] >= 0.95 and rows[runs[2][0]]["C_vec"] >= 0.95
