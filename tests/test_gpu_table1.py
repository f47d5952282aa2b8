"""The Table 1 comparison experiment on the GPU: Low & Lou n=3, m=1, l=0.3, Phi=4pi/5, 192x192 lower
boundary, 64x64x64 test region, the five metrics of Schrijver et al. (2006) against the exact field.

The paper's own numbers come from its implementation (Nelder-Mead from its own start values, its
Eq. 15 quadrature); this one solves per point with the library's searches from lambda = 0 on the
nodal rule. The assertions are the paper's qualitative claims, not its digits: the lambda search
improves markedly on the field without it, and the field direction is recovered almost everywhere
(C_vec close to 1). The measured rows are printed next to the paper's row.
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


@pytest.fixture(scope="module")
def case():
    w = lowlou_table1()
    bd = w.boundaries[0]
    jj, ii = w.meta["bottom_idx"]
    bottom = bd.B0[:, jj, ii]
    exact = np.concatenate([bottom, w.meta["ll"].field(*w.xyz)], axis=1)
    return w, bd, bottom, exact


def test_table1_metrics(case):
    w, bd, bottom, exact = case
    paper = json.load(open(os.path.join(HERE, "golden", "paper_table1_present_dbie.json")))
    rows = {}
    runs = (("no lambda search (lambda = 0)", "fp32c", None, 0),
            ("FP32C Levenberg-Marquardt, 20 trials", "fp32c", "lm", 20),
            ("FP32C Nelder-Mead, 50 trials", "fp32c", "nm", 50))
    for name, prec, meth, bud in runs:
        ctx = D.dbie_init([dict(B0=T(bd.B0), x0=bd.x0, y0=bd.y0, h=bd.h)], T(w.xyz), precision=prec)
        lam = torch.zeros(3, w.n_points, dtype=torch.float64, device="cuda:0")
        if meth is None:
            B = D.dbie_eval_field(ctx, lam)["B"]
            conv = float("nan")
        else:
            r = D.dbie_solve_lambda(ctx, lam, method=meth, max_trials=bud, eps=1e-4)
            B = r["B"]
            conv = float((r["status"] == 0).double().mean())
        torch.cuda.synchronize()
        model = np.concatenate([bottom, B.cpu().numpy()], axis=1)
        rows[name] = oracle.schrijver_metrics(exact, model)
        rows[name]["converged"] = conv
        print(name, {k: round(v, 3) for k, v in rows[name].items()}, flush=True)
    print("paper, present DBIE", {k: paper[k] for k in ("C_vec", "C_cs", "E_n", "E_m", "eps")}, flush=True)
    base = rows[runs[0][0]]
    for name, _, meth, _ in runs[1:]:
        m = rows[name]
        assert m["C_vec"] >= 0.9, (name, m)
        assert m["C_vec"] > base["C_vec"] and m["E_n"] > base["E_n"], (name, m, base)
