"""A caller-owned workspace (dbie_workspace_bytes / dbie_set_workspace): every call gives the same
results, bitwise, with the library's own work memory and with the caller's; a call that needs more
than one trial's sums is refused; going back to library memory works."""
import numpy as np
import pytest
import torch

import paper_1306_1122_amd as D

pytestmark = pytest.mark.gpu


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def run_all(ctx, lam, n):
    out = {}
    e = D.dbie_eval_field(ctx, T(lam), want_tan=True)
    out.update({"eval_" + k: v.clone() for k, v in e.items()})
    sc = D.dbie_eval_field_scalar(ctx, T(lam[:1]), want_tan=True)
    out.update({"scalar_" + k: v.clone() for k, v in sc.items()})
    for m in ("nm", "lm"):
        r = D.dbie_solve_lambda(ctx, T(np.abs(lam) * 0.3), method=m, max_trials=8, fp64_accept=True)
        out.update({m + "_" + k: v.clone() for k, v in r.items()})
    g = D.dbie_grad(ctx, T(lam), gB=T(np.ones((3, n))), gdB=T(np.ones((9, n))), want_resid_jac=True)
    out.update({"grad_" + k: v.clone() for k, v in g.items() if v is not None})
    lg = T(np.full((3, 1, 1, 1), 0.05))
    tr = D.dbie_trace_lines(ctx, lg, (0, 0, 0), (1, 1, 1), (0.0, 0.0, 0.3, 40.0, 36.0, 30.0), 0.5, 6)
    out.update({"trace_" + k: v.clone() for k, v in tr.items()})
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("precision,G", [("fp32c", 0), ("fp64", 0), ("fp32c", 2)])
def test_results_identical_with_a_caller_workspace(precision, G):
    rng = np.random.default_rng(31)
    nx, ny, n = 41, 37, 3000
    B0 = rng.normal(size=(3, ny, nx)).astype(np.float32).astype(np.float64)
    xyz = np.stack([rng.uniform(0, nx - 1, n), rng.uniform(0, ny - 1, n), rng.uniform(0.4, 20, n)])
    lam = rng.uniform(-0.3, 0.3, size=(3, n))
    ctx = D.dbie_init([dict(B0=T(B0), x0=0.0, y0=0.0, h=1.0)], T(xyz), precision=precision, quad_points=G)
    ref = run_all(ctx, lam, n)
    nbytes = D.dbie_workspace_bytes(ctx)
    assert nbytes > 0
    with pytest.raises(D.DbieError, match="smaller"):
        D.dbie_set_workspace(ctx, torch.empty(nbytes - 256, dtype=torch.uint8, device="cuda:0"))
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    D.dbie_set_workspace(ctx, ws)
    got = run_all(ctx, lam, n)
    for k in ref:
        assert torch.equal(ref[k], got[k]) or (torch.isnan(ref[k]).any() and torch.equal(
            torch.nan_to_num(ref[k], nan=-7.0), torch.nan_to_num(got[k], nan=-7.0))), k
    with pytest.raises(D.DbieError, match="workspace"):
        D.dbie_eval_field(ctx, T(np.stack([lam, lam])))
    D.dbie_set_workspace(ctx, None)
    two = D.dbie_eval_field(ctx, T(np.stack([lam, lam])), want_tan=True)
    assert torch.equal(two["B"][0], ref["eval_B"]) and torch.equal(two["B"][1], ref["eval_B"])
