"""GPU field-line and current-line tracing (dbie_trace_lines, through the C ABI) against the oracle's
RK4 tracer through its own DBIE field: the same lines point by point, the stop rule, and the context
left as it was."""
import numpy as np
import pytest
import torch

import oracle
import paper_1306_1122_amd as D
from workloads import config1

pytestmark = pytest.mark.gpu


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


@pytest.fixture(scope="module")
def case():
    rng = np.random.default_rng(77)
    w = config1()
    bd = w.boundaries[0]
    seeds = np.stack([rng.uniform(-0.6, 0.6, 12), rng.uniform(-0.6, 0.6, 12), rng.uniform(0.1, 0.6, 12)])
    lam_grid = rng.uniform(0.0, 1.5, size=(3, 3, 4, 5))
    origin, spacing = (-1.0, -1.0, 0.05), (0.5, 2.0 / 3.0, 0.5)
    box = (-0.9, -0.9, 0.05, 0.9, 0.9, 1.0)
    return bd, seeds, lam_grid, origin, spacing, box


@pytest.mark.parametrize("precision,mode,sense", [("fp64", "field", 1.0), ("fp64", "current", -1.0),
                                                  ("fp32c", "field", 1.0), ("fp32c", "current", 1.0)])
def test_lines_match_the_oracle(case, precision, mode, sense):
    bd, seeds, lam_grid, origin, spacing, box = case
    ctx = D.dbie_init([dict(B0=T(bd.B0), x0=bd.x0, y0=bd.y0, h=bd.h)], T(seeds), precision=precision)
    ds, n_steps = 0.02, 40
    out = D.dbie_trace_lines(ctx, T(lam_grid), origin, spacing, box, ds, n_steps, mode=mode, sense=sense)
    torch.cuda.synchronize()
    xyz = out["xyz"].cpu().numpy()
    cnt = out["count"].cpu().numpy()
    direction = oracle.dbie_direction(bd.B0, bd.x0, bd.y0, bd.h, lam_grid, origin, spacing,
                                      current=(mode == "current"))
    ref, rc = oracle.rk4_trace(direction, seeds, ds, n_steps, box[:3], box[3:], sense=sense)
    print(precision, mode, "points per line", cnt.tolist(), flush=True)
    assert np.array_equal(cnt, rc), (cnt, rc)
    assert cnt.max() > 5 and cnt.min() >= 1
    tol = 1e-9 if precision == "fp64" else 1e-4
    for j in range(seeds.shape[1]):
        a, b = xyz[: cnt[j], :, j], ref[: rc[j], :, j]
        assert np.max(np.abs(a - b)) <= tol, (j, np.max(np.abs(a - b)))
        assert np.all(np.isnan(xyz[cnt[j]:, :, j]))
    # the context still evaluates at its own points
    lam = T(np.full((3, seeds.shape[1]), 0.3))
    B = D.dbie_eval_field(ctx, lam)["B"].cpu().numpy()
    Bo, _ = oracle.field(bd.B0, bd.x0, bd.y0, bd.h, seeds, np.full((3, seeds.shape[1]), 0.3))
    assert np.linalg.norm(B - Bo) / np.linalg.norm(Bo) <= (1e-10 if precision == "fp64" else 1e-5)


def test_seed_outside_the_box_and_zero_steps(case):
    bd, seeds, lam_grid, origin, spacing, box = case
    s = seeds[:, :3].copy()
    s[0, 1] = 0.95   # outside x_hi
    ctx = D.dbie_init([dict(B0=T(bd.B0), x0=bd.x0, y0=bd.y0, h=bd.h)], T(s), precision="fp64")
    out = D.dbie_trace_lines(ctx, T(lam_grid), origin, spacing, box, 0.05, 10)
    cnt = out["count"].cpu().numpy()
    assert cnt[1] == 1 and cnt[0] > 1
    np.testing.assert_array_equal(out["xyz"][0].cpu().numpy(), s)
    out0 = D.dbie_trace_lines(ctx, T(lam_grid), origin, spacing, box, 0.05, 0)
    assert out0["xyz"].shape == (1, 3, 3) and np.all(out0["count"].cpu().numpy() == 1)
    with pytest.raises(D.DbieError, match="z_lo"):
        D.dbie_trace_lines(ctx, T(lam_grid), origin, spacing, (-1, -1, 0.0, 1, 1, 1), 0.05, 3)
    with pytest.raises(D.DbieError, match="sense"):
        D.dbie_trace_lines(ctx, T(lam_grid), origin, spacing, box, 0.05, 3, sense=0.5)


def test_lines_through_the_element_field_and_several_magnetograms():
    """Tracing in a context with 9-node elements (Eq. 15, G = 3) and two magnetograms: each line
    follows the oracle's element field of its own magnetogram."""
    rng = np.random.default_rng(78)
    mags = [(rng.normal(size=(3, 15, 17)), -1.0, -1.0, 0.125), (rng.normal(size=(3, 11, 13)), 0.5, 0.0, 0.1)]
    seeds, seg = [], [0]
    for B0, x0, y0, h in mags:
        ny, nx = B0.shape[1:]
        s = np.stack([rng.uniform(x0 + 0.3, x0 + (nx - 1) * h - 0.3, 4), rng.uniform(y0 + 0.3, y0 + (ny - 1) * h - 0.3, 4),
                      rng.uniform(0.2, 0.6, 4)])
        seeds.append(s)
        seg.append(seg[-1] + 4)
    seeds = np.concatenate(seeds, axis=1)
    lam_grid = np.full((3, 1, 1, 1), 0.4)
    box = (-2.0, -2.0, 0.05, 3.0, 3.0, 2.0)
    ctx = D.dbie_init([dict(B0=T(B0), x0=x0, y0=y0, h=h) for B0, x0, y0, h in mags], T(seeds), seg=seg,
                      precision="fp64", quad_points=3)
    out = D.dbie_trace_lines(ctx, T(lam_grid), (0, 0, 0), (1, 1, 1), box, 0.03, 15)
    torch.cuda.synchronize()
    xyz, cnt = out["xyz"].cpu().numpy(), out["count"].cpu().numpy()
    for b, (B0, x0, y0, h) in enumerate(mags):
        def direction(p, B0=B0, x0=x0, y0=y0, h=h):
            lam = np.full(p.shape, 0.4)
            B, _ = oracle.field_quad9(B0, x0, y0, h, p, lam, G=3)
            return B / np.sqrt(np.sum(B * B, axis=0))
        s0, s1 = seg[b], seg[b + 1]
        ref, rc = oracle.rk4_trace(direction, seeds[:, s0:s1], 0.03, 15, box[:3], box[3:])
        assert np.array_equal(cnt[s0:s1], rc), (b, cnt[s0:s1], rc)
        for j in range(s1 - s0):
            k = rc[j]
            assert np.max(np.abs(xyz[:k, :, s0 + j] - ref[:k, :, j])) <= 1e-9, (b, j)
