"""The FP64 path near full double precision: its branch-free sin/cos (reduced by pi with k from one
FMA), the refined hardware 1/sqrt and the folded -3 leave the results within rounding of the
oracle's compensated sums, far inside the 1e-10 parity bar. A bar of 1e-12 catches a sin/cos, 1/sqrt
or reduction that lost a few digits, which the parity bar would let through.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1306_1122_amd as D

pytestmark = pytest.mark.gpu

BAR = 1e-12


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.mark.parametrize("case", ["moderate", "large_phase", "lowest_layers"])
def test_fp64_results_within_rounding_of_the_oracle(case):
    rng = np.random.default_rng({"moderate": 41, "large_phase": 42, "lowest_layers": 43}[case])
    if case == "large_phase":
        # |lambda| h up to 2.9 on a 300-pixel-wide magnetogram: |lambda r| up to ~900, k up to ~290
        nx, ny, n = 300, 24, 160
        lam = rng.uniform(2.0, 2.9, size=(3, n)) * rng.choice([-1.0, 1.0], size=(3, n))
    else:
        nx, ny, n = 48, 40, 500
        lam = rng.uniform(-0.5, 0.5, size=(3, n))
    B0 = rng.normal(size=(3, ny, nx))
    z = rng.uniform(0.3, 2.0, n) if case == "lowest_layers" else rng.uniform(0.3, 30.0, n)
    xyz = np.stack([rng.uniform(0, nx - 1, n), rng.uniform(0, ny - 1, n), z])
    ctx = D.dbie_init([dict(B0=T(B0), x0=0.0, y0=0.0, h=1.0)], T(xyz), precision="fp64")
    out = D.dbie_eval_field(ctx, T(lam), want_tan=True)
    torch.cuda.synchronize()
    B, dB, tan = oracle.field(B0, 0.0, 0.0, 1.0, xyz, lam, tangents=True)
    errs = {k: rel(out[k].cpu(), r) for k, r in (("B", B), ("dB", dB), ("tan", tan))}
    print(case, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, e in errs.items():
        assert e <= BAR, (case, k, e)


@pytest.mark.parametrize("case", ["moderate", "large_phase"])
def test_fp64_adjoint_within_rounding_of_the_oracle(case):
    """dbie_grad in an FP64 context (the same sin/cos and 1/sqrt in the pixel-output transpose):
    dL/dB0 and dL/dlambda against the oracle's VJP at the same bar."""
    rng = np.random.default_rng({"moderate": 51, "large_phase": 52}[case])
    if case == "large_phase":
        nx, ny, n = 300, 24, 120
        lam = rng.uniform(2.0, 2.9, size=(3, n)) * rng.choice([-1.0, 1.0], size=(3, n))
    else:
        nx, ny, n = 40, 36, 300
        lam = rng.uniform(-0.5, 0.5, size=(3, n))
    B0 = rng.normal(size=(3, ny, nx))
    xyz = np.stack([rng.uniform(0, nx - 1, n), rng.uniform(0, ny - 1, n), rng.uniform(0.3, 20.0, n)])
    gB, gdB = rng.normal(size=(3, n)), rng.normal(size=(9, n))
    ctx = D.dbie_init([dict(B0=T(B0), x0=0.0, y0=0.0, h=1.0)], T(xyz), precision="fp64")
    g = D.dbie_grad(ctx, T(lam), gB=T(gB), gdB=T(gdB))
    torch.cuda.synchronize()
    gB0_ref, glam_ref, _ = oracle.vjp(B0, 0.0, 0.0, 1.0, xyz, lam, gB, gdB)
    errs = dict(gB0=rel(g["gB0"].cpu().numpy().reshape(gB0_ref.shape), gB0_ref),
                glam=rel(g["glambda"].cpu(), glam_ref))
    print(case, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, e in errs.items():
        assert e <= BAR, (case, k, e)
