"""GPU adjoint (dbie_grad) and the torch.autograd.Function against the oracle, finite differences
and the dot-product test."""
import numpy as np
import pytest
import torch

import oracle
import paper_1306_1122_amd as D
from workloads import config2, config3

pytestmark = pytest.mark.gpu


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def case(seed=31, nx=23, ny=19, n=400, h=0.5):
    rng = np.random.default_rng(seed)
    B0 = rng.normal(size=(3, ny, nx)).astype(np.float32).astype(np.float64)
    x0, y0 = -1.0, 2.0
    xyz = np.stack([rng.uniform(x0, x0 + nx * h, n), rng.uniform(y0, y0 + ny * h, n), rng.uniform(0.4 * h, 8 * h, n)])
    lam = rng.uniform(0.1, 1.2, size=(3, n))
    gB = rng.normal(size=(3, n))
    gdB = rng.normal(size=(9, n))
    return B0, x0, y0, h, xyz, lam, gB, gdB


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32c", 1e-5)])
def test_grad_matches_oracle(precision, tol):
    B0, x0, y0, h, xyz, lam, gB, gdB = case()
    ctx = D.dbie_init([dict(B0=T(B0), x0=x0, y0=y0, h=h)], T(xyz), precision=precision)
    r = D.dbie_grad(ctx, T(lam), gB=T(gB), gdB=T(gdB), want_resid_jac=True)
    torch.cuda.synchronize()
    gB0_ref, glam_ref, _ = oracle.vjp(B0, x0, y0, h, xyz, lam, gB, gdB)
    # points down to 0.4 h: the FP32C adjoint sums their near pairs in FP64
    assert rel(r["gB0"].cpu().numpy().reshape(3, *B0.shape[1:]), gB0_ref) <= tol
    assert rel(r["glambda"].cpu(), glam_ref) <= tol
    B, dB, tan = oracle.field(B0, x0, y0, h, xyz, lam, tangents=True)
    jac = oracle.residual_jacobian(B, dB, tan, h)
    assert rel(r["resid_jac"].cpu(), jac) <= 10 * tol


@pytest.mark.parametrize("sizes", [((24, 17), (40, 9)), ((24, 17), (21, 9))])
def test_fp32c_adjoint_row_quads_and_strided_outputs_match_the_oracle(sizes):
    """When every magnetogram row is a multiple of four pixels long (24 and 40), each lane of the FP32C
    transpose owns four consecutive pixels of one row and forms the point's dy terms once for them;
    with a 21-pixel row in the batch the outputs are 256 apart. Both match the oracle's transpose,
    with points down to z = 0.4 (near-field pairs) and over the magnetogram edges."""
    rng = np.random.default_rng(37)
    bds, xyzs, seg, B0s = [], [], [0], []
    for nx, ny in sizes:
        n = 450
        B0 = rng.normal(size=(3, ny, nx)).astype(np.float32).astype(np.float64)
        B0s.append(B0)
        bds.append(dict(B0=T(B0), x0=0.0, y0=0.0, h=1.0))
        xyzs.append(np.stack([rng.uniform(-1, nx, n), rng.uniform(-1, ny, n), rng.uniform(0.4, 8.0, n)]))
        seg.append(seg[-1] + n)
    xyz = np.concatenate(xyzs, axis=1)
    n = xyz.shape[1]
    lam = rng.uniform(-0.6, 0.6, size=(3, n))
    gB, gdB = rng.normal(size=(3, n)), rng.normal(size=(9, n))
    ctx = D.dbie_init(bds, T(xyz), seg=seg, precision="fp32c")
    r = D.dbie_grad(ctx, T(lam), gB=T(gB), gdB=T(gdB))
    torch.cuda.synchronize()
    parts = D.split_gB0(ctx, r["gB0"])
    for b in range(2):
        s0, s1 = seg[b], seg[b + 1]
        ref, _, _ = oracle.vjp(B0s[b], 0.0, 0.0, 1.0, xyz[:, s0:s1], lam[:, s0:s1], gB[:, s0:s1], gdB[:, s0:s1])
        e = rel(parts[b].cpu(), ref)
        print("adjoint", sizes, b, "%.2e" % e, flush=True)
        assert e <= 1e-5, (sizes, b)


def test_fp32c_adjoint_on_batched_boundaries_and_determinism():
    rng = np.random.default_rng(35)
    bds, xyzs, seg, B0s = [], [], [0], []
    for nx, ny, n in ((21, 17, 500), (40, 9, 300)):
        B0 = rng.normal(size=(3, ny, nx)).astype(np.float32).astype(np.float64)
        B0s.append(B0)
        bds.append(dict(B0=T(B0), x0=0.0, y0=0.0, h=1.0))
        xyzs.append(np.stack([rng.uniform(0, nx, n), rng.uniform(0, ny, n), rng.uniform(0.5, 6.0, n)]))
        seg.append(seg[-1] + n)
    xyz = np.concatenate(xyzs, axis=1)
    n = xyz.shape[1]
    lam = rng.uniform(0.0, 0.5, size=(3, n))
    gB = rng.normal(size=(3, n))
    gdB = rng.normal(size=(9, n))
    ctx = D.dbie_init(bds, T(xyz), seg=seg, precision="fp32c")
    r1 = D.dbie_grad(ctx, T(lam), gB=T(gB), gdB=T(gdB))
    r2 = D.dbie_grad(ctx, T(lam), gB=T(gB), gdB=T(gdB))
    assert torch.equal(r1["gB0"], r2["gB0"]) and torch.equal(r1["glambda"], r2["glambda"])
    parts = D.split_gB0(ctx, r1["gB0"])
    for b in range(2):
        s0, s1 = seg[b], seg[b + 1]
        ref, _, _ = oracle.vjp(B0s[b], 0.0, 0.0, 1.0, xyz[:, s0:s1], lam[:, s0:s1], gB[:, s0:s1], gdB[:, s0:s1])
        assert rel(parts[b].cpu(), ref) <= 1e-5, b


def test_dot_product_on_the_gpu():
    B0, x0, y0, h, xyz, lam, gB, gdB = case(seed=32)
    x = np.random.default_rng(5).normal(size=B0.shape)
    cx = D.dbie_init([dict(B0=T(x), x0=x0, y0=y0, h=h)], T(xyz), precision="fp64")
    out = D.dbie_eval_field(cx, T(lam))
    lhs = float((out["B"] * T(gB)).sum() + (out["dB"] * T(gdB)).sum())
    r = D.dbie_grad(cx, T(lam), gB=T(gB), gdB=T(gdB))
    rhs = float((r["gB0"].view(3, *B0.shape[1:]) * T(x)).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_lambda_gradient_against_differences_on_the_large_grid():
    """The 256x256 magnetogram of the gradient workload, 1e3 seeded random interior points: the
    lambda gradient from the tangents against central differences of the GPU field in mu."""
    w = config3(nz=4)
    bd = w.boundaries[0]
    rng = np.random.default_rng(33)
    idx = rng.choice(w.n_points, 1000, replace=False)
    xyz = w.xyz[:, idx].copy()
    xyz[2] = rng.uniform(1.0, 128.0, 1000)
    lam = rng.uniform(0.01, 4 * np.pi / 256, size=(3, 1000))
    gB = rng.normal(size=(3, 1000))
    gdB = rng.normal(size=(9, 1000))
    ctx = D.dbie_init([dict(B0=T(bd.B0), x0=bd.x0, y0=bd.y0, h=bd.h)], T(xyz), precision="fp64")
    g = D.dbie_grad(ctx, T(lam), gB=T(gB), gdB=T(gdB), want_gB0=False)["glambda"].cpu().numpy()
    mu = lam * lam
    fd = np.zeros_like(lam)
    for p in range(3):
        d = 1e-6 * mu[p]
        mp, mm = mu.copy(), mu.copy()
        mp[p] += d
        mm[p] -= d
        op = D.dbie_eval_field(ctx, T(np.sqrt(mp)))
        om = D.dbie_eval_field(ctx, T(np.sqrt(mm)))
        Lp = (op["B"] * T(gB)).sum(0) + (op["dB"] * T(gdB)).sum(0)
        Lm = (om["B"] * T(gB)).sum(0) + (om["dB"] * T(gdB)).sum(0)
        fd[p] = ((Lp - Lm) / (2 * T(d))).cpu().numpy() * 2 * lam[p]
    assert rel(g, fd) <= 1e-6
    # and the oracle's gradient on a subset
    sub = slice(0, 40)
    _, glam_ref, _ = oracle.vjp(bd.B0, bd.x0, bd.y0, bd.h, xyz[:, sub], lam[:, sub], gB[:, sub], gdB[:, sub])
    assert rel(g[:, sub], glam_ref) <= 1e-10


def test_autograd_function():
    B0, x0, y0, h, xyz, lam, gB, gdB = case(seed=34, n=200)
    B0t = T(B0).requires_grad_(True)
    lamt = T(lam).requires_grad_(True)
    B, dB = D.dbie_field(B0t, lamt, T(xyz), x0, y0, h, precision="fp64")
    loss = (B * T(gB)).sum() + (dB * T(gdB)).sum()
    loss.backward()
    gB0_ref, glam_ref, _ = oracle.vjp(B0, x0, y0, h, xyz, lam, gB, gdB)
    assert rel(B0t.grad.cpu(), gB0_ref) <= 1e-10
    assert rel(lamt.grad.cpu(), glam_ref) <= 1e-10


@pytest.mark.parametrize("shape", [(600, 40, 2.5, 2.7), (1001, 31, 2.9, 3.14), (2001, 16, 3.0, 3.14), (4001, 8, 3.0, 3.14)])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32c", 1e-5)])
def test_grad_at_large_lambda_matches_oracle(precision, tol, shape):
    """|lambda| h up to 2.7 over a 600 x 40 magnetogram, and up to the cap pi / h over a 1001 x 31 one
    (phases up to ~3100 radians: beyond the hardware sin/cos range, so the FP32C adjoint reduces the
    phase first) against the oracle's transpose."""
    nx, ny, lo, hi = shape
    rng = np.random.default_rng(36 + nx)
    n = 160
    B0 = rng.normal(size=(3, ny, nx)).astype(np.float32).astype(np.float64)
    xyz = np.stack([rng.uniform(0, nx, n), rng.uniform(0, ny, n), rng.uniform(0.5, 20, n)])
    lam = rng.uniform(lo, hi, size=(3, n)) * rng.choice([-1.0, 1.0], size=(3, n))
    gB, gdB = rng.normal(size=(3, n)), rng.normal(size=(9, n))
    ctx = D.dbie_init([dict(B0=T(B0), x0=0.0, y0=0.0, h=1.0)], T(xyz), precision=precision)
    r = D.dbie_grad(ctx, T(lam), gB=T(gB), gdB=T(gdB))
    torch.cuda.synchronize()
    gB0_ref, glam_ref, _ = oracle.vjp(B0, 0.0, 0.0, 1.0, xyz, lam, gB, gdB)
    e = rel(r["gB0"].cpu().numpy().reshape(3, ny, nx), gB0_ref)
    print("large-lambda adjoint", precision, nx, ny, "%.2e" % e, flush=True)
    assert e <= tol


@pytest.mark.parametrize("precision", ["fp32c", "fp64"])
def test_full_size_adjoint_sampled(precision):
    """The benchmark's adjoint: the 128x128 bipole magnetogram and all 2^20 points of its grid, one
    trial, seeded upstream gradients; eight pixels (the four corners, edges, the interior) against
    the oracle's sum over every point."""
    w = config2()
    bd = w.boundaries[0]
    rng = np.random.default_rng(36)
    gB = rng.normal(size=(3, w.n_points))
    gdB = rng.normal(size=(9, w.n_points))
    ctx = D.dbie_init([dict(B0=T(bd.B0), x0=bd.x0, y0=bd.y0, h=bd.h)], T(w.xyz), precision=precision)
    r = D.dbie_grad(ctx, T(w.lam), gB=T(gB), gdB=T(gdB), want_glambda=False)
    torch.cuda.synchronize()
    nx = ny = 128
    pix = np.array([0, nx - 1, (ny - 1) * nx, nx * ny - 1, 5, 3 * nx, 64 * nx + 64, int(rng.integers(nx * ny))])
    ref, _, _ = oracle.vjp(bd.B0, bd.x0, bd.y0, bd.h, w.xyz, w.lam, gB, gdB, pixels=pix)
    got = r["gB0"].view(3, -1)[:, pix].cpu().numpy()
    err = rel(got, ref)
    print("full-size adjoint", precision, f"{err:.1e}", flush=True)
    assert err <= (1e-10 if precision == "fp64" else 1e-5)


def test_field_object_matches_the_calls():
    """Field wraps a context: its methods return what the free functions return on the same
    context, bitwise."""
    B0, x0, y0, h, xyz, lam, gB, gdB = case(seed=37, n=300)
    f = D.Field([dict(B0=T(B0), x0=x0, y0=y0, h=h)], T(xyz), precision="fp32c")
    a = f.eval(T(lam), want_tan=True)
    b = D.dbie_eval_field(f.ctx, T(lam), want_tan=True)
    for k in ("B", "dB", "fg", "tan"):
        assert torch.equal(a[k], b[k]), k
    ga = f.grad(T(lam), gB=T(gB), gdB=T(gdB))
    gb = D.dbie_grad(f.ctx, T(lam), gB=T(gB), gdB=T(gdB))
    assert torch.equal(ga["gB0"], gb["gB0"]) and torch.equal(ga["glambda"], gb["glambda"])
    sa = f.solve(T(lam), method="lm", max_trials=4, fp64_accept=False)
    sb = D.dbie_solve_lambda(f.ctx, T(lam), method="lm", max_trials=4, fp64_accept=False)
    for k in ("lam", "status", "trials"):
        assert torch.equal(sa[k], sb[k]), k
    f.close()
