"""Shared parity checks of GPU outputs against the oracle (imported by the GPU tests).

Relative L2 over the compared points (the bar of each path), and a pointwise bound for every output
of every point, |x_gpu - x_ref| <= c u S, where S is the row's sum of absolute terms
(oracle.field(..., absolute=True)) and u the path's unit roundoff, with c = c0 + 4 t^2 and t the
point's largest phase max_p |lambda_p| r_max in radians: c0 = 512 for FP64 (recursive sums of
128-term tiles and of the tile partials, sin/cos and 1/sqrt to a few ulp, the oracle's own rounding),
c0 = 1024 for FP32C (partial sums of up to 512 FP32 terms, each term to ~10 u); 4 t^2 covers the rounding of
the distance r (relative u, so a phase error t u) times the kernel's sensitivity to the phase (~t),
in both the path and the oracle. f and g are compared where they are well conditioned: |J| and
|div B| at least 1e-2 of |grad B| (no cancellation), f >= 1e-2, and, where the sums of absolute
terms are known, |B| at least 1e-2 of its own (f and g divide by |B| (Eqs. 8 and 9), so a point where
the field cancels carries the FP32 rounding of its terms into both).
"""
import numpy as np

import oracle

UNIT = {"fp64": 2.0 ** -53, "fp32c": 2.0 ** -24}
TOL = {"fp64": 1e-10, "fp32c": 1e-5}


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_phase(bd, xyz, lam):
    ny, nx = bd.B0.shape[1:]
    u = (xyz[0] - bd.x0) / bd.h
    v = (xyz[1] - bd.y0) / bd.h
    dx = np.maximum(np.abs(u), np.abs(nx - 1 - u))
    dy = np.maximum(np.abs(v), np.abs(ny - 1 - v))
    rmax = bd.h * np.sqrt(dx * dx + dy * dy + (xyz[2] / bd.h) ** 2)
    return np.max(np.abs(lam), axis=0) * rmax


def check_pointwise(out, ref, absref, precision, tmax, label):
    """Asserts the pointwise bound for every row in ref; returns the largest err / (u S) seen."""
    c = (512.0 if precision == "fp64" else 1024.0) + 4.0 * tmax ** 2
    worst = 0.0
    for k in ref:
        err = np.abs(np.asarray(out[k], np.float64) - ref[k])
        scale = UNIT[precision] * absref[k]
        bad = ~(err <= scale * c[None, :])
        worst = max(worst, float(np.max(err / np.maximum(scale, 1e-300))))
        assert not np.any(bad), (label, k, int(np.count_nonzero(bad)))
    return worst


def well_conditioned_fg(B, dB, res, aB=None):
    """Points where f and g are well conditioned; aB: the sums of absolute terms of B, if known."""
    J = np.stack([dB[7] - dB[5], dB[2] - dB[6], dB[3] - dB[1]])
    nJ, nG = np.linalg.norm(J, axis=0), np.linalg.norm(dB, axis=0)
    D_ = np.abs(dB[0] + dB[4] + dB[8])
    okf = np.isfinite(res["f"]) & (nJ >= 1e-2 * nG) & (res["f"] >= 1e-2)
    okg = np.isfinite(res["g"]) & (D_ >= 1e-2 * nG)
    if aB is not None:
        okB = np.linalg.norm(B, axis=0) >= 1e-2 * np.linalg.norm(aB, axis=0)
        okf, okg = okf & okB, okg & okB
    return okf, okg


def check_sampled(got, bd, xyz, lam, precision, label, fg=None, tol=None):
    """got: dict of numpy rows at the sampled points (B [3, n], dB [9, n], optionally tan [12, n]);
    fg [2, n] optional. Asserts relative L2 <= the path's bar, the pointwise bound, and f, g at the
    bar where well conditioned. Returns the errors."""
    tol = TOL[precision] if tol is None else tol
    tangents = "tan" in got
    B, dB, tan, aB, adB, atan = oracle.field(bd.B0, bd.x0, bd.y0, bd.h, xyz, lam, tangents=True, absolute=True)
    ref, absref = dict(B=B, dB=dB), dict(B=aB, dB=adB)
    if tangents:
        ref["tan"], absref["tan"] = tan, atan
    errs = {k: rel(got[k], ref[k]) for k in ref}
    errs["pointwise"] = check_pointwise(got, ref, absref, precision, max_phase(bd, xyz, lam), label)
    if fg is not None:
        res = oracle.residuals(B, dB, bd.h)
        okf, okg = well_conditioned_fg(B, dB, res, aB)
        errs["f"] = rel(fg[0][okf], res["f"][okf]) if okf.any() else 0.0
        errs["g"] = rel(fg[1][okg], res["g"][okg]) if okg.any() else 0.0
    print(label, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k in ("B", "dB", "tan", "f", "g"):
        if k in errs:
            assert errs[k] <= tol, (label, k, errs[k])
    return errs
