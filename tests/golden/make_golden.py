"""Writes oracle_tiny_case.json: inputs and FP64 oracle outputs for a tiny seeded case.

Calls only oracle/ (and numpy for the seeded inputs). The paper prints no worked numeric example of
the kernel sum or the lambda solve, so the stored values are the oracle's; they guard the oracle
against unintended changes. Any change to them must name, in its commit message, the passage of the
paper (or the reading of it) that justifies the change.

Also writes oracle_elements_trace_case.json (9-node elements, a short field line).

Run from the repository root:  python tests/golden/make_golden.py  (or `... elements` for the second file only)
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402


def tiny_inputs():
    rng = np.random.default_rng(20130605)
    nx, ny, h, x0, y0 = 6, 5, 0.5, -1.0, -0.75
    B0 = rng.normal(size=(3, ny, nx))
    xyz = np.stack([rng.uniform(-1.2, 2.0, 7), rng.uniform(-1.0, 1.5, 7), rng.uniform(0.2, 2.5, 7)])
    lam = rng.uniform(-1.5, 1.5, size=(3, 7))
    gB = rng.normal(size=(3, 7))
    gdB = rng.normal(size=(9, 7))
    return dict(nx=nx, ny=ny, h=h, x0=x0, y0=y0, B0=B0, xyz=xyz, lam=lam, gB=gB, gdB=gdB)


def main():
    c = tiny_inputs()
    B, dB, tan = oracle.field(c["B0"], c["x0"], c["y0"], c["h"], c["xyz"], c["lam"], tangents=True)
    res = oracle.residuals(B, dB, c["h"])
    gB0, glam, _ = oracle.vjp(c["B0"], c["x0"], c["y0"], c["h"], c["xyz"], c["lam"], c["gB"], c["gdB"])
    out = {k: (v.tolist() if isinstance(v, np.ndarray) else v) for k, v in c.items()}
    out.update(B=B.tolist(), dB=dB.tolist(), tan=tan.tolist(), f=res["f"].tolist(),
               g=res["g"].tolist(), gB0=gB0.tolist(), glam=glam.tolist(),
               source="oracle/dbie_oracle.py via tests/golden/make_golden.py")
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_tiny_case.json"), "w") as fh:
        json.dump(out, fh, indent=0)


def elements_and_trace():
    """A 7 x 5 magnetogram with 9-node elements (G = 3) and a short field line through the nodal
    field: written to oracle_elements_trace_case.json."""
    rng = np.random.default_rng(20130606)
    nx, ny, h, x0, y0 = 7, 5, 0.5, -1.5, -1.0
    B0 = rng.normal(size=(3, ny, nx))
    xyz = np.stack([rng.uniform(-1.6, 1.8, 6), rng.uniform(-1.1, 1.2, 6), rng.uniform(0.1, 2.0, 6)])
    lam = rng.uniform(-1.5, 1.5, size=(3, 6))
    B, dB, tan = oracle.field_quad9(B0, x0, y0, h, xyz, lam, G=3, tangents=True)
    lam_grid = rng.uniform(0.0, 1.0, size=(3, 2, 2, 2))
    origin, spacing = (-1.5, -1.0, 0.1), (3.0, 2.0, 2.0)
    d = oracle.dbie_direction(B0, x0, y0, h, lam_grid, origin, spacing)
    seeds = np.array([[0.1, -0.4], [0.2, 0.3], [0.5, 0.8]])
    pts, cnt = oracle.rk4_trace(d, seeds, 0.05, 12, (-1.5, -1.0, 0.1), (1.5, 1.0, 2.0))
    out = dict(nx=nx, ny=ny, h=h, x0=x0, y0=y0, G=3, B0=B0.tolist(), xyz=xyz.tolist(), lam=lam.tolist(),
               B=B.tolist(), dB=dB.tolist(), tan=tan.tolist(), lam_grid=lam_grid.tolist(),
               origin=list(origin), spacing=list(spacing), seeds=seeds.tolist(), ds=0.05, n_steps=12,
               box=[-1.5, -1.0, 0.1, 1.5, 1.0, 2.0], trace=np.nan_to_num(pts, nan=-999.0).tolist(),
               count=cnt.tolist(), source="oracle/ via tests/golden/make_golden.py")
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_elements_trace_case.json"),
              "w") as fh:
        json.dump(out, fh, indent=0)


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "elements":
        elements_and_trace()
    else:
        main()
        elements_and_trace()
