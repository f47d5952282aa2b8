"""The oracle still reproduces its stored tiny-case outputs (no GPU)."""
import json
import os

import numpy as np

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_reproduces_tiny_case():
    with open(os.path.join(HERE, "golden", "oracle_tiny_case.json")) as fh:
        g = json.load(fh)
    a = {k: np.asarray(v) for k, v in g.items() if isinstance(v, list)}
    B, dB, tan = oracle.field(a["B0"], g["x0"], g["y0"], g["h"], a["xyz"], a["lam"], tangents=True)
    res = oracle.residuals(B, dB, g["h"])
    gB0, glam, _ = oracle.vjp(a["B0"], g["x0"], g["y0"], g["h"], a["xyz"], a["lam"], a["gB"], a["gdB"])
    for name, v in dict(B=B, dB=dB, tan=tan, f=res["f"], g=res["g"], gB0=gB0, glam=glam).items():
        np.testing.assert_allclose(v, a[name], rtol=1e-13, atol=1e-15 * np.abs(a[name]).max(), err_msg=name)


def test_table1_fixture_is_well_formed():
    with open(os.path.join(HERE, "golden", "paper_table1_present_dbie.json")) as fh:
        t = json.load(fh)
    assert set(t["exact"]) == {"C_vec", "C_cs", "E_n", "E_m", "eps"}
    assert all(isinstance(t[k], float) for k in t["exact"])
