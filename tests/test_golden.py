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


def test_oracle_reproduces_elements_and_trace_case():
    with open(os.path.join(HERE, "golden", "oracle_elements_trace_case.json")) as fh:
        g = json.load(fh)
    a = {k: np.asarray(v) for k, v in g.items() if isinstance(v, list)}
    B, dB, tan = oracle.field_quad9(a["B0"], g["x0"], g["y0"], g["h"], a["xyz"], a["lam"], G=g["G"], tangents=True)
    for name, v in dict(B=B, dB=dB, tan=tan).items():
        np.testing.assert_allclose(v, a[name], rtol=1e-13, atol=1e-15 * np.abs(a[name]).max(), err_msg=name)
    d = oracle.dbie_direction(a["B0"], g["x0"], g["y0"], g["h"], a["lam_grid"], g["origin"], g["spacing"])
    pts, cnt = oracle.rk4_trace(d, a["seeds"], g["ds"], g["n_steps"], g["box"][:3], g["box"][3:])
    np.testing.assert_array_equal(cnt, a["count"])
    np.testing.assert_allclose(np.nan_to_num(pts, nan=-999.0), a["trace"], rtol=1e-12, atol=1e-13)
    assert cnt.min() > 2
