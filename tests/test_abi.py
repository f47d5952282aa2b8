"""The C-ABI library loads, exports every symbol include/dbie.h declares, and rejects invalid
arguments on the host before touching the GPU (no compute calls; runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1306_1122_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dbie.h")


def declared_symbols():
    txt = open(HEADER).read()
    return re.findall(r"DBIE_API\s+[\w\s\*]+?\b(dbie_\w+)\s*\(", txt)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIBPATH):
        import __graft_entry__
        __graft_entry__.build()
    return L.load()


def test_header_declares_the_four_entry_points():
    names = declared_symbols()
    for n in ("dbie_init", "dbie_eval_field", "dbie_solve_lambda", "dbie_grad", "dbie_destroy",
              "dbie_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
        assert n in L.SIGNATURES, n


def declared_arity():
    """Number of parameters of every declared entry point, from the header text."""
    txt = re.sub(r"/\*.*?\*/", " ", open(HEADER).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"DBIE_API\s+[\w\s\*]+?\b(dbie_\w+)\s*\((.*?)\)\s*;", txt, re.S):
        params = m.group(2).strip()
        out[m.group(1)] = 0 if params in ("", "void") else params.count(",") + 1
    return out


def test_binding_signatures_match_the_header():
    """The ctypes declarations take as many arguments as the header declares (a changed signature
    cannot go unnoticed by the binding)."""
    ar = declared_arity()
    assert len(ar) == len(declared_symbols())
    for name, n in ar.items():
        assert len(L.SIGNATURES[name][1]) == n, (name, n, len(L.SIGNATURES[name][1]))


def test_defaults(lib):
    o = L.dbie_options()
    assert lib.dbie_default_options(ctypes.byref(o)) == 0
    assert o.precision == L.DBIE_FP32C and o.nearfield_radius_h == 2.0
    assert abs(o.dv_over_dsigma_h - 1 / 6) < 1e-16
    assert o.quad_points == 0
    s = L.dbie_solve_opts()
    assert lib.dbie_default_solve_opts(ctypes.byref(s)) == 0
    assert s.max_trials == 50 and s.eps == 1e-4 and s.method == L.DBIE_NELDER_MEAD
    assert s.lm_radius == 0.0 and s.lm_damping == 0.0   # the simplex edge, nu0 = 1
    assert lib.dbie_default_options(None) == L.DBIE_E_INVAL


def _problem(nx=4, ny=3, h=1.0, n=5, nb=1, seg=None):
    arr = (L.dbie_boundary * nb)()
    for b in range(nb):
        arr[b].nx, arr[b].ny, arr[b].x0, arr[b].y0, arr[b].h, arr[b].B0 = nx, ny, 0.0, 0.0, h, 0x1000
    p = L.dbie_problem()
    p.n_boundaries = nb
    p.boundaries = arr
    p.n_points = n
    p.xyz = 0x2000
    keep = [arr]
    if seg is not None:
        s = (ctypes.c_int64 * len(seg))(*seg)
        p.seg = s
        keep.append(s)
    return p, keep


@pytest.mark.parametrize("case,msg", [
    ("null_out", "out is NULL"),
    ("null_problem", "problem is NULL"),
    ("precision", "precision"),
    ("radius", "nearfield_radius_h"),
    ("dvds", "dv_over_dsigma_h"),
    ("no_boundary", "at least one boundary"),
    ("h", "h must be positive"),
    ("nx", "nx or ny"),
    ("seg_missing", "seg is required"),
    ("seg_order", "non-decreasing"),
    ("seg_end", "end at n_points"),
    ("quad_points", "quad_points must be"),
    ("quad_even", "odd nx, ny"),
])
def test_init_argument_checks(lib, case, msg):
    p, keep = _problem()
    o = L.dbie_options()
    lib.dbie_default_options(ctypes.byref(o))
    out = ctypes.c_void_p()
    args = [ctypes.byref(out), ctypes.byref(p), ctypes.byref(o), None]
    if case == "null_out":
        args[0] = None
    elif case == "null_problem":
        args[1] = None
    elif case == "precision":
        o.precision = 7
    elif case == "radius":
        o.nearfield_radius_h = 2.5
    elif case == "dvds":
        o.dv_over_dsigma_h = 0.0
    elif case == "no_boundary":
        p.n_boundaries = 0
    elif case == "h":
        p.boundaries[0].h = -1.0
    elif case == "nx":
        p.boundaries[0].nx = 0
    elif case == "seg_missing":
        p, keep = _problem(nb=2)
        args[1] = ctypes.byref(p)
    elif case == "seg_order":
        p, keep = _problem(nb=2, seg=[0, 6, 5])
        args[1] = ctypes.byref(p)
    elif case == "seg_end":
        p, keep = _problem(nb=2, seg=[0, 2, 4])
        args[1] = ctypes.byref(p)
    elif case == "quad_points":
        o.precision, o.quad_points = L.DBIE_FP64, 1
    elif case == "quad_even":
        o.precision, o.quad_points = L.DBIE_FP64, 4   # the default magnetogram is 4 x 3
    rc = lib.dbie_init(*args)
    assert rc == L.DBIE_E_INVAL
    assert msg in lib.dbie_last_error(None).decode()
    assert not out.value


def test_workspace_calls_on_null_context(lib):
    assert lib.dbie_workspace_bytes(None) == L.DBIE_E_INVAL
    assert lib.dbie_set_workspace(None, None, 0) == L.DBIE_E_INVAL


def test_calls_on_null_context_are_rejected(lib):
    assert lib.dbie_eval_field(None, None, 1, None, None, None, None, None) == L.DBIE_E_INVAL
    assert lib.dbie_eval_field_noalloc(None, None, 1, None, None, None, None, None) == L.DBIE_E_INVAL
    assert lib.dbie_timing(None, 1) == L.DBIE_E_INVAL
    lib.dbie_destroy(None)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """With no built library the binding raises instead of computing anything some other way."""
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIBPATH", str(tmp_path / "libdbie.so"))
    with pytest.raises(RuntimeError, match="not built"):
        L.load()
