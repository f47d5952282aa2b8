"""Thin Python binding of the C ABI (include/dbie.h), with the same function names.

Argument marshalling only: every step of the computation runs in the HIP library. Tensors must be
CUDA (ROCm) tensors, contiguous, float64 (int32 for status/trials). Outputs left as None are allocated
here with torch and returned. Streams default to torch's current stream.
"""
from __future__ import annotations

import ctypes
from typing import Dict, List, Optional, Sequence

import torch

from . import _lib as L


class DbieError(RuntimeError):
    pass


def _lib():
    return L.load()


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, name: str, shape: Sequence[int], dtype=torch.float64, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the context on {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _on(device: torch.device):
    """Make the context's device current for a call (the library requires it)."""
    return torch.cuda.device(device)


class Context:
    """Owns a dbie_ctx handle (destroyed with the object)."""

    def __init__(self, handle: ctypes.c_void_p, n_points: int, shapes: List[tuple], precision: int,
                 device: torch.device):
        self.handle = handle
        self.n_points = n_points
        self.shapes = shapes
        self.precision = precision
        self.device = device
        self._ws = None   # a caller-owned workspace handed to the context (kept alive until close)

    @property
    def n_pixels(self) -> int:
        return sum(nx * ny for nx, ny in self.shapes)

    def close(self):
        if self.handle:
            with _on(self.device):
                _lib().dbie_destroy(self.handle)
            self.handle = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check(rc: int, ctx: Optional[Context], what: str):
    if rc != L.DBIE_OK:
        msg = _lib().dbie_last_error(ctx.handle if ctx is not None else None)
        raise DbieError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")


def dbie_default_options() -> L.dbie_options:
    o = L.dbie_options()
    _lib().dbie_default_options(ctypes.byref(o))
    return o


def dbie_default_solve_opts() -> L.dbie_solve_opts:
    o = L.dbie_solve_opts()
    _lib().dbie_default_solve_opts(ctypes.byref(o))
    return o


def dbie_init(boundaries: List[Dict], xyz: torch.Tensor, seg: Optional[Sequence[int]] = None,
              precision: str = "fp32c", nearfield_radius_h: float = 2.0,
              dv_over_dsigma_h: float = 1.0 / 6.0, tune: bool = False,
              tune_cache: Optional[str] = None, quad_points: int = 0, pixel_split: int = 0,
              stream=None) -> Context:
    """boundaries: list of dict(B0=[3, ny, nx] float64 CUDA tensor, x0=, y0=, h=); xyz: [3, N].
    quad_points = 0 selects the nodal sum (Eq. 16); 2..4 the 9-node elements of Eq. (15) with that many
    Gauss points per element side."""
    lib = _lib()
    nb = len(boundaries)
    arr = (L.dbie_boundary * nb)()
    shapes = []
    for b, bd in enumerate(boundaries):
        B0 = bd["B0"]
        if B0.dim() != 3 or B0.shape[0] != 3:
            raise ValueError("B0 must have shape [3, ny, nx]")
        _need(B0, "B0", tuple(B0.shape))
        arr[b].nx, arr[b].ny = int(B0.shape[2]), int(B0.shape[1])
        arr[b].x0, arr[b].y0, arr[b].h = float(bd.get("x0", 0.0)), float(bd.get("y0", 0.0)), float(bd.get("h", 1.0))
        arr[b].B0 = B0.data_ptr()
        shapes.append((int(B0.shape[2]), int(B0.shape[1])))
    if xyz.dim() != 2 or xyz.shape[0] != 3:
        raise ValueError("xyz must have shape [3, N]")
    _need(xyz, "xyz", tuple(xyz.shape))
    for bd in boundaries:
        if bd["B0"].device != xyz.device:
            raise ValueError("every B0 must be on the device of xyz")
    N = int(xyz.shape[1])
    prob = L.dbie_problem()
    prob.n_boundaries = nb
    prob.boundaries = arr
    prob.n_points = N
    prob.xyz = xyz.data_ptr()
    segarr = None
    if seg is not None:
        if len(seg) != nb + 1:
            raise ValueError(f"seg must hold n_boundaries + 1 = {nb + 1} offsets")
        segarr = (ctypes.c_int64 * len(seg))(*[int(s) for s in seg])
        prob.seg = segarr
    opt = dbie_default_options()
    opt.precision = {"fp64": L.DBIE_FP64, "fp32c": L.DBIE_FP32C}[precision]
    opt.nearfield_radius_h = float(nearfield_radius_h)
    opt.dv_over_dsigma_h = float(dv_over_dsigma_h)
    opt.tune = int(bool(tune))
    opt.tune_cache = tune_cache.encode() if tune_cache else None
    opt.quad_points = int(quad_points)
    opt.pixel_split = int(pixel_split)
    h = ctypes.c_void_p()
    with _on(xyz.device):
        rc = lib.dbie_init(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(opt), _stream(stream))
    if rc != L.DBIE_OK:
        msg = lib.dbie_last_error(None)
        raise DbieError(f"dbie_init failed ({rc}): {msg.decode() if msg else ''}")
    return Context(h, N, shapes, opt.precision, xyz.device)


def dbie_eval_field(ctx: Context, lam: torch.Tensor, B=None, dB=None, fg=None, tan=None,
                    want_dB: bool = True, want_fg: bool = True, want_tan: bool = False, stream=None):
    """lam: [3, N] or [L, 3, N]. Returns dict(B, dB, fg, tan) with a leading L axis only if lam has one."""
    return _eval_field("dbie_eval_field", ctx, lam, B, dB, fg, tan, want_dB, want_fg, want_tan, stream)


def dbie_eval_field_noalloc(ctx: Context, lam: torch.Tensor, B=None, dB=None, fg=None, tan=None,
                            want_dB: bool = True, want_fg: bool = True, want_tan: bool = False, stream=None):
    """dbie_eval_field through the entry point that allocates no device memory (its partial sums live
    in the library's static work array; L * N is limited). Outputs not passed in are allocated here,
    by torch, before the call."""
    return _eval_field("dbie_eval_field_noalloc", ctx, lam, B, dB, fg, tan, want_dB, want_fg, want_tan, stream)


def _eval_field(entry, ctx, lam, B, dB, fg, tan, want_dB, want_fg, want_tan, stream):
    N = ctx.n_points
    squeeze = lam.dim() == 2
    lam3 = lam.unsqueeze(0) if squeeze else lam
    Lt = int(lam3.shape[0])
    _need(lam3, "lambda", (Lt, 3, N), device=ctx.device)
    dev = lam.device
    z = lambda *s: torch.empty(*s, dtype=torch.float64, device=dev)  # noqa: E731
    B = z(Lt, 3, N) if B is None else B
    dB = (z(Lt, 9, N) if want_dB else None) if dB is None else dB
    fg = (z(Lt, 2, N) if want_fg else None) if fg is None else fg
    tan = (z(Lt, 12, N) if want_tan else None) if tan is None else tan
    for t, nm, rows in ((B, "B", 3), (dB, "dB", 9), (fg, "fg", 2), (tan, "tan", 12)):
        if t is not None:
            # a 2-D output is accepted for one trial only
            _need(t, nm, (Lt, rows, N) if (t.dim() == 3 or Lt > 1) else (rows, N), device=ctx.device)
    with _on(ctx.device):
        rc = getattr(_lib(), entry)(ctx.handle, _ptr(lam3), Lt, _ptr(B), _ptr(dB), _ptr(fg), _ptr(tan),
                                    _stream(stream))
    _check(rc, ctx, entry)
    out = dict(B=B, dB=dB, fg=fg, tan=tan)
    if squeeze:
        out = {k: (v[0] if v is not None and v.dim() == 3 else v) for k, v in out.items()}
    return out


def dbie_eval_field_scalar(ctx: Context, lam: torch.Tensor, want_dB: bool = True, want_fg: bool = True,
                           want_tan: bool = False, stream=None):
    """lam: [N] or [L, N], one lambda shared by the three components of each point."""
    N = ctx.n_points
    squeeze = lam.dim() == 1
    lam2 = lam.unsqueeze(0) if squeeze else lam
    Lt = int(lam2.shape[0])
    _need(lam2, "lambda", (Lt, N), device=ctx.device)
    dev = lam.device
    z = lambda *s: torch.empty(*s, dtype=torch.float64, device=dev)  # noqa: E731
    B = z(Lt, 3, N)
    dB = z(Lt, 9, N) if want_dB else None
    fg = z(Lt, 2, N) if want_fg else None
    tan = z(Lt, 12, N) if want_tan else None
    with _on(ctx.device):
        rc = _lib().dbie_eval_field_scalar(ctx.handle, _ptr(lam2), Lt, _ptr(B), _ptr(dB), _ptr(fg), _ptr(tan),
                                           _stream(stream))
    _check(rc, ctx, "dbie_eval_field_scalar")
    out = dict(B=B, dB=dB, fg=fg, tan=tan)
    if squeeze:
        out = {k: (v[0] if v is not None else v) for k, v in out.items()}
    return out


def dbie_solve_lambda(ctx: Context, lambda_inout: torch.Tensor, method: str = "nm", max_trials: int = 50,
                      eps: float = 1e-4, init_step: float = 0.0, lambda_cap: float = 0.0,
                      fp64_accept: bool = True, B=None, fg=None, status=None, trials=None,
                      want_B: bool = True, want_fg: bool = True, use_graph: bool = True,
                      lm_radius: float = 0.0, lm_damping: float = 0.0, stream=None):
    """Per-point lambda search (method "nm": Nelder-Mead, "lm": Levenberg-Marquardt in mu = lambda^2)
    from the start values in lambda_inout [3, N], which receives |lambda*|. lm_radius: LM's trust
    radius in lambda at the start (0: the simplex edge; math.inf: none); lm_damping: its initial
    damping nu0 (0: 1). Returns dict(lam, B, fg,
    status, trials): status per point (_lib.DBIE_ST_*), trials = evaluations used."""
    N = ctx.n_points
    _need(lambda_inout, "lambda_inout", (3, N), device=ctx.device)
    dev = lambda_inout.device
    B = (torch.empty(3, N, dtype=torch.float64, device=dev) if want_B else None) if B is None else B
    fg = (torch.empty(2, N, dtype=torch.float64, device=dev) if want_fg else None) if fg is None else fg
    status = torch.empty(N, dtype=torch.int32, device=dev) if status is None else status
    trials = torch.empty(N, dtype=torch.int32, device=dev) if trials is None else trials
    _need(status, "status", (N,), torch.int32, device=ctx.device)
    _need(trials, "trials", (N,), torch.int32, device=ctx.device)
    if B is not None:
        _need(B, "B", (3, N), device=ctx.device)
    if fg is not None:
        _need(fg, "fg", (2, N), device=ctx.device)
    o = dbie_default_solve_opts()
    o.method = {"nm": L.DBIE_NELDER_MEAD, "lm": L.DBIE_LEVENBERG_MARQUARDT}[method]
    o.max_trials = int(max_trials)
    o.eps = float(eps)
    o.init_step = float(init_step)
    o.lambda_cap = float(lambda_cap)
    o.fp64_accept = int(bool(fp64_accept))
    o.use_graph = int(bool(use_graph))
    o.lm_radius = float(lm_radius)
    o.lm_damping = float(lm_damping)
    with _on(ctx.device):
        rc = _lib().dbie_solve_lambda(ctx.handle, _ptr(lambda_inout), ctypes.byref(o), _ptr(B), _ptr(fg),
                                      _ptr(status), _ptr(trials), _stream(stream))
    _check(rc, ctx, "dbie_solve_lambda")
    return dict(lam=lambda_inout, B=B, fg=fg, status=status, trials=trials)


def dbie_grad(ctx: Context, lam: torch.Tensor, gB=None, gdB=None, want_glambda: bool = True,
              want_gB0: bool = True, want_resid_jac: bool = False, glambda=None, gB0=None,
              resid_jac=None, stream=None):
    """Adjoint of the evaluation at lam [3, N] for the upstream gradients gB [3, N] and gdB [9, N]:
    glambda [3, N], gB0 (concatenated [3, ny, nx] per boundary; see split_gB0) and, on request, the
    residual Jacobian d(u, s)/d mu [4, 3, N]."""
    N = ctx.n_points
    _need(lam, "lambda", (3, N), device=ctx.device)
    dev = lam.device
    if gB is not None:
        _need(gB, "gB", (3, N), device=ctx.device)
    if gdB is not None:
        _need(gdB, "gdB", (9, N), device=ctx.device)
    glambda = (torch.empty(3, N, dtype=torch.float64, device=dev) if want_glambda else None) \
        if glambda is None else glambda
    gB0 = (torch.empty(3 * ctx.n_pixels, dtype=torch.float64, device=dev) if want_gB0 else None) \
        if gB0 is None else gB0
    resid_jac = (torch.empty(4, 3, N, dtype=torch.float64, device=dev) if want_resid_jac else None) \
        if resid_jac is None else resid_jac
    for t, nm, shape in ((glambda, "glambda", (3, N)), (gB0, "gB0", (3 * ctx.n_pixels,)),
                         (resid_jac, "resid_jac", (4, 3, N))):
        if t is not None:
            _need(t, nm, shape, device=ctx.device)
    with _on(ctx.device):
        rc = _lib().dbie_grad(ctx.handle, _ptr(lam), _ptr(gB), _ptr(gdB), _ptr(glambda), _ptr(gB0),
                              _ptr(resid_jac), _stream(stream))
    _check(rc, ctx, "dbie_grad")
    return dict(glambda=glambda, gB0=gB0, resid_jac=resid_jac)


def split_gB0(ctx: Context, gB0: torch.Tensor) -> List[torch.Tensor]:
    """View the concatenated gB0 as one [3, ny, nx] tensor per boundary."""
    out, off = [], 0
    for nx, ny in ctx.shapes:
        out.append(gB0[off: off + 3 * nx * ny].view(3, ny, nx))
        off += 3 * nx * ny
    return out


def dbie_timing(ctx: Context, enable: bool = True):
    _check(_lib().dbie_timing(ctx.handle, int(bool(enable))), ctx, "dbie_timing")


def dbie_timing_read(ctx: Context):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(_lib().dbie_timing_read(ctx.handle, ctypes.byref(ms), ctypes.byref(n)), ctx, "dbie_timing_read")
    return ms.value, n.value


def dbie_query(ctx: Context) -> Dict[str, int]:
    a, b = ctypes.c_int64(), ctypes.c_int64()
    p, w, t = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib().dbie_query(ctx.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(p), ctypes.byref(w),
                             ctypes.byref(t)), ctx, "dbie_query")
    return dict(n_points=a.value, n_pixels=b.value, ppl=p.value, waves=w.value, tile_pixels=t.value)


def dbie_query_tan(ctx: Context) -> Dict[str, int]:
    p, w, t = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib().dbie_query_tan(ctx.handle, ctypes.byref(p), ctypes.byref(w), ctypes.byref(t)), ctx,
           "dbie_query_tan")
    return dict(ppl=p.value, waves=w.value, tile_pixels=t.value)


def dbie_set_tile_shape(ctx: Context, ppl: int, waves: int, tile_pixels: int, persistent: bool = False):
    with _on(ctx.device):
        rc = _lib().dbie_set_tile_shape(ctx.handle, int(ppl), int(waves), int(tile_pixels), int(bool(persistent)))
    _check(rc, ctx, "dbie_set_tile_shape")


def dbie_query_persistent(ctx: Context) -> Dict[str, bool]:
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib().dbie_query_persistent(ctx.handle, ctypes.byref(a), ctypes.byref(b)), ctx, "dbie_query_persistent")
    return dict(plain=bool(a.value), with_tangents=bool(b.value))


def dbie_solve_trace(ctx: Context, enable: bool = True):
    _check(_lib().dbie_solve_trace(ctx.handle, int(bool(enable))), ctx, "dbie_solve_trace")


def dbie_solve_trace_read(ctx: Context, max_rounds: int = 100000, with_end: bool = False):
    """Returns (t_ms [rounds], converged [rounds]) of the last traced solve, and with with_end the
    elapsed milliseconds at the end of the call as a third item."""
    import numpy as np
    n = ctypes.c_int32()
    _check(_lib().dbie_solve_trace_read(ctx.handle, None, None, 0, ctypes.byref(n), None), ctx,
           "dbie_solve_trace_read")
    m = max(0, min(n.value, max_rounds))
    t = (ctypes.c_double * max(m, 1))()
    cv = (ctypes.c_int32 * max(m, 1))()
    te = ctypes.c_double()
    _check(_lib().dbie_solve_trace_read(ctx.handle, t, cv, m, ctypes.byref(n), ctypes.byref(te)), ctx,
           "dbie_solve_trace_read")
    out = (np.array(t[:m]), np.array(cv[:m], dtype=np.int64))
    return out + (te.value,) if with_end else out


def dbie_trace_lines(ctx: Context, lam_grid: torch.Tensor, origin, spacing, box, ds: float, n_steps: int,
                     mode: str = "field", sense: float = 1.0, stream=None):
    """Field (mode="field") or current (mode="current") lines from the context's points.
    lam_grid: [3, nz, ny, nx] float64 on the device, node (i, j, k) at origin + (i, j, k) * spacing;
    box = (x_lo, y_lo, z_lo, x_hi, y_hi, z_hi). Returns dict(xyz=[n_steps + 1, 3, N], count=[N])."""
    if lam_grid.dim() != 4 or lam_grid.shape[0] != 3:
        raise ValueError("lam_grid must have shape [3, nz, ny, nx]")
    _need(lam_grid, "lam_grid", tuple(lam_grid.shape), device=ctx.device)
    N = ctx.n_points
    g = L.dbie_lambda_grid()
    g.nz, g.ny, g.nx = (int(v) for v in lam_grid.shape[1:])
    g.x0, g.y0, g.z0 = (float(v) for v in origin)
    g.dx, g.dy, g.dz = (float(v) for v in spacing)
    g.lam = lam_grid.data_ptr()
    bx = (ctypes.c_double * 6)(*[float(v) for v in box])
    xyz = torch.empty(int(n_steps) + 1, 3, N, dtype=torch.float64, device=lam_grid.device)
    count = torch.empty(N, dtype=torch.int32, device=lam_grid.device)
    m = {"field": L.DBIE_TRACE_FIELD, "current": L.DBIE_TRACE_CURRENT}[mode]
    with _on(ctx.device):
        rc = _lib().dbie_trace_lines(ctx.handle, ctypes.byref(g), bx, float(ds), int(n_steps), m, float(sense),
                                     xyz.data_ptr() if N else None, count.data_ptr() if N else None,
                                     _stream(stream))
    _check(rc, ctx, "dbie_trace_lines")
    return dict(xyz=xyz, count=count)


def dbie_residual_stats(ctx: Context, fg: torch.Tensor, eps: float = 1e-4, stream=None) -> Dict[str, float]:
    """Means of f and g over the points with finite residuals, their number, and the number with
    max(f, g) <= eps, reduced on the device."""
    _need(fg, "fg", (2, ctx.n_points), device=ctx.device)
    out = (ctypes.c_double * 4)()
    with _on(ctx.device):
        rc = _lib().dbie_residual_stats(ctx.handle, fg.data_ptr() if ctx.n_points else None, float(eps), out,
                                        _stream(stream))
    _check(rc, ctx, "dbie_residual_stats")
    return dict(mean_f=out[0], mean_g=out[1], finite=int(out[2]), converged=int(out[3]))


def dbie_query_split(ctx: Context) -> int:
    v = ctypes.c_int32()
    _check(_lib().dbie_query_split(ctx.handle, ctypes.byref(v)), ctx, "dbie_query_split")
    return int(v.value)


def dbie_query_tuned(ctx: Context) -> int:
    """0 untuned, 1 timed by this context's init, 2 reused from this process's tuner cache, 3 read from
    the tune_cache file."""
    v = ctypes.c_int32()
    _check(_lib().dbie_query_tuned(ctx.handle, ctypes.byref(v)), ctx, "dbie_query_tuned")
    return int(v.value)


def dbie_workspace_bytes(ctx: Context) -> int:
    return int(_lib().dbie_workspace_bytes(ctx.handle))


def dbie_set_workspace(ctx: Context, ws: Optional[torch.Tensor]):
    """Give the context a caller-owned device workspace (a uint8 tensor of at least
    dbie_workspace_bytes(ctx) bytes, kept alive by the context object), or None to go back."""
    if ws is None:
        with _on(ctx.device):
            rc = _lib().dbie_set_workspace(ctx.handle, None, 0)
        _check(rc, ctx, "dbie_set_workspace")
        ctx._ws = None
        return
    if not ws.is_cuda or not ws.is_contiguous():
        raise ValueError("workspace must be a contiguous device tensor")
    if ws.device != ctx.device:
        raise ValueError(f"workspace is on {ws.device}, the context on {ctx.device}")
    with _on(ctx.device):
        rc = _lib().dbie_set_workspace(ctx.handle, ws.data_ptr(), ws.numel() * ws.element_size())
    _check(rc, ctx, "dbie_set_workspace")
    ctx._ws = ws


def dbie_destroy(ctx: Context):
    ctx.close()


def dbie_last_error(ctx: Optional[Context] = None) -> str:
    m = _lib().dbie_last_error(ctx.handle if ctx is not None else None)
    return m.decode() if m else ""


class Field:
    """The context with its calls as methods (argument marshalling only):

        f = Field([dict(B0=..., x0=..., y0=..., h=...)], xyz, precision="fp32c")
        out = f.eval(lam); sol = f.solve(lam0, method="lm"); g = f.grad(lam, gB=...)

    The keyword arguments of dbie_init, dbie_eval_field, dbie_solve_lambda, dbie_grad and
    dbie_trace_lines pass through unchanged."""

    def __init__(self, boundaries: List[Dict], xyz: torch.Tensor, **init_kw):
        self.ctx = dbie_init(boundaries, xyz, **init_kw)

    def eval(self, lam: torch.Tensor, **kw):
        return dbie_eval_field(self.ctx, lam, **kw)

    def eval_scalar(self, lam: torch.Tensor, **kw):
        return dbie_eval_field_scalar(self.ctx, lam, **kw)

    def solve(self, lambda_inout: torch.Tensor, **kw):
        return dbie_solve_lambda(self.ctx, lambda_inout, **kw)

    def grad(self, lam: torch.Tensor, **kw):
        return dbie_grad(self.ctx, lam, **kw)

    def trace(self, lam_grid: torch.Tensor, origin, spacing, box, ds: float, n_steps: int, **kw):
        return dbie_trace_lines(self.ctx, lam_grid, origin, spacing, box, ds, n_steps, **kw)

    def close(self):
        self.ctx.close()
