"""torch.autograd.Function over the library: forward = dbie_eval_field, backward = dbie_grad.

    B, dB = dbie_field(B0, lam, xyz, x0=0, y0=0, h=1, precision="fp32c")

B0: [3, ny, nx] (one magnetogram), lam: [3, N], xyz: [3, N], all float64 CUDA tensors. Gradients flow
to B0 (the transpose of the Eq. 16 sum and of its gradient rows, computed by the library's adjoint
kernel) and to lam (from the mu-tangents). xyz receives no gradient. A context is created per call
and released with the autograd graph.
"""
import torch

from . import dbie as D


class DbieField(torch.autograd.Function):
    @staticmethod
    def forward(ctx, B0, lam, xyz, x0, y0, h, precision):
        c = D.dbie_init([dict(B0=B0.detach().contiguous(), x0=x0, y0=y0, h=h)], xyz.detach().contiguous(),
                        precision=precision)
        lam_d = lam.detach().contiguous()
        out = D.dbie_eval_field(c, lam_d, want_dB=True, want_fg=False)
        ctx.c = c
        ctx.save_for_backward(lam_d)
        return out["B"], out["dB"]

    @staticmethod
    def backward(ctx, gB, gdB):
        (lam,) = ctx.saved_tensors
        c = ctx.c
        gB = None if gB is None else gB.contiguous()
        gdB = None if gdB is None else gdB.contiguous()
        r = D.dbie_grad(c, lam, gB=gB, gdB=gdB, want_glambda=ctx.needs_input_grad[1],
                        want_gB0=ctx.needs_input_grad[0])
        gB0 = None
        if r["gB0"] is not None:
            nx, ny = c.shapes[0]
            gB0 = r["gB0"].view(3, ny, nx)
        return gB0, r["glambda"], None, None, None, None, None


def dbie_field(B0, lam, xyz, x0=0.0, y0=0.0, h=1.0, precision="fp32c"):
    return DbieField.apply(B0, lam, xyz, float(x0), float(y0), float(h), precision)
