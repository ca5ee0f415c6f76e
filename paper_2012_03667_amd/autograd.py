"""torch.autograd wrapper: the converged solution x*(theta) of the gap equation
as a differentiable function of theta = (D, omega, m) per instance, with the
backward pass by implicit differentiation on the GPU (qdse_grad: GMRES on
(I - J)^T lambda = dL/dx*, then lambda^T dF/dtheta)."""
from __future__ import annotations

import torch

from ._lib import (QDSE_AUTO, QDSE_CONV_MASS, QDSE_NEWTON, QDSE_OK, QDSE_PICARD, QdseError,
                   Solver)

_SOLVERS = {"picard": QDSE_PICARD, "newton": QDSE_NEWTON, "auto": QDSE_AUTO}


class GapFixedPoint(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, opts):
        th = theta.detach().to("cpu", torch.float64)
        params = [tuple(float(v) for v in row) for row in th]
        S = Solver(opts["n_radial"], opts["n_angle"], params, interp_order=opts["interp_order"],
                   s_min=opts["s_min"], s_max=opts["s_max"], solver=_SOLVERS[opts["solver"]])
        x = S.initial(opts["A0"], opts["B0"])
        rc, it, res = S.solve(x, tol=opts["tol"], max_iter=opts["max_iter"],
                              conv_mode=QDSE_CONV_MASS)
        if rc != QDSE_OK:
            # no gradient through an unconverged, diverged or spurious fixed
            # point (one that fails the branch certificate)
            bad = [(k, int(v)) for k, v in enumerate(S.solve_status()) if v != QDSE_OK]
            raise QdseError(rc, f"gap fixed point not certified for (instance, status) {bad[:8]}")
        ctx.solver = S
        ctx.opts = opts
        ctx.theta_device = theta.device
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        S = ctx.solver
        g = gx.detach().to(x.device, torch.float64).contiguous()
        tb, rc = S.grad(x, g, tol=ctx.opts["grad_tol"], max_iter=ctx.opts["grad_max_iter"])
        if rc != QDSE_OK:
            raise QdseError(rc, "adjoint solve did not converge")
        return torch.tensor(tb, dtype=torch.float64, device=ctx.theta_device), None


def solve_gap(theta, n_radial=512, n_angle=128, interp_order=3, s_min=1e-4, s_max=1e4,
              A0=1.0, B0=1.0, tol=1e-12, max_iter=2000, solver="picard", grad_tol=1e-12,
              grad_max_iter=400):
    """x* = [A | B] per instance (shape (n_inst, 2 n_radial), CUDA float64) for
    theta = (D, omega, m) rows; differentiable with respect to theta. solver:
    "picard" (successive approximation), "newton" or "auto" (Newton for the
    instances successive approximation does not certify). Raises QdseError
    unless every instance ends at a certified fixed point."""
    if solver not in _SOLVERS:
        raise ValueError(f"solver must be one of {sorted(_SOLVERS)}")
    opts = dict(n_radial=n_radial, n_angle=n_angle, interp_order=interp_order, s_min=s_min,
                s_max=s_max, A0=A0, B0=B0, tol=tol, max_iter=max_iter, solver=solver,
                grad_tol=grad_tol, grad_max_iter=grad_max_iter)
    return GapFixedPoint.apply(theta, opts)
