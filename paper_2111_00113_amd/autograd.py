"""Differentiable sparse solve x = A^{-1} b through sketched GMRES.

Forward: restarted sGMRES (sgmres_solve) on A x = b.  Backward (adjoint
method): one sGMRES solve of A^T lambda = dL/dx, then dL/db = lambda and
dL/dA_ij = -lambda_i x_j on A's sparsity pattern (sgmres_csr_outer_grad).
Both solves go through one plan of A built in the forward pass (CSR(A^T) and
the sliced ELL copies are built once, not again in the backward pass).  The matrix enters through its CSR values `val`
(float64, requires_grad allowed); the structure is fixed.  Accuracy of both
directions is set by the solve tolerance.
"""

from __future__ import annotations

import torch

from . import sgmres as _sg


class SGMRESSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, val, b, row_ptr, col_idx, opts):
        A = _sg.DeviceCSR(int(row_ptr.numel() - 1), row_ptr, col_idx, val.detach().contiguous())
        plan = _sg.Plan(A, transpose=True)
        x = torch.zeros_like(b)
        rc, info = _sg.sgmres_solve(None, b.detach().contiguous(), x, opts["d"], opts["k"], opts["s"],
                                    opts.get("seed", 0), opts.get("tol", 1e-12), opts.get("restarts", 1000),
                                    plan=plan)
        if rc != _sg.OK:
            plan.close()
            raise RuntimeError(f"forward solve did not converge: {info}")
        ctx.save_for_backward(A.val, row_ptr, col_idx, x)
        ctx.plan = plan
        ctx.opts = opts
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, gx):
        val, row_ptr, col_idx, x = ctx.saved_tensors
        opts = ctx.opts
        A = _sg.DeviceCSR(int(row_ptr.numel() - 1), row_ptr, col_idx, val)
        lam = torch.zeros_like(x)
        g = gx.contiguous()
        plan = ctx.plan
        try:
            if float(g.abs().max()) != 0.0:
                rc, info = _sg.sgmres_solve(None, g, lam, opts["d"], opts["k"], opts["s"], opts.get("seed", 0) + 1,
                                            opts.get("tol", 1e-12), opts.get("restarts", 1000), transposed=True,
                                            plan=plan)
                if rc != _sg.OK:
                    raise RuntimeError(f"adjoint solve did not converge: {info}")
        finally:
            plan.close()
            ctx.plan = None
        gval = _sg.sgmres_csr_outer_grad(A, lam, x, -1.0) if ctx.needs_input_grad[0] else None
        gb = lam if ctx.needs_input_grad[1] else None
        return gval, gb, None, None, None


def sgmres_solve_diff(row_ptr, col_idx, val, b, d, k, s, seed=0, tol=1e-12, restarts=1000):
    """x = A^{-1} b with gradients to `val` (A's CSR values) and `b`."""
    opts = dict(d=d, k=k, s=s, seed=seed, tol=tol, restarts=restarts)
    return SGMRESSolve.apply(val, b, row_ptr, col_idx, opts)
