"""Differentiable KKT solve: ``torch.autograd.Function`` over the C ABI.

Forward: factorization fused with the forward / backward substitution
(kkt_factor_solve).  Backward: the adjoint (kkt_solve_adjoint) reuses the factor
kept in the workspace to solve Psi lambda = dL/dx and writes the gradients
restricted to the block pattern:
    dL/dD_i = -sym(lambda_i x_i^T),  dL/dC_i = -(lambda_{i+1} x_i^T + x_{i+1} lambda_i^T),
    dL/dB_i = -(lambda_g x_i^T + x_g lambda_i^T),  dL/dcorner = -sym(lambda_g x_g^T),
    dL/dr = lambda   (summed over the rhs columns).
All arithmetic runs in the HIP library; this module only marshals tensors.
"""
import torch

from . import kkt

_PLANS = {}


def plan_for(dims, nrhs):
    """A cached plan for a tuple of (N, b, ng, p) shapes."""
    key = (tuple(tuple(d) for d in dims), int(nrhs))
    p = _PLANS.get(key)
    if p is None:
        p = kkt.Plan(list(key[0]), nrhs=nrhs)
        _PLANS[key] = p
    return p


class KKTSolveFn(torch.autograd.Function):
    """x = Psi(D, C, B, corner)^{-1} r on packed pools (see include/kkt.h)."""

    @staticmethod
    def forward(ctx, D, C, B, corner, r, plan):
        for t in (D, C, B, corner, r):
            if t.numel() and (t.dtype != torch.float64 or not t.is_cuda):
                raise TypeError("KKTSolve expects float64 CUDA tensors")
        D, C, B, corner = (t.contiguous() for t in (D, C, B, corner))
        ws = plan.new_workspace(D.device)
        info = torch.zeros(plan.S, dtype=torch.int32, device=D.device)
        x = r.detach().contiguous().clone()
        plan.factor_solve(D, C, B, corner, ws, x, info)
        ctx.plan, ctx.ws, ctx.info = plan, ws, info
        ctx.save_for_backward(x)
        ctx.mark_non_differentiable(info)
        return x, info

    @staticmethod
    def backward(ctx, gx, ginfo):
        (x,) = ctx.saved_tensors
        plan, ws = ctx.plan, ctx.ws
        lam = gx.detach().contiguous().clone()
        n = plan.pool_lengths()
        dev = x.device
        dD = torch.empty(n["D"], dtype=torch.float64, device=dev)
        dC = torch.empty(n["C"], dtype=torch.float64, device=dev)
        dB = torch.empty(n["B"], dtype=torch.float64, device=dev)
        dR = torch.empty(n["corner"], dtype=torch.float64, device=dev)
        plan.solve_adjoint(ws, x, lam, dD, dC, dB, dR)
        return dD, dC, dB, dR, lam, None


def kkt_solve_packed(D, C, B, corner, r, plan):
    """Differentiable solve on packed pools; returns (x, info)."""
    return KKTSolveFn.apply(D, C, B, corner, r, plan)


def kkt_solve(D, C, B, corner, r, segments=1):
    """Differentiable solve for a uniform batch.

    D [S, N, b, b], C [S, N-1, b, b], B [S, N, ng, b], corner [S, ng, ng],
    r [S, N*b + ng, nrhs]  ->  x with the shape of r (and info [S]).
    A uniform batch's pools are exactly these tensors, contiguous."""
    S, N, b = D.shape[0], D.shape[1], D.shape[2]
    ng = B.shape[2]
    nrhs = r.shape[2]
    plan = plan_for([(N, b, ng, segments)] * S, nrhs)
    x, info = KKTSolveFn.apply(D.reshape(-1), C.reshape(-1), B.reshape(-1), corner.reshape(-1),
                               r.reshape(-1), plan)
    return x.view(S, N * b + ng, nrhs), info
