"""torch.autograd front end of the ghost fill, surface evaluation and force
sums.  Every forward and backward step is a call into the gcr library (the
backward ones run its reverse-level adjoint kernels); this module only
allocates outputs and passes pointers.

The fill is affine in (interior field, boundary data): with phi = fill(u, b)
the ghost relations of Sec. 4 (Eqs. A14-A17) make every ghost value a fixed
linear combination of its stencil cells and of b.  Its adjoint therefore
needs no saved activations, only the plan.  Gradients with respect to the
geometry are not provided (the plan is a constant of these functions).
"""
from typing import Optional, Sequence

import torch

from . import Plan


def _f64(t: torch.Tensor) -> torch.Tensor:
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("gcr autograd: expects contiguous float64 tensors")
    return t


class GhostFill(torch.autograd.Function):
    """Filled copies of nf fields (Sec. 3.2 level order, Sec. 4 relations).

    apply(plan, bc_kind, bc_type, nf, *fields, *bc_vals) -> nf tensors.
    Ghost slots of each input are overwritten in the output, so their
    gradient is zero; every other slot of an output is its input.
    Backward runs gcr_fill_adjoint (levels in reverse) and returns
    dJ/d(input field) and dJ/d(bc value) per ghost."""

    @staticmethod
    def forward(ctx, plan: Plan, bc_kind, bc_type, nf: int, *tensors):
        fields = [_f64(t) for t in tensors[:nf]]
        bc_val = [_f64(t) for t in tensors[nf:]]
        out = [f.clone() for f in fields]
        plan.fill(out, bc_kind, bc_val, bc_type)
        ctx.plan, ctx.bc_kind, ctx.bc_type, ctx.nf = plan, list(bc_kind), bc_type, nf
        ctx.dev = fields[0].device
        return tuple(out)

    @staticmethod
    def backward(ctx, *grads):
        plan, nf = ctx.plan, ctx.nf
        lam = [torch.zeros(plan.n_cells, dtype=torch.float64, device=ctx.dev) if g is None
               else g.detach().to(torch.float64).contiguous().clone() for g in grads]
        lam_bc = [torch.empty(plan.n_ghost, dtype=torch.float64, device=ctx.dev)
                  for _ in range(nf)]
        plan.fill_adjoint(lam, ctx.bc_kind, lam_bc, ctx.bc_type)
        return (None, None, None, None, *lam, *lam_bc)


class SurfaceEval(torch.autograd.Function):
    """Values and gradients at caller points xq [dim][nq] (Sec. 6, anchor
    ghost's interpolant).  apply(plan, xq, *fields) -> (val [nf][nq],
    grad [nf][dim][nq]).  Backward: gcr_surface_adjoint into dense zeros."""

    @staticmethod
    def forward(ctx, plan: Plan, xq: torch.Tensor, *fields):
        fields = [_f64(f) for f in fields]
        val, grad, _ = plan.surface(_f64(xq), fields)
        ctx.plan, ctx.xq, ctx.nf, ctx.dev = plan, xq, len(fields), fields[0].device
        return val, grad

    @staticmethod
    def backward(ctx, gval, ggrad):
        plan = ctx.plan
        lam = [torch.zeros(plan.n_cells, dtype=torch.float64, device=ctx.dev)
               for _ in range(ctx.nf)]
        gv = None if gval is None else gval.detach().to(torch.float64).contiguous()
        gg = None if ggrad is None else ggrad.detach().to(torch.float64).contiguous()
        if gv is not None or gg is not None:
            plan.surface_adjoint(ctx.xq, gv, gg, lam)
        return (None, None, *lam)


class Forces(torch.autograd.Function):
    """Force on the body, F = sum_q w_q (-p n_q + mu (grad u + grad u^T) n_q)
    (Sec. 6).  apply(plan, xq, nrm, wq, mu, p, *u) -> F [dim].  Backward:
    gcr_forces_adjoint into dense zeros (no gradient for xq, nrm, wq, mu)."""

    @staticmethod
    def forward(ctx, plan: Plan, xq, nrm, wq, mu: float, p, *u):
        F = plan.forces(_f64(xq), _f64(nrm), _f64(wq), _f64(p), [_f64(c) for c in u], mu)
        ctx.plan, ctx.args, ctx.mu, ctx.nu, ctx.dev = plan, (xq, nrm, wq), mu, len(u), p.device
        return F

    @staticmethod
    def backward(ctx, gF):
        plan = ctx.plan
        xq, nrm, wq = ctx.args
        lam_p = torch.zeros(plan.n_cells, dtype=torch.float64, device=ctx.dev)
        lam_u = [torch.zeros(plan.n_cells, dtype=torch.float64, device=ctx.dev)
                 for _ in range(ctx.nu)]
        plan.forces_adjoint(xq, nrm, wq, ctx.mu, gF.detach().to(torch.float64).contiguous(),
                            lam_p, lam_u)
        return (None, None, None, None, None, lam_p, *lam_u)


def ghost_fill(plan: Plan, fields: Sequence[torch.Tensor], bc_kind: Sequence[int],
               bc_val: Sequence[torch.Tensor], bc_type: Optional[Sequence] = None):
    """Differentiable fill: returns new filled tensors (inputs untouched)."""
    return GhostFill.apply(plan, list(bc_kind), bc_type, len(fields), *fields, *bc_val)


def surface(plan: Plan, xq: torch.Tensor, fields: Sequence[torch.Tensor]):
    return SurfaceEval.apply(plan, xq, *fields)


def forces(plan: Plan, xq, nrm, wq, p, u: Sequence[torch.Tensor], mu: float = 1.0):
    return Forces.apply(plan, xq, nrm, wq, float(mu), p, *u)
