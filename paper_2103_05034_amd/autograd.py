"""The pseudofermion action as a differentiable function of the gauge links.

The Conclusions section motivates the solver by HMC sampling of the
two-flavour determinant det(M^dag M).  Its pseudofermion estimate is

    S(U) = phi^dag (M_pc^dag M_pc)^{-1} phi,

and HMC needs dS/dU.  :class:`PseudofermionAction` exposes S to
``torch.autograd``: the forward pass solves ``A X = phi`` with ``dwf_cg`` and
takes ``S = Re <phi, X>`` from ``dwf_dot``; the backward pass forms
``Y = M_pc X`` with ``dwf_mpc`` and the link gradient with the adjoint kernel
behind ``dwf_force``.  Every step runs in libdwf; this module only marshals
tensors and applies the chain rule's scalar factor.

Gradient convention (PyTorch's for complex inputs): ``U.grad`` holds
``dS/dRe U + i dS/dIm U``, so that ``dS = Re sum(conj(U.grad) * dU)``.  The
gradient with respect to ``phi`` is ``2 X`` on the even sites (A is
Hermitian).
"""

from __future__ import annotations

import torch

from . import DWF_EVEN, DWF_F64, DWFError, DWF_EINVAL


class PseudofermionAction(torch.autograd.Function):
    """S = PseudofermionAction.apply(U, phi, op, tol=1e-12, maxiter=100000).

    ``U``: complex128 links ``[T][Z][Y][X][4][3][3]`` on the operator's device
    (may require grad); ``phi``: complex128 natural 5D field
    ``[Ls][T][Z][Y][X][4][3]`` of which the even sites are used; ``op``: an
    FP64 :class:`Operator` on the same lattice with ``max_cg_rhs >= 1``.  Its
    links are replaced by ``U`` (forward) and restored from the saved ``U``
    before the backward pass if another call changed them.  Returns S as a
    real 0-dim float64 tensor.  Raises :class:`DWFError` if CG does not reach
    ``tol``.
    """

    @staticmethod
    def forward(ctx, U, phi, op, tol=1e-12, maxiter=100000):
        if op.prec != DWF_F64 or op.max_cg_rhs < 1:
            raise DWFError(DWF_EINVAL, "PseudofermionAction needs an FP64 Operator with max_cg_rhs >= 1")
        op.update_links(U.detach())
        phi_p = op.pack(phi.detach()[None], DWF_EVEN)
        X = op.new_field(1)
        op.cg(phi_p, X, 1, tol=tol, maxiter=maxiter)
        s = op.dot(phi_p, X, 1)
        ctx.op = op
        ctx.U = op.U  # the links the saved X belongs to
        ctx.save_for_backward(X)
        return s.real[0].clone()

    @staticmethod
    def backward(ctx, grad_S):
        (X,) = ctx.saved_tensors
        op = ctx.op
        if op.U is not ctx.U:
            op.update_links(ctx.U)
        grad_U = grad_phi = None
        if ctx.needs_input_grad[0]:
            Y = op.new_field(1)
            op.mpc(X, Y, 1, False)
            grad_U = op.force(X, Y) * grad_S
        if ctx.needs_input_grad[1]:
            grad_phi = op.unpack(X, 1, DWF_EVEN)[0] * (2.0 * grad_S)
        return grad_U, grad_phi, None, None, None
