"""torch.autograd.Function around the library's solve and adjoint.

X = K^{-1} B for the block-sparse complex-symmetric K given as the flat K
buffer (see include/d3m.h).  The backward pass reuses the factors: because
K = K^T, lambda = K^{-1} g needs no second factorization, and the gradient on
K lives on K's block pattern (Sec. II of the paper: the dual solution step;
the adjoint is the library's way of differentiating it).

Conventions.  The C ABI is holomorphic: for J = sum_k Re(c_k^T x_k) it takes
G = C and returns Lambda = K^{-1} G and dK = -sym(Lambda X^T) per block.
PyTorch hands backward grad_X = conj(dJ/dX) and expects conjugated
gradients, so this wrapper passes G = conj(grad_X) and returns conj(Lambda)
for B.  For the flat K buffer the library returns the gradient with respect
to the stored entries (d3m_options.dk_stored): a diagonal block is read from
its lower triangle, so its strictly-lower entries carry both (i,j) and (j,i),
its diagonal one entry and its upper triangle none; a stored off-diagonal
block also carries its mirror K_JI = K_IJ^T.  The wrapper only conjugates.
"""
from __future__ import annotations

import torch

from . import C128, Factor


class D3MSolve(torch.autograd.Function):
    """X = D3MSolve.apply(K, B, plan, precision); differentiable in K and B."""

    @staticmethod
    def forward(ctx, K, B, plan, precision=C128, tol=1e-10):
        f = Factor(plan, precision, nrhs_max=B.shape[0], tol=tol, dk_stored=True)
        f.factorize(K.detach())
        X = f.solve(B.detach().contiguous())
        ctx.factor = f
        ctx.save_for_backward(X)
        return X

    @staticmethod
    def backward(ctx, grad_X):
        (X,) = ctx.saved_tensors
        f = ctx.factor
        G = torch.conj(grad_X).resolve_conj().contiguous()
        want_k = ctx.needs_input_grad[0]
        Lam, dK = f.adjoint(X, G, want_dK=want_k)
        gB = torch.conj(Lam).resolve_conj() if ctx.needs_input_grad[1] else None
        gK = torch.conj(dK).resolve_conj() if want_k else None
        return gK, gB, None, None, None


def solve(K, B, plan, precision=C128, tol=1e-10):
    return D3MSolve.apply(K, B, plan, precision, tol)
