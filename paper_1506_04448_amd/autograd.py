"""Autograd wrappers of the sketched objectives and the Adam refinement.

``SketchedTuuu``  f(u) = med_m <s^(m)(T), s^(m)(u (x) u (x) u)>, the T(u,u,u)
                  estimate of Eq. (3), for a batch of vectors; its backward is
                  the sum of the three mode read-offs (Proposition 1 with the
                  modes permuted) of the median's sketch.
``SketchedCPLoss`` (1/B) sum_m ||s^(m)(T) - sum_i lam_i s^(m)(u_i^(x)3)||^2, the
                  CP least-squares objective measured through the sketches
                  (linearity of Section 3.1); when gradients are wanted the
                  forward reads them off the same FP64 residual spectra and
                  the backward scales them.
``refine_adam``   torch.optim.Adam on (lam, U) of that loss, e.g. from the
                  output of the robust tensor power method.

Both functions call the HIP library for every step of the computation; the
Python side only moves tensors and scales.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import contract_tuuu_grad, contract_uuu, cp_loss


@dataclass
class SketchHandle:
    """A library context, its tables and the sketches of one tensor
    (S64 [B][b/2+1][2] float64; S32 its float32 copy, needed for float32 vectors)."""
    ctx: object
    tab: object
    S64: torch.Tensor
    S32: torch.Tensor | None = None


class SketchedTuuu(torch.autograd.Function):
    @staticmethod
    def forward(fctx, U, sk: SketchHandle):
        f_med, _ = contract_uuu(sk.ctx, sk.tab, U.detach().contiguous(), S64=sk.S64, S32=sk.S32)
        fctx.sk = sk
        fctx.save_for_backward(U)
        return f_med

    @staticmethod
    def backward(fctx, grad_f):
        (U,) = fctx.saved_tensors
        sk = fctx.sk
        scale = grad_f.to(U.dtype).contiguous()
        _, _, grad = contract_tuuu_grad(sk.ctx, sk.tab, U.detach().contiguous(), S64=sk.S64,
                                        S32=sk.S32, scale=scale)
        return grad, None


class SketchedCPLoss(torch.autograd.Function):
    @staticmethod
    def forward(fctx, lam, U, sk: SketchHandle):
        # The gradients are linear in the upstream gradient (a scalar), so when
        # they are wanted the one library call that forms the FP64 residual
        # spectra returns them with the loss, and the backward only scales them.
        want = any(fctx.needs_input_grad[:2])
        loss, g_lam, g_U = cp_loss(sk.ctx, sk.tab, sk.S64, lam.detach().contiguous(),
                                   U.detach().contiguous(), grads=want)
        if want:
            fctx.save_for_backward(g_lam, g_U)
        return loss

    @staticmethod
    def backward(fctx, grad_loss):
        g_lam, g_U = fctx.saved_tensors
        scale = grad_loss.to(g_U.dtype)
        return g_lam * scale, g_U * scale, None


def tuuu(U: torch.Tensor, sk: SketchHandle) -> torch.Tensor:
    """Differentiable T(u,u,u) estimates for the rows of U."""
    return SketchedTuuu.apply(U, sk)


def sketched_cp_loss(lam: torch.Tensor, U: torch.Tensor, sk: SketchHandle) -> torch.Tensor:
    """Differentiable sketched CP loss of (lam, U)."""
    return SketchedCPLoss.apply(lam, U, sk)


def refine_adam(sk: SketchHandle, lam0: torch.Tensor, U0: torch.Tensor, steps: int = 200,
                lr: float = 1e-3, dtype=torch.float32):
    """Adam on (lam, U) of the sketched CP loss from (lam0, U0); the vectors are
    not renormalised.  Returns (lam, U, losses [steps + 1] float64 tensor on the
    device: the loss before each step and after the last)."""
    lam = lam0.detach().to(dtype).clone().requires_grad_(True)
    U = U0.detach().to(dtype).clone().requires_grad_(True)
    opt = torch.optim.Adam([lam, U], lr=lr)
    losses = []
    for _ in range(steps):
        opt.zero_grad(set_to_none=True)
        loss = sketched_cp_loss(lam, U, sk)
        loss.backward()
        opt.step()
        losses.append(loss.detach())
    with torch.no_grad():
        losses.append(sketched_cp_loss(lam, U, sk).detach())
    return lam.detach(), U.detach(), torch.stack(losses)
