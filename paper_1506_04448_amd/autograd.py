"""Autograd wrappers of the sketched objectives and the Adam refinement.

``SketchedTuuu``  f(u) = med_m <s^(m)(T), s^(m)(u (x) u (x) u)>, the T(u,u,u)
                  estimate of Eq. (3), for a batch of vectors; its backward is
                  the sum of the three mode read-offs (Proposition 1 with the
                  modes permuted) of the median's sketch.
``SketchedCPLoss`` (1/B) sum_m ||s^(m)(T) - sum_i lam_i s^(m)(u_i^(x)3)||^2, the
                  CP least-squares objective measured through the sketches
                  (linearity of Section 3.1); its backward recomputes the FP64
                  residual spectra and reads the gradients off them.
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
        loss, _, _ = cp_loss(sk.ctx, sk.tab, sk.S64, lam.detach().contiguous(),
                             U.detach().contiguous(), grads=False)
        fctx.sk = sk
        fctx.save_for_backward(lam, U)
        return loss

    @staticmethod
    def backward(fctx, grad_loss):
        lam, U = fctx.saved_tensors
        sk = fctx.sk
        scale = grad_loss.reshape(1).to(U.dtype).contiguous()
        _, g_lam, g_U = cp_loss(sk.ctx, sk.tab, sk.S64, lam.detach().contiguous(),
                                U.detach().contiguous(), scale=scale, grads=True)
        return g_lam, g_U, None


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
