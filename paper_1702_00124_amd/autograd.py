"""Pseudofermion action as a differentiable torch function.

S = PseudofermionAction.apply(omega, phi, lattice, term): the action of one
pseudofermion term (Sec. 2 and 4.1) at the links U = exp(i omega^a T^a) U0,
U0 the lattice's current links, omega a float64 tensor [4, V, 8] of su(3)
coefficients per link.  The backward is the library's force kernel: the Lie
derivative grad^a S = d/de S(exp(i e T^a) U)|_0 at U, times the incoming
gradient.  At omega = 0 this is exactly dS/domega; for omega != 0 it is the
Lie derivative at the rotated links (the derivative the HMC momentum update
uses), not the derivative through the exponential map.

Every computation runs in libwilson_hmc; torch only holds the buffers and the
graph.  The lattice's links are restored to U0 before forward returns.
"""
from __future__ import annotations

import torch

from .lattice import Term, WilsonLattice


class PseudofermionAction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, omega: torch.Tensor, phi: torch.Tensor, lat: WilsonLattice, term: Term):
        if omega.shape != (4, lat.V, 8):
            raise ValueError(f"omega must be [4, {lat.V}, 8]")
        U0 = lat.get_links()
        rotated = bool(torch.any(omega != 0))
        try:
            if rotated:
                lat.link_update(lat.import_su3(omega.detach()), 1.0)
            S = lat.action(term, phi)
            F = lat.export_su3(lat.fermion_force(term, phi)) if ctx.needs_input_grad[0] else None
        finally:
            if rotated:
                lat.set_links(U0)
        ctx.save_for_backward(F if F is not None else torch.empty(0, device=omega.device))
        return torch.tensor(S, dtype=torch.float64, device=omega.device)

    @staticmethod
    def backward(ctx, grad_S):
        (F,) = ctx.saved_tensors
        if F.numel() == 0:
            return None, None, None, None
        return grad_S * F, None, None, None


def pseudofermion_action(omega: torch.Tensor, phi: torch.Tensor, lat: WilsonLattice, term: Term) -> torch.Tensor:
    return PseudofermionAction.apply(omega, phi, lat, term)
