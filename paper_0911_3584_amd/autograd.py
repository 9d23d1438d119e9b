"""torch.autograd.Function for the LNV energy E(L) = 2 Tr(KH), K = 3LSL - 2LSLSL.

The forward pass runs the library's energy+gradient chain once and keeps
dE/dL (the adjoint of the truncated products); the backward pass scales it by
the upstream gradient.  S and H are treated as constants.
"""
import torch


class LNVEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, L, S, H, lnv, prec="fp64"):
        E, G = lnv.energy_grad(L.detach(), S.detach(), H.detach(), prec=prec)
        ctx.save_for_backward(G)
        return E.reshape(())

    @staticmethod
    def backward(ctx, gE):
        (G,) = ctx.saved_tensors
        return gE * G, None, None, None, None
