"""torch.autograd.Functions around the hot path with hand-written adjoints
with respect to the MPO (the derivative pattern on top of DMRG3S).

HeffApply:  y = H_eff(W) psi (d3s_apply_heff, FP64);
            Wbar[w,v,s,t] = sum ybar[a,s,b] L[a,w,x] psi[x,t,y] R[b,v,y]
            (d3s_heff_grad_W), psibar = H_eff^T ybar (d3s_apply_heff with the
            bra/ket legs of L, W, R exchanged).  The environments are inputs
            without gradient.
MPOEnergy:  E(W_1..W_l) = <Psi|H|Psi> at a fixed MPS; backward returns
            dE/dW_i for every site (d3s_energy_gradients), so that for W_i
            depending on a coupling J, autograd yields dE/dJ, which equals
            <Psi|dH/dJ|Psi> (Hellmann-Feynman at an eigenstate).

The arithmetic runs in the HIP library; this module only wires it into
torch's autograd.
"""
import torch


class HeffApply(torch.autograd.Function):
    """y = H_eff(W) psi; backward gives Wbar (d3s_heff_grad_W) and
    psibar = H_eff^T ybar, which is H_eff applied with the bra/ket legs of L,
    W and R exchanged (d3s_apply_heff on transposed copies)."""

    @staticmethod
    def forward(ctx_, lib, L, W, R, psi):
        out = torch.empty_like(psi)
        lib.apply_heff(L, W, R, psi, out)
        ctx_.save_for_backward(L, W, R, psi)
        ctx_.lib = lib
        return out

    @staticmethod
    def backward(ctx_, ybar):
        L, W, R, psi = ctx_.saved_tensors
        lib = ctx_.lib
        ybar = ybar.contiguous()
        Wbar = psibar = None
        if ctx_.needs_input_grad[2]:
            Wbar = torch.empty_like(W)
            lib.heff_grad_W(L, R, psi, ybar, Wbar)
        if ctx_.needs_input_grad[4]:
            Lt = L.transpose(0, 2).contiguous()
            Wt = W.transpose(2, 3).contiguous()
            Rt = R.transpose(0, 2).contiguous()
            psibar = torch.empty_like(psi)
            lib.apply_heff(Lt, Wt, Rt, ybar, psibar)
        return None, None, Wbar, None, psibar


class MPOEnergy(torch.autograd.Function):
    """E(W_1, ..., W_l) = <Psi|H(W)|Psi> at a fixed normalised MPS.

    forward: the MPO tensors are copied into the state's MPO buffers and
    d3s_prepare returns the energy (it re-gauges the state, which leaves it
    unchanged); backward: d3s_energy_gradients gives dE/dW_i for all sites."""

    @staticmethod
    def forward(ctx_, lib, state, *Ws):
        for buf, W in zip(state.mpo, Ws):
            buf.copy_(W.detach().reshape(buf.shape))
        e = lib.prepare(state)
        ctx_.lib = lib
        ctx_.state = state
        return torch.tensor(e, dtype=torch.float64, device=Ws[0].device)

    @staticmethod
    def backward(ctx_, gE):
        grads = ctx_.lib.energy_gradients(ctx_.state)
        return (None, None) + tuple(gE * g for g in grads)


def heff_apply(lib, L, W, R, psi):
    """y = H_eff(W) psi with gradients with respect to W and psi."""
    return HeffApply.apply(lib, L, W, R, psi)


def mpo_energy(lib, state, Ws):
    """E = <Psi|H(W_1..W_l)|Psi>, differentiable in every W_i."""
    return MPOEnergy.apply(lib, state, *Ws)
