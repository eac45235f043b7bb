"""Training of the network on the GPU: spectrum loss, torch autograd
wrapper and Adam (Sec. "Learning Task": Adam on a loss of the energy
spectrum after an unrolled run).

All lattice arithmetic, forward and backward, runs in libnco.so; this module
computes the loss on the (nbins) spectrum values and hands the parameter
vector to torch only so that a torch optimiser can update it.
"""
import numpy as np

from .lattice import Lattice, n_bins


def log_spectrum_loss(E, E_target, kmin, kmax):
    """L = mean over kmin <= k <= kmax of (ln E(k) - ln E_t(k))^2 and dL/dE."""
    ks = np.arange(kmin, kmax + 1)
    r = np.log(E[ks]) - np.log(E_target[ks])
    dE = np.zeros_like(E)
    dE[ks] = 2.0 * r / (len(ks) * E[ks])
    return float(np.mean(r * r)), dE


class Unroll:
    """One training sample: initial populations (or fields), forcing and the
    unroll length; evaluates the loss and its gradient for given parameters
    on a lattice that stays resident on the device."""

    def __init__(self, shape, tau, init, nsteps, ckpt_every, target, kmin, kmax, forcing=None,
                 storage="f32", act="tanh", mlp="f32_mfma", width=32, stream=None):
        self.lat = Lattice(shape, storage, "nco", tau, stream=stream)
        self.init, self.nsteps, self.ckpt_every = init, int(nsteps), int(ckpt_every)
        self.target, self.kmin, self.kmax = np.asarray(target, np.float64), int(kmin), int(kmax)
        self.forcing, self.act, self.mlp, self.width = forcing, act, mlp, width

    def _reset(self, params):
        lat = self.lat
        lat.set_net_weights(params, self.width, self.act, self.mlp)
        if self.init[0] == "eq":
            lat.init_equilibrium(self.init[1], self.init[2])
        else:
            lat.init_populations(self.init[1])
        if self.forcing is None:
            lat.set_forcing(None, None, 0.0, 0.0, 1.0)
        else:
            lat.set_forcing(*self.forcing)

    def loss(self, params):
        self._reset(params)
        self.lat.step(self.nsteps)
        return log_spectrum_loss(self.lat.energy_spectrum(), self.target, self.kmin, self.kmax)[0]

    def loss_and_grad(self, params):
        self._reset(params)
        self.lat.forward_record(self.nsteps, self.ckpt_every)
        E = self.lat.energy_spectrum()
        L, dE = log_spectrum_loss(E, self.target, self.kmin, self.kmax)
        g, _ = self.lat.backward(dL_dE=dE)
        return L, g, E

    def close(self):
        self.lat.close()


def make_autograd(unroll):
    """torch.autograd.Function computing the loss of ``unroll`` from a flat
    float64 parameter tensor, with the hand-written adjoint as backward."""
    import torch

    class NCOUnrollLoss(torch.autograd.Function):
        @staticmethod
        def forward(ctx, params):
            L, g, _ = unroll.loss_and_grad(params.detach().cpu().numpy())
            ctx.save_for_backward(torch.from_numpy(g))
            return params.new_tensor(L)

        @staticmethod
        def backward(ctx, grad_out):
            (g,) = ctx.saved_tensors
            return grad_out * g.to(grad_out.device, grad_out.dtype)

    return NCOUnrollLoss.apply


def train(unrolls, params0, epochs, lr=1e-3, log=None):
    """Adam (torch.optim) over the given samples; returns (params, losses)."""
    import torch
    p = torch.nn.Parameter(torch.tensor(np.asarray(params0, np.float64)))
    opt = torch.optim.Adam([p], lr=lr)
    fns = [make_autograd(u) for u in unrolls]
    history = []
    for ep in range(epochs):
        total = 0.0
        for fn in fns:
            opt.zero_grad()
            loss = fn(p)
            loss.backward()
            opt.step()
            with torch.no_grad():
                p.copy_(p.float().double())          # parameters live as float32 values
            total += float(loss.detach())
        history.append(total / len(fns))
        if log:
            log("epoch %d: loss %.6f" % (ep, history[-1]))
    return p.detach().numpy().copy(), history


__all__ = ["log_spectrum_loss", "Unroll", "make_autograd", "train", "n_bins"]
