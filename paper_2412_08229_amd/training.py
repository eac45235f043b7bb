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


def paper_spectrum_loss(E, E_target, kmin=4, kmax=10, omega=20.0, kappa_max=None):
    """The loss of Eq. (loss) in Sec. "Learning Task": the mean squared gap
    of the spectrum to the target over kmin <= k <= kmax plus omega E(kappa_max),
    which presses down the energy piling up at the grid cutoff; kappa_max is
    the shell N/2 of an N^3 box (without it, the smallest N whose spectrum
    has len(E) shells is taken).  Returns (L, dL/dE)."""
    E = np.asarray(E, np.float64)
    ks = np.arange(kmin, kmax + 1)
    kc = int(kappa_max) if kappa_max is not None else _cutoff_shell(len(E))
    r = E[ks] - E_target[ks]
    dE = np.zeros_like(E)
    dE[ks] = 2.0 * r / len(ks)
    dE[kc] += omega
    return float(np.mean(r * r) + omega * E[kc]), dE


def _cutoff_shell(nbins):
    """N/2 for a spectrum of n_bins(N) shells."""
    for n in range(2, 4 * nbins):
        if n_bins(n) == nbins:
            return n // 2
    raise ValueError("no lattice size has %d shells" % nbins)


class Unroll:
    """One training sample: initial populations (or fields), forcing and the
    unroll length; evaluates the loss and its gradient for given parameters
    on a lattice that stays resident on the device.  forcing: None or the
    arguments of ``Lattice.set_forcing``, (k, draws, amplitude, kf, c) with
    an optional sixth, phase_rule."""

    def __init__(self, shape, tau, init, nsteps, ckpt_every, target, kmin, kmax, forcing=None,
                 storage="f32", act="tanh", mlp="f32_mfma", width=32, stream=None, loss="log", omega=20.0):
        self.lat = Lattice(shape, storage, "nco", tau, stream=stream)
        self.init, self.nsteps, self.ckpt_every = init, int(nsteps), int(ckpt_every)
        self.target, self.kmin, self.kmax = np.asarray(target, np.float64), int(kmin), int(kmax)
        self.forcing, self.act, self.mlp, self.width = forcing, act, mlp, width
        # 'log': mean squared log gap over kmin..kmax; 'paper': Eq. (loss),
        # the squared gap over kmin..kmax plus omega E(N/2).
        self.loss_kind, self.omega = loss, float(omega)

    def _loss(self, E):
        if self.loss_kind == "paper":
            return paper_spectrum_loss(E, self.target, self.kmin, self.kmax, self.omega, self.lat.nx // 2)
        return log_spectrum_loss(E, self.target, self.kmin, self.kmax)

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
        return self._loss(self.lat.energy_spectrum())[0]

    def loss_and_grad(self, params):
        self._reset(params)
        self.lat.forward_record(self.nsteps, self.ckpt_every)
        E = self.lat.energy_spectrum()
        L, dE = self._loss(E)
        g, _ = self.lat.backward(dL_dE=dE)
        return L, g, E

    def close(self):
        self.lat.close()


class DissipationUnroll:
    """One dissipation-rate training sample (the loss of the Taylor-Green
    training of Sec. "Training based on dissipation rates"): a recorded run
    of nsteps steps from the fields (rho, u) whose mean kinetic energy k(t)
    is sampled every ``every`` steps; the dissipation rate eps = -dk/dt
    (centred differences, k in units of u0^2, t in convective units L / u0
    with L = N / 2 pi for a box of N nodes per edge) is compared with
    eps_ref(t) over t_min <= t:  L = mean ((eps - eps_ref) / max eps_ref)^2.

    domain: 'periodic' (the box itself) or 'tgv_octant', the reduced cube of
    Appendix A, whose n nodes per edge stand for the N = 4n box (fields from
    ``inputs.tgv3d_octant``).  depth: hidden layers of the network (3 adds
    the paper's extra layer for this training; vector-unit network, mlp
    'f32')."""

    def __init__(self, shape, tau, rho, u, u0, nsteps, ckpt_every, every, eps_ref, t_min=1.0,
                 storage="f32", act="tanh", mlp="f32_mfma", width=32, stream=None, domain="periodic", depth=2):
        self.lat = Lattice(shape, storage, "nco", tau, stream=stream)
        self.depth = int(depth)
        if domain != "periodic":
            self.lat.set_domain(domain)
        self.rho, self.u, self.u0 = rho, u, float(u0)
        self.nsteps, self.ckpt_every, self.every = int(nsteps), int(ckpt_every), int(every)
        self.act, self.mlp, self.width = act, mlp, width
        L = shape[-1] * (4 if domain == "tgv_octant" else 1) / (2.0 * np.pi)
        self.dt = self.every * self.u0 / L                       # convective time between samples
        m = self.nsteps // self.every + 1
        self.t = np.arange(m) * self.dt
        self.inner = np.arange(1, m - 1)
        self.inner = self.inner[self.t[self.inner] >= t_min]
        self.eps_ref = np.array([eps_ref(t) for t in self.t[self.inner]])
        self.scale = float(np.max(np.abs(self.eps_ref)))

    def _run(self, params):
        lat = self.lat
        lat.set_net_weights(params, self.width, self.act, self.mlp, depth=self.depth)
        lat.init_equilibrium(self.rho, self.u)
        k = lat.forward_record(self.nsteps, self.ckpt_every, energy_every=self.every) / self.u0 ** 2
        eps = -(k[self.inner + 1] - k[self.inner - 1]) / (2.0 * self.dt)
        r = (eps - self.eps_ref) / self.scale
        return k, eps, r

    def curve(self, params):
        """(t, eps) of the run with these parameters."""
        _, eps, _ = self._run(params)
        return self.t[self.inner], eps

    def loss(self, params):
        return float(np.mean(self._run(params)[2] ** 2))

    def loss_and_grad(self, params):
        k, eps, r = self._run(params)
        L = float(np.mean(r ** 2))
        # dL/deps_m = 2 r_m / (scale |window|); eps_m = -(k_{m+1} - k_{m-1}) / (2 dt); k = k_raw / u0^2.
        de = 2.0 * r / (self.scale * len(r))
        dk = np.zeros_like(k)
        np.add.at(dk, self.inner + 1, -de / (2.0 * self.dt))
        np.add.at(dk, self.inner - 1, de / (2.0 * self.dt))
        g, _ = self.lat.backward(dL_dk=dk / self.u0 ** 2, energy_every=self.every)
        return L, g, None

    def close(self):
        self.lat.close()


def tgv_cube_energy(kind, n, re, u0, t_end, samples, params=None, tau=None, every=None, nsamp=None,
                    width=32, act="tanh", mlp="f32_mfma", stream=None, depth=2):
    """Mean kinetic energy k(t) / u0^2 of the Taylor-Green vortex on the
    reduced n^3 cube of Appendix A (the box of 4n nodes per edge), sampled
    at t = 0, every, 2 every, ... steps; t in convective units.

    Either (re, t_end, samples): tau from the Reynolds number of the 4n box
    and ``samples`` intervals over [0, t_end]; or (tau, every, nsamp)
    directly.  kind: 'bgk', 'mrt' (orders 3..6 relaxed at 4/3, the network's
    rates at a zero output) or 'nco' with ``params``.  A run whose global
    sums stop being finite ends there.  Returns (t, k, status)."""
    from . import inputs
    from . import _lib as L
    N = 4 * n
    tc = N / (2.0 * np.pi) / u0                      # steps per convective time
    if tau is None:
        tau = inputs.viscosity(N, u0, re)[1]
    if every is None:
        every = max(1, int(round(t_end * tc / samples)))
        nsamp = int(round(t_end * tc / every))
    rho, u = inputs.tgv3d_octant(n, u0)
    ts, ks, status = [0.0], [], "stable"
    with Lattice((n, n, n), "f32", kind, tau, stream=stream) as lat:
        lat.set_domain("tgv_octant")
        if kind == "nco":
            lat.set_net_weights(params, width, act, mlp, depth=depth)
        if kind == "mrt":
            lat.set_rates([4.0 / 3.0] * 4)
        lat.init_equilibrium(rho, u)
        ks.append(lat.global_sums()[4] / lat.n / u0 ** 2)
        for i in range(nsamp):
            lat.step(every)
            try:
                s = lat.global_sums()
            except L.NCOError:
                status = "unstable at t = %.2f" % ((i + 1) * every / tc)
                break
            ts.append((i + 1) * every / tc)
            ks.append(s[4] / lat.n / u0 ** 2)
    return np.array(ts), np.array(ks), status


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


def curriculum_steps(epoch, start=200, grow=200, every=10):
    """Unroll length of the curriculum of Sec. "Learning Task": the loss is
    first taken after 200 steps, and 200 more every ten epochs."""
    return start + grow * (epoch // every)


ADAM_EPS_REL = 1e-8


def _scale_free_eps(opt, grad):
    """Adam's epsilon as a fraction of the first gradient's RMS (once).  Adam's
    step is then independent of the loss's scale: the paper's loss on
    lattice-unit spectra (~1e-5, losses ~1e-10 on small lattices) would
    otherwise leave every update under a fixed epsilon of 1e-8."""
    group = opt.param_groups[0]
    if group.get("eps_set"):
        return
    rms = float(np.sqrt(np.mean(np.square(np.asarray(grad, np.float64)))))
    if rms > 0.0 and np.isfinite(rms):
        group["eps"] = ADAM_EPS_REL * rms
        group["eps_set"] = True


def train(unrolls, params0, epochs, lr=1e-3, log=None, schedule=None):
    """Adam (torch.optim, epsilon relative to the first gradient) over the
    given samples; returns (params, losses).  schedule: None, or a function
    epoch -> unroll length (e.g. ``curriculum_steps``) applied to every
    sample at the start of an epoch."""
    import torch
    p = torch.nn.Parameter(torch.tensor(np.asarray(params0, np.float64)))
    opt = torch.optim.Adam([p], lr=lr)
    fns = [make_autograd(u) for u in unrolls]
    history = []
    for ep in range(epochs):
        if schedule is not None:
            for u in unrolls:
                u.nsteps = int(schedule(ep))
        total = 0.0
        for fn in fns:
            opt.zero_grad()
            loss = fn(p)
            loss.backward()
            _scale_free_eps(opt, p.grad.detach().numpy())
            opt.step()
            with torch.no_grad():
                p.copy_(p.float().double())          # parameters live as float32 values
            total += float(loss.detach())
        history.append(total / len(fns))
        if log:
            log("epoch %d: loss %.6f" % (ep, history[-1]))
    return p.detach().numpy().copy(), history


def train_batched(unrolls, params0, epochs, lr=1e-3, log=None, schedule=None):
    """Adam (epsilon relative to the first gradient) with one step per epoch
    on the mean loss of all samples.  The
    samples' recorded runs and reverse sweeps go concurrently, one host
    thread per sample, each lattice on its own stream (the library's calls
    on different lattices are independent and release the interpreter
    lock), so that small lattices share the device instead of queueing.
    schedule: None, or a function epoch -> unroll length set on every sample
    before that epoch (the curriculum of Sec. "Learning Task").
    Returns (params, mean loss per epoch)."""
    from concurrent.futures import ThreadPoolExecutor

    import torch
    p = torch.nn.Parameter(torch.tensor(np.asarray(params0, np.float64)))
    opt = torch.optim.Adam([p], lr=lr)
    history = []
    with ThreadPoolExecutor(max_workers=len(unrolls)) as pool:
        for ep in range(epochs):
            if schedule is not None:
                for u in unrolls:
                    u.nsteps = int(schedule(ep))
            x = p.detach().numpy().copy()
            res = list(pool.map(lambda u: _loss_and_grad_or_none(u, x), unrolls))
            # A sample whose run has blown up (non-finite loss or gradient)
            # sits this epoch out instead of poisoning the step.
            ok = [r for r in res if r is not None]
            history.append(float(np.mean([r[0] for r in ok])) if ok else float("nan"))
            if log:
                log("epoch %d: loss %.6f (%d of %d samples finite)" % (ep, history[-1], len(ok), len(res)))
            if not ok:
                break
            opt.zero_grad()
            p.grad = torch.from_numpy(np.mean([r[1] for r in ok], axis=0))
            _scale_free_eps(opt, p.grad.numpy())
            opt.step()
            with torch.no_grad():
                p.copy_(p.float().double())          # parameters live as float32 values
    return p.detach().numpy().copy(), history


def _loss_and_grad_or_none(unroll, params):
    from ._lib import NCOError
    try:
        L, g, _ = unroll.loss_and_grad(params)
    except NCOError:
        return None
    if not (np.isfinite(L) and np.all(np.isfinite(g))):
        return None
    return L, g


__all__ = ["log_spectrum_loss", "paper_spectrum_loss", "curriculum_steps", "Unroll", "DissipationUnroll", "tgv_cube_energy", "make_autograd", "train",
           "train_batched", "n_bins"]
