"""A thin object wrapper over the C ABI: one ``Lattice`` owns one nco_lattice.

Shapes follow the C ABI: populations (27, nz, ny, nx), velocity (3, nz, ny,
nx), node order x fastest.  Nothing here computes; it only reshapes arrays
and forwards calls to libnco.so.
"""
import math

import numpy as np

from . import _lib as L


def n_bins(n):
    """Number of spectrum shells for a cubic lattice of edge n."""
    return int(math.floor(math.sqrt(3.0) * (n // 2) + 0.5)) + 1


def batch_step(lattices, nsteps):
    """Advance lattice i by nsteps[i] steps in grouped dispatches
    (nco_batch_step); all lattices share one device and stream."""
    if len(nsteps) != len(lattices):
        raise ValueError("one step count per lattice")
    L.nco_batch_step([lat._h for lat in lattices], [int(s) for s in nsteps])


class Lattice:
    def __init__(self, shape, storage="f32", op="bgk", tau=0.6, stream=None):
        """shape = (nz, ny, nx).  stream: an integer hipStream_t (for example
        ``torch.cuda.current_stream().cuda_stream``) or None."""
        self.nz, self.ny, self.nx = (int(s) for s in shape)
        self.n = self.nx * self.ny * self.nz
        self.storage = storage
        self.op = op
        self.tau = float(tau)
        self.n_params = 2084          # width-32, depth-2 network until set_net_weights
        self._h = L.nco_lattice_create(self.nx, self.ny, self.nz, L.STORAGE[storage], L.OPS[op],
                                       self.tau, stream)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def close(self):
        if getattr(self, "_h", None):
            L.nco_lattice_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @staticmethod
    def bytes(shape, storage="f32"):
        nz, ny, nx = shape
        return L.nco_lattice_bytes(nx, ny, nz, L.STORAGE[storage])

    def set_op(self, op, tau=None):
        self.op = op
        if tau is not None:
            self.tau = float(tau)
        L.nco_set_op(self._h, L.OPS[op], self.tau)

    def set_rates(self, omega_high):
        L.nco_set_rates(self._h, omega_high)

    def set_net_weights(self, params, width, act="tanh", mlp_prec="f32", depth=2):
        """Network weights (order W1, b1, W2, b2, [W2b, b2b,] W3, b3); depth
        3 adds the third hidden layer (any arithmetic).
        mlp_prec: "f32" (vector units), "f32_mfma" (float32 matrix cores),
        "bf16" (bf16 products) or "f32_split" (float32-class products split
        over the 16-bit matrix cores)."""
        L.nco_set_net_weights(self._h, width, L.ACTS[act], L.MLP_PREC[mlp_prec], params, depth)
        self.n_params = int(np.asarray(params).size)

    def init_equilibrium(self, rho, u):
        L.nco_init_equilibrium(self._h, self.n, None if rho is None else np.asarray(rho).ravel(),
                               np.asarray(u).ravel())

    def init_populations(self, f):
        L.nco_init_populations(self._h, self.n, np.asarray(f).ravel())

    def step(self, nsteps=1):
        L.nco_step(self._h, int(nsteps))

    def sync(self):
        L.nco_sync(self._h)

    def restrict_from(self, fine):
        """Set this (coarse) lattice's state from the finer lattice ``fine``
        by acoustic scaling (Sec. "Learning Task"); see nco_restrict."""
        L.nco_restrict(fine._h, self._h)

    def set_domain(self, domain):
        """'periodic' (default) or 'tgv_octant': the cube [0, pi/2]^3 of the
        Taylor-Green vortex standing for the symmetric 4n box (Appendix A);
        initialise it with ``inputs.tgv3d_octant``."""
        L.nco_set_domain(self._h, domain)

    def set_stochastic_rounding(self, enable, seed=0):
        """Stochastic rounding of 16-bit deviation storage in the following
        steps (nco_set_stochastic_rounding)."""
        L.nco_set_stochastic_rounding(self._h, 1 if enable else 0, seed)

    def set_reverse_cache(self, nbytes):
        """Memory for network values kept between a recomputed step and its
        adjoint (nco_set_reverse_cache; 0: off)."""
        L.nco_set_reverse_cache(self._h, nbytes)

    def set_inplace(self, enable):
        """True (the default): pairs of BGK / fixed-rate steps run in place on
        one buffer where it fits the last-level cache (nco_set_inplace)."""
        L.nco_set_inplace(self._h, 1 if enable else 0)

    def set_check(self, every, mass_rel_tol):
        """Stability check every ``every`` steps (0: off); ``sync`` raises
        NCOError(NCO_E_UNSTABLE) once it has failed."""
        L.nco_set_check(self._h, every, mass_rel_tol)

    def populations(self):
        return L.nco_read_populations(self._h, self.n).reshape((27,) + self.shape)

    def macroscopic(self):
        rho, u = L.nco_read_macroscopic(self._h, self.n)
        return rho.reshape(self.shape), u.reshape((3,) + self.shape)

    def rates(self):
        return L.nco_read_rates(self._h, self.n).reshape((4,) + self.shape)

    def global_sums(self):
        return L.nco_global_sums(self._h)

    def energy_spectrum(self):
        return L.nco_energy_spectrum(self._h, n_bins(self.nx))

    def device_populations(self):
        return L.nco_device_populations(self._h)

    def set_forcing(self, k, draws, amplitude, kf, c, phase_rule=False):
        """Spectral forcing for the following steps; k=None switches it off.
        phase_rule: Alvelius' velocity-dependent theta1 (the reverse mode
        follows the force back to the state through it)."""
        L.nco_set_forcing(self._h, k, draws, amplitude, kf, c, phase_rule)

    def set_forcing_power(self, k, draws, power, ka, kb, kf, c, phase_rule=False):
        """Spectral forcing with the amplitude from the power input (lattice
        units: kinetic energy per unit mass per step) over the band
        ka <= |k| <= kb."""
        L.nco_set_forcing_power(self._h, k, draws, power, ka, kb, kf, c, phase_rule)

    def forward_record(self, nsteps, ckpt_every, energy_every=0):
        """Recorded run for backward(); with energy_every > 0 it returns the
        mean kinetic energy k(t) of the states t = 0, energy_every, ..."""
        if energy_every > 0:
            return L.nco_forward_record_energy(self._h, int(nsteps), int(ckpt_every), int(energy_every))
        L.nco_forward_record(self._h, int(nsteps), int(ckpt_every))
        return None

    def backward(self, dL_dE=None, dL_df=None, n_params=None, want_df0=False, dL_dk=None, energy_every=0):
        """Gradient of the recorded run: (dL/dtheta, dL/df0 or None), dL/dtheta
        in the order of the parameters given to set_net_weights.  dL_dk:
        loss gradient on the kinetic-energy samples of forward_record."""
        n_params = self.n_params if n_params is None else n_params
        df = None if dL_df is None else np.asarray(dL_df).ravel()
        if dL_dk is not None:
            g, df0 = L.nco_backward_energy(self._h, self.n, n_params, dL_dk, int(energy_every), dL_dE, df, want_df0)
        else:
            g, df0 = L.nco_backward(self._h, self.n, n_params, dL_dE, df, want_df0)
        return g, (None if df0 is None else df0.reshape((27,) + self.shape))
