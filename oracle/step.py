"""One lattice Boltzmann time step, literally (Sec. II.A), in float64.

Test infrastructure (see ``oracle/__init__``): never used by the product path.

Reading of the step order (the paper states f_i(x + c_i, t+1) =
f_i(x, t) + Omega_i + S_i and nothing about storage): the stored state is the
post-collision population; one step pull-streams it, f_i(x) <- f_i(x - c_i)
with periodic wrap, and then applies collision (and source) at every node.
Populations have shape (27, nz, ny, nx), x fastest.
"""
import numpy as np

from . import collision, lattice

_C = lattice.velocities()


def stream(f):
    """Pull streaming with periodic wrap: out_i(x) = f_i(x - c_i)."""
    out = np.empty_like(f)
    for i, (cx, cy, cz) in enumerate(_C):
        out[i] = np.roll(f[i], shift=(cz, cy, cx), axis=(0, 1, 2))
    return out


def unstream(f):
    """Inverse of ``stream`` (push streaming): out_i(x) = f_i(x + c_i)."""
    out = np.empty_like(f)
    for i, (cx, cy, cz) in enumerate(_C):
        out[i] = np.roll(f[i], shift=(-cz, -cy, -cx), axis=(0, 1, 2))
    return out


class Operator:
    """A collision operator and its parameters.

    kind: 'bgk' | 'mrt' (fixed higher-order rates) | 'nco'."""

    def __init__(self, kind, tau, omega_high=None, layers=None, act="tanh"):
        self.kind, self.tau, self.act = kind, float(tau), act
        self.omega_high = None if omega_high is None else np.asarray(omega_high, np.float64)
        self.layers = layers

    def collide(self, f):
        if self.kind == "bgk":
            return collision.bgk(f, self.tau)
        if self.kind == "mrt":
            w = self.omega_high.reshape((4,) + (1,) * (f.ndim - 1))
            return collision.moment_relaxation(f, self.tau, np.broadcast_to(w, (4,) + f.shape[1:]))
        if self.kind == "nco":
            return collision.nco(f, self.tau, self.layers, self.act)
        raise ValueError(self.kind)


def step(f, op, force=None):
    """One time step: pull-stream, collide, add the Kupershtokh source of the
    streamed state when a force field (3, nz, ny, nx) is given."""
    fs = stream(f)
    out = op.collide(fs)
    if force is not None:
        out = out + collision.kupershtokh_source(fs, force)
    return out


def run(f, op, nsteps, forces=None):
    """``nsteps`` steps; ``forces`` is None or a callable t -> force field."""
    for t in range(nsteps):
        f = step(f, op, None if forces is None else forces(t))
    return f
