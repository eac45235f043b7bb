"""Pins of the reduced Taylor-Green domain (Appendix A) in the oracle.

The reduced step is defined through the symmetry group of the vortex; these
tests tie that group to the analytic initial field of Eq. tgv3d_equation and
to the periodic oracle, independently of how the group is used.
"""
import numpy as np
import pytest

from oracle import collision, lattice, observables, reduced, step
from paper_2412_08229_amd import inputs

U0 = 0.05


def _field_at(u, rho, A, b, n):
    """rho and u of the full offset-grid box at the images g x of all nodes."""
    N = 4 * n
    P = 2 * np.arange(N) + 1
    Z, Y, X = np.meshgrid(P, P, P, indexing="ij")
    img = (np.tensordot(A, np.stack([X, Y, Z]), axes=1) + b.reshape(3, 1, 1, 1)) % (8 * n)
    jx, jy, jz = (img - 1) // 2
    return rho[jz, jy, jx], u[:, jz, jy, jx]


@pytest.mark.parametrize("n", [1, 2, 3])
def test_group_order_and_tiling(n):
    G = reduced.symmetry_group(n)
    assert len(G) == 64
    for A, _ in G:  # signed permutation matrices
        assert (np.abs(A).sum(0) == 1).all() and (np.abs(A).sum(1) == 1).all()
    # The cube's images cover every node of the 4n box exactly once.
    reduced.unfold(np.zeros((27, n, n, n)))


@pytest.mark.parametrize("n", [2, 3])
def test_every_symmetry_maps_the_vortex_to_itself(n):
    """rho(g x) = rho(x), u(g x) = A u(x) at every node of the box, for every
    group element (the group is generated from maps read off the field)."""
    rho, u = inputs.tgv3d(4 * n, U0, offset=0.5)
    for A, b in reduced.symmetry_group(n):
        rg, ug = _field_at(u, rho, A, b, n)
        assert np.abs(rg - rho).max() < 1e-15
        assert np.abs(ug - np.tensordot(A, u, axes=1)).max() < 1e-15


def test_unfold_equals_the_full_vortex():
    n = 3
    rho, u = inputs.tgv3d_octant(n, U0)
    rhoF, uF = inputs.tgv3d(4 * n, U0, offset=0.5)
    full = reduced.unfold(collision.equilibrium(rho, u))
    assert np.abs(full - collision.equilibrium(rhoF, uF)).max() < 1e-15


def test_wrong_generator_is_caught(monkeypatch):
    """A plausible mistake (the quarter turn taken about the box's z axis
    instead of the vortex axis x = y = pi/2) no longer reproduces the vortex."""
    n = 2
    good = reduced.generators

    def bad(nn):
        g = good(nn)
        A, b = g[3]
        g[3] = (A, np.zeros_like(b))
        return g

    monkeypatch.setattr(reduced, "generators", bad)
    rho, u = inputs.tgv3d_octant(n, U0)
    rhoF, uF = inputs.tgv3d(4 * n, U0, offset=0.5)
    try:
        full = reduced.unfold(collision.equilibrium(rho, u))
    except AssertionError:
        return  # the images no longer tile the box
    assert np.abs(full - collision.equilibrium(rhoF, uF)).max() > 1e-3


@pytest.mark.parametrize("kind", ["bgk", "nco"])
def test_reduced_run_equals_the_periodic_box(kind):
    """The periodic dynamics keep the vortex's symmetries (equivariant
    collision, Sec. II.B): the reduced lattice run equals the 4n box run,
    restricted, to float64 rounding."""
    n = 2
    rho, u = inputs.tgv3d_octant(n, U0)
    rhoF, uF = inputs.tgv3d(4 * n, U0, offset=0.5)
    layers = collision.unpack_params(inputs.mlp_params(32, 0), 32)
    op = step.Operator(kind, 0.51, layers=layers)
    fr = reduced.run(collision.equilibrium(rho, u), op, 4)
    ff = step.run(collision.equilibrium(rhoF, uF), op, 4)
    assert np.abs(fr - reduced.restrict(ff, n)).max() < 1e-14
    assert np.abs(fr - collision.equilibrium(rho, u)).max() > 1e-4  # the state moved
    # Mean kinetic energy of the cube = that of the box.
    assert abs(observables.kinetic_energy(fr) - observables.kinetic_energy(ff)) < 1e-15


@pytest.mark.parametrize("n", [1, 2, 3])
def test_reduced_streaming_is_a_permutation(n):
    """Streaming on the reduced lattice moves every population slot to
    exactly one slot, so its adjoint is its inverse (a scatter)."""
    labels = np.arange(27 * n ** 3, dtype=np.float64).reshape(27, n, n, n)
    moved = reduced.restrict(step.stream(reduced.unfold(labels)), n)
    assert np.array_equal(np.sort(moved.ravel()), labels.ravel())
    # Rest populations stay in place; a population never changes speed class.
    assert np.array_equal(moved[13], labels[13])
    C = lattice.velocities()
    speed = (C ** 2).sum(1)
    src = moved.astype(np.int64) // n ** 3
    assert (speed[src] == speed.reshape(27, 1, 1, 1)).all()
