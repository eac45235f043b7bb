"""The reduced Taylor-Green domain of Appendix A ("Reduced Taylor-Green
vortex"), in float64.

Test infrastructure (see ``oracle/__init__``): never used by the product path.

The three-dimensional Taylor-Green vortex (Eq. tgv3d_equation) keeps the
symmetries of its initial field for all time, because the lattice Boltzmann
step commutes with every signed permutation of the axes that maps the lattice
to itself (streaming does, and the collision is equivariant by construction,
Sec. II.B).  The appendix therefore simulates only the cube [0, pi/2]^3, with
nodes half a spacing from its faces, and sends populations that leave the
cube back in through reflections S_a, rotations R_b and the swap T_xy.

Here the reduced step is defined by what it stands for: unfold the cube's
populations to the whole periodic box [0, 2 pi)^3 through the symmetry group
of the vortex, take one ordinary periodic step there (``step.step``), and keep
the cube.  Nothing of the appendix's displacement tables is used (they are
partly garbled); the group is generated from five symmetries read off the
initial field, each checked against it by the tests:

* the mirrors x -> -x, y -> -y, z -> -z (S_x, S_y, S_z at the planes through
  the origin), which reverse the matching velocity component;
* the rotation by +90 degrees about the z-parallel line x = y = pi/2,
  (x, y) -> (pi - y, x), velocity (u, v) -> (-v, u) (an R_z rotation about
  the vortex axis);
* the rotation by 180 degrees about the line x = y, z = pi/2,
  (x, y, z) -> (y, x, pi - z), velocity (u, v, w) -> (v, u, -w) (T_xy with S_z).

A reduced lattice of n nodes per edge stands for the box of N = 4n nodes per
edge at x_j = (j + 1/2) 2 pi / N; the cube holds the nodes j < n on every
axis.  Positions are handled as odd integers P = 2 j + 1 in units of half a
spacing, period 2N = 8n, so that every map is exact integer arithmetic.
"""
import numpy as np

from . import lattice, step as _step

_C = lattice.velocities()
_INDEX = {tuple(int(v) for v in c): i for i, c in enumerate(_C)}


def generators(n):
    """The five generating symmetries as (A, b): P -> A P + b (mod 8n) on
    half-spacing positions (x, y, z); A acts on velocities too."""
    q = 4 * n  # pi in half spacings
    gens = []
    for a in range(3):
        A = np.eye(3, dtype=np.int64)
        A[a, a] = -1
        gens.append((A, np.zeros(3, np.int64)))
    gens.append((np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]], np.int64), np.array([q, 0, 0], np.int64)))
    gens.append((np.array([[0, 1, 0], [1, 0, 0], [0, 0, -1]], np.int64), np.array([0, 0, q], np.int64)))
    return gens


def symmetry_group(n):
    """All products of the generators, modulo the period 2 pi: a list of
    (A, b).  The cube [0, pi/2]^3 is a fundamental domain of this group, so
    it has 64 elements (checked by the tests)."""
    h = 8 * n
    gens = generators(n)
    eye = (np.eye(3, dtype=np.int64), np.zeros(3, np.int64))
    seen = {(eye[0].tobytes(), eye[1].tobytes()): eye}
    frontier = [eye]
    while frontier:
        nxt = []
        for A, b in frontier:
            for G, c in gens:
                A2, b2 = G @ A, (G @ b + c) % h
                key = (A2.tobytes(), b2.tobytes())
                if key not in seen:
                    seen[key] = (A2, b2)
                    nxt.append((A2, b2))
        frontier = nxt
    return list(seen.values())


def _cube_positions(n):
    """Half-spacing positions (3, n, n, n) of the cube's nodes, [z, y, x] order."""
    P = 2 * np.arange(n, dtype=np.int64) + 1
    Z, Y, X = np.meshgrid(P, P, P, indexing="ij")
    return np.stack([X, Y, Z])


def images(n):
    """For every group element: the full-box node indices (jz, jy, jx) of the
    images of the cube's nodes and the population index map i -> index of
    A c_i."""
    h = 8 * n
    pos = _cube_positions(n)
    out = []
    for A, b in symmetry_group(n):
        img = (np.tensordot(A, pos, axes=1) + b.reshape(3, 1, 1, 1)) % h
        jx, jy, jz = (img - 1) // 2
        perm = np.array([_INDEX[tuple(int(v) for v in A @ c)] for c in _C])
        out.append(((jz, jy, jx), perm))
    return out


def unfold(f):
    """Populations (27, n, n, n) of the cube -> the symmetric field (27, 4n,
    4n, 4n) on the whole box: f(g x, A_g c) = f(x, c) for every symmetry g.
    Raises if the images do not cover every node of the box exactly once."""
    n = f.shape[-1]
    assert f.shape == (27, n, n, n)
    N = 4 * n
    full = np.empty((27, N, N, N))
    hits = np.zeros((N, N, N), np.int64)
    for (jz, jy, jx), perm in images(n):
        for i in range(27):
            full[perm[i], jz, jy, jx] = f[i]
        np.add.at(hits, (jz, jy, jx), 1)
    if not (hits == 1).all():
        raise AssertionError("the cube's images do not tile the box")
    return full


def restrict(full, n):
    """The cube's nodes of a full-box field."""
    return full[..., :n, :n, :n].copy()


def step(f, op):
    """One step of the reduced lattice: unfold, periodic step, restrict."""
    n = f.shape[-1]
    return restrict(_step.step(unfold(f), op), n)


def run(f, op, nsteps):
    for _ in range(nsteps):
        f = step(f, op)
    return f
