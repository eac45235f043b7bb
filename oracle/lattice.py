"""D3Q27 lattice constants built from coordinates, in float64.

Test infrastructure (see ``oracle/__init__``): never used by the product path.

Sources in the paper:
* Sec. II.A (lattice Boltzmann equation): discrete velocities c_i of the DdQq
  stencil, lattice weights w_i, speed of sound c_s.  The paper names D3Q27 in
  Sec. II.B but prints neither the velocities nor the weights; the textbook
  D3Q27 set is used: c in {-1,0,1}^3, w the tensor product of the D1Q3 weights
  (1/6, 2/3, 1/6), c_s^2 = 1/3.
* Sec. II.B (definition of M): rows are the Hermite polynomials
  H^(n) = (-1)^n / omega(xi) * nabla^n omega(xi) of the Gaussian omega,
  evaluated at xi_i = sqrt(3) c_i, in the printed order (orders 0..6).  The
  printed last row "xyxzyz" is read as the sixth-order xxyyzz polynomial, the
  only sixth-order Hermite polynomial D3Q27 supports.
* Sec. II.B (equivariance): the full octahedral group O_h of order 48 acting
  on the velocities by rotations and reflections, each element giving a
  permutation matrix Pi_g of the populations.
"""
import itertools

import numpy as np
from numpy.polynomial import hermite_e

CS2 = 1.0 / 3.0  # squared lattice speed of sound

# Row labels of M exactly as listed in Sec. II.B (last one read as xxyyzz).
MOMENT_LABELS = (
    "", "x", "y", "z",
    "xx", "xy", "xz", "yy", "yz", "zz",
    "xxy", "xxz", "xyy", "xyz", "xzz", "yyz", "yzz",
    "xxyy", "xxyz", "xxzz", "xyyz", "xyzz", "yyzz",
    "xxyyz", "xxyzz", "xyyzz",
    "xxyyzz",
)


def velocities():
    """The 27 discrete velocities, shape (27, 3) int, ordered with c_x fastest:
    i = 9 (c_z + 1) + 3 (c_y + 1) + (c_x + 1).  The rest velocity is i = 13
    and the opposite of i is 26 - i."""
    return np.array([(cx, cy, cz)
                     for cz in (-1, 0, 1) for cy in (-1, 0, 1) for cx in (-1, 0, 1)],
                    dtype=np.int64)


def weights(C=None):
    """Lattice weights w_i = w1(c_x) w1(c_y) w1(c_z), w1(0) = 2/3, w1(+-1) = 1/6."""
    C = velocities() if C is None else C
    w1 = {-1: 1.0 / 6.0, 0: 2.0 / 3.0, 1: 1.0 / 6.0}
    return np.array([w1[a] * w1[b] * w1[c] for a, b, c in C], dtype=np.float64)


def multi_index(label):
    """Hermite multi-index (n_x, n_y, n_z) of a row label such as 'xxy'."""
    return (label.count("x"), label.count("y"), label.count("z"))


def moment_orders():
    """Order n_x + n_y + n_z of each row of M, in row order."""
    return np.array([sum(multi_index(l)) for l in MOMENT_LABELS], dtype=np.int64)


def hermite_1d(n, xi):
    """Probabilists' Hermite polynomial He_n(xi) = (-1)^n e^{xi^2/2} d^n/dxi^n
    e^{-xi^2/2}, which is the one-dimensional factor of H^(n) in Sec. II.B."""
    coef = np.zeros(n + 1)
    coef[n] = 1.0
    return hermite_e.hermeval(xi, coef)


def hermite_matrix(C=None):
    """M[k, i] = H_k(xi_i) with xi_i = sqrt(3) c_i (Sec. II.B, definition of M).

    A multivariate Hermite polynomial of the normalised Gaussian factorises into
    a product of one-dimensional ones, one per coordinate, with the number of
    derivatives taken along that coordinate as degree."""
    C = velocities() if C is None else C
    xi = np.sqrt(3.0) * C.astype(np.float64)
    M = np.empty((27, 27), dtype=np.float64)
    for k, label in enumerate(MOMENT_LABELS):
        nx, ny, nz = multi_index(label)
        M[k] = hermite_1d(nx, xi[:, 0]) * hermite_1d(ny, xi[:, 1]) * hermite_1d(nz, xi[:, 2])
    return M


def hermite_matrix_inverse(M=None):
    """M^{-1}, obtained by solving M X = I (no closed form is assumed here)."""
    M = hermite_matrix() if M is None else M
    return np.linalg.solve(M, np.eye(27))


def octahedral_group():
    """The 48 elements of O_h as 3x3 integer matrices: one nonzero entry, +-1,
    in every row and column (all axis permutations times all axis
    reflections).  Element 0 is the identity."""
    mats = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            R = np.zeros((3, 3), dtype=np.int64)
            for row in range(3):
                R[row, perm[row]] = signs[row]
            mats.append(R)
    ident = [k for k, R in enumerate(mats) if np.array_equal(R, np.eye(3, dtype=np.int64))]
    order = ident + [k for k in range(48) if k not in ident]
    return [mats[k] for k in order]


def population_permutation(R, C=None):
    """Permutation matrix Pi_g of a group element R acting on the populations:
    (Pi_g f)_i = f_j where c_i = R c_j, i.e. the distribution carried along by
    the rotation/reflection R."""
    C = velocities() if C is None else C
    index = {tuple(c): i for i, c in enumerate(C)}
    P = np.zeros((27, 27), dtype=np.float64)
    for j, c in enumerate(C):
        i = index[tuple(R @ c)]
        P[i, j] = 1.0
    return P


def group_permutations(C=None):
    """Pi_g for all 48 g in O_h, shape (48, 27, 27)."""
    return np.stack([population_permutation(R, C) for R in octahedral_group()])
