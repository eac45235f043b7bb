"""Collision operators of the paper, literally, in float64.

Test infrastructure (see ``oracle/__init__``): never used by the product path.

Populations are arrays of shape (27, ...) - the first axis is the velocity
index of ``oracle.lattice.velocities()``, the remaining axes are nodes.
"""
import numpy as np

from . import lattice

_C = lattice.velocities().astype(np.float64)
_W = lattice.weights()
_M = lattice.hermite_matrix()
_MINV = lattice.hermite_matrix_inverse(_M)
_ORDER = lattice.moment_orders()
_PI = lattice.group_permutations()


def macroscopic(f):
    """rho = sum_i f_i and rho u = sum_i c_i f_i (Sec. II.A); returns (rho, u)
    with u of shape (3, ...)."""
    rho = f.sum(axis=0)
    j = np.tensordot(_C.T, f, axes=(1, 0))
    return rho, j / rho


def equilibrium(rho, u):
    """Quadratic equilibrium (Eq. EquilibriumDistribution):
    f_i^eq = w_i rho (1 + u.c_i/cs^2 + (u.c_i)^2/(2 cs^4) - u.u/(2 cs^2))."""
    cs2 = lattice.CS2
    cu = np.tensordot(_C, u, axes=(1, 0))          # (27, ...)
    uu = (u * u).sum(axis=0)                        # (...)
    shape = (27,) + (1,) * np.ndim(rho)
    return _W.reshape(shape) * rho * (1.0 + cu / cs2 + cu * cu / (2.0 * cs2 * cs2)
                                      - uu / (2.0 * cs2))


def moments(f):
    """m = M f (Sec. II.B)."""
    return np.tensordot(_M, f, axes=(1, 0))


def from_moments(m):
    """f = M^{-1} m."""
    return np.tensordot(_MINV, m, axes=(1, 0))


def bgk(f, tau):
    """Post-collision populations with the BGK operator (Sec. II.A):
    f + Omega with Omega_i = -(f_i - f_i^eq)/tau."""
    rho, u = macroscopic(f)
    feq = equilibrium(rho, u)
    return f - (f - feq) / tau


def rate_vector(tau, omega_high):
    """Diagonal of S (Eq. omegatheta): 1 for the conserved moments (orders 0
    and 1), omega_nu = 1/tau for all six second-order moments, and
    omega_high[n-3] for the moments of order n = 3..6 (the four order groups).

    ``omega_high`` has shape (4, ...) so that the rates may vary per node."""
    omega_high = np.asarray(omega_high, dtype=np.float64)
    node_shape = omega_high.shape[1:]
    s = np.empty((27,) + node_shape, dtype=np.float64)
    for k in range(27):
        n = _ORDER[k]
        if n <= 1:
            s[k] = 1.0
        elif n == 2:
            s[k] = 1.0 / tau
        else:
            s[k] = omega_high[n - 3]
    return s


def moment_relaxation(f, tau, omega_high):
    """f + Omega with Omega = -M^{-1} S (M f - m^eq) and m^eq = M f^eq
    (Eq. omegatheta); the equilibrium is the quadratic one (reading: the
    paper's only stated equilibrium)."""
    rho, u = macroscopic(f)
    m = moments(f)
    meq = moments(equilibrium(rho, u))
    s = rate_vector(tau, omega_high)
    return f - from_moments(s * (m - meq))


# --------------------------------------------------------------------------
# The invariant network (Sec. II.B, Eq. gconv_m and the rate squashing).
# --------------------------------------------------------------------------

def activation(name):
    if name == "tanh":
        return np.tanh
    if name == "relu":
        return lambda x: np.maximum(x, 0.0)
    raise ValueError(name)


def unpack_params(params, width, depth=2, n_in=27, n_out=4):
    """Split a flat parameter vector into [(W, b), ...] with W stored
    [in, out] row-major, in the order W1, b1, W2, b2, ..., W_last, b_last."""
    params = np.asarray(params, dtype=np.float64)
    sizes = [n_in] + [width] * depth + [n_out]
    layers, pos = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = params[pos:pos + a * b].reshape(a, b)
        pos += a * b
        bias = params[pos:pos + b]
        pos += b
        layers.append((W, bias))
    if pos != params.size:
        raise ValueError("parameter count %d does not match the architecture (%d)"
                         % (params.size, pos))
    return layers


def n_params(width, depth=2, n_in=27, n_out=4):
    sizes = [n_in] + [width] * depth + [n_out]
    return sum(a * b + b for a, b in zip(sizes[:-1], sizes[1:]))


def mlp(x, layers, act="tanh"):
    """Phi(x): affine -> activation for every hidden layer, affine output.
    ``x`` has shape (..., 27); returns (..., 4)."""
    g = activation(act)
    h = x
    for W, b in layers[:-1]:
        h = g(h @ W + b)
    W, b = layers[-1]
    return h @ W + b


def invariant_network(f, layers, act="tanh"):
    """tilde tau = N_Phi(f) = (1/|G|) sum_g Phi(M Pi_g f)  (Eq. gconv_m).

    The mean is taken over the network outputs, literally as printed.
    ``f`` has shape (27, ...); returns (4, ...)."""
    node_shape = f.shape[1:]
    fl = f.reshape(27, -1)
    acc = np.zeros((fl.shape[1], 4))
    for P in _PI:
        mg = _M @ (P @ fl)                     # m^(g) = M Pi_g f, (27, nodes)
        acc += mlp(mg.T, layers, act)
    acc /= len(_PI)
    return acc.T.reshape((4,) + node_shape)


def squash(tau_tilde):
    """tau_n = 1 / (2 (1 + exp(tilde tau_n))) + 1/2, so tau_n in (1/2, 1)
    (Sec. II.B, the sigmoid applied to the network output)."""
    return 1.0 / (2.0 * (1.0 + np.exp(tau_tilde))) + 0.5


def nco_rates(f, layers, act="tanh"):
    """omega_n = 1/tau_n for the four higher-order groups, shape (4, ...)."""
    return 1.0 / squash(invariant_network(f, layers, act))


def nco(f, tau, layers, act="tanh"):
    """f + Omega(f, theta), Omega = -M^{-1} S_theta (M f - m^eq) with the
    higher-order rates from the invariant network (Eq. omegatheta)."""
    return moment_relaxation(f, tau, nco_rates(f, layers, act))


def kupershtokh_source(f, force):
    """Exact-difference source S_i = f^eq(rho, u + du) - f^eq(rho, u),
    du = F dt / rho with dt = 1 (Sec. II.A, forcing).  ``force`` (3, ...)."""
    rho, u = macroscopic(f)
    return equilibrium(rho, u + force / rho) - equilibrium(rho, u)
