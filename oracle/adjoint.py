"""Reverse-mode derivative of an unrolled lattice Boltzmann run, in float64.

Test infrastructure (see ``oracle/__init__``): never used by the product path.

The paper trains the network parameters with Adam on a loss of the energy
spectrum after an unrolled run (Sec. "Learning Task"); this module computes
that gradient by hand, step by step backwards through the literal forward
definitions of ``oracle.collision`` and ``oracle.step``:

    y_t   = stream(x_t)                      pull streaming
    x_t+1 = collide(y_t; theta) + S(y_t; F_t)

    lambda_y  = (d collide/d y)^T lambda_t+1 + (d S/d y)^T lambda_t+1
    grad     += (d collide/d theta)^T lambda_t+1
    lambda_t  = stream^T lambda_y             (push streaming)

Populations are (27, nz, ny, nx).  Parameters are the list of (W, b) layers
of ``collision.unpack_params``; gradients come back in the same structure and
can be flattened with ``flatten``.
"""
import numpy as np

from . import collision, forcing, lattice, observables, step

_C = lattice.velocities().astype(np.float64)
_W = lattice.weights()
_M = collision._M
_MINV = collision._MINV
_ORDER = lattice.moment_orders()
_PI = lattice.group_permutations()


def flatten(grads):
    return np.concatenate([np.concatenate([dW.ravel(), db.ravel()]) for dW, db in grads])


# ------------------------------------------------------------- pieces -------

def equilibrium_vjp(rho, j, v):
    """(d f^eq / d f)^T v for f^eq written in (rho, j): f^eq_i = w_i (rho +
    3 c.j + 9/2 (c.j)^2 / rho - 3/2 j.j / rho), with rho = sum f, j = sum c f.
    ``v`` has shape (27, N); returns (27, N)."""
    cj = _C @ j                                   # (27, N)
    jj = (j * j).sum(axis=0)
    w = _W[:, None]
    dfeq_drho = w * (1.0 - 4.5 * cj * cj / rho ** 2 + 1.5 * jj / rho ** 2)
    g_rho = (v * dfeq_drho).sum(axis=0)           # (N,)
    # d f^eq_i / d j_a = w_i (3 c_ia + 9 (c.j) c_ia / rho - 3 j_a / rho)
    coeff = w * (3.0 + 9.0 * cj / rho)            # multiplies c_ia
    g_j = _C.T @ (v * coeff) - 3.0 * j / rho * (v * w).sum(axis=0)   # (3, N)
    return g_rho[None, :] + _C @ g_j


def _act(name):
    if name == "tanh":
        return np.tanh, lambda h: 1.0 - h * h          # derivative from the output
    return (lambda z: np.maximum(z, 0.0)), (lambda h: (h > 0.0).astype(np.float64))


def network_forward(m_all, layers, act):
    """Literal forward of tilde tau = mean_g Phi(M Pi_g f) keeping the
    activations of every group element.  m_all: (48, N, 27) inputs."""
    g, _ = _act(act)
    hs = [m_all]
    h = m_all
    for W, b in layers[:-1]:
        h = g(h @ W + b)
        hs.append(h)
    W, b = layers[-1]
    out = (h @ W + b).mean(axis=0)                 # (N, 4)
    return out, hs


def network_vjp(hs, layers, act, d_out):
    """Backward of ``network_forward``: d_out (N, 4) = dL/d tilde tau.
    Returns (dL/d inputs (48, N, 27), parameter gradients)."""
    _, dg = _act(act)
    ng = hs[0].shape[0]
    grads = [None] * len(layers)
    W, _ = layers[-1]
    d = np.broadcast_to(d_out / ng, (ng,) + d_out.shape)       # dL/d(output of group g)
    grads[-1] = (np.einsum("gni,gno->io", hs[-1], d), d.sum(axis=(0, 1)))
    dh = d @ W.T
    for li in range(len(layers) - 2, -1, -1):
        W, _ = layers[li]
        dz = dh * dg(hs[li + 1])
        grads[li] = (np.einsum("gni,gno->io", hs[li], dz), dz.sum(axis=(0, 1)))
        dh = dz @ W.T
    return dh, grads


def nco_collide_vjp(f, lam, tau, layers, act, force=None):
    """VJP of one NCO collision (plus Kupershtokh source when ``force`` is
    given) at pre-collision populations f (27, N) for lambda = dL/d f_post.
    Returns (dL/d f, parameter gradients)."""
    rho = f.sum(axis=0)
    j = _C.T @ f
    u = j / rho
    m = _M @ f
    meq = _M @ collision.equilibrium(rho, u)
    # Network forward on the 48 transformed moment vectors.
    m_all = np.stack([(_M @ (P @ f)).T for P in _PI])          # (48, N, 27)
    tt, hs = network_forward(m_all, layers, act)               # (N, 4)
    tau_n = collision.squash(tt.T)                              # (4, N)
    omega = 1.0 / tau_n
    s = collision.rate_vector(tau, omega)                       # (27, N)
    # f_post = f - M^{-1} (s (m - meq)) [+ S]
    mu = _MINV.T @ lam                                          # dL/d(M^{-1} x) = M^{-T} lam
    d_q = -mu                                                   # q = s (m - meq)
    d_s = d_q * (m - meq)
    d_diff = d_q * s
    g = lam + _M.T @ d_diff                                     # through m = M f
    g -= equilibrium_vjp(rho, j, _M.T @ d_diff)                 # through m^eq = M f^eq
    # Rates: s_k = omega_{order(k) - 3} for orders 3..6.
    d_omega = np.zeros_like(omega)
    for k in range(27):
        if _ORDER[k] >= 3:
            d_omega[_ORDER[k] - 3] += d_s[k]
    e = np.exp(tt.T)
    dtau_dt = -e / (2.0 * (1.0 + e) ** 2)
    d_tt = (d_omega * (-1.0 / tau_n ** 2) * dtau_dt).T          # (N, 4)
    d_in, pgrads = network_vjp(hs, layers, act, d_tt)           # (48, N, 27)
    for gi, P in enumerate(_PI):
        g += P.T @ (_M.T @ d_in[gi].T)
    if force is not None:
        jf = j + force
        # S = f^eq(rho, j + F) - f^eq(rho, j): same rho, shifted momentum.
        g += equilibrium_vjp(rho, jf, lam) - equilibrium_vjp(rho, j, lam)
    return g, pgrads


def force_vjp(rho, j, force, lam):
    """(d S / d F)^T lam for the exact-difference source S = f^eq(rho, j + F)
    - f^eq(rho, j) of one collision: dS_i/dF_a is d f^eq_i / d j_a taken at
    j + F, w_i (3 c_ia + 9 (c_i . (j + F)) c_ia / rho - 3 (j + F)_a / rho).
    rho (N,), j and force (3, N), lam (27, N); returns dL/dF (3, N)."""
    jf = j + force
    w = _W[:, None]
    cj = _C @ jf
    return _C.T @ (lam * w * (3.0 + 9.0 * cj / rho)) - 3.0 * jf / rho * (lam * w).sum(axis=0)


def spectrum_vjp(f, dL_dE):
    """(dE / d f)^T dL_dE for the shell spectrum of ``observables``."""
    n = f.shape[1]
    rho = f.sum(axis=0)
    j = np.tensordot(_C.T, f, axes=(1, 0))
    u = j / rho
    uh = np.fft.fftn(u, axes=(1, 2, 3)) / n ** 3
    a = np.asarray(dL_dE)[observables.shell_index(n)]           # dL/dE at each wavevector
    lam_u = np.real(np.fft.ifftn(a * uh, axes=(1, 2, 3)))
    lam_j = lam_u / rho
    lam_rho = -(lam_u * u).sum(axis=0) / rho
    return lam_rho[None] + np.tensordot(_C, lam_j, axes=(1, 0))


def log_spectrum_loss(E, E_target, kmin, kmax):
    """L = mean over kmin <= k <= kmax of (ln E(k) - ln E_t(k))^2 and dL/dE."""
    ks = np.arange(kmin, kmax + 1)
    r = np.log(E[ks]) - np.log(E_target[ks])
    L = float((r * r).mean())
    dE = np.zeros_like(E)
    dE[ks] = 2.0 * r / (len(ks) * E[ks])
    return L, dE


# ---------------------------------------------------------------- driver ----

def kinetic_energy_vjp(f):
    """d k / d f for the mean kinetic energy k = <|u|^2> / 2, u = j / rho:
    per node, d(|j|^2 / (2 rho^2)) / d f_i = (u . c_i - |u|^2) / rho, divided
    by the number of nodes."""
    C = lattice.velocities().astype(float)
    rho, u = collision.macroscopic(f)
    uc = np.einsum("ia,a...->i...", C, u)
    uu = (u * u).sum(axis=0)
    return (uc - uu) / rho / rho.size


def run_and_grad(f0, tau, layers, act, nsteps, loss_grad, forces=None, traj_grad=None, state_forcing=None):
    """Forward nsteps NCO steps from f0, then the exact gradient of
    L = loss(x_T) (+ terms on the intermediate states) with respect to the
    network parameters and to f0.

    loss_grad(x_T) -> (L, dL/dx_T).  forces: None or callable t -> (3, ...).
    traj_grad: None or callable (t, x_t) -> dL/dx_t (or None) for the loss
    terms on the state after t steps, t = 0 .. nsteps, whose values the
    caller adds to L.  state_forcing: None or (ks, draws, amplitude, kf, c),
    the spectral forcing with Alvelius' velocity-dependent theta1: step t
    takes the coefficients ``forcing.coefficients_state`` of draws[t mod
    len(draws)] and of the velocity of x_t, and the reverse mode follows the
    force back to x_t through them.  Returns (L, parameter gradients,
    dL/df0)."""
    if forces is not None and state_forcing is not None:
        raise ValueError("give forces or state_forcing, not both")
    op = step.Operator("nco", tau, layers=layers, act=act)
    shape = f0.shape
    xs, us, Fs = [f0], [], []
    for t in range(nsteps):
        F = None if forces is None else forces(t)
        if state_forcing is not None:
            ks, draws, amp, kf, c = state_forcing
            _, u = collision.macroscopic(xs[-1])
            F = forcing.field(ks, forcing.coefficients_state(ks, draws[t % len(draws)], amp, kf, c, u), shape[1:])
            us.append(u)
        Fs.append(F)
        xs.append(step.step(xs[-1], op, F))
    L, lam = loss_grad(xs[-1])

    def add_traj(t, lam):
        extra = None if traj_grad is None else traj_grad(t, xs[t])
        return lam if extra is None else lam + extra

    lam = add_traj(nsteps, lam)
    total = [(np.zeros_like(W), np.zeros_like(b)) for W, b in layers]
    for t in range(nsteps - 1, -1, -1):
        y = step.stream(xs[t]).reshape(27, -1)
        F = None if Fs[t] is None else Fs[t].reshape(3, -1)
        lam_next = lam.reshape(27, -1)
        g, pg = nco_collide_vjp(y, lam_next, tau, layers, act, F)
        total = [(a + c, b + d) for (a, b), (c, d) in zip(total, pg)]
        lam = step.unstream(g.reshape(shape))
        if state_forcing is not None:
            # The force of step t depends on x_t through u = j / rho.
            ks, draws, amp, kf, c = state_forcing
            gF = force_vjp(y.sum(axis=0), _C.T @ y, F, lam_next).reshape((3,) + shape[1:])
            du = forcing.coefficients_state_vjp(ks, draws[t % len(draws)], amp, kf, c, us[t],
                                                forcing.field_vjp(ks, gF))
            rho, u = collision.macroscopic(xs[t])
            lam = lam + (np.einsum("ia,a...->i...", _C, du) - (u * du).sum(axis=0)) / rho
        lam = add_traj(t, lam)
    return L, total, lam
