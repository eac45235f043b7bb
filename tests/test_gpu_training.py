"""Training of the network on the GPU (forced isotropic turbulence, loss on
the log energy spectrum): full-size gradient check by finite differences and
the gain of the trained network over the untrained one, the fixed-rate
operator and BGK on the same seeded workload."""
import numpy as np
import pytest

from paper_2412_08229_amd import Lattice, inputs
from paper_2412_08229_amd import _lib as L
from paper_2412_08229_amd.training import Unroll, curriculum_steps, log_spectrum_loss, n_bins, train

pytestmark = pytest.mark.gpu


def forced_turbulence(n, nsteps, seed, tau, urms=0.05, k0=4.0, amp=2e-6):
    """Small forced-turbulence sample: random-phase solenoidal start with
    E(k) ~ k^4 exp(-2 (k/k0)^2), Alvelius forcing on 0 < |k| <= 2 at a given
    amplitude; the target spectrum is the initial one."""
    rho, u = inputs.turbulence(n, seed=seed, k0=k0, urms=urms)
    ks = inputs.forcing_half_modes(2.0)
    draws = inputs.uniform_draws(nsteps, len(ks), seed + 1)
    with Lattice((n, n, n), "f64", "bgk", tau) as lat:
        lat.init_equilibrium(rho, u)
        target = lat.energy_spectrum()
    return rho, u, (ks, draws, amp, 1.5, 1.0), target


# Forced band of the training workload: every integer wavevector with
# 0.5 <= |k| <= 2.5, Gaussian force density peaked at k_f = 1.5, width c = 1.
C4_BAND = (0.5, 2.5, 1.5, 1.0)


def c4_sample(seed, n=64, nsteps=200, tau=0.52, phase_rule=False):
    """The forced-turbulence training sample at its full size.  A random-
    phase solenoidal field with E(k) ~ k^4 exp(-2 (k/4)^2), u_rms 0.05, is
    set on a 2n lattice and restricted to the n lattice (the coarse start).
    The force's power input is the start's dissipation 2 nu sum (2 pi k / n)^2
    E(k) (lattice units), its amplitude from the power by the equation for A
    (Sec. "Training Data - Forced Isotropic Turbulence").  The target is the
    same setup run with BGK on the 2n lattice by acoustic scaling (tau_f =
    6 nu + 1/2, 2 nsteps steps, each draw held for two fine steps with a
    quarter of the amplitude: the same force per unit physical time) and
    restricted to n (Sec. "Learning Task").  Returns the coarse start's
    populations, the coarse forcing, the target spectrum and the power."""
    nu = (tau - 0.5) / 3.0
    nf = 2 * n
    rho_f, u_f = inputs.turbulence(nf, seed=seed, k0=4.0, urms=0.05)
    ka, kb, kf, c = C4_BAND
    ks = inputs.forcing_half_modes(kb, ka)
    draws = inputs.uniform_draws(nsteps, len(ks), seed + 1)
    with Lattice((nf,) * 3, "f32", "bgk", 6.0 * nu + 0.5) as fine, Lattice((n,) * 3, "f32", "bgk", tau) as coarse:
        fine.init_equilibrium(rho_f, u_f)
        coarse.restrict_from(fine)
        f0 = coarse.populations()
        E0 = coarse.energy_spectrum()
        power = 2.0 * nu * float(np.sum((2.0 * np.pi * np.arange(len(E0)) / n) ** 2 * E0))
        amp = L.nco_forcing_amplitude(power, 1.0, ka, kb, kf, c)
        fine.set_forcing(ks, np.repeat(draws, 2, axis=0), amp / 4.0, kf, c, phase_rule)
        fine.step(2 * nsteps)
        coarse.restrict_from(fine)
        target = coarse.energy_spectrum()
    return f0, (ks, draws, amp, kf, c, phase_rule), target, power


@pytest.mark.parametrize("phase_rule", [False, True])
def test_c4_gradient_matches_finite_differences(phase_rule):
    """64^3, 200-step unroll, checkpoints every 20, forcing from the power
    input, target from the restricted 128^3 BGK run: the adjoint's
    directional derivative against a central difference of the loss, with
    drawn forcing phases or Alvelius' velocity-dependent phase."""
    n, T, K, tau = 64, 200, 20, 0.52
    f0, frc, target, _ = c4_sample(11, n, T, tau, phase_rule)
    params = inputs.mlp_params(32, 0)
    run = Unroll((n, n, n), tau, ("pop", f0), T, K, target, 2, 16, forcing=frc)
    L0, g, _ = run.loss_and_grad(params)
    v = np.random.Generator(np.random.PCG64(12)).standard_normal(params.size)
    v /= np.linalg.norm(v)
    h = 2e-3
    Lp = run.loss(params + h * v)
    Lm = run.loss(params - h * v)
    run.close()
    fd = (Lp - Lm) / (2 * h)
    an = float(g @ v)
    print("C4 64^3 x200 (phase rule %s): loss %.6e, directional derivative adjoint %.6e, finite difference %.6e"
          % (phase_rule, L0, an, fd))
    assert np.isfinite(L0) and abs(fd - an) < 3e-2 * abs(an)


def test_training_reduces_loss_below_untrained_fixed_rate_and_bgk():
    n, T, K, tau = 16, 60, 20, 0.505
    rho, u, frc, target = forced_turbulence(n, T, seed=21, tau=tau, urms=0.06)
    kmin, kmax = 2, 6
    params0 = inputs.mlp_params(32, 1)
    run = Unroll((n, n, n), tau, ("eq", rho, u), T, K, target, kmin, kmax, forcing=frc)
    L_untrained = run.loss(params0)
    params, hist = train([run], params0, epochs=40, lr=2e-2)
    L_trained = run.loss(params)
    run.close()
    others = {}
    for kind in ("mrt", "bgk"):
        with Lattice((n, n, n), "f32", kind, tau) as lat:
            lat.set_rates([4.0 / 3.0] * 4)
            lat.set_forcing(*frc)
            lat.init_equilibrium(rho, u)
            lat.step(T)
            E = lat.energy_spectrum()
        others[kind] = log_spectrum_loss(E, target, kmin, kmax)[0] if np.all(np.isfinite(E)) else np.inf
    print("loss: untrained NCO %.5f, trained NCO %.5f, fixed-rate %.5f, BGK %.5f; history %s"
          % (L_untrained, L_trained, others["mrt"], others["bgk"], np.round(hist, 5).tolist()))
    assert L_trained < 0.9 * L_untrained
    assert L_trained < others["mrt"] and L_trained < others["bgk"]


def test_c4_training_gain_64():
    """The forced-turbulence training at its full size: 64^3, 200-step
    unrolls, checkpoints every 20, forcing from the power input, target the
    restricted 128^3 BGK run (``c4_sample``), loss on the log-spectrum gap
    over 2 <= k <= 16.  30 Adam epochs on the GPU's own forward and reverse
    kernels (~18 s) cut the loss far below the untrained network's, the
    fixed-rate operator's and BGK's (measured: 3.73e-3 -> 9.0e-5, against
    3.73e-3 fixed-rate and 3.7e-4 BGK: the seeded network relaxes the
    higher orders at ~4/3 and damps the shells above k = 8, which the
    trained one restores)."""
    n, T, K, tau = 64, 200, 20, 0.52
    f0, frc, target, power = c4_sample(31, n, T, tau)
    params0 = inputs.mlp_params(32, 1)
    run = Unroll((n, n, n), tau, ("pop", f0), T, K, target, 2, 16, forcing=frc)
    L_untrained = run.loss(params0)
    params, hist = train([run], params0, epochs=30, lr=1e-2)
    L_trained = run.loss(params)
    run.close()
    others = {}
    ka, kb, kf, c = C4_BAND
    for kind in ("mrt", "bgk"):
        with Lattice((n, n, n), "f32", kind, tau) as lat:
            lat.set_rates([4.0 / 3.0] * 4)
            lat.set_forcing_power(frc[0], frc[1], power, ka, kb, kf, c)
            lat.init_populations(f0)
            lat.step(T)
            others[kind] = log_spectrum_loss(lat.energy_spectrum(), target, 2, 16)[0]
    print("64^3 loss (power input %.4e): untrained NCO %.4e, trained NCO %.4e, fixed-rate %.4e, BGK %.4e; "
          "history %s" % (power, L_untrained, L_trained, others["mrt"], others["bgk"],
                          np.round(hist, 6).tolist()))
    assert L_trained < 0.1 * L_untrained
    assert L_trained < 0.1 * others["mrt"] and L_trained < 0.5 * others["bgk"]


def _tgv_energy(kind, n, t_end, params=None, u0=0.1 / np.sqrt(3.0), re=1600.0):
    """k(t) / u0^2 of the 3-D Taylor-Green vortex (Re 1600, Ma 0.1) sampled
    every ~0.1 convective times; t in convective units."""
    nu, tau = inputs.viscosity(n, u0, re)
    tc = n / (2 * np.pi) / u0
    every = max(1, int(round(0.1 * tc)))
    m = int(round(t_end * tc / every))
    rho, u = inputs.tgv3d(n, u0)
    with Lattice((n, n, n), "f32", kind, tau) as lat:
        if kind == "nco":
            lat.set_net_weights(params, 32, "tanh", "f32_mfma")
        if kind == "mrt":
            lat.set_rates([4.0 / 3.0] * 4)
        lat.init_equilibrium(rho, u)
        ks = [lat.global_sums()[4] / lat.n / u0 ** 2]
        for _ in range(m):
            lat.step(every)
            ks.append(lat.global_sums()[4] / lat.n / u0 ** 2)
    return np.arange(m + 1) * every / tc, np.array(ks)


def test_dissipation_training_gain_tgv32():
    """The dissipation-rate training of Sec. "Learning Task" (there on the
    reduced Taylor-Green box), here on the under-resolved periodic 32^3
    vortex at Re 1600: the loss is the mean squared gap of -dk/dt to a 128^3
    BGK run over 1 <= t <= 8, through the energy-trajectory reverse mode.
    40 Adam epochs (~20 s) cut it about tenfold (measured 0.150 -> 0.014),
    far below the fixed-rate operator (0.151) and BGK (1.85), and the trained
    operator stays stable to t = 12, past the time BGK blows up at 32^3."""
    from paper_2412_08229_amd.training import DissipationUnroll
    u0, n = 0.1 / np.sqrt(3.0), 32
    tr, kr = _tgv_energy("bgk", 128, 8.5)
    er = -np.gradient(kr, tr)
    _, tau = inputs.viscosity(n, u0, 1600.0)
    tc = n / (2 * np.pi) / u0
    every = int(round(0.1 * tc))
    nsteps = int(round(8.0 * tc / every)) * every
    rho, u = inputs.tgv3d(n, u0)
    run = DissipationUnroll((n, n, n), tau, rho, u, u0, nsteps, 20, every,
                            lambda t: float(np.interp(t, tr, er)), t_min=1.0)
    p0 = inputs.mlp_params(32, 1)
    L0 = run.loss(p0)
    params, hist = train([run], p0, epochs=40, lr=1e-2)
    L1 = run.loss(params)
    others = {}
    for kind in ("mrt", "bgk"):
        t, k = _tgv_energy(kind, n, 8.0)
        kk = np.interp(run.t, t, k)
        eps = -(kk[run.inner + 1] - kk[run.inner - 1]) / (2 * run.dt)
        others[kind] = float(np.mean(((eps - run.eps_ref) / run.scale) ** 2))
    run.close()
    t, k = _tgv_energy("nco", n, 12.0, params=params)
    print("dissipation loss: untrained NCO %.4f, trained %.4f, fixed-rate %.4f, BGK %.4f; trained k(12) = %.4f"
          % (L0, L1, others["mrt"], others["bgk"], k[-1]))
    assert L1 < 0.3 * L0 and L1 < 0.3 * others["mrt"] and L1 < others["bgk"]
    assert np.all(np.isfinite(k)) and t[-1] > 11.9


# Measured in a 40-epoch run over the full Re 400/800/1600 x cube 10/16/25/32
# grid at Ma 0.1 (512^3-box reference): the cube-10 losses fall 3-4x and the
# mean 3.3x.  Here 25 epochs on four samples must halve the mean.
EPOCHS_REDUCED = 25
REDUCED_GAIN = 0.5


def test_dissipation_training_reduced_cubes():
    """The dissipation-rate training of Sec. "Training based on dissipation
    rates" on the reduced Taylor-Green cube of Appendix A, over part of the
    paper's case grid: Re 400 and 1600 at Ma 0.1 on cubes of 10 and 16 nodes
    per edge (the 40^3 and 64^3 boxes).  Loss: -dk/dt at 100 points over
    0 <= t <= 15 against BGK on the 64^3 cube (the 256^3 box); one Adam step
    per epoch on the mean loss, the four samples concurrently on their own
    streams.  The trained network beats the untrained one, the fixed-rate
    operator and BGK on the mean loss."""
    from paper_2412_08229_amd.training import DissipationUnroll, tgv_cube_energy, train_batched
    u0, t_end, samples = 0.1 / np.sqrt(3.0), 15.0, 100
    runs = []
    for re in (400.0, 1600.0):
        t, k, st = tgv_cube_energy("bgk", 64, re, u0, t_end, 300)
        assert st == "stable"
        er = -np.gradient(k, t)
        for n in (10, 16):
            _, tau = inputs.viscosity(4 * n, u0, re)
            tc = 4 * n / (2 * np.pi) / u0
            every = int(round(t_end * tc / samples))
            nsteps = int(round(t_end * tc / every)) * every
            rho, u = inputs.tgv3d_octant(n, u0)
            runs.append(DissipationUnroll((n, n, n), tau, rho, u, u0, nsteps, 50, every,
                                          lambda x, t=t, er=er: float(np.interp(x, t, er)), t_min=0.0,
                                          domain="tgv_octant"))
    p0 = inputs.mlp_params(32, 1)
    L0 = np.array([r.loss(p0) for r in runs])
    params, hist = train_batched(runs, p0, epochs=EPOCHS_REDUCED, lr=1e-2)
    L1 = np.array([r.loss(params) for r in runs])
    other = {"mrt": [], "bgk": []}
    for r in runs:
        for kind in other:
            t, k, st = tgv_cube_energy(kind, r.lat.nx, None, u0, t_end, None, tau=r.lat.tau, every=r.every,
                                       nsamp=r.nsteps // r.every)
            if st != "stable":
                other[kind].append(np.inf)
                continue
            eps = -(k[r.inner + 1] - k[r.inner - 1]) / (2.0 * r.dt)
            other[kind].append(float(np.mean(((eps - r.eps_ref) / r.scale) ** 2)))
        r.close()
    print("reduced-cube dissipation loss per sample (Re 400 n10, n16, Re 1600 n10, n16): untrained %s, "
          "trained %s, fixed-rate %s, BGK %s" % (np.round(L0, 5), np.round(L1, 5), np.round(other["mrt"], 5),
                                                  np.round(other["bgk"], 5)))
    assert L1.mean() < REDUCED_GAIN * L0.mean()
    assert L1.mean() < REDUCED_GAIN * np.mean(other["mrt"]) and L1.mean() < np.mean(other["bgk"])


def test_paper_spectrum_training_pipeline():
    """The data side of Sec. "Learning Task" at a small scale: a 32^3 BGK
    run (fine) forced with Alvelius' velocity-dependent phase, restricted by
    acoustic scaling to 16^3 (coarse, tau_c = 1/2 + (tau_f - 1/2) / 2); the
    coarse NCO runs from the restricted state, forced by the same rule (the
    phases are redrawn every step and the rule leaves no correlation with u,
    so a step injects |F|^2 / 2, in proportion to the amplitude of F(k): one
    coarse step must inject what two fine steps do, amplitude x2), under the
    paper's loss (squared
    spectrum gap over 2 <= k <= 6 plus 20 E(8); target: the fine spectrum at
    the restriction time) with the unroll curriculum (20 steps, 20 more every
    3 epochs).  The gradient runs through the phase rule.  Training lowers
    the loss at the final unroll length below the untrained network's."""
    nf, nc = 32, 16
    tau_f = 0.52
    tau_c = 0.5 + (tau_f - 0.5) / 2
    rho, u, frc, _ = forced_turbulence(nf, 200, seed=41, tau=tau_f, urms=0.06)
    ks, draws, amp, kf, cw = frc
    with Lattice((nf,) * 3, "f32", "bgk", tau_f) as fine, Lattice((nc,) * 3, "f32", "nco", tau_c) as coarse:
        fine.set_forcing(*frc, phase_rule=True)
        fine.init_equilibrium(rho, u)
        fine.step(200)
        target = fine.energy_spectrum()[:n_bins(nc)]
        coarse.restrict_from(fine)
        f0 = coarse.populations()
    assert np.all(np.isfinite(target)) and np.all(np.isfinite(f0))

    def sched(ep):
        return curriculum_steps(ep, start=20, grow=20, every=3)
    epochs = 9
    run = Unroll((nc,) * 3, tau_c, ("pop", f0), sched(0), 10, target, 2, 6, loss="paper", omega=20.0,
                 forcing=(ks, draws, 2.0 * amp, kf, cw, True))
    p0 = inputs.mlp_params(32, 1)
    run.nsteps = sched(epochs - 1)
    L_untrained = run.loss(p0)
    params, hist = train([run], p0, epochs=epochs, lr=1e-2, schedule=sched)
    run.nsteps = sched(epochs - 1)
    L_trained = run.loss(params)
    run.close()
    print("paper loss at %d steps: untrained %.4e, trained %.4e; history %s"
          % (sched(epochs - 1), L_untrained, L_trained, ["%.3e" % h for h in hist]))
    assert L_trained < 0.95 * L_untrained
