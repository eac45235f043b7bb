"""Pins of the fine-to-coarse restriction (Sec. "Learning Task") in the oracle."""
import numpy as np
import pytest

from oracle import collision, lattice, restrict, step
from paper_2412_08229_amd import inputs

C = lattice.velocities().astype(float)
W = lattice.weights()


def _ce_pre(n, u0, tau):
    """Pre-collision Chapman-Enskog state of the 2-D Taylor-Green vortex on
    an n^3 box: f^eq - tau (w_i / cs^2) rho c_ia c_ib d_a u_b (lattice units)."""
    rho, u, g = inputs.tgv2d(n, u0)
    cc = np.einsum("ia,ib,ab...->i...", C, C, g)
    return collision.equilibrium(rho, u) - tau * 3.0 * W.reshape(27, 1, 1, 1) * rho * cc


def test_identity_at_ratio_one():
    f = inputs.random_populations((5, 6, 7), seed=1)
    out = restrict.restrict(f, 1, 0.6, 0.6)
    assert np.abs(out - f).max() < 1e-16


def test_factor_is_the_printed_one_at_ratio_two():
    assert restrict.factor(2, 0.52, 0.51) == 2 * 0.52 / 0.51


@pytest.mark.parametrize("r", [2, 4])
def test_chapman_enskog_state_maps_to_the_coarse_one(r):
    """The fine Chapman-Enskog state, restricted, is the coarse one built
    directly at the coarse nodes with tau_c (acoustic scaling: the same
    velocity, nu_c = nu_f / r): exact to rounding, since the gradient in
    lattice units is r times larger on the coarse lattice."""
    n, u0 = 8, 0.05
    tau_f = 0.52
    tau_c = 0.5 + (tau_f - 0.5) / r
    fine_stored = step.unstream(_ce_pre(r * n, u0, tau_f))
    coarse_stored = restrict.restrict(fine_stored, r, tau_c, tau_f)
    assert np.abs(step.stream(coarse_stored) - _ce_pre(n, u0, tau_c)).max() < 1e-15
    # A plausible mistake: the printed factor 2 tau_c / tau_f at r = 4.
    if r == 4:
        pre = step.stream(fine_stored)[:, ::r, ::r, ::r]
        rho, u = collision.macroscopic(pre)
        feq = collision.equilibrium(rho, u)
        bad = feq + 2 * tau_c / tau_f * (pre - feq)
        assert np.abs(bad - _ce_pre(n, u0, tau_c)).max() > 1e-6


def test_mass_and_momentum_of_the_sampled_node():
    f = inputs.random_populations((8, 8, 8), seed=2, lo=0.8, hi=1.2)
    out = step.stream(restrict.restrict(f, 2, 0.55, 0.6))
    pre = step.stream(f)[:, ::2, ::2, ::2]
    assert np.abs(out.sum(0) - pre.sum(0)).max() < 1e-15
    assert np.abs(np.tensordot(C.T, out, 1) - np.tensordot(C.T, pre, 1)).max() < 1e-15
