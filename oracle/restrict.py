"""Fine-to-coarse restriction by acoustic scaling (Sec. "Learning Task",
the equation for f_{i,c}), in float64.

Test infrastructure (see ``oracle/__init__``): never used by the product path.

The coarse distribution at a coarse node is the equilibrium of the density
and velocity of the fine node at the same position plus the fine node's
non-equilibrium part f - f^eq scaled by (dx_c / dx_f)(tau_c / tau_f).  The
paper prints the factor 2 tau_c / tau_f, the value for a spacing ratio of 2;
the ratio-general form is used for any integer ratio r (the paper coarsens
256^3 to 32^3).  The scaling follows from the Chapman-Enskog form of the
non-equilibrium part, -tau (w_i / cs^2) rho c_i c_i : grad u, whose lattice
velocity gradient grows with the spacing at a fixed Mach number.

Reading of the state: the formula holds for the distribution entering the
collision (that form of the non-equilibrium part is the pre-collision one).
The stored state here is post-collision (see ``step``), so the fine state is
streamed first, restricted at the coarse nodes (coarse node X on fine node
r X), and the result is un-streamed on the coarse lattice: the coarse run's
first step then streams it back and collides exactly the restricted
distribution.
"""
import numpy as np

from . import collision, step


def factor(r, tau_c, tau_f):
    """(dx_c / dx_f)(tau_c / tau_f) for the spacing ratio r."""
    return r * tau_c / tau_f


def restrict_pre(f_pre, r, tau_c, tau_f):
    """Restriction of a pre-collision distribution (27, nz, ny, nx) to every
    r-th node on each axis."""
    fs = f_pre[:, ::r, ::r, ::r]
    rho, u = collision.macroscopic(fs)
    feq = collision.equilibrium(rho, u)
    return feq + factor(r, tau_c, tau_f) * (fs - feq)


def restrict(f_fine, r, tau_c, tau_f):
    """Stored (post-collision) fine state -> stored coarse state."""
    return step.unstream(restrict_pre(step.stream(f_fine), r, tau_c, tau_f))
