"""Convergence study of Sec. "Convergence": the extruded two-dimensional
Taylor-Green vortex, one time step at several resolutions, the deviation of
velocity and pressure from the analytic solution in the relative L2 norm.

Setup (the paper gives no numbers): u0 = 0.05, Re = 100 at every
resolution (nu = u0 (n / 2 pi) / Re, tau = 3 nu + 1/2), NCO with the seeded
27-32-32-4 tanh network on the float32 matrix cores.  Analytic solution at
step t: u = u(0) exp(-2 nu k^2 t), p = p(0) exp(-4 nu k^2 t), k^2 = (2 pi / n)^2,
with p(0) = -u0^2/4 (cos 2x + cos 2y) (the pressure of the printed
velocity) and p = cs^2 (rho - 1) on the lattice.  Two starts: the
post-collision Chapman-Enskog state (first-order non-equilibrium part
included) and the equilibrium alone.  At every resolution the GPU's fields
after the step equal the oracle's to float32 rounding; the errors fall with
the resolution (measured orders printed; bounds below carry a margin).
"""
import json
import math

import numpy as np
import pytest

from oracle import collision, lattice, step
from paper_2412_08229_amd import Lattice, inputs

pytestmark = pytest.mark.gpu

U0, RE = 0.05, 100.0
C = lattice.velocities()
W = lattice.weights()


def _start(n, tau, kind):
    rho, u, g = inputs.tgv2d(n, U0)
    feq = collision.equilibrium(rho, u)
    if kind == "equilibrium":
        return feq
    cc = np.einsum("ia,ib,ab...->i...", C.astype(float), C.astype(float), g)
    return feq - (tau - 1.0) * 3.0 * W.reshape(27, 1, 1, 1) * rho * cc


def _errors(rho, u, n, nu):
    _, u_a, _ = inputs.tgv2d(n, U0)
    rho_a, _, _ = inputs.tgv2d(n, U0)
    k2 = (2.0 * math.pi / n) ** 2
    u_a = u_a * math.exp(-2.0 * nu * k2)
    p_a = (rho_a - 1.0) / 3.0 * math.exp(-4.0 * nu * k2)
    p = (rho - 1.0) / 3.0
    eu = math.sqrt(((u - u_a) ** 2).sum() / (u_a ** 2).sum())
    ep = math.sqrt(((p - p_a) ** 2).sum() / (p_a ** 2).sum())
    return eu, ep


@pytest.mark.parametrize("start", ["chapman_enskog", "equilibrium"])
def test_tgv2d_convergence_one_step(start):
    params = inputs.mlp_params(32, 0)
    layers = collision.unpack_params(params, 32)
    out = {}
    for n in (8, 16, 32, 64):
        nu, tau = inputs.viscosity(n, U0, RE)
        f0 = _start(n, tau, start)
        with Lattice((n, n, n), "f32", "nco", tau) as lat:
            lat.set_net_weights(params, 32, "tanh", "f32_mfma")
            lat.init_populations(f0)
            fs = lat.populations()
            lat.step(1)
            rho_g, u_g = lat.macroscopic()
        f1 = step.run(fs, step.Operator("nco", tau, layers=layers, act="tanh"), 1)
        rho_o, u_o = collision.macroscopic(f1)
        assert np.abs(u_g - u_o).max() < 1e-7 and np.abs(rho_g - rho_o).max() < 1e-6
        out[n] = _errors(rho_g, u_g, n, nu)
    ns = sorted(out)
    order_u = [math.log2(out[a][0] / out[b][0]) for a, b in zip(ns, ns[1:])]
    order_p = [math.log2(out[a][1] / out[b][1]) for a, b in zip(ns, ns[1:])]
    print("CONVERGENCE", start, json.dumps({"errors": {str(k): v for k, v in out.items()},
                                            "order_u": order_u, "order_p": order_p}))
    for a, b in zip(ns, ns[1:]):
        assert out[b][0] < out[a][0] and out[b][1] < out[a][1]
    assert order_u[-1] > 1.5
