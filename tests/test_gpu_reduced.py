"""The reduced Taylor-Green domain of Appendix A on the GPU, through the C ABI.

A lattice of n^3 nodes in the domain 'tgv_octant' is the cube [0, pi/2]^3 of
the vortex and stands for the symmetric box of 4n nodes per edge.  It is
checked against the oracle's reduced step (unfold to the box, periodic step,
restrict: ``oracle.reduced``), against the oracle's periodic reverse mode on
the unfolded box, and against the GPU's own periodic run of the 4n box on the
same offset grid.

Tolerances: streaming is bit-exact; float64 storage agrees to rounding
(1e-13); the float32 and 16-bit forms use the bounds of the periodic parity
tests for the same storage and network arithmetic.
"""
import functools

import numpy as np
import pytest

from oracle import adjoint, collision, observables, reduced, step
from paper_2412_08229_amd import Lattice, inputs
from paper_2412_08229_amd import _lib as L

pytestmark = pytest.mark.gpu

U0 = 0.05
WIDTH = 32
OMEGA = np.array([1.15, 1.35, 1.55, 1.75])


def _lat(n, storage, kind, tau, mlp="f32", act="tanh", seed=0):
    lat = Lattice((n, n, n), storage, kind, tau)
    lat.set_domain("tgv_octant")
    if kind == "nco":
        lat.set_net_weights(inputs.mlp_params(WIDTH, seed), WIDTH, act, mlp)
    if kind == "mrt":
        lat.set_rates(OMEGA)
    return lat


def _op(kind, tau, act="tanh", seed=0):
    layers = collision.unpack_params(inputs.mlp_params(WIDTH, seed), WIDTH) if kind == "nco" else None
    return step.Operator(kind, tau, omega_high=OMEGA, layers=layers, act=act)


def _reduced_stream(f):
    n = f.shape[-1]
    return reduced.restrict(step.stream(reduced.unfold(f)), n)


@pytest.mark.parametrize("storage", ["f32", "f64", "f16", "bf16"])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 12])
def test_reduced_streaming_is_bit_exact(storage, n):
    f0 = inputs.random_populations((n, n, n), seed=3)
    with _lat(n, storage, "stream", 0.6) as lat:
        lat.init_populations(f0)
        q = lat.populations()
        lat.step(1)
        g = lat.populations()
        lat.step(2)
        g3 = lat.populations()
    assert np.array_equal(g, _reduced_stream(q))
    assert np.array_equal(g3, _reduced_stream(_reduced_stream(_reduced_stream(q))))


@pytest.mark.parametrize("kind", ["bgk", "mrt", "nco"])
@pytest.mark.parametrize("n", [2, 3])
def test_reduced_f64_matches_oracle(kind, n):
    """Far from equilibrium, every moment exercised: float64 storage equals
    the oracle's reduced step to rounding."""
    f0 = inputs.random_populations((n, n, n), seed=4)
    with _lat(n, "f64", kind, 0.6) as lat:
        lat.init_populations(f0)
        lat.step(5)
        got = lat.populations()
    want = reduced.run(f0, _op(kind, 0.6), 5)
    assert np.abs(got - want).max() < 1e-13


N_TGV, STEPS_TGV = 4, 40


@functools.lru_cache(maxsize=None)
def _oracle_tgv(kind):
    tau = inputs.viscosity(4 * N_TGV, U0, 100.0)[1] if kind == "nco" else 0.6
    rho, u = inputs.tgv3d_octant(N_TGV, U0)
    return tau, rho, u, reduced.run(collision.equilibrium(rho, u), _op(kind, tau), STEPS_TGV)


TGV_BOUNDS = {
    ("f32", "bgk", "f32"): 1e-5, ("f32", "mrt", "f32"): 1e-5,
    ("f32", "nco", "f32"): 1e-5, ("f32", "nco", "f32_mfma"): 1e-5, ("f32", "nco", "bf16"): 3e-5,
    ("f16", "nco", "f32_mfma"): 3e-5, ("bf16", "nco", "bf16"): 3e-4,
}


@pytest.mark.parametrize("storage,kind,mlp", sorted(TGV_BOUNDS))
def test_reduced_tgv_matches_oracle(storage, kind, mlp):
    """The vortex on the 4^3 cube (the 16^3 box), 40 steps, every storage
    and network arithmetic against the oracle's reduced run."""
    tau, rho, u, want = _oracle_tgv(kind)
    with _lat(N_TGV, storage, kind, tau, mlp=mlp) as lat:
        lat.init_equilibrium(rho, u)
        lat.step(STEPS_TGV)
        got = lat.populations()
    err = np.abs(got - want).max()
    print("reduced 4^3 %s/%s/%s x%d: max err %.3e" % (storage, kind, mlp, STEPS_TGV, err))
    assert err < TGV_BOUNDS[(storage, kind, mlp)]


@pytest.mark.parametrize("kind,mlp", [("bgk", "f32"), ("nco", "f32_mfma"), ("nco", "bf16")])
def test_reduced_cube_equals_gpu_box(kind, mlp):
    """The 16^3 cube and the 64^3 box (offset grid) at Re 1600, Ma 0.1, 300
    steps on the GPU: the cube holds the box's values (to float32 rounding,
    the summation order differs between images) and the same kinetic
    energy."""
    n, u0 = 16, 0.1 / np.sqrt(3.0)
    _, tau = inputs.viscosity(4 * n, u0, 1600.0)
    rho, u = inputs.tgv3d(4 * n, u0, offset=0.5)
    rho_c, u_c = inputs.tgv3d_octant(n, u0)
    with Lattice((4 * n,) * 3, "f32", kind, tau) as box:
        if kind == "nco":
            box.set_net_weights(inputs.mlp_params(WIDTH, 0), WIDTH, "tanh", mlp)
        box.init_equilibrium(rho, u)
        box.step(300)
        fb = reduced.restrict(box.populations(), n)
        kb = box.global_sums()[4] / box.n
    with _lat(n, "f32", kind, tau, mlp=mlp) as cube:
        cube.init_equilibrium(rho_c, u_c)
        cube.step(300)
        fc = cube.populations()
        kc = cube.global_sums()[4] / cube.n
    err = np.abs(fc - fb).max()
    print("cube 16^3 vs box 64^3 %s/%s x300: max |f| diff %.3e, k rel diff %.3e"
          % (kind, mlp, err, abs(kc - kb) / kb))
    assert err < 1e-5 and abs(kc - kb) < 1e-5 * kb


@pytest.mark.parametrize("mlp", ["f32", "f32_mfma"])
@pytest.mark.parametrize("n", [2, 3])
def test_reduced_energy_gradient_matches_oracle_box(mlp, n):
    """dL/dtheta of L = sum_m a_m k(t_m) on the cube equals the oracle's
    periodic reverse mode on the unfolded 4n box (k is the same function of
    theta on both), and dL/df0 on the cube is the sum over the 64 images of
    the box's, i.e. 64 times its value on the cube's own nodes."""
    width, tau, T, K, every = WIDTH, 0.56, 6, 4, 2
    params = inputs.mlp_params(width, 21)
    rho, u = inputs.random_velocity((n, n, n), seed=22, amp=0.08)
    a = np.random.Generator(np.random.PCG64(23)).standard_normal(T // every + 1)
    with Lattice((n, n, n), "f32", "nco", tau) as lat:
        lat.set_domain("tgv_octant")
        lat.set_net_weights(params, width, "tanh", mlp)
        lat.init_equilibrium(rho, u)
        fs = lat.populations()
        k = lat.forward_record(T, K, energy_every=every)
        g, df0 = lat.backward(dL_dk=a, energy_every=every, want_df0=True)
    layers = collision.unpack_params(params, width)
    full = reduced.unfold(fs)
    op = step.Operator("nco", tau, layers=layers, act="tanh")
    x, k_o = full, [observables.kinetic_energy(full)]
    for t in range(1, T + 1):
        x = step.step(x, op)
        if t % every == 0:
            k_o.append(observables.kinetic_energy(x))
    assert np.abs(k - np.array(k_o)).max() < 1e-6 * max(k_o)

    def traj(t, xt):
        return a[t // every] * adjoint.kinetic_energy_vjp(xt) if t % every == 0 else None
    _, go, gfo = adjoint.run_and_grad(full, tau, layers, "tanh", T, lambda xt: (0.0, np.zeros_like(xt)),
                                      traj_grad=traj)
    go = adjoint.flatten(go)
    gfo = 64.0 * reduced.restrict(gfo, n)
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    relf = np.linalg.norm(df0 - gfo) / np.linalg.norm(gfo)
    print("reduced %d^3 energy gradient %s: rel err %.2e, dL/df0 rel err %.2e" % (n, mlp, rel, relf))
    assert rel < 2e-3 and relf < 2e-3


def test_reduced_gradient_equals_gpu_box():
    """The same energy-trajectory gradient from the 8^3 cube and the 32^3
    box on the GPU (the vortex at Re 1600, 60 steps, checkpoints every 20)."""
    n, u0, T, K, every = 8, 0.1 / np.sqrt(3.0), 60, 20, 10
    _, tau = inputs.viscosity(4 * n, u0, 1600.0)
    params = inputs.mlp_params(WIDTH, 5)
    a = np.random.Generator(np.random.PCG64(6)).standard_normal(T // every + 1)
    out = []
    for domain, shape, (rho, u) in (("periodic", (4 * n,) * 3, inputs.tgv3d(4 * n, u0, offset=0.5)),
                                    ("tgv_octant", (n,) * 3, inputs.tgv3d_octant(n, u0))):
        with Lattice(shape, "f32", "nco", tau) as lat:
            lat.set_domain(domain)
            lat.set_net_weights(params, WIDTH, "tanh", "f32_mfma")
            lat.init_equilibrium(rho, u)
            k = lat.forward_record(T, K, energy_every=every)
            g, _ = lat.backward(dL_dk=a, energy_every=every)
        out.append((k, g))
    (kb, gb), (kc, gc) = out
    rel = np.linalg.norm(gc - gb) / np.linalg.norm(gb)
    print("gradient cube 8^3 vs box 32^3: k max rel diff %.2e, grad rel diff %.2e"
          % (np.abs(kc - kb).max() / kb.max(), rel))
    assert np.abs(kc - kb).max() < 1e-5 * kb.max() and rel < 1e-3


def test_reduced_domain_arguments():
    with Lattice((4, 4, 5), "f32", "bgk", 0.6) as lat:
        with pytest.raises(L.NCOError) as e:
            lat.set_domain("tgv_octant")
        assert e.value.status == L.NCO_E_INVALID
        with pytest.raises(L.NCOError) as e:
            L.nco_set_domain(lat._h, 7)
        assert e.value.status == L.NCO_E_INVALID
    with _lat(4, "f32", "bgk", 0.6) as lat:
        rho, u = inputs.tgv3d_octant(4, U0)
        lat.init_equilibrium(rho, u)
        with pytest.raises(L.NCOError) as e:
            lat.energy_spectrum()
        assert e.value.status == L.NCO_E_UNSUPPORTED
        lat.set_domain("periodic")
        assert lat.energy_spectrum().shape[0] > 0
