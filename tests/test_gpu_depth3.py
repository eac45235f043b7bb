"""Networks with a third hidden layer (the network of Sec. "Training based
on dissipation rates") on the vector units and the matrix cores (float32,
split over the 16-bit ones, bf16), through the C ABI, against the oracle.
Depth 3 runs at width 32; narrower networks are zero-padded, so float64
storage must match the oracle to rounding at every width."""
import numpy as np
import pytest

from oracle import adjoint, collision, observables, step
from paper_2412_08229_amd import Lattice, inputs
from paper_2412_08229_amd import _lib as L

pytestmark = pytest.mark.gpu


def _setup(width, act, seed, n=8, amp=0.05):
    params = inputs.mlp_params(width, seed, depth=3)
    layers = collision.unpack_params(params, width, depth=3)
    rho, u = inputs.random_velocity((n, n, n), seed=seed + 1, amp=amp)
    return params, layers, rho, u


@pytest.mark.parametrize("storage,tol", [("f64", 1e-13), ("f32", 1e-5)])
@pytest.mark.parametrize("width,act", [(20, "relu"), (32, "tanh"), (8, "tanh")])
def test_depth3_steps_match_oracle(storage, tol, width, act):
    params, layers, rho, u = _setup(width, act, 40)
    tau, n = 0.56, 8
    with Lattice((n, n, n), storage, "nco", tau) as lat:
        lat.set_net_weights(params, width, act, "f32", depth=3)
        lat.init_equilibrium(rho, u)
        f0 = lat.populations()
        lat.step(10)
        got = lat.populations()
    want = step.run(f0, step.Operator("nco", tau, layers=layers, act=act), 10)
    err = np.abs(got - want).max()
    print("depth 3, width %d %s, %s storage, 10 steps: max err %.3e" % (width, act, storage, err))
    assert err < tol


@pytest.mark.parametrize("mlp", ["f32_mfma", "f32_split"])
@pytest.mark.parametrize("width,act", [(20, "relu"), (32, "tanh")])
def test_depth3_matrix_cores_match_oracle(width, act, mlp):
    """The third layer on the matrix cores (float32, or split over the
    16-bit ones; one more product per group element, chained on the second
    layer's accumulator): 10 steps and the rates readout against the
    oracle, in float32 storage; on a 9^3 lattice (ragged against the 64-node
    blocks)."""
    params, layers, rho, u = _setup(width, act, 48, n=9)
    tau, n = 0.56, 9
    with Lattice((n, n, n), "f32", "nco", tau) as lat:
        lat.set_net_weights(params, width, act, mlp, depth=3)
        lat.init_equilibrium(rho, u)
        f0 = lat.populations()
        om = lat.rates()
        lat.step(10)
        got = lat.populations()
    want = step.run(f0, step.Operator("nco", tau, layers=layers, act=act), 10)
    err = np.abs(got - want).max()
    rerr = np.abs(om - collision.nco_rates(f0, layers, act)).max()
    print("depth 3 on matrix cores (%s), width %d %s: max err %.3e, rates %.3e" % (mlp, width, act, err, rerr))
    assert err < 1e-5 and rerr < 1e-5


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("width,act", [(20, "relu"), (32, "tanh")])
def test_depth3_bf16_network_close_to_oracle(width, act, storage):
    """The third layer on the bf16 matrix cores (one more bf16 product per
    group element, fed by the second layer's activations rounded to bf16):
    rates within bf16 rounding of the oracle on the stored state (the bound
    of the depth-2 bf16 network's rates test) and 10 steps within the bound
    of the depth-2 bf16 network's 100-step parity case in the same storage,
    on a 9^3 lattice (ragged against the 64-node blocks)."""
    params, layers, rho, u = _setup(width, act, 49, n=9)
    tau, n = 0.56, 9
    with Lattice((n, n, n), storage, "nco", tau) as lat:
        lat.set_net_weights(params, width, act, "bf16", depth=3)
        lat.init_equilibrium(rho, u)
        f0 = lat.populations()
        om = lat.rates()
        lat.step(10)
        got = lat.populations()
    want = step.run(f0, step.Operator("nco", tau, layers=layers, act=act), 10)
    err = np.abs(got - want).max()
    rerr = np.abs(om - collision.nco_rates(f0, layers, act)).max()
    print("depth 3 on bf16 matrix cores, width %d %s, %s storage: max err %.3e, rates %.3e"
          % (width, act, storage, err, rerr))
    assert rerr < 5e-3
    assert err < {"f32": 3e-5, "bf16": 3e-4}[storage]


@pytest.mark.parametrize("mlp,tol", [("f32_mfma", 1e-6), ("f32_split", 1e-6), ("bf16", 1e-5)])
@pytest.mark.parametrize("n", [41, 128])
def test_depth3_sampled_against_oracle_at_size(n, mlp, tol):
    """The 27-20-20-20-4 ReLU network in the block shapes of larger
    lattices: 64-node blocks of four tiles per wavefront (41^3, a ragged
    last block) and 256-node blocks (128^3, the benchmark's launch), one step
    of the Taylor-Green vortex checked on 256 sampled nodes.  Bounds: those
    of the depth-2 sampled checks of the same arithmetics."""
    u0 = 0.1 / np.sqrt(3.0)
    _, tau = inputs.viscosity(n, u0, 1600.0)
    rho, u = inputs.tgv3d(n, u0)
    params = inputs.mlp_params(20, 50, depth=3)
    layers = collision.unpack_params(params, 20, depth=3)
    with Lattice((n, n, n), "f32", "nco", tau) as lat:
        lat.set_net_weights(params, 20, "relu", mlp, depth=3)
        lat.init_equilibrium(rho, u)
        lat.step(3)
        before = lat.populations()
        lat.step(1)
        after = lat.populations()
    pts = np.random.Generator(np.random.PCG64(51)).integers(0, n, size=(256, 3))
    C = [(cx, cy, cz) for cz in (-1, 0, 1) for cy in (-1, 0, 1) for cx in (-1, 0, 1)]
    pulled = np.empty((27, len(pts)))
    for i, (cx, cy, cz) in enumerate(C):
        pulled[i] = before[i, (pts[:, 0] - cz) % n, (pts[:, 1] - cy) % n, (pts[:, 2] - cx) % n]
    want = step.Operator("nco", tau, layers=layers, act="relu").collide(pulled)
    got = after[:, pts[:, 0], pts[:, 1], pts[:, 2]]
    err = np.abs(got - want).max()
    print("depth 3 %s at %d^3, sampled: max err %.3e" % (mlp, n, err))
    assert err < tol


def test_depth3_rates_match_oracle():
    params, layers, _, _ = _setup(20, "relu", 41)
    f = inputs.random_populations((6, 5, 7), seed=42, lo=0.8, hi=1.2)
    with Lattice((6, 5, 7), "f64", "nco", 0.6) as lat:
        lat.set_net_weights(params, 20, "relu", "f32", depth=3)
        lat.init_populations(f)
        got = lat.rates()
    want = collision.nco_rates(f, layers, "relu")
    assert np.abs(got - want).max() < 1e-13


@pytest.mark.parametrize("width,act,mlp", [(20, "relu", "f32"), (32, "tanh", "f32"), (20, "relu", "f32_mfma")])
def test_depth3_energy_gradient_matches_oracle(width, act, mlp):
    """Gradient of sum_m a_m k(t_m) over a 6-step run (checkpoints every 4)
    against the oracle's reverse mode, in the caller's parameter order
    (the padded units dropped)."""
    n, tau, T, K, every = 6, 0.56, 6, 4, 2
    params, layers, rho, u = _setup(width, act, 43, n=n, amp=0.08)
    a = np.random.Generator(np.random.PCG64(44)).standard_normal(T // every + 1)
    with Lattice((n, n, n), "f32", "nco", tau) as lat:
        lat.set_net_weights(params, width, act, mlp, depth=3)
        lat.init_equilibrium(rho, u)
        fs = lat.populations()
        k = lat.forward_record(T, K, energy_every=every)
        g, df0 = lat.backward(dL_dk=a, energy_every=every, want_df0=True)
    assert g.size == collision.n_params(width, depth=3)
    op = step.Operator("nco", tau, layers=layers, act=act)
    x, k_o = fs, [observables.kinetic_energy(fs)]
    for t in range(1, T + 1):
        x = step.step(x, op)
        if t % every == 0:
            k_o.append(observables.kinetic_energy(x))
    assert np.abs(k - np.array(k_o)).max() < 1e-6 * max(k_o)

    def traj(t, xt):
        return a[t // every] * adjoint.kinetic_energy_vjp(xt) if t % every == 0 else None
    _, go, gfo = adjoint.run_and_grad(fs, tau, layers, act, T, lambda xt: (0.0, np.zeros_like(xt)),
                                      traj_grad=traj)
    go = adjoint.flatten(go)
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    relf = np.linalg.norm(df0 - gfo) / np.linalg.norm(gfo)
    print("depth 3 width %d %s %s energy gradient: rel err %.2e, dL/df0 rel err %.2e" % (width, act, mlp, rel, relf))
    assert rel < 2e-3 and relf < 2e-3


def test_depth3_arguments_and_switching_back():
    params3 = inputs.mlp_params(20, 45, depth=3)
    params2 = inputs.mlp_params(32, 46)
    rho, u = inputs.random_velocity((4, 4, 4), seed=47, amp=0.05)
    with Lattice((4, 4, 4), "f32", "nco", 0.6) as lat:
        # Batched stepping takes depth-2 networks only.
        lat.set_net_weights(params3, 20, "relu", "f32_mfma", depth=3)
        from paper_2412_08229_amd.lattice import batch_step
        with pytest.raises(L.NCOError) as e:
            batch_step([lat], [1])
        assert e.value.status == L.NCO_E_UNSUPPORTED
        with pytest.raises(L.NCOError) as e:
            lat.set_net_weights(params3[:-1], 20, "relu", "f32", depth=3)
        assert e.value.status == L.NCO_E_INVALID
        with pytest.raises(L.NCOError) as e:
            L.nco_set_net_weights(lat._h, 20, 1, 0, params3, depth=4)
        assert e.value.status == L.NCO_E_INVALID
        # Depth 3, then back to depth 2 on the same lattice: the same as a
        # fresh lattice with the depth-2 network.
        lat.set_net_weights(params3, 20, "relu", "f32", depth=3)
        lat.init_equilibrium(rho, u)
        lat.step(2)
        lat.set_net_weights(params2, 32, "tanh", "f32_mfma")
        lat.init_equilibrium(rho, u)
        lat.step(3)
        got = lat.populations()
    with Lattice((4, 4, 4), "f32", "nco", 0.6) as ref:
        ref.set_net_weights(params2, 32, "tanh", "f32_mfma")
        ref.init_equilibrium(rho, u)
        ref.step(3)
        want = ref.populations()
    assert np.array_equal(got, want)
