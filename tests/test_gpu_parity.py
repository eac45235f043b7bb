"""GPU parity of the HIP path against the CPU float64 oracle, through the C ABI.

Tolerances: streaming is bit-exact (a permutation of stored values); float64
storage agrees with the oracle to rounding (1e-13); the float32 path stays
within 1e-5 max-abs population error after 100 steps at 16^3.
"""
import numpy as np
import pytest

from oracle import collision, observables, step
from paper_2412_08229_amd import Lattice, inputs
from paper_2412_08229_amd import _lib as L

pytestmark = pytest.mark.gpu

WIDTH = 32
OMEGA = np.array([1.15, 1.35, 1.55, 1.75])


def _params(width=WIDTH, seed=0):
    return inputs.mlp_params(width, seed)


def _oracle_op(kind, tau, width=WIDTH, seed=0, act="tanh"):
    layers = collision.unpack_params(_params(width, seed), width) if kind == "nco" else None
    return step.Operator(kind, tau, omega_high=OMEGA, layers=layers, act=act)


def _lattice(shape, storage, kind, tau, width=WIDTH, seed=0, act="tanh", mlp="f32"):
    lat = Lattice(shape, storage, kind, tau)
    if kind == "nco":
        lat.set_net_weights(_params(width, seed), width, act, mlp)
    if kind == "mrt":
        lat.set_rates(OMEGA)
    return lat


# ------------------------------------------------------------- streaming ----

@pytest.mark.parametrize("storage", ["f32", "f64", "f16", "bf16"])
@pytest.mark.parametrize("shape", [(5, 7, 9), (1, 1, 1), (3, 1, 2), (16, 16, 16), (2, 3, 130)])
def test_streaming_is_bit_exact(storage, shape):
    f0 = inputs.random_populations(shape, seed=1)
    with Lattice(shape, storage, "stream", 0.6) as lat:
        lat.init_populations(f0)
        q = lat.populations()          # the stored values, decoded exactly
        lat.step(1)
        g = lat.populations()
        lat.step(2)
        g3 = lat.populations()
    assert np.array_equal(g, step.stream(q))
    assert np.array_equal(g3, step.stream(step.stream(step.stream(q))))


# ------------------------------------------------- float32 path, C1 config --

def _tgv16():
    n, u0 = 16, 0.05
    rho, u = inputs.tgv3d(n, u0)
    return n, rho, u


@pytest.mark.parametrize("kind,mlp", [("bgk", "f32"), ("mrt", "f32"), ("nco", "f32"), ("nco", "f32_mfma"),
                                      ("nco", "f32_split")])
def test_f32_tgv16_100_steps_within_1e5(kind, mlp):
    n, rho, u = _tgv16()
    tau = inputs.viscosity(n, 0.05, 100.0)[1] if kind == "nco" else 0.6
    with _lattice((n, n, n), "f32", kind, tau, mlp=mlp) as lat:
        lat.init_equilibrium(rho, u)
        lat.step(100)
        got = lat.populations()
    want = step.run(collision.equilibrium(rho, u), _oracle_op(kind, tau), 100)
    err = np.abs(got - want).max()
    print("%s/%s f32 16^3 x100: max err %.3e" % (kind, mlp, err))
    assert err < 1e-5


# ---------------------------------------------------- float64 storage -------

@pytest.mark.parametrize("kind", ["bgk", "mrt", "nco"])
@pytest.mark.parametrize("shape", [(6, 5, 7), (1, 4, 3)])
def test_f64_matches_oracle_to_rounding(kind, shape):
    f0 = inputs.random_populations(shape, seed=2, lo=0.8, hi=1.2)
    tau = 0.57
    with _lattice(shape, "f64", kind, tau, width=20, seed=3) as lat:
        lat.init_populations(f0)
        lat.step(3)
        got = lat.populations()
    want = step.run(f0, _oracle_op(kind, tau, width=20, seed=3), 3)
    assert np.abs(got - want).max() < 1e-13


@pytest.mark.parametrize("width,act", [(8, "tanh"), (16, "relu"), (20, "relu"), (32, "tanh")])
def test_network_rates_match_oracle(width, act):
    shape = (3, 4, 5)
    rho, u = inputs.random_velocity(shape, seed=4, amp=0.1)
    f0 = collision.equilibrium(rho, u) + 0.01 * (inputs.random_populations(shape, seed=5) - 1.0 / 27)
    layers = collision.unpack_params(_params(width, 6), width)
    want = collision.nco_rates(f0, layers, act)
    for storage, tol in (("f64", 1e-13), ("f32", 2e-6)):
        with _lattice(shape, storage, "nco", 0.6, width=width, seed=6, act=act) as lat:
            lat.init_populations(f0)
            got = lat.rates()
            f_stored = lat.populations()
        want_s = collision.nco_rates(f_stored, layers, act)
        assert np.abs(got - want_s).max() < tol, (storage, np.abs(got - want_s).max())
        assert np.abs(got - want).max() < max(tol, 1e-5)


# -------------------------------------------------------- observables -------

@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_global_sums_match_oracle(storage):
    shape = (7, 6, 5)
    rho, u = inputs.random_velocity(shape, seed=7)
    with Lattice(shape, storage, "bgk", 0.6) as lat:
        lat.init_equilibrium(rho, u)
        s = lat.global_sums()
        f = lat.populations()
        r2, u2 = lat.macroscopic()
    want = observables.global_sums(f)
    np.testing.assert_allclose(s, want, rtol=1e-13, atol=1e-15)
    rr, uu = collision.macroscopic(f)
    np.testing.assert_allclose(r2, rr, rtol=1e-14)
    np.testing.assert_allclose(u2, uu, atol=1e-16)


# 40 and 70: several 32-long input chunks and 64-frequency blocks of the
# DFT, each with a ragged tail, and a ragged last block of lines.
@pytest.mark.parametrize("n", [8, 9, 12, 16, 40, 70])
def test_energy_spectrum_matches_oracle(n):
    rho, u = inputs.turbulence(n, seed=8, k0=2.0, urms=0.05)
    with Lattice((n, n, n), "f64", "bgk", 0.6) as lat:
        lat.init_equilibrium(rho, u)
        E = lat.energy_spectrum()
        f = lat.populations()
    want = observables.spectrum(f)
    assert E.shape == want.shape
    np.testing.assert_allclose(E, want, rtol=1e-11, atol=1e-18)


@pytest.mark.parametrize("storage,mlp,tol", [("f64", "f32", 1e-12), ("f32", "f32", 1e-7),
                                             ("f32", "f32_mfma", 1e-7), ("f32", "f32_split", 1e-7)])
def test_conservation_on_gpu(storage, mlp, tol):
    n = 16
    rho, u = inputs.random_velocity((n, n, n), seed=9, amp=0.05)
    with _lattice((n, n, n), storage, "nco", 0.52, mlp=mlp) as lat:
        lat.init_equilibrium(rho, u)
        s0 = lat.global_sums()
        lat.step(100)
        s1 = lat.global_sums()
    assert abs(s1[0] - s0[0]) / s0[0] < tol
    assert np.abs(s1[1:4] - s0[1:4]).max() / s0[0] < tol


# Lattice symmetries as (matrix R acting on velocities, the node map as a
# function on [z][y][x] arrays): a rotation by 90 degrees about z, the
# reflection x -> -x, and the cyclic axis permutation (x, y, z) -> (y, z, x).
_SYMMETRIES = {
    "rot_z": (np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]]), lambda a: np.rot90(a, k=1, axes=(2, 1))),
    "reflect_x": (np.diag([-1, 1, 1]), lambda a: np.roll(a[:, :, ::-1], 1, axis=2)),
    "cycle_xyz": (np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]]), lambda a: np.transpose(a, (1, 2, 0))),
}


def _apply_symmetry(f, name):
    R, nodes = _SYMMETRIES[name]
    C = np.array([(cx, cy, cz) for cz in (-1, 0, 1) for cy in (-1, 0, 1) for cx in (-1, 0, 1)])
    index = {tuple(c): i for i, c in enumerate(C)}
    out = np.empty_like(f)
    for j in range(27):
        out[index[tuple(R @ C[j])]] = nodes(f[j])
    return out


@pytest.mark.parametrize("sym", sorted(_SYMMETRIES))
@pytest.mark.parametrize("storage, mlp, tol", [("f64", "f32", 1e-13), ("f32", "f32", 1e-6),
                                               ("f32", "f32_mfma", 1e-6), ("f32", "f32_split", 1e-6),
                                               ("f32", "bf16", 1e-5)])
def test_lattice_symmetry_equivariance_on_gpu(sym, storage, mlp, tol):
    """A lattice symmetry applied to the whole field commutes with two NCO
    steps (Sec. II.B: the group-averaged rates are invariant, the collision
    equivariant), on the vector-unit and both matrix-core networks.  Only
    the order of the group sum changes, so agreement is to rounding."""
    n = 8
    f0 = inputs.random_populations((n, n, n), seed=10, lo=0.9, hi=1.1)
    res = []
    for start in (f0, _apply_symmetry(f0, sym)):
        with _lattice((n, n, n), storage, "nco", 0.55, mlp=mlp) as lat:
            lat.init_populations(start)
            lat.step(2)
            res.append(lat.populations())
    assert np.abs(_apply_symmetry(res[0], sym) - res[1]).max() < tol


def test_symmetry_maps_are_lattice_symmetries():
    """The node maps above move a field the way its velocities say: a single
    population travelling along c ends, after streaming, where the mapped
    one travels along R c (checked with the streaming-only operator)."""
    n = 6
    for name in _SYMMETRIES:
        f0 = inputs.random_populations((n, n, n), seed=12, lo=0.9, hi=1.1)
        res = []
        for start in (f0, _apply_symmetry(f0, name)):
            with Lattice((n, n, n), "f64", "stream", 0.6) as lat:
                lat.init_populations(start)
                lat.step(1)
                res.append(lat.populations())
        assert np.array_equal(_apply_symmetry(res[0], name), res[1]), name


@pytest.mark.parametrize("mlp", ["f32", "f32_mfma", "f32_split"])
def test_bench_size_sampled_against_oracle(mlp):
    """128^3 float32 NCO in the benchmark's launch configuration: one step
    checked node by node on a sample of 256 nodes."""
    n = 128
    _, tau = inputs.viscosity(n, 0.1 / np.sqrt(3.0), 1600.0)
    rho, u = inputs.tgv3d(n, 0.1 / np.sqrt(3.0))
    with _lattice((n, n, n), "f32", "nco", tau, mlp=mlp) as lat:
        lat.init_equilibrium(rho, u)
        lat.step(3)
        before = lat.populations()
        lat.step(1)
        after = lat.populations()
    assert np.isfinite(after).all()
    rng = np.random.Generator(np.random.PCG64(11))
    pts = rng.integers(0, n, size=(256, 3))
    C = np.array([(cx, cy, cz) for cz in (-1, 0, 1) for cy in (-1, 0, 1) for cx in (-1, 0, 1)])
    pulled = np.empty((27, len(pts)))
    for i, (cx, cy, cz) in enumerate(C):
        pulled[i] = before[i, (pts[:, 0] - cz) % n, (pts[:, 1] - cy) % n, (pts[:, 2] - cx) % n]
    want = _oracle_op("nco", tau).collide(pulled)
    got = after[:, pts[:, 0], pts[:, 1], pts[:, 2]]
    assert np.abs(got - want).max() < 1e-6


@pytest.mark.parametrize("mlp", ["f32", "f32_mfma", "f32_split"])
def test_repeatable_bitwise(mlp):
    n = 12
    rho, u = inputs.random_velocity((n, n, n), seed=12)
    out = []
    for _ in range(2):
        with _lattice((n, n, n), "f32", "nco", 0.55, mlp=mlp) as lat:
            lat.init_equilibrium(rho, u)
            lat.step(5)
            out.append((lat.populations(), lat.global_sums(), lat.energy_spectrum()))
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_state_and_argument_errors():
    with Lattice((4, 4, 4), "f32", "nco", 0.6) as lat:
        with pytest.raises(L.NCOError) as e:
            lat.step(1)
        assert e.value.status == L.NCO_E_STATE
        with pytest.raises(L.NCOError) as e:
            lat.rates()
        assert e.value.status == L.NCO_E_STATE
        with pytest.raises(L.NCOError) as e:
            lat.set_net_weights(np.zeros(10), 32)
        assert e.value.status == L.NCO_E_INVALID
        with pytest.raises(L.NCOError) as e:
            lat.set_net_weights(np.zeros(inputs.n_params(12)), 12)
        assert e.value.status == L.NCO_E_INVALID
        with pytest.raises(L.NCOError) as e:
            lat.set_rates([1.0, 2.5, 1.0, 1.0])
        assert e.value.status == L.NCO_E_INVALID
        with pytest.raises(L.NCOError):
            lat.set_op("bgk", 0.5)
    with Lattice((4, 5, 4), "f32", "bgk", 0.6) as lat:
        with pytest.raises(L.NCOError):
            lat.energy_spectrum()


def test_zero_steps_and_rest_state():
    """A new lattice holds the rest state w_i, which every operator keeps."""
    with _lattice((3, 3, 3), "f64", "nco", 0.7) as lat:
        f = lat.populations()
        lat.step(0)
        assert np.array_equal(lat.populations(), f)
        lat.step(4)
        g = lat.populations()
    w = collision.equilibrium(np.ones((3, 3, 3)), np.zeros((3, 3, 3, 3)))
    assert np.abs(f - w).max() < 1e-16 and np.abs(g - w).max() < 1e-15


# ------------------------------------------------- matrix-core network -------

@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("act", ["tanh", "relu"])
def test_mfma_network_rates_match_oracle(storage, act):
    """Rates of the matrix-core network path on a ragged node count (315 =
    one full block and a partial one) against the oracle on the stored state."""
    shape = (5, 7, 9)
    rho, u = inputs.random_velocity(shape, seed=13, amp=0.1)
    f0 = collision.equilibrium(rho, u) + 0.01 * (inputs.random_populations(shape, seed=14) - 1.0 / 27)
    layers = collision.unpack_params(_params(32, 15), 32)
    with _lattice(shape, storage, "nco", 0.6, width=32, seed=15, act=act, mlp="f32_mfma") as lat:
        lat.init_populations(f0)
        got = lat.rates()
        f_stored = lat.populations()
    want = collision.nco_rates(f_stored, layers, act)
    err = np.abs(got - want).max()
    print("mfma rates %s/%s: %.3e" % (storage, act, err))
    assert err < 2e-6


@pytest.mark.parametrize("mlp", ["f32_mfma", "f32_split"])
@pytest.mark.parametrize("shape", [(5, 7, 9), (1, 1, 1), (16, 16, 16), (41, 43, 45), (67, 65, 66)])
def test_mfma_step_matches_oracle_ragged(shape, mlp):
    """Two steps against the oracle, from a ragged partial block to
    lattices of 64-node blocks of four tiles per wavefront (41 x 43 x 45 =
    79,335 nodes) and of 256-node blocks (67 x 65 x 66 = 287,430 nodes),
    each with a partial last block."""
    f0 = inputs.random_populations(shape, seed=16, lo=0.9, hi=1.1)
    tau = 0.56
    if shape[0] > 16:
        # The oracle on a sample of nodes (their pulled neighbourhoods).
        with _lattice(shape, "f32", "nco", tau, mlp=mlp) as lat:
            lat.init_populations(f0)
            lat.step(1)
            before = lat.populations()
            lat.step(1)
            after = lat.populations()
        rng = np.random.Generator(np.random.PCG64(21))
        pts = np.concatenate([rng.integers(0, shape, size=(200, 3)), [[s - 1 for s in shape], [0, 0, 0]]])
        C = np.array([(cx, cy, cz) for cz in (-1, 0, 1) for cy in (-1, 0, 1) for cx in (-1, 0, 1)])
        pulled = np.empty((27, len(pts)))
        for i, (cx, cy, cz) in enumerate(C):
            pulled[i] = before[i, (pts[:, 0] - cz) % shape[0], (pts[:, 1] - cy) % shape[1],
                               (pts[:, 2] - cx) % shape[2]]
        want = _oracle_op("nco", tau).collide(pulled)
        assert np.abs(after[:, pts[:, 0], pts[:, 1], pts[:, 2]] - want).max() < 1e-6
        return
    with _lattice(shape, "f32", "nco", tau, mlp=mlp) as lat:
        lat.init_populations(f0)
        f_stored = lat.populations()
        lat.step(2)
        got = lat.populations()
    want = step.run(f_stored, _oracle_op("nco", tau), 2)
    assert np.abs(got - want).max() < 2e-6


def test_mfma_requires_float_storage():
    with Lattice((4, 4, 4), "f64", "nco", 0.6) as lat:
        with pytest.raises(L.NCOError) as e:
            lat.set_net_weights(_params(32), 32, "tanh", "f32_mfma")
        assert e.value.status == L.NCO_E_UNSUPPORTED


@pytest.mark.parametrize("width, act", [(20, "relu"), (20, "tanh"), (8, "tanh"), (16, "relu")])
@pytest.mark.parametrize("mlp, tol", [("f32_mfma", 2e-6), ("bf16", 5e-3), ("f32_split", 2e-6)])
def test_mfma_narrow_networks_match_oracle(width, act, mlp, tol):
    """Widths below 32 on the matrix cores (zero-padded to 32), among them
    the paper's 27-20-20-4 ReLU network: rates on a ragged lattice against
    the oracle at the true width, and two steps."""
    shape = (5, 7, 9)
    rho, u = inputs.random_velocity(shape, seed=17, amp=0.1)
    f0 = collision.equilibrium(rho, u) + 0.01 * (inputs.random_populations(shape, seed=18) - 1.0 / 27)
    layers = collision.unpack_params(_params(width, 19), width)
    with _lattice(shape, "f32", "nco", 0.58, width=width, seed=19, act=act, mlp=mlp) as lat:
        lat.init_populations(f0)
        f_stored = lat.populations()
        got = lat.rates()
        lat.step(2)
        after = lat.populations()
    want = collision.nco_rates(f_stored, layers, act)
    assert np.abs(got - want).max() < tol
    op = step.Operator("nco", 0.58, layers=layers, act=act)
    assert np.abs(after - step.run(f_stored, op, 2)).max() < (1e-4 if mlp == "bf16" else 2e-6)


# ------------------------------------------- float32 split over f16 products --

@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("act", ["tanh", "relu"])
@pytest.mark.parametrize("layer, scale", [(2, 1.0), (2, 1e-3), (2, 40.0), (1, 1e-3), (1, 40.0)])
def test_split_network_rates_match_oracle(storage, act, layer, scale):
    """Split arithmetic (f16 products of heads and remainders for tanh, bf16
    products of three parts for ReLU): rates on a ragged lattice against the
    float64 oracle at the float32 matrix cores' bound, with the first or the
    second layer's weights scaled over five decades (for tanh, the
    power-of-two scales that keep the f16 parts in range), and its error
    within a few times that of the float32 matrix cores on the same state."""
    shape = (5, 7, 9)
    rho, u = inputs.random_velocity(shape, seed=13, amp=0.1)
    f0 = collision.equilibrium(rho, u) + 0.01 * (inputs.random_populations(shape, seed=14) - 1.0 / 27)
    params = _params(32, 15).copy()
    n1 = 27 * 32 + 32
    if layer == 2:
        params[n1:n1 + 32 * 32] *= scale
    else:
        params[:27 * 32] *= scale
    params = params.astype(np.float32).astype(np.float64)      # the weights the lattice holds
    layers = collision.unpack_params(params, 32)
    errs = {}
    for mlp in ("f32_mfma", "f32_split"):
        with Lattice(shape, storage, "nco", 0.6) as lat:
            lat.set_net_weights(params, 32, act, mlp)
            lat.init_populations(f0)
            got = lat.rates()
            f_stored = lat.populations()
        want = collision.nco_rates(f_stored, layers, act)
        errs[mlp] = np.abs(got - want).max()
    print("rates %s %s, W%d x %g: float32 matrix cores %.3e, split %.3e" % (storage, act, layer, scale,
                                                                            errs["f32_mfma"], errs["f32_split"]))
    assert errs["f32_split"] < 2e-6
    assert errs["f32_split"] < 4 * errs["f32_mfma"] + 1e-7



# ------------------------------------------------------ precision forms -------

@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("act", ["tanh", "relu"])
def test_bf16_network_rates_close_to_oracle(storage, act):
    """bf16 matrix-core network: rates within bf16 rounding of the float64
    oracle on the stored state (error printed)."""
    shape = (5, 7, 9)
    rho, u = inputs.random_velocity(shape, seed=17, amp=0.1)
    f0 = collision.equilibrium(rho, u) + 0.01 * (inputs.random_populations(shape, seed=18) - 1.0 / 27)
    layers = collision.unpack_params(_params(32, 19), 32)
    with _lattice(shape, storage, "nco", 0.6, width=32, seed=19, act=act, mlp="bf16") as lat:
        lat.init_populations(f0)
        got = lat.rates()
        f_stored = lat.populations()
    want = collision.nco_rates(f_stored, layers, act)
    err = np.abs(got - want).max()
    print("bf16 network rates %s/%s: max |omega - omega_oracle| = %.3e" % (storage, act, err))
    assert err < 5e-3


# Measured errors against the float64 oracle after 100 steps of the 16^3
# Taylor-Green case (NCO, 27-32-32-4 tanh); bounds carry a margin of ~3x.
PRECISION_BOUNDS = {
    ("f32", "f32"): 1e-5, ("f32", "f32_mfma"): 1e-5, ("f32", "f32_split"): 1e-5, ("f32", "bf16"): 3e-5,
    ("f16", "f32_mfma"): 3e-5, ("f16", "bf16"): 5e-5,
    ("bf16", "f32_mfma"): 3e-4, ("bf16", "bf16"): 3e-4,
}


@pytest.mark.parametrize("storage,mlp", sorted(PRECISION_BOUNDS))
def test_precision_forms_tgv16_100_steps(storage, mlp):
    n, rho, u = _tgv16()
    tau = inputs.viscosity(n, 0.05, 100.0)[1]
    with _lattice((n, n, n), storage, "nco", tau, mlp=mlp) as lat:
        lat.init_equilibrium(rho, u)
        lat.step(100)
        got = lat.populations()
        ke = lat.global_sums()[4] / n ** 3
    want = step.run(collision.equilibrium(rho, u), _oracle_op("nco", tau), 100)
    err = np.abs(got - want).max()
    ke_ref = observables.kinetic_energy(want)
    print("storage %s, network %s: max |f - f_oracle| = %.3e, kinetic energy rel. err %.3e"
          % (storage, mlp, err, abs(ke - ke_ref) / ke_ref))
    assert err < PRECISION_BOUNDS[(storage, mlp)]


def _pulled(state, pts, n):
    C = np.array([(cx, cy, cz) for cz in (-1, 0, 1) for cy in (-1, 0, 1) for cx in (-1, 0, 1)])
    out = np.empty((27, len(pts)))
    for i, (cx, cy, cz) in enumerate(C):
        out[i] = state[i, (pts[:, 0] - cz) % n, (pts[:, 1] - cy) % n, (pts[:, 2] - cx) % n]
    return out


@pytest.mark.parametrize("kind", ["bgk", "mrt"])
def test_bench_256_datapath_sampled_against_oracle(kind):
    """The 256^3 stream-collide datapath in the benchmark's configuration
    (float32, Taylor-Green at Re 1600, fixed rates 4/3): one step checked
    node by node on 512 sampled nodes."""
    n = 256
    _, tau = inputs.viscosity(n, 0.1 / np.sqrt(3.0), 1600.0)
    rho, u = inputs.tgv3d(n, 0.1 / np.sqrt(3.0))
    with Lattice((n, n, n), "f32", kind, tau) as lat:
        if kind == "mrt":
            lat.set_rates([4.0 / 3.0] * 4)
        lat.init_equilibrium(rho, u)
        del rho, u
        lat.step(2)
        before = lat.populations()
        lat.step(1)
        after = lat.populations()
    pts = np.random.Generator(np.random.PCG64(13)).integers(0, n, size=(512, 3))
    pulled = _pulled(before, pts, n)
    del before
    op = step.Operator(kind, tau, omega_high=np.array([4.0 / 3.0] * 4))
    want = op.collide(pulled)
    got = after[:, pts[:, 0], pts[:, 1], pts[:, 2]]
    err = np.abs(got - want).max()
    print("256^3 %s, sampled: max err %.3e" % (kind, err))
    # float32 arithmetic: rho is a 27-term float32 sum (~3e-7 relative) and at
    # tau = 0.5044 the update is ~2 f^eq - f, which doubles f^eq's rounding
    # on the 0.3 rest population; the 128^3 NCO check uses the same bound.
    assert err < 1e-6


@pytest.mark.parametrize("n", [43, 128])
def test_bench_size_bf16_network_sampled_against_oracle(n):
    """128^3 NCO with the bf16 matrix-core network (the benchmark's
    nco_bf16net variant), and 43^3 (64-node blocks of four tiles, a ragged
    last block): one step on 256 sampled nodes, within the bf16 network's
    rounding (its rates carry ~1e-3 relative error)."""
    _, tau = inputs.viscosity(n, 0.1 / np.sqrt(3.0), 1600.0)
    rho, u = inputs.tgv3d(n, 0.1 / np.sqrt(3.0))
    with _lattice((n, n, n), "f32", "nco", tau, mlp="bf16") as lat:
        lat.init_equilibrium(rho, u)
        lat.step(3)
        before = lat.populations()
        lat.step(1)
        after = lat.populations()
    pts = np.random.Generator(np.random.PCG64(14)).integers(0, n, size=(256, 3))
    want = _oracle_op("nco", tau).collide(_pulled(before, pts, n))
    got = after[:, pts[:, 0], pts[:, 1], pts[:, 2]]
    err = np.abs(got - want).max()
    print("%d^3 bf16 network, sampled: max err %.3e" % (n, err))
    assert err < 1e-5
