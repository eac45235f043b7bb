"""Grouped multi-lattice steps (nco_batch_step) and the solve server on the GPU.

A lattice advanced inside a batch, next to lattices of other sizes, kinds and
step counts, must end bit-identical to the same lattice advanced alone with
nco_step: both run the same per-node code, and a grouped dispatch only maps
blocks to lattices.  The float32 NCO members are also checked against the
oracle.
"""
import numpy as np
import pytest

from oracle import collision, step
from paper_2412_08229_amd import Lattice, inputs
from paper_2412_08229_amd import _lib as L
from paper_2412_08229_amd.lattice import batch_step

pytestmark = pytest.mark.gpu

WIDTH = 32
OMEGA = np.array([1.15, 1.35, 1.55, 1.75])


@pytest.fixture(scope="module")
def stream():
    import torch
    return torch.cuda.Stream().cuda_stream


# (shape, storage, op, network arithmetic, activation, steps)
MIX = [
    ((16, 16, 16), "f32", "nco", "f32_mfma", "tanh", 7),
    ((5, 7, 9), "f32", "nco", "f32_mfma", "tanh", 4),
    ((3, 11, 13), "bf16", "nco", "bf16", "tanh", 6),
    ((8, 8, 8), "f16", "nco", "bf16", "relu", 5),
    ((9, 4, 6), "f32", "nco", "f32_mfma", "relu", 0),
    ((7, 5, 3), "f32", "bgk", None, None, 6),
    ((16, 3, 17), "f64", "bgk", None, None, 3),
    ((6, 6, 6), "f16", "mrt", None, None, 5),
    ((1, 1, 1), "bf16", "bgk", None, None, 2),
    ((4, 9, 2), "f32", "mrt", None, None, 7),
    ((6, 10, 7), "f32", "nco", "f32_split", "tanh", 5),
    ((12, 12, 12), "bf16", "nco", "f32_split", "tanh", 3),
    ((7, 9, 8), "f16", "nco", "f32_split", "relu", 4),
]


def _make(case, seed, stream):
    shape, storage, op, mlp, act, _ = case
    lat = Lattice(shape, storage, op, 0.56 + 0.01 * seed, stream=stream)
    if op == "nco":
        lat.set_net_weights(inputs.mlp_params(WIDTH, seed), WIDTH, act, mlp)
    if op == "mrt":
        lat.set_rates(OMEGA)
    lat.init_populations(inputs.random_populations(shape, seed=seed, lo=0.9, hi=1.1))
    return lat


def test_batch_equals_individual_steps(stream):
    alone = []
    for s, case in enumerate(MIX):
        with _make(case, s, stream) as lat:
            lat.step(case[-1])
            alone.append(lat.populations())
    lats = [_make(case, s, stream) for s, case in enumerate(MIX)]
    try:
        batch_step(lats, [c[-1] for c in MIX])
        for lat, ref, case in zip(lats, alone, MIX):
            assert np.array_equal(lat.populations(), ref), case
    finally:
        for lat in lats:
            lat.close()


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_reduced_cube_batch_equals_individual_steps(stream, storage):
    """Reduced Taylor-Green cubes (App. A, streaming folded at the faces)
    with the float32 matrix-core network: stepped alone, lattices up to 4096
    nodes run six-wavefront tiles whose threads share the tile's pulls; in a
    batch, 256-node blocks in which each thread pulls its own node.  The two
    must agree bit for bit (16^3, and 12^3 and 5^3 with a partial last
    tile)."""
    u0 = 0.1 / np.sqrt(3.0)

    def make(n, seed):
        lat = Lattice((n, n, n), storage, "nco", 0.56 + 0.01 * seed, stream=stream)
        lat.set_domain("tgv_octant")
        lat.set_net_weights(inputs.mlp_params(WIDTH, seed), WIDTH, "tanh", "f32_mfma")
        lat.init_equilibrium(*inputs.tgv3d_octant(n, u0))
        return lat

    sizes = [16, 12, 5]
    alone = []
    for s, n in enumerate(sizes):
        with make(n, s) as lat:
            lat.step(6)
            alone.append(lat.populations())
    lats = [make(n, s) for s, n in enumerate(sizes)]
    try:
        batch_step(lats, [6] * len(sizes))
        for lat, ref, n in zip(lats, alone, sizes):
            assert np.array_equal(lat.populations(), ref), n
    finally:
        for lat in lats:
            lat.close()


def test_batch_nco_matches_oracle(stream):
    case = MIX[1]
    shape, _, _, _, act, nsteps = case
    lats = [_make(c, s, stream) for s, c in enumerate(MIX[:3])]
    try:
        batch_step(lats, [c[-1] for c in MIX[:3]])
        got = lats[1].populations()
    finally:
        for lat in lats:
            lat.close()
    op = step.Operator("nco", 0.57, layers=collision.unpack_params(inputs.mlp_params(WIDTH, 1), WIDTH), act=act)
    ref = step.run(inputs.random_populations(shape, seed=1, lo=0.9, hi=1.1), op, nsteps)
    assert np.abs(got - ref).max() < 1e-5


def test_more_members_than_one_group(stream):
    # 37 BGK lattices of one kind: three grouped dispatches per step.
    shapes = [(1 + s % 5, 2 + s % 3, 3 + s % 7) for s in range(37)]
    steps = [s % 4 for s in range(37)]
    lats = [Lattice(sh, "f32", "bgk", 0.6, stream=stream) for sh in shapes]
    try:
        for s, lat in enumerate(lats):
            lat.init_populations(inputs.random_populations(lat.shape, seed=100 + s))
        batch_step(lats, steps)
        for s, lat in enumerate(lats):
            op = step.Operator("bgk", 0.6)
            ref = step.run(inputs.random_populations(lat.shape, seed=100 + s), op, steps[s])
            assert np.abs(lat.populations() - ref).max() < 2e-6, s
    finally:
        for lat in lats:
            lat.close()


def test_empty_batch_and_zero_steps(stream):
    batch_step([], [])
    with Lattice((4, 4, 4), "f32", "bgk", 0.6, stream=stream) as lat:
        f0 = inputs.random_populations(lat.shape, seed=3)
        lat.init_populations(f0)
        q = lat.populations()
        batch_step([lat], [0])
        assert np.array_equal(lat.populations(), q)


def test_batch_errors(stream):
    a = Lattice((4, 4, 4), "f32", "bgk", 0.6, stream=stream)
    b = Lattice((4, 4, 4), "f32", "bgk", 0.6)                  # its own stream
    c = Lattice((4, 4, 4), "f32", "nco", 0.6, stream=stream)
    d = Lattice((4, 4, 4), "f32", "stream", 0.6, stream=stream)
    try:
        with pytest.raises(L.NCOError) as e:
            batch_step([a, a], [1, 1])
        assert e.value.status == L.NCO_E_INVALID
        with pytest.raises(L.NCOError) as e:
            batch_step([a, b], [1, 1])
        assert e.value.status == L.NCO_E_INVALID
        with pytest.raises(L.NCOError) as e:
            batch_step([a], [-1])
        assert e.value.status == L.NCO_E_INVALID
        with pytest.raises(L.NCOError) as e:        # NCO without a network
            batch_step([c], [1])
        assert e.value.status == L.NCO_E_UNSUPPORTED
        c.set_net_weights(inputs.mlp_params(WIDTH, 0), WIDTH, "tanh", "f32")
        with pytest.raises(L.NCOError) as e:        # VALU network is not batched
            batch_step([c], [1])
        assert e.value.status == L.NCO_E_UNSUPPORTED
        with pytest.raises(L.NCOError) as e:
            batch_step([d], [1])
        assert e.value.status == L.NCO_E_UNSUPPORTED
    finally:
        for lat in (a, b, c, d):
            lat.close()


def test_forcing_inside_a_batch(stream):
    # The forcing clock of each member advances with its own steps.
    ks = inputs.forcing_half_modes(2.0)
    draws = inputs.uniform_draws(3, len(ks), seed=5)
    out = []
    for batched in (False, True):
        lats = [Lattice((8, 8, 8), "f32", "bgk", 0.6, stream=stream) for _ in range(2)]
        for lat in lats:
            lat.init_equilibrium(None, np.zeros((3, 8, 8, 8)))
            lat.set_forcing(ks, draws, 1e-3, 1.5, 0.25)
        if batched:
            batch_step(lats, [5, 2])
        else:
            lats[0].step(5)
            lats[1].step(2)
        out.append([lat.populations() for lat in lats])
        for lat in lats:
            lat.close()
    for x, y in zip(*out):
        assert np.array_equal(x, y)


def test_server_results_alone_and_in_mix(stream):
    """A request's result does not depend on what else the server runs."""
    from paper_2412_08229_amd import serve
    eng = serve.GpuEngine(stream=stream)
    mix = [serve.Request(rid=i, arrival=0.0, n=n, re=re, steps=st, flow=fl, cls=cl)
           for i, (n, re, st, fl, cl) in enumerate([(32, 800.0, 40, "tgv", "f32"), (16, 1600.0, 25, "turb", "bf16"),
                                                   (24, 400.0, 60, "turb", "f32"), (16, 3000.0, 10, "tgv", "bf16")])]
    srv = serve.Server(eng, budget_bytes=1 << 30, max_slots=3, chunk=7)
    rep = srv.run(mix)
    assert rep["status"] == {"done": 4}
    for r in mix:
        lone = serve.Request(rid=r.rid, arrival=0.0, n=r.n, re=r.re, steps=r.steps, flow=r.flow, cls=r.cls)
        serve.Server(eng, budget_bytes=1 << 30, max_slots=1, chunk=1000).run([lone])
        assert lone.result == r.result, r.rid
