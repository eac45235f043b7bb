"""Stochastic rounding of 16-bit deviation storage (nco_set_stochastic_rounding),
through the C ABI.

* The storage rounds each deviation up with probability equal to the dropped
  fraction: averaged over many seeds, one step's stored values converge to
  the float32 values before rounding, while round-to-nearest-even keeps its
  error of a quarter of a bfloat16 step on average.
* The random bits are a counter-based hash of (seed, step, node, population):
  runs repeat bit for bit, another seed changes them, and batched steps store
  what single steps store.
* Only the 16-bit deviation storages accept it."""
import numpy as np
import pytest

from paper_2412_08229_amd import Lattice, inputs
from paper_2412_08229_amd.lattice import batch_step
from paper_2412_08229_amd import _lib as L

pytestmark = pytest.mark.gpu

SHAPE = (20, 18, 22)


def _start(storage):
    rho, u = inputs.random_velocity(SHAPE, seed=31, amp=0.05)
    with Lattice(SHAPE, storage, "bgk", 0.56) as lat:
        lat.init_equilibrium(rho, u)
        return lat.populations()            # exactly representable in that storage


def _one_step(f0, storage, sr=None):
    with Lattice(SHAPE, storage, "bgk", 0.56) as lat:
        if sr is not None:
            lat.set_stochastic_rounding(True, sr)
        lat.init_populations(f0)
        lat.step(1)
        return lat.populations()


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_stochastic_rounding_is_unbiased(storage):
    f0 = _start(storage)
    x = _one_step(f0, "f32")                   # the values before rounding (float32 arithmetic)
    y_rne = _one_step(f0, storage)
    K = 64
    acc = np.zeros_like(x)
    for seed in range(K):
        acc += _one_step(f0, storage, sr=seed)
    y_sr = acc / K
    e_rne = np.sqrt(np.mean((y_rne - x) ** 2))
    e_one = np.sqrt(np.mean((_one_step(f0, storage, sr=1000) - x) ** 2))
    e_avg = np.sqrt(np.mean((y_sr - x) ** 2))
    bias = abs(np.mean(y_sr - x))
    print("%s rms error: nearest-even %.3e, one stochastic step %.3e, mean of %d seeds %.3e, bias %.2e"
          % (storage, e_rne, e_one, K, e_avg, bias))
    # One stochastic rounding has rms error sqrt(2/3)/sqrt(2) ~ 1.4x that of
    # nearest-even (uniform fractions); the mean of K independent ones falls
    # as 1/sqrt(K): 8x below a single one for K = 64.
    assert 1.1 * e_rne < e_one < 2.0 * e_rne
    assert e_avg < 0.25 * e_one
    assert bias < 0.05 * e_rne


def test_stochastic_rounding_repeats_and_depends_on_the_seed():
    rho, u = inputs.random_velocity(SHAPE, seed=32, amp=0.05)

    def run(seed, nsteps=6):
        with Lattice(SHAPE, "bf16", "mrt", 0.56) as lat:
            lat.set_rates([1.3, 1.1, 1.2, 1.4])
            if seed is not None:
                lat.set_stochastic_rounding(True, seed)
            lat.init_equilibrium(rho, u)
            lat.step(nsteps)
            return lat.populations()
    a, b, c, d = run(5), run(5), run(6), run(None)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c) and not np.array_equal(a, d)


def test_stochastic_rounding_in_a_batch_equals_single_steps():
    """A BGK and an NCO (bf16 network) lattice with stochastic rounding,
    stepped together in grouped dispatches, store what they store alone."""
    import torch
    st = torch.cuda.Stream().cuda_stream
    cases = [(SHAPE, "bgk", 9, 7), ((12, 12, 12), "nco", 10, 4)]

    def make(shape, op, seed):
        lat = Lattice(shape, "bf16", op, 0.58, stream=st)
        if op == "nco":
            lat.set_net_weights(inputs.mlp_params(32, seed), 32, "tanh", "bf16")
        lat.set_stochastic_rounding(True, seed)
        rho, u = inputs.random_velocity(shape, seed=seed, amp=0.05)
        lat.init_equilibrium(rho, u)
        return lat
    want = []
    for shape, op, seed, nsteps in cases:
        with make(shape, op, seed) as lat:
            lat.step(nsteps)
            want.append(lat.populations())
    lats = [make(shape, op, seed) for shape, op, seed, _ in cases]
    batch_step(lats, [c[3] for c in cases])
    got = [lat.populations() for lat in lats]
    for lat in lats:
        lat.close()
    for g, w in zip(got, want):
        assert np.array_equal(g, w)


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_stochastic_rounding_needs_16_bit_storage(storage):
    with Lattice((4, 4, 4), storage, "bgk", 0.6) as lat:
        with pytest.raises(L.NCOError):
            lat.set_stochastic_rounding(True, 1)
        lat.set_stochastic_rounding(False, 1)      # switching it off is always accepted
    with Lattice((4, 4, 4), "bf16", "bgk", 0.6) as lat:
        with pytest.raises(L.NCOError):
            L.nco_set_stochastic_rounding(lat._h, 2, 0)
