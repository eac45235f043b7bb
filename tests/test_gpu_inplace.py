"""Pairs of BGK / fixed-rate steps in place on one buffer (nco_set_inplace)
against the two-buffer steps, through the C ABI: the populations must agree
bit for bit.  The sizes are those where the pairs run (one buffer fits the
256 MB last-level cache, two do not): 128^3 float32, a non-cubic float64
lattice, 16-bit deviation lattices (also with stochastic rounding).  Seven steps with a stability check
every three mix pairs and single steps (a pair never straddles a check)."""
import numpy as np
import pytest

from paper_2412_08229_amd import Lattice, inputs

pytestmark = pytest.mark.gpu


def _run(shape, storage, op, forced, inplace, nsteps=7):
    rho, u = inputs.random_velocity(shape, seed=21, amp=0.05)
    sr = storage.endswith("sr")              # with stochastic rounding
    with Lattice(shape, storage[:-2] if sr else storage, op, 0.56) as lat:
        lat.set_inplace(inplace)
        if sr:
            lat.set_stochastic_rounding(True, 3)
        if op == "mrt":
            lat.set_rates([1.3, 1.1, 1.2, 1.4])
        if forced:
            ks = inputs.forcing_half_modes(2.0)
            lat.set_forcing(ks, inputs.uniform_draws(nsteps, len(ks), 22), 2e-6, 1.5, 1.0)
        lat.set_check(3, 1e-3)
        lat.init_equilibrium(rho, u)
        lat.step(nsteps)
        lat.sync()
        return lat.populations(), lat.global_sums()


@pytest.mark.parametrize("shape,storage,op,forced", [
    ((128, 128, 128), "f32", "bgk", False),
    ((128, 128, 128), "f32", "mrt", True),
    ((94, 92, 90), "f64", "bgk", True),
    ((170, 160, 150), "bf16", "mrt", False),
    ((170, 160, 150), "bf16sr", "bgk", True),
    ((170, 160, 150), "f16sr", "mrt", False),
])
def test_inplace_pairs_equal_two_buffer_steps(shape, storage, op, forced):
    print("in-place pairs vs two buffers: %s %s %s forced=%s" % (shape, storage, op, forced), flush=True)
    f_pair, s_pair = _run(shape, storage, op, forced, True)
    f_ab, s_ab = _run(shape, storage, op, forced, False)
    assert np.array_equal(f_pair, f_ab)
    assert np.array_equal(s_pair, s_ab)


def test_inplace_switch_rejects_other_values():
    from paper_2412_08229_amd import _lib as L
    with Lattice((4, 4, 4), "f32", "bgk", 0.6) as lat:
        with pytest.raises(L.NCOError):
            L.nco_set_inplace(lat._h, 2)
