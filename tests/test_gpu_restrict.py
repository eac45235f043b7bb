"""Fine-to-coarse restriction (nco_restrict, Sec. "Learning Task") on the
GPU against the oracle's restriction of the same stored fine state."""
import numpy as np
import pytest

from oracle import lattice, restrict
from paper_2412_08229_amd import Lattice, inputs
from paper_2412_08229_amd import _lib as L

pytestmark = pytest.mark.gpu

# Coarse storage -> bound on |coarse - oracle|: float64 arithmetic, then the
# storage's rounding.  float32 rounds the value (half an ulp, 6e-8 of it),
# the 16-bit forms round the deviation d = f - w (2^-11 of |d| for FP16,
# 2^-8 for BF16).  The factor r tau_c / tau_f amplifies the
# non-equilibrium part of these far-from-equilibrium states, so values and
# deviations reach ~1 at r = 4.
BOUNDS = {"f64": 1e-15, "f32": 1.2e-7, "f16": 2.0 ** -11 * 1.01, "bf16": 2.0 ** -8 * 1.01}


@pytest.mark.parametrize("fine_shape,r", [((16, 8, 12), 2), ((16, 16, 16), 4), ((6, 5, 7), 1), ((9, 6, 3), 3)])
@pytest.mark.parametrize("fine_storage,coarse_storage", [("f64", "f64"), ("f32", "f32"), ("f64", "f16"),
                                                         ("f32", "bf16"), ("bf16", "f32")])
def test_restriction_matches_oracle(fine_shape, r, fine_storage, coarse_storage):
    coarse_shape = tuple(s // r for s in fine_shape)
    tau_f = 0.53
    tau_c = 0.5 + (tau_f - 0.5) / r
    f0 = inputs.random_populations(fine_shape, seed=7, lo=0.8, hi=1.2)
    with Lattice(fine_shape, fine_storage, "bgk", tau_f) as fine, \
            Lattice(coarse_shape, coarse_storage, "bgk", tau_c) as coarse:
        fine.init_populations(f0)
        ff = fine.populations()
        coarse.restrict_from(fine)
        got = coarse.populations()
    want = restrict.restrict(ff, r, tau_c, tau_f)
    err = np.abs(got - want).max()
    print("restrict %s -> %s, r = %d: max err %.3e" % (fine_shape, coarse_shape, r, err))
    w = lattice.weights().reshape(27, 1, 1, 1)
    scale = {"f64": 1.0, "f32": np.abs(want).max()}.get(coarse_storage, np.abs(want - w).max())
    assert err < BOUNDS[coarse_storage] * scale


def test_restriction_arguments():
    with Lattice((8, 8, 8), "f32", "bgk", 0.6) as fine, Lattice((3, 4, 4), "f32", "bgk", 0.6) as odd, \
            Lattice((4, 4, 4), "f32", "bgk", 0.6) as coarse:
        with pytest.raises(L.NCOError) as e:
            odd.restrict_from(fine)
        assert e.value.status == L.NCO_E_INVALID
        with pytest.raises(L.NCOError) as e:
            L.nco_restrict(fine._h, fine._h)
        assert e.value.status == L.NCO_E_INVALID
        coarse.set_domain("tgv_octant")
        with pytest.raises(L.NCOError) as e:
            coarse.restrict_from(fine)
        assert e.value.status == L.NCO_E_UNSUPPORTED
