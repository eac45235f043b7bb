"""CPU checks of the C ABI: the library loads, exports every function that
include/nco.h declares, and rejects bad arguments before touching a GPU."""
import os
import re

import numpy as np
import pytest

from paper_2412_08229_amd import _lib as L
from paper_2412_08229_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "nco.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nco_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = L.lib()
    declared = _declared()
    assert len(declared) >= 18
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(L.SIGNATURES) == declared
    assert L.nco_version() >= 100


def test_lattice_bytes_host_only():
    b32 = L.nco_lattice_bytes(128, 128, 128, L.F32)
    b16 = L.nco_lattice_bytes(128, 128, 128, L.BF16_DEV)
    assert b32 >= 2 * 27 * 4 * 128 ** 3
    assert b16 >= 2 * 27 * 2 * 128 ** 3 and b16 < b32
    with pytest.raises(L.NCOError) as e:
        L.nco_lattice_bytes(0, 4, 4, L.F32)
    assert e.value.status == L.NCO_E_INVALID
    with pytest.raises(L.NCOError):
        L.nco_lattice_bytes(4, 4, 4, 17)


@pytest.mark.parametrize("tau", [0.5, 0.3, float("nan")])
def test_create_rejects_tau_at_or_below_half(tau):
    with pytest.raises(L.NCOError) as e:
        L.nco_lattice_create(4, 4, 4, L.F32, L.OP_BGK, tau)
    assert e.value.status == L.NCO_E_INVALID
    assert "tau" in str(e.value)


def test_create_rejects_bad_extent_storage_operator():
    for args in [(0, 4, 4, L.F32, L.OP_BGK), (4, 4, 4, 9, L.OP_BGK), (4, 4, 4, L.F32, 11)]:
        with pytest.raises(L.NCOError) as e:
            L.nco_lattice_create(*args, 0.6)
        assert e.value.status == L.NCO_E_INVALID


def test_parameter_count_of_the_abi():
    for w in (8, 16, 20, 32):
        assert inputs.n_params(w) == w * (27 + w + 4) + 2 * w + 4
    assert inputs.mlp_params(32, 0).dtype == np.float64


def test_forcing_amplitude_from_power_matches_the_oracle():
    """The host-side amplitude of the power input (the equation for A in
    Sec. "Training Data - Forced Isotropic Turbulence") against the oracle's,
    and its argument checks; no device is needed."""
    from oracle import forcing
    for args in [(0.1, 1.0, 0.5, 2.5, 1.5, 1.0), (2e-6, 0.5, 1.0, 2.0, 1.5, 0.3), (1e-3, 2.0, 3.0, 9.0, 4.0, 5.0),
                 (1e-5, 1.0, 0.5, 2.5, -1.0, 0.5), (3e-7, 1.0, 4.0, 6.0, 1.0, 2.0)]:
        got = L.nco_forcing_amplitude(*args)
        want = forcing.amplitude_from_power(*args)
        assert abs(got / want - 1.0) < 1e-12, (args, got, want)
    for bad in [(-1.0, 1.0, 0.5, 2.5, 1.5, 1.0), (1.0, 0.0, 0.5, 2.5, 1.5, 1.0), (1.0, 1.0, 2.5, 0.5, 1.5, 1.0),
                (1.0, 1.0, 0.5, 2.5, 1.5, 0.0), (1.0, 1.0, 0.5, float("inf"), 1.5, 1.0),
                (1.0, 1.0, 500.0, 501.0, 0.0, 1.0)]:
        with pytest.raises(L.NCOError) as e:
            L.nco_forcing_amplitude(*bad)
        assert e.value.status == L.NCO_E_INVALID
