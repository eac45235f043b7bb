"""Failure detection and save/resume on the GPU.

* The stability check (nco_set_check): a NaN written into the populations,
  and a mass change forced from the host into device memory, are reported
  by nco_sync as NCO_E_UNSTABLE; an ordinary run within the tolerance is
  not.  The collision conserves mass (the zeroth moment relaxes with rate
  1, Sec. II.B), so drift comes only from rounding or a blow-up.
* Save and resume: populations read to the host and set again continue
  bit-identically to an uninterrupted run, in every storage format.
* Creation arguments outside the method's domain (tau <= 1/2, empty sizes)
  are rejected.
"""
import ctypes
import os

import numpy as np
import pytest

from paper_2412_08229_amd import Lattice, inputs
from paper_2412_08229_amd import _lib as L

pytestmark = pytest.mark.gpu


def _hip():
    import torch  # noqa: F401  (the HIP runtime torch loaded, which libnco.so shares)
    L.lib()
    hip = ctypes.CDLL("libamdhip64.so.7", mode=os.RTLD_NOLOAD | os.RTLD_GLOBAL)
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipMemcpy.restype = ctypes.c_int
    return hip


def test_nan_is_reported_by_the_check_and_by_the_sums():
    shape = (6, 5, 4)
    f = inputs.random_populations(shape, seed=3, lo=0.9, hi=1.1)
    f[7, 2, 3, 1] = np.nan
    with Lattice(shape, "f32", "bgk", 0.6) as lat:
        lat.init_populations(f)
        lat.step(2)
        lat.sync()                                   # no check configured: nothing reported here
        with pytest.raises(L.NCOError) as e:
            lat.global_sums()
        assert e.value.status == L.NCO_E_UNSTABLE
    with Lattice(shape, "f32", "bgk", 0.6) as lat:
        lat.init_populations(f)
        lat.set_check(1, 1e-6)
        lat.step(1)
        with pytest.raises(L.NCOError) as e:
            lat.sync()
        assert e.value.status == L.NCO_E_UNSTABLE
        # A new initialisation clears the failure.
        lat.init_populations(inputs.random_populations(shape, seed=4, lo=0.9, hi=1.1))
        lat.step(3)
        lat.sync()


@pytest.mark.parametrize("storage, kind, tol", [("f32", "bgk", 1e-6), ("f32", "nco", 1e-6), ("bf16", "nco", 1e-4)])
def test_ordinary_run_passes_the_check(storage, kind, tol):
    n = 16
    rho, u = inputs.tgv3d(n, 0.05)
    with Lattice((n, n, n), storage, kind, 0.55) as lat:
        if kind == "nco":
            lat.set_net_weights(inputs.mlp_params(32, 0), 32, "tanh", "bf16" if storage == "bf16" else "f32_mfma")
        lat.init_equilibrium(rho, u)
        lat.set_check(5, tol)
        lat.step(100)
        lat.sync()


def test_mass_drift_forced_from_the_host_is_reported():
    hip = _hip()
    shape = (8, 8, 8)
    with Lattice(shape, "f32", "bgk", 0.6) as lat:
        lat.init_populations(inputs.random_populations(shape, seed=5, lo=0.9, hi=1.1))
        lat.set_check(2, 1e-6)
        lat.step(1)
        lat.sync()
        ptr, nbytes = lat.device_populations()
        assert nbytes == 27 * 512 * 4
        # Add 0.01 to one population (the total mass is ~512): relative drift 2e-5.
        val = np.empty(1, np.float32)
        off = 4 * (13 * 512 + 100)
        assert hip.hipMemcpy(val.ctypes.data, ptr + off, 4, 2) == 0        # device to host
        val += np.float32(0.01)
        assert hip.hipMemcpy(ptr + off, val.ctypes.data, 4, 1) == 0        # host to device
        lat.step(1)                                                         # second step: check runs
        with pytest.raises(L.NCOError) as e:
            lat.sync()
        assert e.value.status == L.NCO_E_UNSTABLE
        assert "stability check" in L.lib().nco_last_error().decode()


def test_batch_reports_the_unstable_member_only():
    import torch
    stream = torch.cuda.Stream().cuda_stream
    shape = (5, 6, 7)
    good = inputs.random_populations(shape, seed=6, lo=0.9, hi=1.1)
    bad = good.copy()
    bad[0, 0, 0, 0] = np.inf
    lats = [Lattice(shape, "f32", "mrt", 0.6, stream=stream) for _ in range(3)]
    try:
        for lat, f in zip(lats, (good, bad, good)):
            lat.set_rates([1.2, 1.3, 1.4, 1.5])
            lat.init_populations(f)
            lat.set_check(3, 1e-6)
        from paper_2412_08229_amd.lattice import batch_step
        batch_step(lats, [6, 6, 6])
        lats[0].sync()
        with pytest.raises(L.NCOError) as e:
            lats[1].sync()
        assert e.value.status == L.NCO_E_UNSTABLE
        lats[2].sync()
    finally:
        for lat in lats:
            lat.close()


@pytest.mark.parametrize("storage, kind, mlp", [("f32", "nco", "f32_mfma"), ("f16", "nco", "bf16"),
                                                ("bf16", "mrt", None), ("f64", "bgk", None)])
def test_save_and_resume_is_bit_exact(storage, kind, mlp):
    shape = (9, 8, 12)
    rho, u = inputs.random_velocity(shape, seed=8)

    def make():
        lat = Lattice(shape, storage, kind, 0.57)
        if kind == "nco":
            lat.set_net_weights(inputs.mlp_params(32, 2), 32, "tanh", mlp)
        if kind == "mrt":
            lat.set_rates([1.1, 1.2, 1.3, 1.4])
        return lat

    with make() as a:
        a.init_equilibrium(rho, u)
        a.step(10)
        saved = a.populations()
        a.step(10)
        straight = a.populations()
    with make() as b:
        b.init_populations(saved)
        assert np.array_equal(b.populations(), saved)
        b.step(10)
        resumed = b.populations()
    assert np.array_equal(resumed, straight)


def test_creation_arguments_outside_the_domain():
    for shape, tau in [((4, 4, 4), 0.5), ((4, 4, 4), 0.4), ((0, 4, 4), 0.6)]:
        with pytest.raises(L.NCOError) as e:
            Lattice(shape, "f32", "bgk", tau)
        assert e.value.status == L.NCO_E_INVALID
    with Lattice((4, 4, 4), "f32", "bgk", 0.6) as lat:
        with pytest.raises(L.NCOError) as e:
            lat.set_check(-1, 1e-3)
        assert e.value.status == L.NCO_E_INVALID


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_footprint_matches_device_memory(storage):
    """nco_lattice_bytes (the serving admission figure) against the device
    memory a lattice takes once created and initialised with an equilibrium."""
    import torch
    n = 96
    rho, u = inputs.tgv3d(n, 0.05)
    with Lattice((4, 4, 4), storage, "bgk", 0.6) as warm:      # load the library's code first
        warm.init_equilibrium(None, np.zeros((3, 4, 4, 4)))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    lat = Lattice((n, n, n), storage, "bgk", 0.6)
    lat.init_equilibrium(rho, u)
    lat.sync()
    used = free0 - torch.cuda.mem_get_info()[0]
    want = Lattice.bytes((n, n, n), storage)
    lat.close()
    print("%s: reported %d bytes, device memory used %d" % (storage, want, used))
    assert abs(used - want) < 0.05 * want + (4 << 20)
