"""ctypes binding of libnco.so (the C ABI in include/nco.h).

Argument marshalling only: every function here converts numpy arrays to
pointers, calls the C function of the same name and raises ``NCOError`` on
a non-zero status.  All computation happens in the HIP library; if the
library is missing, loading fails loudly.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnco.so")

NCO_OK, NCO_E_INVALID, NCO_E_OOM, NCO_E_HIP, NCO_E_UNSTABLE, NCO_E_STATE, NCO_E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
F32, F16_DEV, BF16_DEV, F64 = 0, 1, 2, 3
OP_BGK, OP_MRT, OP_NCO, OP_STREAM = 0, 1, 2, 3
MLP_F32, MLP_F32_MFMA, MLP_BF16, MLP_F32_SPLIT = 0, 1, 2, 3
ACT_TANH, ACT_RELU = 0, 1

STORAGE = {"f32": F32, "f16": F16_DEV, "bf16": BF16_DEV, "f64": F64}
OPS = {"bgk": OP_BGK, "mrt": OP_MRT, "nco": OP_NCO, "stream": OP_STREAM}
ACTS = {"tanh": ACT_TANH, "relu": ACT_RELU}
MLP_PREC = {"f32": MLP_F32, "f32_mfma": MLP_F32_MFMA, "bf16": MLP_BF16, "f32_split": MLP_F32_SPLIT}

# Every exported symbol with (restype, argtypes); the CPU tests check that
# the library exports exactly these names.
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_F = ctypes.POINTER(ctypes.c_float)
_I = ctypes.c_int
_SZ = ctypes.c_size_t
SIGNATURES = {
    "nco_version": (_I, []),
    "nco_last_error": (ctypes.c_char_p, []),
    "nco_lattice_bytes": (_I, [_I, _I, _I, _I, ctypes.POINTER(_SZ)]),
    "nco_lattice_create": (_I, [_I, _I, _I, _I, _I, ctypes.c_double, _P, ctypes.POINTER(_P)]),
    "nco_lattice_destroy": (_I, [_P]),
    "nco_set_op": (_I, [_P, _I, ctypes.c_double]),
    "nco_set_rates": (_I, [_P, _D]),
    "nco_set_domain": (_I, [_P, _I]),
    "nco_set_inplace": (_I, [_P, _I]),
    "nco_set_reverse_cache": (_I, [_P, ctypes.c_size_t]),
    "nco_set_stochastic_rounding": (_I, [_P, _I, ctypes.c_uint]),
    "nco_restrict": (_I, [_P, _P]),
    "nco_set_net_weights": (_I, [_P, _I, _I, _I, _F, _SZ]),
    "nco_set_net_weights_depth": (_I, [_P, _I, _I, _I, _I, _F, _SZ]),
    "nco_init_equilibrium": (_I, [_P, _D, _D]),
    "nco_init_populations": (_I, [_P, _D]),
    "nco_step": (_I, [_P, _I]),
    "nco_sync": (_I, [_P]),
    "nco_set_check": (_I, [_P, _I, ctypes.c_double]),
    "nco_read_populations": (_I, [_P, _D]),
    "nco_read_macroscopic": (_I, [_P, _D, _D]),
    "nco_read_rates": (_I, [_P, _D]),
    "nco_global_sums": (_I, [_P, _D]),
    "nco_energy_spectrum": (_I, [_P, _D, _I]),
    "nco_energy_spectrum_noalloc": (_I, [_P, _P, _I]),
    "nco_device_populations": (_I, [_P, ctypes.POINTER(_P), ctypes.POINTER(_SZ)]),
    "nco_set_forcing": (_I, [_P, _I, ctypes.POINTER(ctypes.c_int), _D, _I, ctypes.c_double, ctypes.c_double,
                             ctypes.c_double]),
    "nco_set_forcing_ex": (_I, [_P, _I, ctypes.POINTER(ctypes.c_int), _D, _I, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, _I]),
    "nco_forcing_amplitude": (_I, [ctypes.c_double] * 6 + [_D]),
    "nco_set_forcing_power": (_I, [_P, _I, ctypes.POINTER(ctypes.c_int), _D, _I] + [ctypes.c_double] * 5 + [_I]),
    "nco_forward_record": (_I, [_P, _I, _I]),
    "nco_forward_record_energy": (_I, [_P, _I, _I, _I, _D]),
    "nco_backward_energy": (_I, [_P, _D, _I, _D, _I, _D, _D, _SZ, _D]),
    "nco_batch_step": (_I, [ctypes.POINTER(_P), _I, ctypes.POINTER(ctypes.c_int)]),
    "nco_backward": (_I, [_P, _D, _I, _D, _D, _SZ, _D]),
}


class NCOError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("NCO status %d: %s" % (status, message))
        self.status = status


_lib = None


def lib():
    """Load libnco.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libnco.so not built: run __graft_entry__.build() "
                              "(or python paper_2412_08229_amd/build.py)")
        # PyTorch wheels carry their own HIP runtime under the same soname as
        # the system one libnco.so links.  Whichever loads first serves the
        # whole process, and torch does not work on a runtime other than its
        # own, so torch (when installed) is loaded first: the library and
        # torch then share one runtime, and torch streams are valid handles.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != NCO_OK:
        raise NCOError(status, lib().nco_last_error().decode(errors="replace"))
    return status


def dptr(a):
    return a.ctypes.data_as(_D)


def fptr(a):
    return a.ctypes.data_as(_F)


def as_f64(a, size=None):
    out = np.ascontiguousarray(a, dtype=np.float64)
    if size is not None and out.size != size:
        raise ValueError("expected %d values, got %d" % (size, out.size))
    return out


def nco_version():
    return lib().nco_version()


def nco_lattice_bytes(nx, ny, nz, storage):
    b = _SZ()
    check(lib().nco_lattice_bytes(nx, ny, nz, storage, ctypes.byref(b)))
    return b.value


def nco_lattice_create(nx, ny, nz, storage, op, tau, stream=None):
    h = _P()
    check(lib().nco_lattice_create(nx, ny, nz, storage, op, tau, stream, ctypes.byref(h)))
    return h


def nco_lattice_destroy(h):
    check(lib().nco_lattice_destroy(h))


def nco_set_op(h, op, tau):
    check(lib().nco_set_op(h, op, tau))


def nco_set_rates(h, omega_high):
    w = as_f64(omega_high, 4)
    check(lib().nco_set_rates(h, dptr(w)))


def nco_set_net_weights(h, width, act, mlp_prec, params, depth=2):
    p = np.ascontiguousarray(params, dtype=np.float32)
    if depth == 2:
        check(lib().nco_set_net_weights(h, width, act, mlp_prec, fptr(p), p.size))
    else:
        check(lib().nco_set_net_weights_depth(h, depth, width, act, mlp_prec, fptr(p), p.size))


def nco_init_equilibrium(h, n, rho, u):
    u = as_f64(u, 3 * n)
    if rho is None:
        check(lib().nco_init_equilibrium(h, None, dptr(u)))
    else:
        r = as_f64(rho, n)
        check(lib().nco_init_equilibrium(h, dptr(r), dptr(u)))


def nco_init_populations(h, n, f):
    f = as_f64(f, 27 * n)
    check(lib().nco_init_populations(h, dptr(f)))


def nco_step(h, nsteps):
    check(lib().nco_step(h, nsteps))


def nco_sync(h):
    check(lib().nco_sync(h))


def nco_restrict(fine, coarse):
    check(lib().nco_restrict(fine, coarse))


DOMAINS = {"periodic": 0, "tgv_octant": 1}


def nco_set_domain(h, domain):
    check(lib().nco_set_domain(h, DOMAINS[domain] if isinstance(domain, str) else int(domain)))


def nco_set_stochastic_rounding(h, enable, seed):
    check(lib().nco_set_stochastic_rounding(h, int(enable), int(seed) & 0xffffffff))


def nco_set_reverse_cache(h, nbytes):
    check(lib().nco_set_reverse_cache(h, int(nbytes)))


def nco_set_inplace(h, enable):
    check(lib().nco_set_inplace(h, int(enable)))


def nco_set_check(h, every, mass_rel_tol):
    check(lib().nco_set_check(h, int(every), float(mass_rel_tol)))


def nco_read_populations(h, n):
    out = np.empty(27 * n)
    check(lib().nco_read_populations(h, dptr(out)))
    return out


def nco_read_macroscopic(h, n):
    rho = np.empty(n)
    u = np.empty(3 * n)
    check(lib().nco_read_macroscopic(h, dptr(rho), dptr(u)))
    return rho, u


def nco_read_rates(h, n):
    out = np.empty(4 * n)
    check(lib().nco_read_rates(h, dptr(out)))
    return out


def nco_global_sums(h):
    out = np.empty(5)
    check(lib().nco_global_sums(h, dptr(out)))
    return out


def nco_energy_spectrum(h, nbins):
    out = np.empty(nbins)
    check(lib().nco_energy_spectrum(h, dptr(out), nbins))
    return out


def nco_energy_spectrum_noalloc(h, E_dev_ptr, nbins):
    """E(k) into nbins doubles of caller-owned device memory at E_dev_ptr
    (an integer address), asynchronously on the lattice's stream."""
    check(lib().nco_energy_spectrum_noalloc(h, ctypes.c_void_p(E_dev_ptr), nbins))


def nco_set_forcing(h, k, draws, amplitude, kf, c, phase_rule=False):
    if k is None or len(k) == 0:
        check(lib().nco_set_forcing(h, 0, None, None, 0, 0.0, 0.0, 1.0))
        return
    kk = np.ascontiguousarray(k, dtype=np.int32)
    d = np.ascontiguousarray(draws, dtype=np.float64)
    n_modes = kk.shape[0]
    if d.ndim != 3 or d.shape[1] != n_modes or d.shape[2] != 3:
        raise ValueError("draws must have shape (n_steps, n_modes, 3)")
    check(lib().nco_set_forcing_ex(h, n_modes, kk.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), dptr(d),
                                   d.shape[0], amplitude, kf, c, int(bool(phase_rule))))


def nco_forcing_amplitude(power, dt, ka, kb, kf, c):
    out = ctypes.c_double(0.0)
    check(lib().nco_forcing_amplitude(power, dt, ka, kb, kf, c, ctypes.byref(out)))
    return out.value


def nco_set_forcing_power(h, k, draws, power, ka, kb, kf, c, phase_rule=False):
    kk = np.ascontiguousarray(k, dtype=np.int32)
    d = np.ascontiguousarray(draws, dtype=np.float64)
    n_modes = kk.shape[0]
    if d.ndim != 3 or d.shape[1] != n_modes or d.shape[2] != 3:
        raise ValueError("draws must have shape (n_steps, n_modes, 3)")
    check(lib().nco_set_forcing_power(h, n_modes, kk.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), dptr(d),
                                      d.shape[0], power, ka, kb, kf, c, int(bool(phase_rule))))


def nco_batch_step(handles, nsteps):
    n = len(handles)
    arr = (_P * max(n, 1))(*[h.value if isinstance(h, _P) else h for h in handles])
    steps = (ctypes.c_int * max(n, 1))(*[int(s) for s in nsteps])
    check(lib().nco_batch_step(arr, n, steps))


def nco_forward_record(h, nsteps, ckpt_every):
    check(lib().nco_forward_record(h, nsteps, ckpt_every))


def nco_forward_record_energy(h, nsteps, ckpt_every, every):
    k = np.empty(nsteps // every + 1)
    check(lib().nco_forward_record_energy(h, nsteps, ckpt_every, every, dptr(k)))
    return k


def nco_backward_energy(h, n, n_params, dL_dk, every, dL_dE=None, dL_df=None, want_df0=False):
    grad = np.empty(n_params)
    k = as_f64(dL_dk)
    e = None if dL_dE is None else as_f64(dL_dE)
    df = None if dL_df is None else as_f64(dL_df, 27 * n)
    df0 = np.empty(27 * n) if want_df0 else None
    check(lib().nco_backward_energy(h, dptr(k), every, None if e is None else dptr(e), 0 if e is None else e.size,
                                    None if df is None else dptr(df), dptr(grad), n_params,
                                    None if df0 is None else dptr(df0)))
    return grad, df0


def nco_backward(h, n, n_params, dL_dE=None, dL_df=None, want_df0=False):
    grad = np.empty(n_params)
    e = None if dL_dE is None else as_f64(dL_dE)
    df = None if dL_df is None else as_f64(dL_df, 27 * n)
    df0 = np.empty(27 * n) if want_df0 else None
    check(lib().nco_backward(h, None if e is None else dptr(e), 0 if e is None else e.size,
                             None if df is None else dptr(df), dptr(grad), n_params,
                             None if df0 is None else dptr(df0)))
    return grad, df0


def nco_device_populations(h):
    p = _P()
    b = _SZ()
    check(lib().nco_device_populations(h, ctypes.byref(p), ctypes.byref(b)))
    return p.value, b.value
