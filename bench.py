"""Benchmark of the NCO stream-collide hot path on one MI355X.

Workload: Taylor-Green vortex on a periodic 128^3 D3Q27 lattice, float32
populations, Re = 1600, Ma = 0.1 (u0 = 0.1/sqrt(3)), NCO collision with a
27-32-32-4 tanh network (seeded N(0, 0.1) weights), forward only.  One
"step" is one lattice time step: one fused pull-stream + moments + network +
relax + back-transform launch over all 128^3 nodes.  BGK and fixed-rate
moment relaxation are timed on the same grid and reported beside it.

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, GB/s
FP32_PEAK_TFLOPS = 157.3         # MI355X float32 (vector and dense matrix)
T_START = time.perf_counter()
METRIC = "NCO stream-collide GLUPS & % HBM peak, FP32 vs low-precision; p99 solve latency"

# HBM bytes per launch at 128^3 from rocprofv3 FETCH_SIZE / WRITE_SIZE runs,
# scaled by a plain copy of known size (profiles/*_hbm_counters.md).  An entry
# is removed whenever its kernel changes, until the counters are taken again.
TRAFFIC_BYTES = {"nco": 337.0e6 + 226.5e6}


# Timed variants: name -> (operator, population storage, network arithmetic,
# activation).  "nco" is the headline (float32 storage and network).
VARIANTS = {
    "nco": ("nco", "f32", "f32_mfma", "tanh"),
    # Float32-class network products split over the f16 matrix cores.
    "nco_f32split": ("nco", "f32", "f32_split", "tanh"),
    "nco_bf16net": ("nco", "f32", "bf16", "tanh"),
    "nco_f16store_bf16net": ("nco", "f16", "bf16", "tanh"),
    "nco_bf16store_bf16net": ("nco", "bf16", "bf16", "tanh"),
    "nco_relu_bf16net": ("nco", "f32", "bf16", "relu"),
    "nco_valu": ("nco", "f32", "f32", "tanh"),
    "bgk": ("bgk", "f32", None, None),
    "bgk_f16store": ("bgk", "f16", None, None),
    "bgk_bf16store": ("bgk", "bf16", None, None),
    "mrt": ("mrt", "f32", None, None),
    "mrt_f16store": ("mrt", "f16", None, None),
    # The stream-collide datapath on a lattice that does not fit the 256 MB
    # last-level cache (3.6 GB of float32 populations).
    "bgk_256": ("bgk", "f32", None, None),
    "mrt_256": ("mrt", "f32", None, None),
}
GRID = {"bgk_256": 256, "mrt_256": 256}
# The paper's own network, 27-20-20-4 with ReLU (zero-padded to width 32 on
# the matrix cores).
VARIANTS["nco_w20_relu"] = ("nco", "f32", "f32_mfma", "relu")
VARIANTS["nco_w20_relu_bf16net"] = ("nco", "f32", "bf16", "relu")
VARIANTS["nco_w20_relu_f32split"] = ("nco", "f32", "f32_split", "relu")
NET_WIDTH = {"nco_w20_relu": 20, "nco_w20_relu_bf16net": 20, "nco_w20_relu_f32split": 20}
# The paper's network for the dissipation training, 27-20-20-20-4 ReLU (third
# hidden layer; on the matrix cores zero-padded to width 32).
VARIANTS["nco_d3_w20_relu"] = ("nco", "f32", "f32_mfma", "relu")
VARIANTS["nco_d3_w20_relu_valu"] = ("nco", "f32", "f32", "relu")
VARIANTS["nco_d3_w20_relu_f32split"] = ("nco", "f32", "f32_split", "relu")
VARIANTS["nco_d3_w20_relu_bf16net"] = ("nco", "f32", "bf16", "relu")
NET_DEPTH = {}
for _v in ("nco_d3_w20_relu", "nco_d3_w20_relu_valu", "nco_d3_w20_relu_f32split", "nco_d3_w20_relu_bf16net"):
    NET_WIDTH[_v], NET_DEPTH[_v] = 20, 3
# The same Taylor-Green vortex on the reduced cube of Appendix A: an n/4
# cube standing for the n box (the node grid is offset by half a spacing).
VARIANTS["nco_octant"] = ("nco", "f32", "f32_mfma", "tanh")
DOMAIN = {"nco_octant": "tgv_octant"}


def nco_flops_per_node(width):
    """Multiply-adds of the group-averaged network, counted as 2 flops each:
    48 x (27 W + W^2) for the two hidden layers of every group element plus
    4 W for the output layer applied once to the group mean."""
    return 2 * (48 * (27 * width + width * width) + 4 * width)


# Matrix-core flop the float32 network kernel executes per node: layer 1
# once per axis permutation over the parity classes (10 K-steps of
# 16x16x4, two 16-row tiles), turned into the 8 reflections by a
# Walsh-Hadamard transform; layer 2 per group element (2 x 2 x 4 K-steps);
# per 16-node tile, 2048 flop per 16x16x4 product.
def nco_executed_flops_per_node():
    per_tile = 6 * (2 * 10) * 2048 + 48 * (2 * 2 * 4) * 2048
    return per_tile // 16


def bytes_per_node(storage):
    return 2 * 27 * {"f32": 4, "f16": 2, "bf16": 2, "f64": 8}[storage]


def time_op(lat, steps, warmup, torch, stream):
    """Average time of one step (one kernel launch) from HIP events recorded
    on the stream the lattice launches on (a torch stream handed to the
    library), bracketed by device synchronisation."""
    lat.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    lat.step(steps)
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


def train_step(n, tau, rho, u, params, width, stream, T=40, K=10, cache_bytes=None):
    """One training step of the float32 matrix-core NCO on the benchmark
    lattice: a T-step recorded forward (checkpoints every K) and the reverse
    pass (segment recompute + matrix-core adjoint) for a population loss.
    cache_bytes: the reverse-mode budget for kept network values (library
    default if None)."""
    from paper_2412_08229_amd import Lattice
    w = np.random.Generator(np.random.PCG64(1)).standard_normal((27, n, n, n)) * 1e-3
    with Lattice((n, n, n), "f32", "nco", tau, stream=stream) as lat:
        lat.set_net_weights(params, width, "tanh", "f32_mfma")
        if cache_bytes is not None:
            lat.set_reverse_cache(cache_bytes)
        for rep in range(2):                    # the first pass allocates the checkpoints
            lat.init_equilibrium(rho, u)
            t0 = time.perf_counter()
            lat.forward_record(T, K)
            lat.sync()
            t1 = time.perf_counter()
            g, _ = lat.backward(dL_df=w)
            t2 = time.perf_counter()
        if not np.all(np.isfinite(g)):
            raise RuntimeError("non-finite gradient")
    fwd = (t1 - t0) / T * 1e3
    rev = (t2 - t1) / T * 1e3
    out = {"forward_ms_per_step": fwd, "reverse_ms_per_step": rev,
           "train_glups": n ** 3 / ((t2 - t0) / T) / 1e9, "steps": T, "checkpoint_every": K,
           "lattice": n, "network": "f32_mfma", "activation": "tanh"}
    if cache_bytes is not None:
        out["reverse_cache_bytes"] = cache_bytes
    return out


def cpu_baseline(n_sample=64, nsteps=6):
    """The float64 oracle timed on the host, on a bounded sample: the same
    workload at n_sample^3 for nsteps steps."""
    from oracle import collision, step
    from paper_2412_08229_amd import inputs
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threads = 1
    u0 = 0.1 / math.sqrt(3.0)
    _, tau = inputs.viscosity(n_sample, u0, 1600.0)
    rho, u = inputs.tgv3d(n_sample, u0)
    layers = collision.unpack_params(inputs.mlp_params(32, 0), 32)
    op = step.Operator("nco", tau, layers=layers, act="tanh")
    f = collision.equilibrium(rho, u)
    t0 = time.perf_counter()
    step.run(f, op, nsteps)
    dt = time.perf_counter() - t0
    glups = n_sample ** 3 * nsteps / dt / 1e9
    return {"value": glups, "unit": "GLUPS", "cores": int(threads), "kind": "oracle",
            "sample": "NCO 27-32-32-4 tanh, TGV %d^3, %d steps, float64 numpy, %.1f s"
                      % (n_sample, nsteps, dt)}


def precision_horizon(n, convective_times, every, f64_steps):
    """Reduced-precision forms over a long Taylor-Green run (Re 1600, Ma 0.1)
    against the float32 path: kinetic energy k(t) every ``every`` steps, the
    mean dissipation rate over each tenth of the run, the energy spectrum at
    the end, and wall time.  The float32 path itself is compared with the
    library's float64 path (float64 storage and arithmetic) over the first
    ``f64_steps`` steps.  Prints one JSON line."""
    import torch
    from paper_2412_08229_amd import Lattice, inputs

    u0 = 0.1 / math.sqrt(3.0)
    _, tau = inputs.viscosity(n, u0, 1600.0)
    rho, u = inputs.tgv3d(n, u0)
    t_c = n / (2 * math.pi) / u0                       # steps per convective time L / u0
    nsteps = int(round(convective_times * t_c / every)) * every
    stream = torch.cuda.Stream().cuda_stream
    params = inputs.mlp_params(32, seed=0)

    def run(storage, mlp, steps, samples):
        sr = storage.endswith("sr")           # 16-bit deviation storage, stochastic rounding
        with Lattice((n, n, n), storage[:-2] if sr else storage, "nco", tau, stream=stream) as lat:
            lat.set_net_weights(params, 32, "tanh", mlp)
            if sr:
                lat.set_stochastic_rounding(True, 0)
            lat.init_equilibrium(rho, u)
            ke = [lat.global_sums()[4] / lat.n]
            t0 = time.perf_counter()
            for i in range(steps // samples):
                lat.step(samples)
                ke.append(lat.global_sums()[4] / lat.n)
                if (i + 1) % 10 == 0:
                    print("# %s/%s: step %d" % (storage, mlp, (i + 1) * samples), file=sys.stderr, flush=True)
            wall = time.perf_counter() - t0
            print("# %s/%s: %d steps in %.1f s" % (storage, mlp, steps, wall), file=sys.stderr, flush=True)
            return np.array(ke), lat.energy_spectrum(), wall

    out = {"workload": "Taylor-Green vortex %d^3, Re 1600, Ma 0.1, NCO 27-32-32-4 tanh" % n,
           "steps": nsteps, "convective_times": nsteps / t_c, "sample_every": every}
    if f64_steps > 0:
        k64, e64, _ = run("f64", "f32", f64_steps, f64_steps // 4)
        k32, e32, _ = run("f32", "f32_mfma", f64_steps, f64_steps // 4)
        out["f32_vs_f64"] = {"steps": f64_steps, "kinetic_energy_err": float(np.max(np.abs(k32 - k64) / k64)),
                             "spectrum_err": float(np.abs(e32 - e64).sum() / e64.sum())}
    ref = run("f32", "f32_mfma", nsteps, every)
    out["f32/f32_mfma"] = {"wall_s": ref[2], "kinetic_energy_final": float(ref[0][-1] / ref[0][0])}
    seg = len(ref[0]) // 10
    for storage, mlp in [("f32", "bf16"), ("f16", "bf16"), ("bf16", "bf16"), ("f16sr", "bf16"), ("bf16sr", "bf16")]:
        ke, spec, wall = run(storage, mlp, nsteps, every)
        d = [(ke[i * seg] - ke[(i + 1) * seg]) for i in range(10)]
        d_r = [(ref[0][i * seg] - ref[0][(i + 1) * seg]) for i in range(10)]
        sh = np.arange(len(spec))
        sh = sh[(sh >= 1) & (sh <= n // 4) & (ref[1] >= 1e-6 * ref[1].max())]
        out["%s/%s" % (storage, mlp)] = {
            "kinetic_energy_err": float(np.max(np.abs(ke - ref[0]) / ref[0])),
            "dissipation_err_per_tenth": float(max(abs(a - b) / abs(b) for a, b in zip(d, d_r))),
            "spectrum_err": float(np.abs(spec - ref[1]).sum() / ref[1].sum()),
            "spectrum_max_shell_err": float(np.max(np.abs(spec[sh] - ref[1][sh]) / ref[1][sh])),
            "wall_s": wall, "speedup": ref[2] / wall}
    print(json.dumps(out), flush=True)


def convergence(sizes, u0=0.05, re=100.0):
    """The convergence study of Sec. "Convergence": the extruded 2-D
    Taylor-Green vortex from its equilibrium, one step, relative L2 errors of
    velocity and pressure against the analytic solution, at fixed Re and
    Ma, for BGK, the fixed-rate operator and the NCO (float32 matrix cores).
    Prints one JSON line."""
    import torch
    from paper_2412_08229_amd import Lattice, inputs

    stream = torch.cuda.Stream().cuda_stream
    params = inputs.mlp_params(32, seed=0)
    out = {"workload": "Taylor-Green vortex 2-D extruded along z, u0 %g, Re %g, one step from equilibrium" % (u0, re),
           "errors": {}}
    for kind in ("bgk", "mrt", "nco"):
        rows = {}
        for n in sizes:
            nu, tau = inputs.viscosity(n, u0, re)
            rho0, u_0, _ = inputs.tgv2d(n, u0)
            with Lattice((n, n, n), "f32", kind, tau, stream=stream) as lat:
                if kind == "nco":
                    lat.set_net_weights(params, 32, "tanh", "f32_mfma")
                if kind == "mrt":
                    lat.set_rates([4.0 / 3.0] * 4)
                lat.init_equilibrium(rho0, u_0)
                lat.step(1)
                rho, u = lat.macroscopic()
            k2 = (2.0 * math.pi / n) ** 2
            u_a = u_0 * math.exp(-2.0 * nu * k2)
            p_a = (rho0 - 1.0) / 3.0 * math.exp(-4.0 * nu * k2)
            eu = math.sqrt(((u - u_a) ** 2).sum() / (u_a ** 2).sum())
            ep = math.sqrt((((rho - 1.0) / 3.0 - p_a) ** 2).sum() / (p_a ** 2).sum())
            rows[n] = {"velocity_l2": eu, "pressure_l2": ep}
        ns = sorted(rows)
        for a, b in zip(ns, ns[1:]):
            rows[b]["velocity_order"] = math.log2(rows[a]["velocity_l2"] / rows[b]["velocity_l2"])
            rows[b]["pressure_order"] = math.log2(rows[a]["pressure_l2"] / rows[b]["pressure_l2"])
        out["errors"][kind] = {str(n): r for n, r in rows.items()}
        print("# convergence %s done" % kind, file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


def tgv_dissipation(sizes, ref_n, t_end=20.0, dt=0.1, re=1600.0):
    """The 3-D Taylor-Green vortex of Sec. "Three-dimensional Taylor-Green
    Vortex" at Re 1600, Ma 0.1: kinetic energy k(t) and dissipation rate
    -dk/dt (both in units of u0 and L = n / 2 pi) up to t_end convective
    times, for BGK, the fixed-rate operator and the NCO (seeded network,
    float32 matrix cores) at the coarse sizes, against a BGK run at ref_n.
    A run whose state stops being finite is reported with the time it did.
    Prints one JSON line."""
    import torch
    from paper_2412_08229_amd import Lattice, inputs
    from paper_2412_08229_amd import _lib as L

    u0 = 0.1 / math.sqrt(3.0)
    stream = torch.cuda.Stream().cuda_stream
    params = inputs.mlp_params(32, seed=0)

    def run(kind, n):
        nu, tau = inputs.viscosity(n, u0, re)
        t_c = n / (2.0 * math.pi) / u0                  # steps per convective time
        every = max(1, int(round(dt * t_c)))
        nsamp = int(round(t_end * t_c / every))
        rho, u = inputs.tgv3d(n, u0)
        ts, ks, status = [0.0], [], "stable"
        with Lattice((n, n, n), "f32", kind, tau, stream=stream) as lat:
            if kind == "nco":
                lat.set_net_weights(params, 32, "tanh", "f32_mfma")
            if kind == "mrt":
                lat.set_rates([4.0 / 3.0] * 4)
            lat.init_equilibrium(rho, u)
            del rho, u
            ks.append(lat.global_sums()[4] / lat.n / u0 ** 2)
            for i in range(nsamp):
                lat.step(every)
                try:
                    s = lat.global_sums()
                except L.NCOError:
                    status = "unstable at t = %.2f" % ((i + 1) * every / t_c)
                    break
                ts.append((i + 1) * every / t_c)
                ks.append(s[4] / lat.n / u0 ** 2)
                if (i + 1) % max(1, nsamp // 10) == 0:
                    print("# %s %d^3: t = %.1f" % (kind, n, ts[-1]), file=sys.stderr, flush=True)
        ts, ks = np.array(ts), np.array(ks)
        eps = -np.gradient(ks, ts) if len(ts) > 2 else np.zeros_like(ts)
        return ts, ks, eps, status

    t_r, k_r, e_r, st_r = run("bgk", ref_n)
    out = {"workload": "Taylor-Green vortex Re %g, Ma 0.1, t <= %g convective times" % (re, t_end),
           "reference": {"operator": "bgk", "lattice": ref_n, "status": st_r,
                         "peak_dissipation": float(e_r.max()), "t_peak": float(t_r[np.argmax(e_r)])},
           "runs": {}}
    for n in sizes:
        for kind in ("bgk", "mrt", "nco"):
            t, k, e, st = run(kind, n)
            e_ref = np.interp(t, t_r, e_r)
            k_ref = np.interp(t, t_r, k_r)
            out["runs"]["%s_%d" % (kind, n)] = {
                "status": st, "t_reached": float(t[-1]),
                "dissipation_err": float(np.max(np.abs(e - e_ref)) / e_r.max()),
                "kinetic_energy_err": float(np.max(np.abs(k - k_ref) / k_ref)),
                "peak_dissipation": float(e.max()), "t_peak": float(t[np.argmax(e)])}
    print(json.dumps(out), flush=True)


# The case table of Sec. "Training based on dissipation rates": cube sizes per
# Mach number, at every Reynolds number.
PAPER_TGV_GRID = {0.05: (16,), 0.1: (10, 16, 25), 0.15: (10, 16, 25, 32), 0.2: (10, 16, 25, 32)}


def tgv_training(cubes, res, mas, ref_cube, epochs, lr, t_end=15.0, samples=100, width=32, act="tanh", depth=2,
                 mlp="f32_mfma", grid=None):
    """Dissipation-rate training of Sec. "Training based on dissipation
    rates" on the reduced Taylor-Green cube of Appendix A: every (Re, Ma,
    cube) of the grid is one sample, its loss the mean squared gap of -dk/dt
    to a BGK run on the ref_cube cube at ``samples`` points over
    0 <= t <= t_end; one Adam step per epoch on the mean loss, the samples
    run concurrently on their own streams.  Reports the loss per sample
    before and after training, for the fixed-rate operator and BGK (or the
    time they became unstable), and the time per epoch.  The network is
    27-width-...-4 with ``depth`` hidden layers (depth 3 with width 20 and
    ReLU is the paper's network for this training; it runs on the vector
    units, mlp 'f32').  Prints one JSON line."""
    from paper_2412_08229_amd import inputs
    from paper_2412_08229_amd.training import DissipationUnroll, tgv_cube_energy, train_batched

    t0 = time.time()
    refs = {}
    for re in res:
        for ma in mas:
            u0 = ma / math.sqrt(3.0)
            t, k, st = tgv_cube_energy("bgk", ref_cube, re, u0, t_end, 3 * samples)
            refs[(re, ma)] = (t, -np.gradient(k, t), st)
            print("# reference Re %g Ma %g: %s, %.1f s" % (re, ma, st, time.time() - t0), file=sys.stderr, flush=True)
    p0 = inputs.mlp_params(width, seed=1, depth=depth)
    runs, keys = [], []
    for re in res:
        for ma in mas:
            u0 = ma / math.sqrt(3.0)
            tr, er, _ = refs[(re, ma)]
            for n in (grid[ma] if grid else cubes):
                _, tau = inputs.viscosity(4 * n, u0, re)
                tc = 4 * n / (2.0 * math.pi) / u0
                every = max(1, int(round(t_end * tc / samples)))
                nsteps = int(round(t_end * tc / every)) * every
                rho, u = inputs.tgv3d_octant(n, u0)
                runs.append(DissipationUnroll((n, n, n), tau, rho, u, u0, nsteps, 50, every,
                                              lambda t, tr=tr, er=er: float(np.interp(t, tr, er)), t_min=0.0,
                                              domain="tgv_octant", width=width, act=act, mlp=mlp, depth=depth))
                keys.append("Re%g_Ma%g_n%d" % (re, ma, n))
    L0 = [r.loss(p0) for r in runs]
    t1 = time.time()
    params, hist = train_batched(runs, p0, epochs, lr=lr,
                                 log=lambda m: print("# " + m, file=sys.stderr, flush=True))
    t_epoch = (time.time() - t1) / max(1, epochs)
    L1 = [r.loss(params) for r in runs]
    out = {"workload": "Taylor-Green dissipation training on the reduced cube, t <= %g, %d points" % (t_end, samples),
           "reference": {"operator": "bgk", "cube": ref_cube, "box": 4 * ref_cube,
                         "status": {"Re%g_Ma%g" % k: v[2] for k, v in refs.items()}},
           "network": {"width": width, "depth": depth, "activation": act, "arithmetic": mlp},
           "epochs": epochs, "lr": lr, "seconds_per_epoch": t_epoch,
           "history": [h if np.isfinite(h) else None for h in hist], "samples": {}}
    for key, run, l0, l1 in zip(keys, runs, L0, L1):
        other = {}
        for kind in ("mrt", "bgk"):
            n = run.lat.nx
            t, k, st = tgv_cube_energy(kind, n, None, run.u0, t_end, None, tau=run.lat.tau, every=run.every,
                                       nsamp=run.nsteps // run.every)
            if st != "stable":
                other[kind] = st
                continue
            eps = -(k[run.inner + 1] - k[run.inner - 1]) / (2.0 * run.dt)
            other[kind] = float(np.mean(((eps - run.eps_ref) / run.scale) ** 2))
        def fin(v):
            return v if isinstance(v, str) or np.isfinite(v) else "non-finite"
        out["samples"][key] = {"untrained": fin(l0), "trained": fin(l1), "fixed_rate": fin(other["mrt"]),
                               "bgk": fin(other["bgk"])}
        run.close()
    print(json.dumps(out), flush=True)


def spectrum_training(n_fine, n_coarse, n_snap, epochs, lr, tau_f=0.6, amp_f=1e-6, urms=0.05, spinup=20.0,
                      start=200, grow=200, every=10, kmin=4, kmax=10, omega=20.0):
    """The spectrum training of Sec. "Learning Task" at the paper's grid
    sizes.  A forced n_fine^3 BGK run stands in for the DNS: Alvelius
    forcing on |k| <= 2 with the velocity-dependent phase, from a seeded
    random-phase field of rms velocity ``urms``, tau_f = 0.6 (nu = 1/30),
    forcing amplitude amp_f (the kinetic energy is printed every large-eddy
    time of the spin-up, which must stay finite).  After
    ``spinup`` large-eddy times, n_snap snapshots half a large-eddy time
    apart are restricted by acoustic scaling to n_coarse^3 (tau_c = 1/2 +
    (tau_f - 1/2) / r); each is a sample whose coarse NCO run is forced by
    the same rule, amplitude x r: the phases are redrawn every step and the
    rule leaves no correlation with u, so a step injects |F|^2 / 2, in
    proportion to the amplitude, and one coarse step must inject what r fine
    steps do.  The loss is the paper's (squared
    spectrum gap over kmin <= k <= kmax plus omega E(N/2)) against the fine
    run's spectrum averaged over the snapshots.  Adam over the samples with
    the unroll curriculum (start steps, grow more every ``every`` epochs).
    Reports the loss per sample at the final unroll length for the untrained
    and trained network, the fixed-rate operator and BGK, and the times.
    Prints one JSON line."""
    from paper_2412_08229_amd import Lattice, inputs
    from paper_2412_08229_amd._lib import NCOError
    from paper_2412_08229_amd.training import (Unroll, curriculum_steps, n_bins, paper_spectrum_loss,
                                               train_batched)

    r = n_fine // n_coarse
    if r * n_coarse != n_fine:
        raise ValueError("the fine extent must be a multiple of the coarse one")
    tau_c = 0.5 + (tau_f - 0.5) / r
    amp_c = amp_f * r
    ks = inputs.forcing_half_modes(2.0)
    t_large = int(round(n_fine / (2.0 * math.pi * 1.5) / urms))     # large-eddy time in fine steps
    t0 = time.time()
    rho, u = inputs.turbulence(n_fine, seed=101, k0=4.0, urms=urms)
    snaps, spectra = [], []
    with Lattice((n_fine,) * 3, "f32", "bgk", tau_f) as fine:
        fine.set_forcing(ks, inputs.uniform_draws(4096, len(ks), 102), amp_f, 1.5, 1.0, phase_rule=True)
        fine.init_equilibrium(rho, u)
        del rho, u
        for i in range(int(math.ceil(spinup))):
            fine.step(t_large)
            k = fine.global_sums()[4] / fine.n
            print("# fine spin-up: %d large-eddy times, mean kinetic energy %.4e (u_rms %.4f)"
                  % (i + 1, k, math.sqrt(2.0 * k / 3.0)), file=sys.stderr, flush=True)
        t_spin = time.time() - t0
        print("# fine %d^3 spun up over %d steps in %.1f s" % (n_fine, int(math.ceil(spinup)) * t_large, t_spin),
              file=sys.stderr, flush=True)
        with Lattice((n_coarse,) * 3, "f32", "bgk", tau_c) as coarse:
            for i in range(n_snap):
                fine.step(t_large // 2)
                spectra.append(fine.energy_spectrum()[:n_bins(n_coarse)])
                coarse.restrict_from(fine)
                snaps.append(coarse.populations())
        kin = fine.global_sums()[4] / fine.n
    t_data = time.time() - t0
    target = np.mean(spectra, axis=0)

    def sched(ep):
        return curriculum_steps(ep, start=start, grow=grow, every=every)
    final = sched(epochs - 1)
    forcing = (ks, inputs.uniform_draws(4096, len(ks), 103), amp_c, 1.5, 1.0, True)
    runs = [Unroll((n_coarse,) * 3, tau_c, ("pop", f0), final, 20, target, kmin, kmax, forcing=forcing,
                   loss="paper", omega=omega) for f0 in snaps]
    p0 = inputs.mlp_params(32, seed=1)

    spec = {"untrained": [], "trained": [], "fixed_rate": [], "bgk": []}

    def safe_loss(run, params, key):
        try:
            v = run.loss(params)
        except NCOError:
            return "unstable"
        if not np.isfinite(v):
            return "non-finite"
        spec[key].append(run.lat.energy_spectrum())
        return v
    L0 = [safe_loss(run, p0, "untrained") for run in runs]
    t1 = time.time()
    params, hist = train_batched(runs, p0, epochs, lr=lr, schedule=sched,
                                 log=lambda m: print("# " + m, file=sys.stderr, flush=True))
    t_epoch = (time.time() - t1) / max(1, epochs)
    for run in runs:
        run.nsteps = final
    L1 = [safe_loss(run, params, "trained") for run in runs]
    out = {"workload": "forced isotropic turbulence spectrum training, %d^3 BGK -> %d^3 NCO" % (n_fine, n_coarse),
           "fine": {"n": n_fine, "tau": tau_f, "forcing_amplitude": amp_f, "large_eddy_steps": t_large,
                    "spinup_large_eddy_times": spinup, "mean_kinetic_energy": float(kin),
                    "seconds": t_data},
           "coarse": {"n": n_coarse, "ratio": r, "tau": tau_c, "forcing_amplitude": amp_c},
           "loss": {"kmin": kmin, "kmax": kmax, "omega": omega, "target": "fine spectrum averaged over the snapshots"},
           "curriculum": {"start": start, "grow": grow, "every": every, "final": final},
           "epochs": epochs, "lr": lr, "seconds_per_epoch": t_epoch,
           "history": [h if np.isfinite(h) else None for h in hist], "samples": {}}
    for i, (run, f0, l0, l1) in enumerate(zip(runs, snaps, L0, L1)):
        other = {}
        for kind in ("mrt", "bgk"):
            with Lattice((n_coarse,) * 3, "f32", kind, tau_c) as lat:
                if kind == "mrt":
                    lat.set_rates([4.0 / 3.0] * 4)
                lat.set_forcing(*forcing)
                lat.init_populations(f0)
                try:
                    lat.step(final)
                    E = lat.energy_spectrum()
                    v = paper_spectrum_loss(E, target, kmin, kmax, omega, n_coarse // 2)[0]
                    other[kind] = v if np.isfinite(v) else "non-finite"
                    if np.isfinite(v):
                        spec["fixed_rate" if kind == "mrt" else kind].append(E)
                except NCOError:
                    other[kind] = "unstable"
        out["samples"]["snapshot%d" % i] = {"untrained": l0, "trained": l1, "fixed_rate": other["mrt"],
                                            "bgk": other["bgk"]}
        run.close()
    # Energy spectra at the final unroll length, averaged over the snapshots
    # each operator kept finite, next to the target (k = 0 .. N/2).
    out["spectra"] = {"k": list(range(n_coarse // 2 + 1)), "target": [float(x) for x in target[:n_coarse // 2 + 1]]}
    for key, es in spec.items():
        out["spectra"][key] = [float(x) for x in np.mean(es, axis=0)[:n_coarse // 2 + 1]] if es else None
    print(json.dumps(out), flush=True)


def serving_leg(n_requests, load, seed=0, chunk=50, slots=16, stream=None):
    """The serving form on the request mix of the serving workload (grids
    {32, 64, 96, 128, 192}^3, Re uniform in [400, 3000], 500-2000 steps,
    Taylor-Green or decaying turbulence, FP32 or BF16 class, 50/50 each):
    Poisson arrivals at the given fraction of the measured capacity, served
    by the continuous-batching server with the free device memory as budget.
    Returns the server's report (p50/p99 latency per class, aggregate GLUPS,
    wall time) with the capacity and offered load."""
    import torch
    from paper_2412_08229_amd import serve
    engine = serve.GpuEngine(stream=stream)
    cap = serve.capacity_glups(engine, chunk=chunk)
    mean_work = float(np.mean([g ** 3 for g in serve.GRIDS])) * 1250.0
    rate = load * cap * 1e9 / mean_work
    reqs = serve.poisson_requests(n_requests, rate, seed)
    budget = int(0.9 * torch.cuda.mem_get_info()[0])
    srv = serve.Server(engine, budget, max_slots=slots, chunk=chunk, prep_workers=2)
    t0 = time.perf_counter()
    rep = srv.run(reqs, log=lambda m: print("# serving: " + m, file=sys.stderr, flush=True))
    rep.update({"offered_load": load, "capacity_glups": cap, "arrival_rate_per_s": rate,
                "mean_request_node_steps": mean_work, "leg_wall_s": time.perf_counter() - t0,
                "mix": "grids %s^3, Re 400-3000, 500-2000 steps, TGV/turbulence, FP32/BF16 class" %
                       (list(serve.GRIDS),)})
    return rep


def precision_leg(n, nsteps, tstream, torch):
    """The precision form at its size: the Taylor-Green vortex at n^3 (Re
    1600, Ma 0.1) for nsteps steps with the float32 path (float32 storage and
    network) and with FP16- and BF16-deviation storage under the bf16
    network; energy spectra (float64 on the device) compared with the
    float32 run's: energy-weighted error sum |E - E_f32| / sum E_f32 and the
    largest relative error of one shell among the shells holding at least
    1e-6 of the peak shell's energy; kinetic-energy error; ms per step.
    The 16-bit deviation storages run with round-to-nearest-even (f16_dev,
    bf16_dev) and with stochastic rounding (f16_dev_sr, bf16_dev_sr)."""
    from paper_2412_08229_amd import Lattice, inputs
    u0 = 0.1 / math.sqrt(3.0)
    _, tau = inputs.viscosity(n, u0, 1600.0)
    rho, u = inputs.tgv3d(n, u0)
    params = inputs.mlp_params(32, seed=0)
    runs = {}
    for name, storage, mlp in [("f32", "f32", "f32_mfma"), ("f16_dev", "f16", "bf16"), ("bf16_dev", "bf16", "bf16"),
                               ("f16_dev_sr", "f16", "bf16"), ("bf16_dev_sr", "bf16", "bf16")]:
        with Lattice((n, n, n), storage, "nco", tau, stream=tstream.cuda_stream) as lat:
            lat.set_net_weights(params, 32, "tanh", mlp)
            if name.endswith("_sr"):
                lat.set_stochastic_rounding(True, 0)
            lat.init_equilibrium(rho, u)
            ms = time_op(lat, nsteps, 0, torch, tstream)
            runs[name] = (ms, lat.energy_spectrum(), lat.global_sums()[4])
    ms0, e0, k0 = runs["f32"]
    sh = np.arange(len(e0))
    sh = sh[(sh >= 1) & (e0 >= 1e-6 * e0.max())]
    out = {"lattice": n, "steps": nsteps, "reference": "float32 storage + float32 network",
           "shells": "1 <= k with E_f32(k) >= 1e-6 max E_f32", "f32_ms_per_step": ms0}
    for name in ("f16_dev", "bf16_dev", "f16_dev_sr", "bf16_dev_sr"):
        ms, e, k = runs[name]
        out[name] = {"ms_per_step": ms, "speedup": ms0 / ms,
                     "spectrum_err": float(np.abs(e - e0).sum() / e0.sum()),
                     "spectrum_max_shell_err": float(np.max(np.abs(e[sh] - e0[sh]) / e0[sh])),
                     "kinetic_energy_err": float(abs(k - k0) / k0)}
        print("# precision %d^3 x %d: %s %.3f ms/step (f32 %.3f), spectrum err %.2e, worst shell %.2e"
              % (n, nsteps, name, ms, ms0, out[name]["spectrum_err"], out[name]["spectrum_max_shell_err"]),
              file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--tgv-dissipation", default="",
                    help="instead of the benchmark: coarse sizes and the reference size last, e.g. 32,64,128,512")
    ap.add_argument("--convergence", default="", help="instead of the benchmark: the TGV2D convergence study "
                                                      "at these comma-separated sizes")
    ap.add_argument("--precision-horizon", type=float, default=0.0,
                    help="instead of the benchmark: the reduced-precision study over this many convective times")
    ap.add_argument("--f64-steps", type=int, default=20)
    ap.add_argument("--tgv-training", default="",
                    help="instead of the benchmark: dissipation training on reduced cubes of these sizes")
    ap.add_argument("--re", default="400,800,1600")
    ap.add_argument("--ma", default="0.1")
    ap.add_argument("--ref-cube", type=int, default=128)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=1e-2)
    ap.add_argument("--net", default="32,2,tanh,f32_mfma", help="width,depth,activation,arithmetic of --tgv-training")
    ap.add_argument("--paper-grid", action="store_true",
                    help="--tgv-training over the paper's case table (cube sizes per Mach number, every Re)")
    ap.add_argument("--spectrum-training", default="",
                    help="instead of the benchmark: FINE,COARSE[,TAU_FINE[,AMPLITUDE[,SPINUP]]] (e.g. 256,32,0.6; "
                         "SPINUP in large-eddy times, default 20), the "
                         "forced-turbulence spectrum training at those grid sizes; with --snapshots, --epochs, "
                         "--lr, --curriculum")
    ap.add_argument("--snapshots", type=int, default=8)
    ap.add_argument("--curriculum", default="200,200,10",
                    help="START,GROW,EVERY of the --spectrum-training unroll curriculum (coarse steps)")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ops", default=",".join(list(VARIANTS) + ["nco_train", "nco_train_stored"]))
    ap.add_argument("--reverse-cache", type=int, default=None,
                    help="bytes of kept network values for nco_train's reverse mode (library default if unset; "
                         "0: every adjoint runs the network forward)")
    ap.add_argument("--serving-requests", type=int, default=16,
                    help="requests of the serving leg (0: no serving leg)")
    ap.add_argument("--serving-load", type=float, default=0.8)
    ap.add_argument("--precision-steps", type=int, default=500,
                    help="steps of the 256^3 precision leg (0: no precision leg)")
    ap.add_argument("--precision-n", type=int, default=256)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the lattice path runs on a single MI355X; "
              "multi-GPU domain decomposition is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.tgv_dissipation:
        sizes = [int(x) for x in args.tgv_dissipation.split(",")]
        tgv_dissipation(sizes[:-1], sizes[-1])
        return
    if args.convergence:
        convergence([int(x) for x in args.convergence.split(",")])
        return
    if args.tgv_training:
        w, d, a, m = args.net.split(",")
        mas = sorted(PAPER_TGV_GRID) if args.paper_grid else [float(x) for x in args.ma.split(",")]
        tgv_training([int(x) for x in args.tgv_training.split(",")], [float(x) for x in args.re.split(",")],
                     mas, args.ref_cube, args.epochs, args.lr, width=int(w), depth=int(d), act=a, mlp=m,
                     grid=PAPER_TGV_GRID if args.paper_grid else None)
        return
    if args.spectrum_training:
        f = args.spectrum_training.split(",")
        start, grow, every = (int(x) for x in args.curriculum.split(","))
        extra = {}
        if len(f) > 2:
            extra["tau_f"] = float(f[2])
        if len(f) > 3:
            extra["amp_f"] = float(f[3])
        if len(f) > 4:
            extra["spinup"] = float(f[4])
        spectrum_training(int(f[0]), int(f[1]), args.snapshots, args.epochs, args.lr, start=start, grow=grow,
                          every=every, **extra)
        return
    if args.precision_horizon > 0:
        precision_horizon(args.n, args.precision_horizon, 100, args.f64_steps)
        return

    import torch
    from paper_2412_08229_amd import Lattice, inputs

    n = args.n
    u0 = 0.1 / math.sqrt(3.0)
    _, tau = inputs.viscosity(n, u0, 1600.0)
    rho, u = inputs.tgv3d(n, u0)
    tstream = torch.cuda.Stream()          # default priority
    stream = tstream.cuda_stream
    if not stream:
        raise RuntimeError("expected a non-null HIP stream handle")
    width = 32
    params = inputs.mlp_params(width, seed=0)
    nodes = n ** 3
    results = {}
    spectra = {}
    fields = {n: (tau, rho, u)}
    for op in args.ops.split(","):
        if op in ("nco_train", "nco_train_stored"):
            # nco_train_stored: every state a checkpoint (no recompute) and
            # every step's network values kept (40 x 0.3 GB at 128^3 beside
            # the 40 x 0.23 GB of states), the memory-rich form.
            kw = {"cache_bytes": args.reverse_cache} if op == "nco_train" else {"K": 1, "cache_bytes": 16 << 30}
            results[op] = train_step(n, tau, rho, u, params, width, stream, **kw)
            print("# %s: forward %.4f ms/step, reverse %.4f ms/step" % (
                op, results[op]["forward_ms_per_step"], results[op]["reverse_ms_per_step"]), file=sys.stderr,
                flush=True)
            continue
        kind, storage, mlp, act = VARIANTS[op]
        domain = DOMAIN.get(op, "periodic")
        if domain == "tgv_octant":
            n_op = n // 4
            tau_op, (rho_op, u_op) = tau, inputs.tgv3d_octant(n_op, u0)
        else:
            n_op = GRID.get(op, n)
            if n_op not in fields:
                fields[n_op] = (inputs.viscosity(n_op, u0, 1600.0)[1],) + inputs.tgv3d(n_op, u0)
            tau_op, rho_op, u_op = fields[n_op]
        lat = Lattice((n_op, n_op, n_op), storage, kind, tau_op, stream=stream)
        lat.set_domain(domain)
        if kind == "nco":
            w_op, d_op = NET_WIDTH.get(op, width), NET_DEPTH.get(op, 2)
            p_op = params if (w_op, d_op) == (width, 2) else inputs.mlp_params(w_op, seed=0, depth=d_op)
            lat.set_net_weights(p_op, w_op, act, mlp, depth=d_op)
        if kind == "mrt":
            lat.set_rates([4.0 / 3.0] * 4)
        lat.init_equilibrium(rho_op, u_op)
        # The per-node vector-unit network is kept as a reference variant; it
        # is two orders slower, so it is timed on fewer steps.
        slow = kind == "nco" and mlp == "f32"
        steps = min(args.steps, 10) if slow else args.steps
        ms = time_op(lat, steps, min(args.warmup, 2) if slow else args.warmup, torch, tstream)
        s = lat.global_sums()
        if not np.all(np.isfinite(s)):
            raise RuntimeError("non-finite state after the %s run" % op)
        if n_op == n and domain == "periodic":
            spectra[op] = (steps, lat.energy_spectrum(), s[4])
        lat.close()
        glups = n_op ** 3 / (ms * 1e-3) / 1e9
        gbs = bytes_per_node(storage) * n_op ** 3 / (ms * 1e-3) / 1e9
        results[op] = {"ms_per_step": ms, "glups": glups, "hbm_gbs": gbs, "lattice": n_op,
                       "hbm_frac": gbs / HBM_PEAK_GBS, "steps": steps, "storage": storage,
                       "network": mlp if kind == "nco" else None,
                       "width": NET_WIDTH.get(op, width) if kind == "nco" else None,
                       "depth": NET_DEPTH.get(op, 2) if kind == "nco" else None,
                       "activation": act if kind == "nco" else None}
        if domain == "tgv_octant":
            results[op]["domain"] = domain
            results[op]["box"] = 4 * n_op
            results[op]["box_equivalent_glups"] = (4 * n_op) ** 3 / (ms * 1e-3) / 1e9
        print("# %s: %.4f ms/step, %.3f GLUPS, %.0f GB/s" % (op, ms, glups, gbs), file=sys.stderr,
              flush=True)

    # Reduced-precision forms against the float32 run of the same operator
    # after the same number of steps: energy-weighted spectrum error
    # sum_k |E - E_f32| / sum_k E_f32, the largest relative error of one shell
    # over 1 <= k <= n/4, the kinetic-energy error and the speedup.
    for op, r in results.items():
        if op not in VARIANTS:
            continue
        ref = VARIANTS[op][0]
        if (op == ref or ref not in spectra or op not in spectra or spectra[ref][0] != spectra[op][0]
                or VARIANTS[op][3] != VARIANTS[ref][3]):
            continue
        _, e_ref, k_ref = spectra[ref]
        _, e, k = spectra[op]
        # Shells 1..n/4 that hold energy (symmetry leaves some of the
        # Taylor-Green shells empty).
        sh = np.arange(len(e_ref))
        sh = sh[(sh >= 1) & (sh <= n // 4) & (e_ref > 1e-10 * e_ref.max())]
        r["vs_f32"] = {"spectrum_err": float(np.abs(e - e_ref).sum() / e_ref.sum()),
                       "spectrum_max_shell_err": float(np.max(np.abs(e[sh] - e_ref[sh]) / e_ref[sh])),
                       "kinetic_energy_err": float(abs(k - k_ref) / k_ref),
                       "speedup": r["glups"] / results[ref]["glups"]}

    # Attainable HBM bandwidth on this device: a plain device-to-device copy of
    # the bytes one float32 step moves (27 reads + 27 writes per node).
    nbytes = bytes_per_node("f32") * nodes // 2
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    with torch.cuda.stream(tstream):
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(tstream)
        for _ in range(20):
            dst.copy_(src)
        t1.record(tstream)
        torch.cuda.synchronize()
    copy_gbs = 2 * nbytes / (t0.elapsed_time(t1) / 20 * 1e-3) / 1e9
    del src, dst

    # The headline variant, else the first timed one (an --ops list of
    # training legs only has no roofline and no value).
    timed = [k for k in results if "ms_per_step" in results[k]]
    main_op = "nco" if "nco" in results else (timed[0] if timed else None)
    r = results[main_op] if main_op else {"glups": None, "ms_per_step": None}
    if main_op is None:
        roof = None
    elif main_op == "nco":
        flops = nco_flops_per_node(width) * nodes
        achieved = flops / (r["ms_per_step"] * 1e-3) / 1e12
        executed = nco_executed_flops_per_node() * nodes / (r["ms_per_step"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_PEAK_TFLOPS, "traffic": TRAFFIC_BYTES.get("nco"),
                "kernel": "k_nco_mfma<f32 storage, tanh, float32 matrix cores>",
                "algorithmic_per_node": "%d flop (network) + %d B" % (nco_flops_per_node(width),
                                                                     bytes_per_node("f32")),
                # What the matrix cores execute: the Walsh-Hadamard fold of
                # layer 1 over the reflections removes 37 % of the network's
                # flop, so this rate, not `achieved`, is the matrix-core
                # utilisation.
                "executed_flop_per_node": nco_executed_flops_per_node(),
                "executed_achieved": executed, "executed_frac": executed / FP32_PEAK_TFLOPS}
    else:
        roof = {"bound": "hbm", "achieved": r["hbm_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": r["hbm_frac"], "traffic": TRAFFIC_BYTES.get(main_op)}
    out = {
        "metric": METRIC,
        "value": r["glups"],
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "Taylor-Green vortex %d^3 D3Q27, Re 1600, Ma 0.1, %s collision, "
                               "27-32-32-4 tanh network, float32 storage, forward only" % (n, (main_op or "nco").upper()),
                   "lattice": [n, n, n], "operator": main_op, "storage": "f32", "width": width},
        "roofline": roof,
        "operators": results,
        "copy_gbs": copy_gbs,
    }
    if args.precision_steps > 0:
        out["precision"] = precision_leg(args.precision_n, args.precision_steps, tstream, torch)
    if args.serving_requests > 0:
        out["serving"] = serving_leg(args.serving_requests, args.serving_load, stream=stream)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    out["bench_wall_s"] = time.perf_counter() - T_START
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
