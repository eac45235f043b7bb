/*
 * nco.h - C ABI of the MI355X (gfx950) neural-collision-operator lattice
 * Boltzmann engine.
 *
 * The engine advances a periodic D3Q27 lattice by the lattice Boltzmann
 * equation f_i(x + c_i, t + 1) = f_i(x, t) + Omega_i(f) + S_i(f)
 * (paper Sec. II.A) with one of three collision operators:
 *   NCO_OP_BGK  Omega_i = -(f_i - f_i^eq) / tau                (Sec. II.A)
 *   NCO_OP_MRT  Omega = -M^{-1} S (M f - m^eq), fixed rates    (Eq. omegatheta
 *               with constant higher-order rates)
 *   NCO_OP_NCO  the same with the four higher-order rates from the
 *               group-averaged invariant network               (Eq. omegatheta,
 *               Eq. gconv_m and the sigmoid rate squashing of Sec. II.B)
 *   NCO_OP_STREAM no collision: streaming alone (a pure permutation of the
 *               stored values, exact in every storage format)
 * where M is the Hermite moment matrix of Sec. II.B, S has rate 1 for the
 * conserved moments, 1/tau for all second-order moments and one rate per
 * order 3, 4, 5, 6.
 *
 * Conventions shared by every call:
 *  - Every call returns an nco_status; on failure nco_last_error() holds a
 *    message for the calling thread.  Nothing aborts the process.
 *  - Host arrays are float64 (network parameters float32), borrowed for the
 *    duration of the call only; copies are synchronous with respect to the
 *    lattice's stream.
 *  - Node order is [z][y][x] with x fastest.  Populations are [27][z][y][x]
 *    with velocity index i = 9 (c_z + 1) + 3 (c_y + 1) + (c_x + 1); a
 *    velocity field is [3][z][y][x].
 *  - The stored state is the post-collision population.  One step pulls
 *    f_i(x - c_i) into x (periodic wrap) and collides there.
 *  - The library owns all device memory it allocates.  A lattice lives on
 *    the device that was current when it was created and runs its work on
 *    one HIP stream; calls on different lattices may come from different
 *    threads, calls on one lattice must not overlap.
 */
#ifndef NCO_H
#define NCO_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nco_lattice nco_lattice;

typedef enum {
    NCO_OK = 0,
    NCO_E_INVALID = -1,     /* bad argument (size, tau <= 1/2, weight count, ...) */
    NCO_E_OOM = -2,         /* device allocation failed */
    NCO_E_HIP = -3,         /* a HIP runtime call failed */
    NCO_E_UNSTABLE = -4,    /* non-finite state or failed stability check */
    NCO_E_STATE = -5,       /* call not valid in the lattice's current state */
    NCO_E_UNSUPPORTED = -6  /* valid request this library does not implement */
} nco_status;

/* Storage of the populations in HBM.  *_DEV stores the deviation from the
 * rest state, (f_i - w_i) * 2^e_i, with a power-of-two scale per velocity
 * class (e = 2, 4, 6, 8 for |c|^2 = 0, 1, 2, 3) that keeps the values in the
 * normal range of the 16-bit formats; arithmetic is float32 in every case
 * except NCO_F64, which computes in float64. */
typedef enum { NCO_F32 = 0, NCO_F16_DEV = 1, NCO_BF16_DEV = 2, NCO_F64 = 3 } nco_storage;

typedef enum { NCO_OP_BGK = 0, NCO_OP_MRT = 1, NCO_OP_NCO = 2, NCO_OP_STREAM = 3 } nco_op;

/* Arithmetic of the network: float32 (VALU), float32 matrix cores, bf16
 * matrix-core products with float32 accumulation, or float32 split over the
 * 16-bit matrix cores (NCO_MLP_F32_SPLIT: the first layer on the float32
 * matrix cores; each hidden-to-hidden layer's weights and activations split
 * into parts whose products, accumulated in float32, give the float32
 * product to a few units of its rounding: an f16 head and remainder of
 * power-of-two-scaled operands and three products for tanh, three bf16
 * parts and six products for ReLU, whose activations are unbounded). */
typedef enum { NCO_MLP_F32 = 0, NCO_MLP_F32_MFMA = 1, NCO_MLP_BF16 = 2, NCO_MLP_F32_SPLIT = 3 } nco_mlp_prec;

typedef enum { NCO_ACT_TANH = 0, NCO_ACT_RELU = 1 } nco_act;

/* Lattice domain: the periodic box, or the reduced Taylor-Green cube of
 * Appendix A ("Reduced Taylor-Green vortex"). */
typedef enum { NCO_DOMAIN_PERIODIC = 0, NCO_DOMAIN_TGV_OCTANT = 1 } nco_domain;

/* Library version, major * 10000 + minor * 100 + patch. */
int nco_version(void);

/* Message describing the last failure on the calling thread ("" if none). */
const char* nco_last_error(void);

/* Device bytes a lattice of this size and storage holds once created and
 * initialised with nco_init_equilibrium: both population buffers, per-lattice
 * work space and the 4 doubles per node of host-transfer staging that call
 * uses; used for admission decisions.  Not included: calls that move all
 * populations to or from the host (nco_init_populations,
 * nco_read_populations, nco_backward) grow the staging to 27 doubles per node
 * on first use, and network tables, forcing tables and reverse-mode
 * checkpoints are allocated by the calls that need them. */
int nco_lattice_bytes(int nx, int ny, int nz, int storage, size_t* bytes);

/* Create a lattice of nx*ny*nz nodes (each >= 1) on the current device.
 * tau > 1/2 is the shear relaxation time, nu = (tau - 1/2)/3 (Sec. II.B).
 * stream: a hipStream_t to run on, or NULL for a stream the library creates
 * (default priority) and owns.  Populations start at the rest state w_i. */
int nco_lattice_create(int nx, int ny, int nz, int storage, int op, double tau,
                       void* stream, nco_lattice** out);

int nco_lattice_destroy(nco_lattice* lat);

/* Switch the collision operator and/or tau of an existing lattice. */
int nco_set_op(nco_lattice* lat, int op, double tau);

/* Domain of the streaming (Appendix A, "Reduced Taylor-Green vortex").
 * NCO_DOMAIN_PERIODIC (the default): periodic wrap on every axis.
 * NCO_DOMAIN_TGV_OCTANT: the n^3 lattice (nx = ny = nz = n) is the cube
 * [0, pi/2]^3 of the three-dimensional Taylor-Green vortex, node j at
 * (j + 1/2) pi / (2n), and stands for the symmetric 2 pi box of 4n nodes per
 * edge; populations that stream out of the cube come back in through the
 * vortex's symmetries (mirrors in the planes through the origin, the quarter
 * turns about the vortex axis x = y = pi/2, the half turn about the line
 * x = y, z = pi/2), with their velocity mapped along.  A state that has
 * those symmetries evolves exactly as on the 4n box, with 64 times fewer
 * nodes; global sums and the kinetic energy are those of the box, up to
 * the factor 64 in the sums.  Valid for every operator, storage and network,
 * for nco_step, nco_batch_step and the reverse mode; spectral forcing, the
 * energy spectrum and spectrum losses need the periodic box
 * (NCO_E_UNSUPPORTED).  NCO_E_INVALID for an unknown domain or a non-cubic
 * lattice.  Takes effect from the next step; it drops a recorded run. */
int nco_set_domain(nco_lattice* lat, int domain);

/* Rounding of NCO_BF16_DEV and NCO_F16_DEV storage in the following steps:
 * enable = 0 (the default) rounds each stored deviation to nearest even; 1
 * rounds it stochastically, up (away from zero) with probability equal to
 * its position between the two neighbouring 16-bit values, so that stored
 * values are unbiased (a per-step change below half a 16-bit step is kept
 * on average instead of rounded away).  The random bits are a
 * counter-based hash of (seed, step index, node, population), so runs are
 * repeatable and independent of launch shapes, and two-buffer steps,
 * in-place pairs, batched steps and the recomputation of the reverse mode
 * store the same values.  Initialisation keeps round-to-nearest.  The
 * rounding is a property of the storage format; the paper's method is the
 * arithmetic around it.  NCO_E_UNSUPPORTED for other storages,
 * NCO_E_INVALID for another enable value.  Drops a recorded run. */
int nco_set_stochastic_rounding(nco_lattice* lat, int enable, unsigned seed);

/* Memory the reverse mode may use to keep network values between a forward
 * step and the adjoint of its state (float32 matrix-core networks of depth
 * 2, Sec. "Learning Task"): 144 bytes per node for each of the K - 1
 * recomputed states of a segment (K = ckpt_every), and as many for the last
 * state of each of the ceil(T / K) segments, which nco_forward_record keeps
 * when both fit.  Where they are kept (default budget 4 GiB), the adjoint
 * reads the group sums of the second layer and the pre-squash outputs
 * instead of running the network forward again; the gradient is the same
 * bit for bit.  With K = 1 every state is a checkpoint, nothing is
 * recomputed, and every adjoint reads kept values (T x 144 bytes per node
 * beside the T checkpoints).  0 switches it off.  The recompute's share
 * takes effect at the next nco_backward, the segment ends' at the next
 * nco_forward_record. */
int nco_set_reverse_cache(nco_lattice* lat, size_t bytes);

/* Pairs of steps in place (enable = 1, the default) or always between two
 * buffers (0).  With 1, nco_step runs two consecutive BGK or fixed-rate
 * steps (Sec. II.A) on one population buffer when that buffer fits the
 * device's 256 MB last-level cache and the two buffers together do not (a
 * 128^3 float32 lattice): the first step pulls as usual and writes each
 * post-collision population i to the opposite slot of node x + c_i, the
 * second reads those slots at its own node and writes the standard layout.
 * Every slot is read and written by one node, and the results equal those
 * of two-buffer steps bit for bit; only the memory traffic changes (the
 * lattice stays cache-resident).  Pairs are not split by a stability check,
 * and the periodic domain without the velocity-dependent forcing phase is
 * required (otherwise steps run between two buffers).  NCO_E_INVALID for
 * another value. */
int nco_set_inplace(nco_lattice* lat, int enable);

/* Fixed rates omega_3..omega_6 of the four higher-order groups (NCO_OP_MRT). */
int nco_set_rates(nco_lattice* lat, const double omega_high[4]);

/* Network Phi: 27 -> width -> width -> 4 (two hidden layers, Sec. II.B).
 * params: width*(27 + width + 4) + 2*width + 4 float32 values in the order
 * W1[27][width], b1[width], W2[width][width], b2[width], W3[width][4], b3[4]
 * (each W stored [in][out] row-major).  The input is the full moment vector
 * m^(g) = M Pi_g f in the row order of M; the output is tilde tau_n for the
 * orders 3..6.  width must be 8, 16, 20 or 32 (the paper's network is
 * width 20 with ReLU).  The matrix-core arithmetics (NCO_MLP_F32_MFMA,
 * NCO_MLP_BF16, NCO_MLP_F32_SPLIT) need float32 or 16-bit storage and run
 * narrower networks zero-padded to width 32, at the cost of width 32. */
int nco_set_net_weights(nco_lattice* lat, int width, int act, int mlp_prec,
                        const float* params, size_t n_params);

/* The same with depth = 2 or 3 hidden layers.  Depth 3 is the network of
 * Sec. "Training based on dissipation rates", which adds a hidden layer:
 * 27 -> width -> width -> width -> 4, params in the order W1[27][width],
 * b1, W2[width][width], b2, W2b[width][width], b2b, W3[width][4], b3
 * (n_params = width*(27 + 2 width + 4) + 3 width + 4).  Depth 3 runs in
 * every network arithmetic (the matrix-core ones with narrower networks
 * zero-padded to width 32) and has the reverse mode (vector-unit adjoint): nco_backward
 * returns the gradient in this parameter order.  nco_batch_step refuses
 * depth-3 lattices.  Setting the weights drops a recorded run. */
int nco_set_net_weights_depth(nco_lattice* lat, int depth, int width, int act, int mlp_prec,
                              const float* params, size_t n_params);

/* f = f^eq(rho, u) (Eq. EquilibriumDistribution).  rho: N values or NULL
 * for rho = 1; u: 3N values. */
int nco_init_equilibrium(nco_lattice* lat, const double* rho, const double* u);

/* Fine-to-coarse restriction by acoustic scaling (Sec. "Learning Task",
 * the equation for f_{i,c}): set the state of `coarse` from that of `fine`,
 * whose extent is r times the coarse one on every axis (integer r >= 1;
 * coarse node X sits on fine node r X).  At each coarse node the fine
 * node's density and velocity give f^eq, and the fine non-equilibrium part
 * f - f^eq is scaled by r tau_c / tau_f (the taus of the two lattices; the
 * paper prints 2 tau_c / tau_f, the r = 2 case).  The formula is applied to
 * the distribution entering the collision: the fine state is streamed
 * first, and the result is stored un-streamed, so that the coarse lattice's
 * next step streams it back and collides exactly the restricted
 * distribution.  float64 arithmetic, any storages.  Waits for the fine
 * lattice's stream, runs on the coarse one's and returns when done; the
 * coarse lattice counts as freshly initialised (stability check mass,
 * recorded run dropped).  NCO_E_INVALID for extents that are not an integer
 * multiple or lattices on different devices; NCO_E_UNSUPPORTED for the
 * reduced domain. */
int nco_restrict(const nco_lattice* fine, nco_lattice* coarse);

/* Set the populations directly: f holds 27N values. */
int nco_init_populations(nco_lattice* lat, const double* f);

/* Advance nsteps >= 0 time steps; asynchronous on the lattice's stream. */
int nco_step(nco_lattice* lat, int nsteps);

/* Advance several lattices at once: lattice i by nsteps[i] steps.  Lattices
 * of one kernel kind (operator, storage, network arithmetic, activation) are
 * taken in chunks of up to 16; every step of a chunk is one grouped dispatch
 * over its lattices, so that small lattices share the device instead of
 * queueing one behind another.  The first chunk runs on the shared stream,
 * the others on up to three side streams the library keeps per device,
 * forked from the shared stream and joined back to it before the call
 * returns, so that chunks run concurrently; work queued on the shared
 * stream afterwards sees every result.  All lattices must live on the same
 * device and stream and appear once; NCO lattices must use a matrix-core
 * network (nco_set_net_weights with NCO_MLP_F32_MFMA or NCO_MLP_BF16);
 * streaming-only lattices are not batched.  Each lattice's result is the
 * same, bit for bit, as from nco_step.  Asynchronous on the shared stream. */
int nco_batch_step(nco_lattice** lats, int n, const int* nsteps);

/* Stability check.  Every `every` steps (0: off, the default) the float64
 * global sums of the state are computed on the device, after the step, on
 * the stream that ran it, and compared with the mass of the state at the
 * last nco_init_* or nco_set_check call: a sum that is not finite (a NaN or
 * infinity anywhere in the lattice) or a mass drift beyond
 * mass_rel_tol |mass| marks the lattice unstable.  The collision conserves
 * mass exactly (the zeroth moment relaxes with rate 1, Sec. II.B), so a
 * drift can only come from rounding or from a blow-up.  The check adds no
 * synchronisation; nco_sync reports it.  A new initialisation clears it. */
int nco_set_check(nco_lattice* lat, int every, double mass_rel_tol);

/* Block until the lattice's stream has finished its work.  Returns
 * NCO_E_UNSTABLE if a stability check (nco_set_check) has failed. */
int nco_sync(nco_lattice* lat);

/* Copy the populations (27N values) to the host. */
int nco_read_populations(nco_lattice* lat, double* f);

/* rho = sum_i f_i (N values) and u = sum_i c_i f_i / rho (3N values), either
 * may be NULL (Sec. II.A). */
int nco_read_macroscopic(nco_lattice* lat, double* rho, double* u);

/* Relaxation rates omega_3..omega_6 the network assigns to the current
 * state of every node (4N values, [4][z][y][x]); NCO_OP_NCO only. */
int nco_read_rates(nco_lattice* lat, double* omega);

/* float64 sums over all nodes: out[0] = mass, out[1..3] = momentum,
 * out[4] = 1/2 sum |u|^2 with u = j / rho.  Deterministic. */
int nco_global_sums(nco_lattice* lat, double out[5]);

/* Energy spectrum of u = j / rho on a cubic lattice (nx = ny = nz = n):
 * u_hat = DFT(u) / n^3, E(k) = 1/2 sum of |u_hat|^2 over the wavevectors in
 * [-n/2, n/2)^3 with round(|k|) = k, for k = 0 .. nbins-1, computed in
 * float64 (the loss of Sec. "Learning Task").  nbins must equal
 * floor(sqrt(3) * (n/2) + 1/2) + 1. */
int nco_energy_spectrum(nco_lattice* lat, double* E, int nbins);

/* nco_energy_spectrum for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): it calls
 * no hipMalloc, hipFree or other allocating routine and does not
 * synchronise.  The spectrum is written to E_dev, nbins doubles of device
 * memory the caller owns, asynchronously on the lattice's stream; the
 * values equal those of nco_energy_spectrum bit for bit.  Its work space is
 * a fixed 36 MiB array per device that the library holds from its first
 * call on that device until the process ends, enough for cubic lattices
 * up to 66^3 (NCO_E_INVALID beyond, with the bytes needed in the message).
 * All calls on one device share that array: calls that overlap in time on
 * one device (different streams or threads) race and must be serialised by
 * the caller; the array keeps the last call's contents. */
int nco_energy_spectrum_noalloc(nco_lattice* lat, double* E_dev, int nbins);

/* Borrowed device pointer to the current population buffer and its size in
 * bytes; valid until the next step or destroy. */
int nco_device_populations(nco_lattice* lat, void** dev_ptr, size_t* bytes);

/* Alvelius spectral forcing (Sec. "Training Data - Forced Isotropic
 * Turbulence"), applied through the Kupershtokh exact-difference source
 * (Sec. II.A) in every following step.  k: n_modes integer wavevectors
 * (3 ints each, one of each +-k pair); the force is
 * F(x) = sum_m 2 Re(F_hat_m exp(i k_m . x)), x = 2 pi (node / extent), with
 * F_hat = A_ran e1 + B_ran e2, A_ran, B_ran = sqrt(F(|k|) / (2 pi |k|^2))
 * exp(i theta1, i (theta1 + psi)) (sin 2 phi, cos 2 phi),
 * F(|k|) = amplitude exp(-(|k| - kf)^2 / c), e1 the unit normal of k in the
 * x-y plane and e2 = (k_x k_z, k_y k_z, -(k_x^2 + k_y^2)) / (|k| sqrt(k_x^2 + k_y^2))
 * ((1,0,0) and (0,1,0) when k_x = k_y = 0).  draws: [n_steps][n_modes][3]
 * uniform numbers in [0, 1) giving phi / pi, psi / 2 pi and theta1 / 2 pi;
 * the t-th step after this call uses draws[t mod n_steps].  n_modes = 0
 * switches forcing off.  Before each step the force is synthesised once on
 * every node (float64 arithmetic; stored as float32, or float64 for
 * NCO_F64 storage: 12 or 24 bytes per node of device memory) and the step
 * reads it; NCO_E_UNSUPPORTED for wavevectors with |k_x| > 16. */
int nco_set_forcing(nco_lattice* lat, int n_modes, const int* k, const double* draws, int n_steps,
                    double amplitude, double kf, double c);

/* nco_set_forcing, and with phase_rule = 1 Alvelius' velocity-dependent
 * phase (Sec. "Training Data - Forced Isotropic Turbulence", the tangent
 * equation) instead of the drawn theta1.  Before each step, on the device,
 * the library computes:
 *   - u_hat(k) = N^-1 sum_x u(x) exp(-i k.x) of the state the step starts
 *     from (u = j / rho, float64, fixed-order sums);
 *   - xi_i = u_hat . e_i and Z = g_A conj(xi1) + g_B exp(i psi) conj(xi2);
 *   - theta1 = atan2(Re Z, Im Z), the solution of the printed
 *     tan theta1 = Re Z / Im Z that keeps the force continuous in u_hat.
 * The force then does no work on the velocity at every forced mode.  The
 * draws' third column is not used.  nco_forward_record keeps F_hat and
 * u_hat of every recorded step (12 doubles per mode and step of device
 * memory), and nco_backward follows the force back to the state through
 * them: dL/dF per node, dL/dF_hat per mode, then theta1 -> Z -> u_hat -> u
 * (zero where Z = 0, where theta1 has no derivative).  nco_batch_step
 * refuses such lattices (NCO_E_UNSUPPORTED).  NCO_E_INVALID for phase_rule
 * outside {0, 1} or more than 1024 modes. */
int nco_set_forcing_ex(nco_lattice* lat, int n_modes, const int* k, const double* draws, int n_steps,
                       double amplitude, double kf, double c, int phase_rule);

/* Amplitude A of the force density F(k) = A exp(-(k - kf)^2 / c) for a power
 * input P injected over a time step dt (Sec. "Training Data - Forced
 * Isotropic Turbulence", the equation for A):
 *   A = (P / dt) / integral_{ka}^{kb} exp(-(k - kf)^2 / c) dk,
 * with the Gaussian's integral in closed form (error functions).  ka < kb
 * are the edges of the forced band of wavenumbers (units of the 2 pi box,
 * like the integer wavevectors of nco_set_forcing).  With every integer
 * wavevector of the band forced, a step of length dt raises the kinetic
 * energy per unit mass by P dt (the force does no work on the velocity
 * under the velocity-dependent phase, and none on average with drawn
 * phases), up to the difference between the sum over the band's
 * wavevectors and the integral.  Host arithmetic only: needs no device.
 * NCO_E_INVALID for P < 0, dt <= 0, c <= 0, ka >= kb, non-finite arguments
 * or an integral that underflows to zero. */
int nco_forcing_amplitude(double power, double dt, double ka, double kb, double kf, double c,
                          double* amplitude);

/* nco_set_forcing_ex with the amplitude from the power input: A =
 * nco_forcing_amplitude(power, 1, ka, kb, kf, c), power in lattice units
 * (kinetic energy per unit mass per time step; the lattice's time step is
 * dt = 1 and its velocity changes by F per step). */
int nco_set_forcing_power(nco_lattice* lat, int n_modes, const int* k, const double* draws, int n_steps,
                          double power, double ka, double kb, double kf, double c, int phase_rule);

/* Run nsteps steps (NCO operator, width 32, float storage) keeping a
 * checkpoint of the state every ckpt_every steps in device memory, for a
 * following nco_backward (the gradient of Adam in Sec. "Learning Task").
 * With a float32 matrix-core network of depth 2 it also keeps the network
 * values of the last step of each checkpoint segment when the reverse-mode
 * budget allows (nco_set_reverse_cache); ckpt_every = 1 keeps every state
 * and nco_backward then recomputes nothing. */
int nco_forward_record(nco_lattice* lat, int nsteps, int ckpt_every);

/* nco_forward_record, and the mean kinetic energy k(t) = <|u|^2> / 2
 * (u = j / rho, float64 sums) of the states t = 0, every, 2 every, ... <=
 * nsteps steps after the start, written to k (nsteps / every + 1 values):
 * the trajectory the dissipation-rate loss of Sec. "Learning Task" (the
 * reduced Taylor-Green training) is computed from. */
int nco_forward_record_energy(nco_lattice* lat, int nsteps, int ckpt_every, int every, double* k);

/* Reverse mode through the recorded run (no step may come in between).  The
 * loss gradient at the final state is dL_dE (nbins values: dL/dE(k) of the
 * spectrum defined by nco_energy_spectrum, or NULL) plus dL_df (27N values,
 * or NULL).  Writes grad (n_params = 2084 values, the parameter order of
 * nco_set_net_weights) in float64 and, if dL_df0 is not NULL, dL/d(initial
 * populations) (27N values).  Segments are recomputed from their checkpoints;
 * the result is deterministic (fixed-order reductions).  The recorded and
 * recomputed steps run the lattice's own network arithmetic; the adjoint
 * differentiates the network in float32: on the matrix cores for the
 * depth-2 matrix-core networks (NCO_MLP_F32_MFMA, and NCO_MLP_F32_SPLIT and
 * NCO_MLP_BF16, whose product rounding it does not differentiate), on the
 * vector units for NCO_MLP_F32 and depth 3. */
int nco_backward(nco_lattice* lat, const double* dL_dE, int nbins, const double* dL_df, double* grad,
                 size_t n_params, double* dL_df0);

/* nco_backward with, in addition, a loss on the kinetic-energy trajectory of
 * nco_forward_record_energy: dL_dk[m] = dL/dk(m every) for the states
 * t = m every, m = 0 .. rec_steps / every (the same sampling as the
 * record).  dL_dE and dL_df (terms at the final state) may both be NULL. */
int nco_backward_energy(nco_lattice* lat, const double* dL_dk, int every, const double* dL_dE, int nbins,
                        const double* dL_df, double* grad, size_t n_params, double* dL_df0);

#ifdef __cplusplus
}
#endif

#endif /* NCO_H */
