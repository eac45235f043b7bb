// Host-visible launch interface of the lattice kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "collide.h"

namespace nco {

// Lattice domains: the periodic box, or the reduced Taylor-Green cube of
// Appendix A (n^3 nodes standing for the symmetric 4n box).
constexpr int DOMAIN_PERIODIC = 0;
constexpr int DOMAIN_TGV_OCTANT = 1;

// Everything a stream-collide launch needs, passed by value.
struct StepArgs {
    int nx, ny, nz, n;       // lattice extent and node count
    int op;                  // OP_BGK / OP_MRT / OP_NCO
    int domain;              // DOMAIN_PERIODIC / DOMAIN_TGV_OCTANT (nx = ny = nz)
    int width, act;          // network shape (OP_NCO)
    int depth;               // hidden layers: 2, or 3 (vector-unit network, width 32)
    double omega_nu;         // 1 / tau
    float omega_nu_f;
    double omega_high[4];    // fixed rates of orders 3..6 (OP_MRT)
    float omega_high_f[4];
    const float* net;        // device network buffer (OP_NCO), see net_off_*()
    // Spectral forcing of this step: F(x) = sum_m 2 Re(Fhat_m exp(i k_m.x)),
    // x in [0, 2 pi)^3; n_modes = 0 disables the Kupershtokh source.
    int n_modes;
    const int* fk;           // [n_modes][3] integer wavevectors
    const double* fhat;      // [n_modes][6] Re/Im of Fhat_x, Fhat_y, Fhat_z for this step
    // The same force synthesised on every node for this step ([3][n], by
    // launch_force_field before the step): float64 for float64 storage,
    // float32 otherwise.  The step kernels read it instead of summing modes.
    const float* force32;
    const double* force64;
    // Rounding of 16-bit deviation storage in this step: 0 rounds to
    // nearest even, any other value rounds stochastically with random bits
    // keyed by it (see sr_bits).
    unsigned sr_key;
    // Network values of this step, [node][NET_SUMS_PER_NODE] over the nodes
    // rounded up to a multiple of 256: the 32 group sums of the second layer
    // and the 4 pre-squash outputs tilde tau.  A float32 matrix-core step
    // writes them when set; the matrix-core adjoint of the same step reads
    // them instead of running the network forward again.  nullptr: neither.
    float* net_sums;
};
constexpr int NET_SUMS_PER_NODE = 36;

// Phases of the spectral modes at a node, e^{i 2 pi (k_x x / nx + k_y y / ny
// + k_z z / nz)}, as the product over the axes of integer powers of the
// node's axis phasors e^{i 2 pi x / nx} (one sincospi of an exact fraction
// per axis; binary powering, so a wavevector component k costs about
// log2 |k| complex products).
struct Phasor {
    double c, s;
};

__device__ __forceinline__ Phasor phasor_mul(Phasor a, Phasor b) {
    return Phasor{a.c * b.c - a.s * b.s, a.c * b.s + a.s * b.c};
}

__device__ __forceinline__ Phasor axis_phasor(int x, int n) {
    Phasor p;
    sincospi(2.0 * (double)x / (double)n, &p.s, &p.c);
    return p;
}

__device__ __forceinline__ Phasor phasor_pow(Phasor b, int k) {
    Phasor r{1.0, 0.0};
    Phasor p = k < 0 ? Phasor{b.c, -b.s} : b;
    for (int e = k < 0 ? -k : k; e; e >>= 1) {
        if (e & 1) r = phasor_mul(r, p);
        if (e > 1) p = phasor_mul(p, p);
    }
    return r;
}

struct NodePhasors {
    Phasor x, y, z;
};

__device__ __forceinline__ NodePhasors node_phasors(int x, int y, int z, int nx, int ny, int nz) {
    return NodePhasors{axis_phasor(x, nx), axis_phasor(y, ny), axis_phasor(z, nz)};
}

// e^{i k.x} for wavevector k (3 ints) at the node of `b`.
__device__ __forceinline__ Phasor mode_phase(const int* k, const NodePhasors& b) {
    return phasor_mul(phasor_mul(phasor_pow(b.x, k[0]), phasor_pow(b.y, k[1])), phasor_pow(b.z, k[2]));
}

// Force density at node idx for the current step, from the field
// synthesised by launch_force_field (zero without forcing).
template <typename R>
__device__ __forceinline__ void read_force(const StepArgs& a, int idx, R& Fx, R& Fy, R& Fz) {
    if (a.force64) {
        Fx = (R)a.force64[idx];
        Fy = (R)a.force64[(size_t)a.n + idx];
        Fz = (R)a.force64[2 * (size_t)a.n + idx];
    } else if (a.force32) {
        Fx = (R)a.force32[idx];
        Fy = (R)a.force32[(size_t)a.n + idx];
        Fz = (R)a.force32[2 * (size_t)a.n + idx];
    } else {
        Fx = Fy = Fz = R(0);
    }
}

// Grouped launch: one dispatch advancing up to GROUP_MAX lattices of the same
// kernel kind by one step; blocks [prefix[i], prefix[i+1]) serve lattice i.
// Passed by value (kernel argument segment, read with scalar loads).
constexpr int GROUP_MAX = 16;
struct GroupDesc {
    const void* fin;
    void* fout;
    StepArgs a;
    const float* lane_tab;
    const int* gtab;
};
struct LaunchGroup {
    int count;
    int prefix[GROUP_MAX + 1];
    GroupDesc d[GROUP_MAX];
};

// Lattice of block b of a grouped launch (count <= 16: a linear scan).
__device__ __forceinline__ int group_member(const LaunchGroup& g, int b) {
    int i = 0;
    while (i + 1 < g.count && g.prefix[i + 1] <= b) ++i;
    return i;
}

hipError_t launch_step(int storage, const void* fin, void* fout, const StepArgs& a, hipStream_t st);
// One step of an in-place pair on a single buffer (BGK or fixed-rate,
// periodic): phase 0 from the standard layout, phase 1 back to it.
hipError_t launch_step_inplace(int storage, void* f, const StepArgs& a, int phase, hipStream_t st);
// Velocity-dependent Alvelius phase: F_hat of this step's forced modes from
// the state f (partial: nblocks(n) x n_modes x 6 doubles of work space), and
// u_hat into uhat (6 doubles per mode) unless it is null.
// Force field of one step, F(x) = sum_m 2 Re(Fhat_m e^{i k_m . x}), on every
// node in float64 arithmetic, written to out32 or out64 ([3][n]); kx_max
// is the largest |k_x| of the modes (at most FORCE_KX_MAX).
constexpr int FORCE_KX_MAX = 16;
hipError_t launch_force_field(const StepArgs& a, int kx_max, float* out32, double* out64, hipStream_t st);
hipError_t launch_force_phase(int storage, const void* f, int n, int nx, int ny, int nz, const int* fk,
                              int n_modes, double* partial, const double* basis, const double* draw, double* fhat,
                              double* uhat, hipStream_t st);
// Fine-to-coarse restriction (coarse extent x r = fine extent on every axis).
hipError_t launch_restrict(int fine_storage, const void* fine, int fnx, int fny, int fnz, int coarse_storage,
                           void* coarse, int cnx, int cny, int cnz, int r, double factor, hipStream_t st);
// BGK and fixed-rate lattices (op in a.op of every member, same storage).
hipError_t launch_step_grouped(int storage, int op, const LaunchGroup& g, hipStream_t st);
hipError_t launch_rates(int storage, const void* fin, double* omega, const StepArgs& a, hipStream_t st);
// f = f^eq(rho, u); rho == nullptr: rho = 1; u == nullptr: u = 0.
hipError_t launch_init_equilibrium(int storage, void* f, const double* rho, const double* u, int n,
                                   hipStream_t st);
hipError_t launch_from_double(int storage, void* f, const double* src, int n, hipStream_t st);
hipError_t launch_to_double(int storage, const void* f, double* dst, int n, hipStream_t st);
hipError_t launch_macroscopic(int storage, const void* f, double* rho, double* u, int n, hipStream_t st);
int sums_partial_count(int n);
hipError_t launch_global_sums(int storage, const void* f, double* partial, double* out, int n,
                              hipStream_t st);
// Global sums into sums[0..4], then flag = 1 if they are not finite or the
// mass left [mass0 (1 - tol), mass0 (1 + tol)].
hipError_t launch_check_state(int storage, const void* f, double* partial, double* sums, int n, double mass0,
                              double tol, int* flag, hipStream_t st);

// Matrix-core network path (nco_mfma.hip), width 32, float32 or bf16 operands.
size_t mfma_lane_table_floats();
size_t mfma_group_table_ints();
void mfma_prepare_tables(const float* params, int act, int prec, const int (*gsrc)[27], float* lane_tab,
                         int* gtab, int depth = 2);
hipError_t launch_nco_mfma(int storage, int prec, const void* fin, void* fout, const StepArgs& a,
                           const float* lane_tab, const int* gtab, double* omega_out, hipStream_t st);
hipError_t launch_nco_mfma_grouped(int storage, int prec, int act, const LaunchGroup& g, hipStream_t st);

// Adjoint of a step (adjoint.hip), network width 32, float arithmetic.
int adjoint_param_count();
// Partial gradient rows of one launch_adjoint (several per 64-node block).
int adjoint_blocks(int n, int depth);
size_t adjoint_xwork_floats(int n, int depth);
// xwork: adjoint_xwork_floats(n, depth) floats of exchange space for the
// split reverse step of small depth-3 lattices (may be null when that is 0).
hipError_t launch_adjoint(int storage, const void* xin, const float* lam_in, float* lam_out, const StepArgs& a,
                          const int* gsrc, float* partial, float* xwork, hipStream_t st);
hipError_t launch_grad_reduce(const float* partial, int nblocks, int npar, double* grad, hipStream_t st);
int adjoint_param_count_depth(int depth);
// lam += coef d(sum over nodes of |u|^2 / 2) / df for the state f (float64 arithmetic).
hipError_t launch_add_energy_grad(int storage, const void* f, float* lam, double coef, int n, hipStream_t st);
// grad = sum over rows of partial[nblocks][NPAR] (float64) in row order, in
// two passes over groups of 64 rows; stage holds ceil(nblocks / 64) rows.
hipError_t launch_grad_reduce_f64(const double* partial, int nblocks, double* stage, double* grad, hipStream_t st);
// Reverse mode of the velocity-dependent forcing phase of one step: x the
// state the step started from, lam_next = dL/d(state after it), a.fhat the
// step's coefficients, uhat its u_hat, draw its (phi, psi) per mode;
// lam_out (already holding the rest of dL/dx) gets the path x -> u_hat ->
// theta1 -> F_hat -> source added.  partial: nblocks(n) x n_modes x 6
// doubles of work space, duhat: 6 doubles per mode.  Float storages only.
hipError_t launch_force_phase_adjoint(int storage, const void* x, const float* lam_next, float* lam_out,
                                      const StepArgs& a, double* partial, const double* basis, const double* draw,
                                      const double* uhat, double* duhat, hipStream_t st);

// The same adjoint on the matrix cores (nco_mfma.hip): 256 nodes per block;
// lane_tab and gtab are the float32 forward tables of mfma_prepare_tables,
// adj_tab the table of mfma_prepare_adjoint_table; the step's parameter
// gradient is added to partial[block][NPAR].
size_t mfma_adjoint_table_floats();
void mfma_prepare_adjoint_table(const float* params, float* tab);
int adjoint_mfma_blocks(int n);
hipError_t launch_adjoint_mfma(int storage, int act, const void* xin, const float* lam_in, float* lam_out,
                               const StepArgs& a, const float* lane_tab, const int* gtab, const float* adj_tab,
                               const int* gsrc, double* partial, hipStream_t st);
hipError_t launch_fill_f32(float* p, size_t count, float v, hipStream_t st);
hipError_t launch_fill_f64(double* p, size_t count, double v, hipStream_t st);
hipError_t launch_add_f64_to_f32(float* dst, const double* src, size_t count, hipStream_t st);
hipError_t launch_f32_to_f64(const float* src, double* dst, size_t count, hipStream_t st);
hipError_t launch_spectrum_adjoint(int storage, const void* f, int n, void* work, const double* dE, int nbins,
                                   float* lam, hipStream_t st);

// Energy spectrum (spectrum.hip).
size_t spectrum_workspace_bytes(int n);
size_t spectrum_forward_bytes(int n);
size_t spectrum_scratch_bytes();
hipError_t spectrum_scratch(int device, void** ptr);
hipError_t launch_energy_spectrum(int storage, const void* f, int n, void* work, double* E_dev,
                                  int nbins, hipStream_t st);

}  // namespace nco
