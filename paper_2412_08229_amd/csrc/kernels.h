// Host-visible launch interface of the lattice kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "collide.h"

namespace nco {

// Everything a stream-collide launch needs, passed by value.
struct StepArgs {
    int nx, ny, nz, n;       // lattice extent and node count
    int op;                  // OP_BGK / OP_MRT / OP_NCO
    int width, act;          // network shape (OP_NCO)
    double omega_nu;         // 1 / tau
    float omega_nu_f;
    double omega_high[4];    // fixed rates of orders 3..6 (OP_MRT)
    float omega_high_f[4];
    const float* net;        // device network buffer (OP_NCO), see net_off_*()
};

hipError_t launch_step(int storage, const void* fin, void* fout, const StepArgs& a, hipStream_t st);
hipError_t launch_rates(int storage, const void* fin, double* omega, const StepArgs& a, hipStream_t st);
hipError_t launch_init_equilibrium(int storage, void* f, const double* rho, const double* u, int n,
                                   hipStream_t st);
hipError_t launch_from_double(int storage, void* f, const double* src, int n, hipStream_t st);
hipError_t launch_to_double(int storage, const void* f, double* dst, int n, hipStream_t st);
hipError_t launch_macroscopic(int storage, const void* f, double* rho, double* u, int n, hipStream_t st);
int sums_partial_count(int n);
hipError_t launch_global_sums(int storage, const void* f, double* partial, double* out, int n,
                              hipStream_t st);
hipError_t launch_check_finite(int storage, const void* f, int n, int* flag, hipStream_t st);

// Matrix-core network path (nco_mfma.hip), width 32, float32 or bf16 operands.
size_t mfma_lane_table_floats();
size_t mfma_group_table_ints();
void mfma_prepare_tables(const float* params, int act, int prec, const int (*gsrc)[27], float* lane_tab,
                         int* gtab);
hipError_t launch_nco_mfma(int storage, int prec, const void* fin, void* fout, const StepArgs& a,
                           const float* lane_tab, const int* gtab, double* omega_out, hipStream_t st);

// Energy spectrum (spectrum.hip).
size_t spectrum_workspace_bytes(int n);
hipError_t launch_energy_spectrum(int storage, const void* f, int n, void* work, double* E_dev,
                                  int nbins, hipStream_t st);

}  // namespace nco
