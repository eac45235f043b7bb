// Lattice kernels: fused pull-stream + collide, initialisation, readout and
// float64 reductions.  One thread per node; populations in structure-of-
// arrays layout [27][z][y][x] so that each of the 27 loads and stores of a
// wavefront is a contiguous row segment of one velocity plane.
//
// Multiply-adds are fused only within one source expression (not across
// statements, as hipcc's default allows), before any header is read: the
// collision code inlined into different kernels (two-buffer, in-place pair,
// grouped) then rounds identically, and those kernels agree bit for bit.
#pragma STDC FP_CONTRACT ON
#include <algorithm>

#include "kernels.h"
#include "stream.h"

namespace nco {

namespace {

template <typename R> __device__ __forceinline__ R pick(float f, double d);
template <> __device__ __forceinline__ float pick<float>(float f, double) { return f; }
template <> __device__ __forceinline__ double pick<double>(float, double d) { return d; }

// Collision of one node in place (plus the Kupershtokh source of force F when
// FORCED); OP and W/ACT select the operator.
template <typename R, int OP, int W, int ACT, bool FORCED, int DEPTH = 2>
__device__ __forceinline__ void collide_node(R (&f)[Q], const StepArgs& a, R Fx, R Fy, R Fz) {
    const R omega_nu = pick<R>(a.omega_nu_f, a.omega_nu);
    if constexpr (OP == OP_BGK) {
        bgk<R, FORCED>(f, omega_nu, Fx, Fy, Fz);
    } else {
        R m[Q];
        to_moments(f, m);
        R omega[4];
        if constexpr (OP == OP_NCO) {
            net_rates<R, W, ACT, DEPTH>(m, a.net, omega);
        } else {
#pragma unroll
            for (int n = 0; n < 4; ++n) omega[n] = pick<R>(a.omega_high_f[n], a.omega_high[n]);
        }
        R dm[Q], df[Q];
        collision_delta<R, FORCED>(m, omega_nu, omega, Fx, Fy, Fz, dm);
        from_moments(dm, df);
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] -= df[i];
    }
}

template <int S, int OP, int W, int ACT, int DEPTH = 2>
__device__ __forceinline__ void stream_collide_node(const typename Codec<S>::store_t* __restrict__ fin,
                                                    typename Codec<S>::store_t* __restrict__ fout,
                                                    const StepArgs& a, int idx);

template <int S, int OP, int W, int ACT, int DEPTH = 2>
__global__ __launch_bounds__(256) void k_stream_collide(const typename Codec<S>::store_t* __restrict__ fin,
                                                        typename Codec<S>::store_t* __restrict__ fout,
                                                        StepArgs a) {
    stream_collide_node<S, OP, W, ACT, DEPTH>(fin, fout, a, blockIdx.x * blockDim.x + threadIdx.x);
}

// One step of several lattices of the same kind in one dispatch.
template <int S, int OP>
__global__ __launch_bounds__(256) void k_stream_collide_grouped(LaunchGroup g) {
    using T = typename Codec<S>::store_t;
    const int i = group_member(g, blockIdx.x);
    const GroupDesc& d = g.d[i];
    stream_collide_node<S, OP, 8, ACT_TANH>(static_cast<const T*>(d.fin), static_cast<T*>(d.fout), d.a,
                                            (blockIdx.x - g.prefix[i]) * blockDim.x + threadIdx.x);
}

template <int S, int OP, int W, int ACT, int DEPTH>
__device__ __forceinline__ void stream_collide_node(const typename Codec<S>::store_t* __restrict__ fin,
                                                    typename Codec<S>::store_t* __restrict__ fout,
                                                    const StepArgs& a, int idx) {
    using R = typename Codec<S>::real;
    if (idx >= a.n) return;
    R f[Q];
    const NodeIdx p = node_of(idx, a.nx, a.ny);
    pull<S>(fin, a, p, f);
    if (a.n_modes > 0) {
        R Fx, Fy, Fz;
        read_force(a, idx, Fx, Fy, Fz);
        collide_node<R, OP, W, ACT, true, DEPTH>(f, a, Fx, Fy, Fz);
    } else {
        collide_node<R, OP, W, ACT, false, DEPTH>(f, a, R(0), R(0), R(0));
    }
    store_local<S>(fout, a.n, idx, f, a.sr_key);
}

// Two steps in place on one population buffer (periodic lattices).  With
// opp(i) = 26 - i the population of velocity -c_i:
//   PHASE 0 reads the standard layout by the usual pull, f_i(x) = F(i, x - c_i),
//     and writes the post-collision f_i of node x to slot (opp(i), x + c_i);
//   PHASE 1 reads f_i(x) = F(opp(i), x), which the first step wrote there
//     from node x - c_i (its pull), and writes F(i, x): the standard layout.
// In either phase the slots a node writes are exactly the slots it read
// (PHASE 0: node x is the only reader of (opp(i), x + c_i), the slot its own
// pull of population opp(i) reads), so threads never race and the pair of
// steps computes what two steps between two buffers compute, bit for bit,
// with one buffer: a 128^3 float32 lattice (226 MB) then stays in the 256 MB
// last-level cache instead of streaming 453 MB through it.  Stores are
// cached, since the next step reads them back at once.
template <int S, int OP, int PHASE>
__global__ __launch_bounds__(256) void k_stream_collide_inplace(typename Codec<S>::store_t* f, StepArgs a) {
    using R = typename Codec<S>::real;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.n) return;
    const NodeIdx p = node_of(idx, a.nx, a.ny);
    R v[Q];
    if constexpr (PHASE == 0) {
        pull<S>(f, a, p, v);
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) v[i] = Codec<S>::load(f + (size_t)(Q - 1 - i) * a.n + idx, i);
    }
    if (a.n_modes > 0) {
        R Fx, Fy, Fz;
        read_force(a, idx, Fx, Fy, Fz);
        collide_node<R, OP, 8, ACT_TANH, true>(v, a, Fx, Fy, Fz);
    } else {
        collide_node<R, OP, 8, ACT_TANH, false>(v, a, R(0), R(0), R(0));
    }
    if constexpr (PHASE == 0) {
        // Destination coordinate for c = -1, 0, +1 is x - 1, x, x + 1.
        const int xd[3] = {p.x == 0 ? a.nx - 1 : p.x - 1, p.x, p.x == a.nx - 1 ? 0 : p.x + 1};
        const int yd[3] = {(p.y == 0 ? a.ny - 1 : p.y - 1) * a.nx, p.y * a.nx,
                           (p.y == a.ny - 1 ? 0 : p.y + 1) * a.nx};
        const int nxy = a.nx * a.ny;
        const int zd[3] = {(p.z == 0 ? a.nz - 1 : p.z - 1) * nxy, p.z * nxy,
                           (p.z == a.nz - 1 ? 0 : p.z + 1) * nxy};
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int dst = zd[cz_of(i) + 1] + yd[cy_of(i) + 1] + xd[cx_of(i) + 1];
            store_one_cached<S>(f + (size_t)(Q - 1 - i) * a.n + dst, idx, i, v[i], a.sr_key);
        }
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) store_one_cached<S>(f + (size_t)i * a.n + idx, idx, i, v[i], a.sr_key);
    }
}

// Streaming alone: the raw stored values are moved, so the result is an exact
// permutation in every storage format.
template <int S>
__global__ __launch_bounds__(256) void k_stream_only(const typename Codec<S>::store_t* __restrict__ fin,
                                                     typename Codec<S>::store_t* __restrict__ fout,
                                                     StepArgs a) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.n) return;
    const NodeIdx p = node_of(idx, a.nx, a.ny);
    if (on_octant_face(a, p)) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const Slot s = fold_octant(a.nx, p.x - cx_of(i), p.y - cy_of(i), p.z - cz_of(i), cx_of(i), cy_of(i),
                                       cz_of(i));
            fout[(size_t)i * a.n + idx] = fin[(size_t)s.plane * a.n + s.node];
        }
        return;
    }
    const int xs[3] = {p.x == a.nx - 1 ? 0 : p.x + 1, p.x, p.x == 0 ? a.nx - 1 : p.x - 1};
    const int ys[3] = {(p.y == a.ny - 1 ? 0 : p.y + 1) * a.nx, p.y * a.nx,
                       (p.y == 0 ? a.ny - 1 : p.y - 1) * a.nx};
    const int nxy = a.nx * a.ny;
    const int zs[3] = {(p.z == a.nz - 1 ? 0 : p.z + 1) * nxy, p.z * nxy,
                       (p.z == 0 ? a.nz - 1 : p.z - 1) * nxy};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int src = zs[cz_of(i) + 1] + ys[cy_of(i) + 1] + xs[cx_of(i) + 1];
        fout[(size_t)i * a.n + idx] = fin[(size_t)i * a.n + src];
    }
}

template <int S, int W, int ACT, int DEPTH = 2>
__global__ __launch_bounds__(256) void k_rates(const typename Codec<S>::store_t* __restrict__ fin,
                                               double* __restrict__ omega_out, StepArgs a) {
    using R = typename Codec<S>::real;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.n) return;
    R f[Q], m[Q], omega[4];
    load_local<S>(fin, a.n, idx, f);
    to_moments(f, m);
    net_rates<R, W, ACT, DEPTH>(m, a.net, omega);
#pragma unroll
    for (int k = 0; k < 4; ++k) omega_out[(size_t)k * a.n + idx] = (double)omega[k];
}

// Fine-to-coarse restriction by acoustic scaling (Sec. "Learning Task"):
// for coarse node X on fine node r X, the pre-collision populations of the
// fine node, f_i = fine_i(r X - c_i) (pull on the periodic fine lattice),
// give rho, u and f^eq, and f^eq_i + factor (f_i - f^eq_i) is stored
// un-streamed on the coarse lattice, at slot (i, X - c_i), where the coarse
// step's pull reads it back at X.  float64 arithmetic; every coarse slot is
// written once (un-streaming is a permutation).
template <int SF, int SC>
__global__ __launch_bounds__(256) void k_restrict(const typename Codec<SF>::store_t* __restrict__ fine,
                                                  typename Codec<SC>::store_t* __restrict__ coarse, int fnx,
                                                  int fny, int fnz, int cnx, int cny, int cnz, int r, double factor) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int cn = cnx * cny * cnz;
    if (idx >= cn) return;
    const int X = idx % cnx, Y = (idx / cnx) % cny, Z = idx / (cnx * cny);
    const size_t fn = (size_t)fnx * fny * fnz;
    double f[Q];
    double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int sx = (r * X - cx_of(i) + fnx) % fnx, sy = (r * Y - cy_of(i) + fny) % fny;
        const int sz = (r * Z - cz_of(i) + fnz) % fnz;
        f[i] = Codec<SF>::to_double(fine[(size_t)i * fn + ((size_t)sz * fny + sy) * fnx + sx], i);
        rho += f[i];
        jx += cx_of(i) * f[i];
        jy += cy_of(i) * f[i];
        jz += cz_of(i) * f[i];
    }
    const double ux = jx / rho, uy = jy / rho, uz = jz / rho;
    const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double cu = cx_of(i) * ux + cy_of(i) * uy + cz_of(i) * uz;
        const double feq = weight_of(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        const int dx = (X - cx_of(i) + cnx) % cnx, dy = (Y - cy_of(i) + cny) % cny, dz = (Z - cz_of(i) + cnz) % cnz;
        coarse[(size_t)i * cn + ((size_t)dz * cny + dy) * cnx + dx] =
            Codec<SC>::from_double(feq + factor * (f[i] - feq), i);
    }
}

template <int S>
__global__ __launch_bounds__(256) void k_init_equilibrium(typename Codec<S>::store_t* __restrict__ f,
                                                          const double* __restrict__ rho,
                                                          const double* __restrict__ u, int n) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const double r = rho ? rho[idx] : 1.0;
    const double ux = u ? u[idx] : 0.0, uy = u ? u[(size_t)n + idx] : 0.0, uz = u ? u[2 * (size_t)n + idx] : 0.0;
    const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double cu = cx_of(i) * ux + cy_of(i) * uy + cz_of(i) * uz;
        // f^eq - w computed as w (rho (1 + ...) - 1) keeps the deviation exact
        // for the 16-bit storage forms.
        const double dev = weight_of(i) * ((r - 1.0) + r * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
        typename Codec<S>::store_t v;
        if constexpr (S == ST_F16) {
            v = __float2half_rn((float)(dev * dev_scale(i)));
        } else if constexpr (S == ST_BF16) {
            v = __float2bfloat16((float)(dev * dev_scale(i)));
        } else {
            v = Codec<S>::from_double(weight_of(i) + dev, i);
        }
        f[(size_t)i * n + idx] = v;
    }
}

template <int S>
__global__ __launch_bounds__(256) void k_from_double(typename Codec<S>::store_t* __restrict__ f,
                                                     const double* __restrict__ src, int n) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
#pragma unroll
    for (int i = 0; i < Q; ++i) f[(size_t)i * n + idx] = Codec<S>::from_double(src[(size_t)i * n + idx], i);
}

template <int S>
__global__ __launch_bounds__(256) void k_to_double(const typename Codec<S>::store_t* __restrict__ f,
                                                   double* __restrict__ dst, int n) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
#pragma unroll
    for (int i = 0; i < Q; ++i) dst[(size_t)i * n + idx] = Codec<S>::to_double(f[(size_t)i * n + idx], i);
}

// rho and u = j / rho in float64 from the stored populations.
template <int S>
__device__ __forceinline__ void macro_double(const typename Codec<S>::store_t* __restrict__ f, int n,
                                             int idx, double& rho, double& ux, double& uy, double& uz) {
    double r = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double v = Codec<S>::to_double(f[(size_t)i * n + idx], i);
        r += v;
        jx += cx_of(i) * v;
        jy += cy_of(i) * v;
        jz += cz_of(i) * v;
    }
    rho = r;
    ux = jx / r;
    uy = jy / r;
    uz = jz / r;
}

template <int S>
__global__ __launch_bounds__(256) void k_macroscopic(const typename Codec<S>::store_t* __restrict__ f,
                                                     double* __restrict__ rho_out,
                                                     double* __restrict__ u_out, int n) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    double r, ux, uy, uz;
    macro_double<S>(f, n, idx, r, ux, uy, uz);
    rho_out[idx] = r;
    u_out[idx] = ux;
    u_out[(size_t)n + idx] = uy;
    u_out[2 * (size_t)n + idx] = uz;
}

// Block sum of NSUM doubles: wavefront shuffles, then one value per wave in LDS.
template <int NSUM>
__device__ __forceinline__ void block_sum(double (&v)[NSUM], double* __restrict__ out) {
    __shared__ double part[NSUM][256 / 64];
#pragma unroll
    for (int s = 0; s < NSUM; ++s)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[s] += __shfl_down(v[s], off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int s = 0; s < NSUM; ++s) part[s][wave] = v[s];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int s = 0; s < NSUM; ++s) {
            double t = 0;
            for (int w = 0; w < (int)(blockDim.x / 64); ++w) t += part[s][w];
            out[(size_t)s * gridDim.x + blockIdx.x] = t;
        }
    }
}

// Stage 1 of the global sums: one partial per block for mass, j, 1/2|u|^2.
template <int S>
__global__ __launch_bounds__(256) void k_sums_partial(const typename Codec<S>::store_t* __restrict__ f,
                                                      double* __restrict__ partial, int n) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    double v[5] = {0, 0, 0, 0, 0};
    if (idx < n) {
        double r, ux, uy, uz;
        macro_double<S>(f, n, idx, r, ux, uy, uz);
        v[0] = r;
        v[1] = r * ux;
        v[2] = r * uy;
        v[3] = r * uz;
        v[4] = 0.5 * (ux * ux + uy * uy + uz * uz);
    }
    block_sum<5>(v, partial);
}

// Velocity-dependent forcing phase (Alvelius' rule, Sec. "Training Data -
// Forced Isotropic Turbulence").  Stage 1: per block and forced mode m, the
// partial sums of u(x) exp(-i k_m.x) over the block's nodes, six doubles
// (Re, Im of u_x, u_y, u_z), at partial[(6 m + s) nblocks + block].  A
// thread takes MODE_NPT nodes (coalesced, 256 apart) and keeps their
// velocities in registers; the modes go in chunks of MODE_CHUNK, one block
// reduction per chunk.
constexpr int MODE_NPT = 8, MODE_CHUNK = 8, MODE_BLOCK_NODES = 256 * MODE_NPT;
inline int mode_partial_blocks(int n) { return (n + MODE_BLOCK_NODES - 1) / MODE_BLOCK_NODES; }

template <int S>
__global__ __launch_bounds__(256) void k_mode_partials(const typename Codec<S>::store_t* __restrict__ f, int n,
                                                       int nx, int ny, int nz, const int* __restrict__ fk,
                                                       int n_modes, double* __restrict__ partial) {
    __shared__ double part[6 * MODE_CHUNK][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double u[MODE_NPT][3];
    NodePhasors ph[MODE_NPT];
#pragma unroll
    for (int j = 0; j < MODE_NPT; ++j) {
        const int idx = blockIdx.x * MODE_BLOCK_NODES + j * 256 + threadIdx.x;
        u[j][0] = u[j][1] = u[j][2] = 0.0;
        int x = 0, y = 0, z = 0;
        if (idx < n) {
            double r;
            macro_double<S>(f, n, idx, r, u[j][0], u[j][1], u[j][2]);
            x = idx % nx;
            y = (idx / nx) % ny;
            z = idx / (nx * ny);
        }
        ph[j] = node_phasors(x, y, z, nx, ny, nz);
    }
    for (int m0 = 0; m0 < n_modes; m0 += MODE_CHUNK) {
        double v[MODE_CHUNK][6];
#pragma unroll
        for (int c = 0; c < MODE_CHUNK; ++c) {
#pragma unroll
            for (int q = 0; q < 6; ++q) v[c][q] = 0.0;
            const int m = m0 + c;
            if (m < n_modes) {
                const int* k = fk + 3 * m;
#pragma unroll
                for (int j = 0; j < MODE_NPT; ++j) {
                    const Phasor e = mode_phase(k, ph[j]);
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        v[c][2 * d] += u[j][d] * e.c;
                        v[c][2 * d + 1] -= u[j][d] * e.s;
                    }
                }
            }
        }
#pragma unroll
        for (int c = 0; c < MODE_CHUNK; ++c)
#pragma unroll
            for (int q = 0; q < 6; ++q)
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) v[c][q] += __shfl_down(v[c][q], off, 64);
        if (lane == 0)
#pragma unroll
            for (int c = 0; c < MODE_CHUNK; ++c)
#pragma unroll
                for (int q = 0; q < 6; ++q) part[6 * c + q][wave] = v[c][q];
        __syncthreads();
        if (threadIdx.x < 6 * MODE_CHUNK) {
            const int e = threadIdx.x, m = m0 + e / 6;
            if (m < n_modes)
                partial[(size_t)(6 * m0 + e) * gridDim.x + blockIdx.x] =
                    part[e][0] + part[e][1] + part[e][2] + part[e][3];
        }
        __syncthreads();
    }
}

// Stage 2, one block per mode: u_hat = sum of the partials (fixed order) / N,
// xi_i = u_hat . e_i, Z = g_A conj(xi1) + g_B exp(i psi) conj(xi2),
// theta1 = atan2(Re Z, Im Z) (the force then does no work on the mode), and
// F_hat = |A| (g_A exp(i theta1) e1 + g_B exp(i (theta1 + psi)) e2) into
// fhat[6 m ..] as (Re, Im) of x, y, z.  basis[8 m ..] = e1, e2, |A|;
// draw[2 m ..] = phi, psi of this step.  u_hat goes to uhat[6 m ..] in the
// same layout when uhat is not null (kept for the reverse mode).
__global__ __launch_bounds__(256) void k_force_phase(const double* __restrict__ partial, int nblocks, double inv_n,
                                                     const double* __restrict__ basis,
                                                     const double* __restrict__ draw, double* __restrict__ fhat,
                                                     double* __restrict__ uhat) {
    __shared__ double part[6][4];
    const int m = blockIdx.x;
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
#pragma unroll
        for (int q = 0; q < 6; ++q) v[q] += partial[(size_t)(6 * m + q) * nblocks + b];
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_down(v[q], off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < 6; ++q) part[q][wave] = v[q];
    __syncthreads();
    if (threadIdx.x != 0) return;
    double ur[3], ui[3];
    for (int a = 0; a < 3; ++a) {
        ur[a] = (part[2 * a][0] + part[2 * a][1] + part[2 * a][2] + part[2 * a][3]) * inv_n;
        ui[a] = (part[2 * a + 1][0] + part[2 * a + 1][1] + part[2 * a + 1][2] + part[2 * a + 1][3]) * inv_n;
    }
    const double* e1 = basis + 8 * m;
    const double* e2 = e1 + 3;
    const double mag = e1[6];
    const double x1r = ur[0] * e1[0] + ur[1] * e1[1] + ur[2] * e1[2];
    const double x1i = ui[0] * e1[0] + ui[1] * e1[1] + ui[2] * e1[2];
    const double x2r = ur[0] * e2[0] + ur[1] * e2[1] + ur[2] * e2[2];
    const double x2i = ui[0] * e2[0] + ui[1] * e2[1] + ui[2] * e2[2];
    const double phi = draw[2 * m], psi = draw[2 * m + 1];
    double sp, cp, s2, c2;
    sincos(psi, &sp, &cp);
    sincos(2.0 * phi, &s2, &c2);
    const double ga = s2, gb = c2;
    // Z = ga conj(xi1) + gb (cos psi + i sin psi)(x2r - i x2i).
    const double zr = ga * x1r + gb * (cp * x2r + sp * x2i);
    const double zi = -ga * x1i + gb * (sp * x2r - cp * x2i);
    const double th1 = atan2(zr, zi);
    double s1, c1, s12, c12;
    sincos(th1, &s1, &c1);
    sincos(th1 + psi, &s12, &c12);
    for (int a = 0; a < 3; ++a) {
        fhat[6 * m + 2 * a] = mag * (ga * c1 * e1[a] + gb * c12 * e2[a]);
        fhat[6 * m + 2 * a + 1] = mag * (ga * s1 * e1[a] + gb * s12 * e2[a]);
    }
    if (uhat)
        for (int a = 0; a < 3; ++a) {
            uhat[6 * m + 2 * a] = ur[a];
            uhat[6 * m + 2 * a + 1] = ui[a];
        }
}

// Stage 2: a single block adds the partials in a fixed order.
__global__ __launch_bounds__(256) void k_sums_final(const double* __restrict__ partial, int nblocks,
                                                    double* __restrict__ out) {
    double v[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
#pragma unroll
        for (int s = 0; s < 5; ++s) v[s] += partial[(size_t)s * nblocks + b];
    __shared__ double part[5][4];
#pragma unroll
    for (int s = 0; s < 5; ++s)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[s] += __shfl_down(v[s], off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int s = 0; s < 5; ++s) part[s][wave] = v[s];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int s = 0; s < 5; ++s) out[s] = part[s][0] + part[s][1] + part[s][2] + part[s][3];
}

// Stability check on the float64 global sums (mass, momentum, energy):
// *flag = 1 if any is not finite (a NaN or infinity anywhere in the lattice
// reaches every sum) or the mass has drifted from mass0 by more than
// tol |mass0|.  One thread; a plain store, idempotent.
__global__ void k_check_sums(const double* __restrict__ sums, double mass0, double tol, int* __restrict__ flag) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    bool bad = false;
    for (int s = 0; s < 5; ++s) bad |= !(sums[s] - sums[s] == 0.0);
    bad |= !(fabs(sums[0] - mass0) <= tol * fabs(mass0));
    if (bad) *flag = 1;
}

// Force field of one step, separable in x: with R_m(y, z) = 2 Fhat_m
// e^{i 2 pi (k_y y / ny + k_z z / nz)},
//   F(x, y, z) = sum_kx Re(S_kx(y, z) e^{i 2 pi kx x / nx}),
//   S_kx(y, z) = sum of R_m over the modes m with k_x = kx (in mode order),
// so a node sums 2 kx_max + 1 terms whatever the number of modes.  A block
// serves `rows` consecutive (y, z) rows: its threads first form S for each
// (row, kx) in LDS (one sincospi of an exact fraction per mode and row),
// then each node takes its x phase e^{i 2 pi x / nx} (from an LDS table the
// block fills, one sincospi per x) and the powers up to kx_max by
// products.  float64 throughout.
constexpr int FF_MAX_ROWS = 8;
constexpr int FF_CHUNK = 32;
constexpr int FF_XTAB = 1024;                   // x-phase table in LDS up to this extent

template <typename T>
__global__ __launch_bounds__(256) void k_force_field(StepArgs a, int kx_max, int rows, T* __restrict__ out) {
    __shared__ double2 S[FF_MAX_ROWS][2 * FORCE_KX_MAX + 1][3];
    __shared__ double2 R[FF_MAX_ROWS][FF_CHUNK][3];
    __shared__ int skx[FF_CHUNK];
    __shared__ double2 xph[FF_XTAB];            // e^{i 2 pi x / nx}
    const int row0 = blockIdx.x * rows;
    const int nrows = a.ny * a.nz;
    const int nk = 2 * kx_max + 1;
    if (a.nx <= FF_XTAB)
        for (int x = threadIdx.x; x < a.nx; x += blockDim.x) {
            double sn, cs;
            sincospi(2.0 * (double)x / (double)a.nx, &sn, &cs);
            xph[x] = make_double2(cs, sn);
        }
    for (int e = threadIdx.x; e < rows * nk; e += blockDim.x)
#pragma unroll
        for (int d = 0; d < 3; ++d) S[e / nk][e % nk][d] = make_double2(0.0, 0.0);
    for (int m0 = 0; m0 < a.n_modes; m0 += FF_CHUNK) {
        const int mend = min(FF_CHUNK, a.n_modes - m0);
        // R_m(row) for every (row, mode) of the chunk, one per thread.
        for (int e = threadIdx.x; e < rows * FF_CHUNK; e += blockDim.x) {
            const int rr = e / FF_CHUNK, c = e % FF_CHUNK, m = m0 + c, row = row0 + rr;
            double2 v[3] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
            if (c < mend && row < nrows) {
                const int y = row % a.ny, z = row / a.ny;
                const int* k = a.fk + 3 * m;
                const long py = ((long)k[1] * y) % a.ny, pz = ((long)k[2] * z) % a.nz;
                const double turn = (double)py / a.ny + (double)pz / a.nz;
                double sn, cs;
                sincospi(2.0 * turn, &sn, &cs);
                const double* fh = a.fhat + 6 * m;
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    v[d] = make_double2(2.0 * (fh[2 * d] * cs - fh[2 * d + 1] * sn),
                                        2.0 * (fh[2 * d] * sn + fh[2 * d + 1] * cs));
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) R[rr][c][d] = v[d];
        }
        if (threadIdx.x < FF_CHUNK) skx[threadIdx.x] = (int)threadIdx.x < mend ? a.fk[3 * (m0 + threadIdx.x)] : 0;
        __syncthreads();
        // S_kx += the chunk's modes with that k_x, in mode order.
        for (int e = threadIdx.x; e < rows * nk; e += blockDim.x) {
            const int rr = e / nk, kx = e % nk - kx_max;
            double2 acc[3] = {S[rr][kx + kx_max][0], S[rr][kx + kx_max][1], S[rr][kx + kx_max][2]};
            for (int c = 0; c < mend; ++c)
                if (skx[c] == kx)
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        acc[d].x += R[rr][c][d].x;
                        acc[d].y += R[rr][c][d].y;
                    }
#pragma unroll
            for (int d = 0; d < 3; ++d) S[rr][kx + kx_max][d] = acc[d];
        }
        __syncthreads();
    }
    const int nodes = rows * a.nx;
    for (int local = threadIdx.x; local < nodes; local += blockDim.x) {
        const int r = local / a.nx, x = local - r * a.nx;
        if (row0 + r >= nrows) break;
        double sn, cs;
        if (a.nx <= FF_XTAB) {
            sn = xph[x].y;
            cs = xph[x].x;
        } else {
            sincospi(2.0 * (double)x / (double)a.nx, &sn, &cs);
        }
        double F[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) F[d] = S[r][kx_max][d].x;
        double pc = 1.0, ps = 0.0;                  // e^{i k theta}, k = 1 .. kx_max
        for (int k = 1; k <= kx_max; ++k) {
            const double t = pc * cs - ps * sn;
            ps = pc * sn + ps * cs;
            pc = t;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double2 sp = S[r][kx_max + k][d], sm = S[r][kx_max - k][d];
                // Re(sp e^{i k theta}) + Re(sm e^{-i k theta})
                F[d] += (sp.x + sm.x) * pc - (sp.y - sm.y) * ps;
            }
        }
        const size_t idx = (size_t)row0 * a.nx + local;
#pragma unroll
        for (int d = 0; d < 3; ++d) out[(size_t)d * a.n + idx] = (T)F[d];
    }
}

inline int nblocks(int n) { return (n + 255) / 256; }

template <int S, int OP>
hipError_t launch_step_op(const void* fin, void* fout, const StepArgs& a, hipStream_t st) {
    using T = typename Codec<S>::store_t;
    const T* in = static_cast<const T*>(fin);
    T* out = static_cast<T*>(fout);
    if constexpr (OP == OP_NONE) {
        hipLaunchKernelGGL((k_stream_only<S>), dim3(nblocks(a.n)), dim3(256), 0, st, in, out, a);
    } else if constexpr (OP != OP_NCO) {
        hipLaunchKernelGGL((k_stream_collide<S, OP, 8, ACT_TANH>), dim3(nblocks(a.n)), dim3(256), 0, st, in, out, a);
    } else {
#define NCO_CASE(WW, AA)                                                                               \
    if (a.depth == 2 && a.width == WW && a.act == AA) {                                                \
        hipLaunchKernelGGL((k_stream_collide<S, OP, WW, AA>), dim3(nblocks(a.n)), dim3(256), 0, st, in, \
                           out, a);                                                                    \
        return hipGetLastError();                                                                      \
    }
        // Depth 3 runs at width 32 (narrower networks are zero-padded).
        if (a.depth == 3 && a.width == 32) {
            if (a.act == ACT_TANH)
                hipLaunchKernelGGL((k_stream_collide<S, OP, 32, ACT_TANH, 3>), dim3(nblocks(a.n)), dim3(256), 0, st,
                                   in, out, a);
            else
                hipLaunchKernelGGL((k_stream_collide<S, OP, 32, ACT_RELU, 3>), dim3(nblocks(a.n)), dim3(256), 0, st,
                                   in, out, a);
            return hipGetLastError();
        }
        NCO_CASE(8, ACT_TANH) NCO_CASE(16, ACT_TANH) NCO_CASE(20, ACT_TANH) NCO_CASE(32, ACT_TANH)
        NCO_CASE(8, ACT_RELU) NCO_CASE(16, ACT_RELU) NCO_CASE(20, ACT_RELU) NCO_CASE(32, ACT_RELU)
#undef NCO_CASE
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int S>
hipError_t launch_rates_s(const void* fin, double* out, const StepArgs& a, hipStream_t st) {
    using T = typename Codec<S>::store_t;
    const T* in = static_cast<const T*>(fin);
    if (a.depth == 3 && a.width == 32) {
        if (a.act == ACT_TANH)
            hipLaunchKernelGGL((k_rates<S, 32, ACT_TANH, 3>), dim3(nblocks(a.n)), dim3(256), 0, st, in, out, a);
        else
            hipLaunchKernelGGL((k_rates<S, 32, ACT_RELU, 3>), dim3(nblocks(a.n)), dim3(256), 0, st, in, out, a);
        return hipGetLastError();
    }
#define RATE_CASE(WW, AA)                                                                            \
    if (a.depth == 2 && a.width == WW && a.act == AA) {                                                              \
        hipLaunchKernelGGL((k_rates<S, WW, AA>), dim3(nblocks(a.n)), dim3(256), 0, st, in, out, a); \
        return hipGetLastError();                                                                    \
    }
    RATE_CASE(8, ACT_TANH) RATE_CASE(16, ACT_TANH) RATE_CASE(20, ACT_TANH) RATE_CASE(32, ACT_TANH)
    RATE_CASE(8, ACT_RELU) RATE_CASE(16, ACT_RELU) RATE_CASE(20, ACT_RELU) RATE_CASE(32, ACT_RELU)
#undef RATE_CASE
    return hipErrorInvalidValue;
}

}  // namespace

#define DISPATCH_STORAGE(S, CALL)                \
    switch (S) {                                 \
        case ST_F32: { constexpr int SS = ST_F32; CALL; } \
        case ST_F16: { constexpr int SS = ST_F16; CALL; } \
        case ST_BF16: { constexpr int SS = ST_BF16; CALL; } \
        case ST_F64: { constexpr int SS = ST_F64; CALL; } \
        default: return hipErrorInvalidValue;    \
    }

hipError_t launch_step(int storage, const void* fin, void* fout, const StepArgs& a, hipStream_t st) {
    switch (a.op) {
        case OP_BGK: DISPATCH_STORAGE(storage, return (launch_step_op<SS, OP_BGK>(fin, fout, a, st)))
        case OP_MRT: DISPATCH_STORAGE(storage, return (launch_step_op<SS, OP_MRT>(fin, fout, a, st)))
        case OP_NCO: DISPATCH_STORAGE(storage, return (launch_step_op<SS, OP_NCO>(fin, fout, a, st)))
        case OP_NONE: DISPATCH_STORAGE(storage, return (launch_step_op<SS, OP_NONE>(fin, fout, a, st)))
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step_inplace(int storage, void* f, const StepArgs& a, int phase, hipStream_t st) {
    if (a.domain != DOMAIN_PERIODIC || (a.op != OP_BGK && a.op != OP_MRT) || (phase != 0 && phase != 1))
        return hipErrorInvalidValue;
    const dim3 grid(nblocks(a.n)), block(256);
#define INPLACE(OPV)                                                                                          \
    DISPATCH_STORAGE(storage, {                                                                               \
        using T = typename Codec<SS>::store_t;                                                                \
        if (phase == 0)                                                                                       \
            hipLaunchKernelGGL((k_stream_collide_inplace<SS, OPV, 0>), grid, block, 0, st, static_cast<T*>(f), a); \
        else                                                                                                  \
            hipLaunchKernelGGL((k_stream_collide_inplace<SS, OPV, 1>), grid, block, 0, st, static_cast<T*>(f), a); \
        return hipGetLastError();                                                                             \
    })
    if (a.op == OP_BGK) {
        INPLACE(OP_BGK)
    }
    INPLACE(OP_MRT)
#undef INPLACE
}

hipError_t launch_step_grouped(int storage, int op, const LaunchGroup& g, hipStream_t st) {
    const dim3 grid(g.prefix[g.count]), block(256);
    switch (op) {
        case OP_BGK:
            DISPATCH_STORAGE(storage, {
                hipLaunchKernelGGL((k_stream_collide_grouped<SS, OP_BGK>), grid, block, 0, st, g);
                return hipGetLastError();
            })
        case OP_MRT:
            DISPATCH_STORAGE(storage, {
                hipLaunchKernelGGL((k_stream_collide_grouped<SS, OP_MRT>), grid, block, 0, st, g);
                return hipGetLastError();
            })
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_rates(int storage, const void* fin, double* omega, const StepArgs& a, hipStream_t st) {
    DISPATCH_STORAGE(storage, return launch_rates_s<SS>(fin, omega, a, st))
}

hipError_t launch_init_equilibrium(int storage, void* f, const double* rho, const double* u, int n,
                                   hipStream_t st) {
    DISPATCH_STORAGE(storage, {
        hipLaunchKernelGGL(k_init_equilibrium<SS>, dim3(nblocks(n)), dim3(256), 0, st,
                           static_cast<typename Codec<SS>::store_t*>(f), rho, u, n);
        return hipGetLastError();
    })
}

hipError_t launch_from_double(int storage, void* f, const double* src, int n, hipStream_t st) {
    DISPATCH_STORAGE(storage, {
        hipLaunchKernelGGL(k_from_double<SS>, dim3(nblocks(n)), dim3(256), 0, st,
                           static_cast<typename Codec<SS>::store_t*>(f), src, n);
        return hipGetLastError();
    })
}

hipError_t launch_to_double(int storage, const void* f, double* dst, int n, hipStream_t st) {
    DISPATCH_STORAGE(storage, {
        hipLaunchKernelGGL(k_to_double<SS>, dim3(nblocks(n)), dim3(256), 0, st,
                           static_cast<const typename Codec<SS>::store_t*>(f), dst, n);
        return hipGetLastError();
    })
}

hipError_t launch_macroscopic(int storage, const void* f, double* rho, double* u, int n, hipStream_t st) {
    DISPATCH_STORAGE(storage, {
        hipLaunchKernelGGL(k_macroscopic<SS>, dim3(nblocks(n)), dim3(256), 0, st,
                           static_cast<const typename Codec<SS>::store_t*>(f), rho, u, n);
        return hipGetLastError();
    })
}

hipError_t launch_restrict(int fine_storage, const void* fine, int fnx, int fny, int fnz, int coarse_storage,
                           void* coarse, int cnx, int cny, int cnz, int r, double factor, hipStream_t st) {
    const int cn = cnx * cny * cnz;
#define RESTRICT_TO(SF)                                                                                       \
    DISPATCH_STORAGE(coarse_storage, {                                                                        \
        hipLaunchKernelGGL((k_restrict<SF, SS>), dim3(nblocks(cn)), dim3(256), 0, st,                        \
                           static_cast<const typename Codec<SF>::store_t*>(fine),                            \
                           static_cast<typename Codec<SS>::store_t*>(coarse), fnx, fny, fnz, cnx, cny, cnz, r, \
                           factor);                                                                           \
        return hipGetLastError();                                                                             \
    })
    switch (fine_storage) {
        case ST_F32: RESTRICT_TO(ST_F32)
        case ST_F16: RESTRICT_TO(ST_F16)
        case ST_BF16: RESTRICT_TO(ST_BF16)
        case ST_F64: RESTRICT_TO(ST_F64)
        default: return hipErrorInvalidValue;
    }
#undef RESTRICT_TO
}

int sums_partial_count(int n) { return nblocks(n); }

hipError_t launch_global_sums(int storage, const void* f, double* partial, double* out, int n,
                              hipStream_t st) {
    const int nb = nblocks(n);
    DISPATCH_STORAGE(storage, {
        hipLaunchKernelGGL(k_sums_partial<SS>, dim3(nb), dim3(256), 0, st,
                           static_cast<const typename Codec<SS>::store_t*>(f), partial, n);
        hipLaunchKernelGGL(k_sums_final, dim3(1), dim3(256), 0, st, partial, nb, out);
        return hipGetLastError();
    })
}

hipError_t launch_force_field(const StepArgs& a, int kx_max, float* out32, double* out64, hipStream_t st) {
    if (a.n_modes < 1 || !a.fk || !a.fhat || (!out32 && !out64) || kx_max < 0 || kx_max > FORCE_KX_MAX)
        return hipErrorInvalidValue;
    const int rows = FF_MAX_ROWS;
    const int nrows = a.ny * a.nz;
    const unsigned nb = (unsigned)((nrows + rows - 1) / rows);
    if (out64)
        hipLaunchKernelGGL(k_force_field<double>, dim3(nb), dim3(256), 0, st, a, kx_max, rows, out64);
    else
        hipLaunchKernelGGL(k_force_field<float>, dim3(nb), dim3(256), 0, st, a, kx_max, rows, out32);
    return hipGetLastError();
}

hipError_t launch_force_phase(int storage, const void* f, int n, int nx, int ny, int nz, const int* fk,
                              int n_modes, double* partial, const double* basis, const double* draw, double* fhat,
                              double* uhat, hipStream_t st) {
    const int nb = mode_partial_blocks(n);
    DISPATCH_STORAGE(storage, {
        hipLaunchKernelGGL(k_mode_partials<SS>, dim3(nb), dim3(256), 0, st,
                           static_cast<const typename Codec<SS>::store_t*>(f), n, nx, ny, nz, fk, n_modes, partial);
        if (hipError_t e = hipGetLastError()) return e;
        hipLaunchKernelGGL(k_force_phase, dim3(n_modes), dim3(256), 0, st, partial, nb, 1.0 / n, basis, draw,
                           fhat, uhat);
        return hipGetLastError();
    })
}

hipError_t launch_check_state(int storage, const void* f, double* partial, double* sums, int n, double mass0,
                              double tol, int* flag, hipStream_t st) {
    if (hipError_t e = launch_global_sums(storage, f, partial, sums, n, st)) return e;
    hipLaunchKernelGGL(k_check_sums, dim3(1), dim3(64), 0, st, sums, mass0, tol, flag);
    return hipGetLastError();
}

}  // namespace nco
