// Adjoint (reverse mode) of one stream-collide step with the NCO collision.
//
// The forward step is y = stream(x_t) (pull), x_t+1 = y - M^{-1} dm(y; theta)
// with dm = S (m - m^eq) - dm_source (Eq. omegatheta, Kupershtokh source of
// Sec. II.A).  Given lambda = dL/dx_t+1 at every node, this kernel computes,
// per node, the pre-collision adjoint
//     lambda_y = lambda + M^T g_m,   g_m = (d dm / d m)^T nu,  nu = -M^{-T} lambda,
// including the path through the rates omega_n(theta, m) of the invariant
// network (Eq. gconv_m and the sigmoid squashing), and scatters it back along
// the streaming direction: dL/dx_t,i(x - c_i) = lambda_y,i(x).  The network
// is re-evaluated per node and group element (no activations are stored);
// its parameter gradient
//     dL/dW1 = sum_(nodes, g) x_g dz1^T, dL/dW2 = sum h1 dz2^T, ...
// is reduced over the 64 nodes of a block in LDS, each lane owning a fixed
// block of gradient entries, and written as one partial per block; a second
// kernel adds the partials in a fixed order (deterministic, no atomics).
#include "adjoint.h"
#include "kernels.h"
#include "stream.h"

namespace nco {

namespace {

// DEPTH = 3: a third hidden layer (W2b, b2b) between the second and the
// output layer; its gradient goes to the tail OFF_W2B, OFF_B2B of a partial
// row of NPAR3 values.
//
// A block holds 64 nodes (one per lane) and SPLIT wavefronts.  Wavefront w
// takes the group elements w G .. w G + G - 1, G = 48 / SPLIT (without the
// split over blocks below), of every node in both passes, with its own LDS
// rows, so the serial chain of one lane is G group elements instead of 48.  The per-node parts (the group
// sum of pass 1, the collision adjoint) are formed from the wavefronts'
// partial sums in a fixed order; every wavefront writes its own partial
// gradient row, and wavefront 0 scatters dL/dx.
//
// On lattices too small to fill the device the group elements are also
// split over gridDim.y blocks per 64 nodes (MODE != ADJ_WHOLE), in three
// launches that exchange through xwork: ADJ_SUMS writes each block's share
// of the group sum of pass 1 ([gridDim.y][n][W]); ADJ_MAIN adds the shares
// in block order, runs pass 2 on its own elements and writes its share of
// the network's dL/dm ([gridDim.y][27][n], paper row order), the blocks with
// blockIdx.y = 0 also the collision's part of dL/dx before streaming
// ([27][n]); k_adjoint_finish adds the shares in order and scatters.
// Block (x, y) wavefront w takes the group elements from
// (y SPLIT + w) Gw, Gw = 48 / (gridDim.y SPLIT), and writes gradient row
// (y gridDim.x + x) SPLIT + w.
constexpr int ADJ_WHOLE = 0, ADJ_SUMS = 1, ADJ_MAIN = 2;

typedef const __attribute__((address_space(4))) float cfloat;

template <int S, int ACT, int DEPTH, int SPLIT, int MODE = ADJ_WHOLE>
__global__ __launch_bounds__(64 * SPLIT) void k_adjoint(const typename Codec<S>::store_t* __restrict__ xin,
                                                const float* __restrict__ lam_in, float* __restrict__ lam_out,
                                                StepArgs a, const int* __restrict__ gsrc,
                                                float* __restrict__ partial, float* __restrict__ xwork) {
    constexpr int W = AW;
    constexpr int ROW = DEPTH == 3 ? NPAR3 : NPAR;
    static_assert(NGROUP % SPLIT == 0, "the group elements split evenly over the wavefronts");
    const int GY = gridDim.y, gy = blockIdx.y;
    const int G = NGROUP / (SPLIT * GY);        // group elements per wavefront
    const int g0 = (gy * SPLIT + (int)(threadIdx.x >> 6)) * G;
    // Network (unstacked W1 [27][W], b1, W2 [W][W], b2, W3 [W][4], b3), read
    // by every lane at the same address: through the constant address space,
    // so that the weights come by scalar loads into scalar registers and feed
    // the FMAs directly (no LDS traffic, no vector registers).
    const float* const net = a.net;
    cfloat* __restrict__ c_w1 = (cfloat*)net;     // the identity element's slice
    cfloat* __restrict__ c_b1 = (cfloat*)(net + net_off_b1(W));
    cfloat* __restrict__ c_w2 = (cfloat*)(net + net_off_w2(W));
    cfloat* __restrict__ c_b2 = (cfloat*)(net + net_off_b2(W));
    cfloat* __restrict__ c_w3 = (cfloat*)(net + net_off_w3(W));
    cfloat* __restrict__ c_b3 = (cfloat*)(net + net_off_b3(W));
    cfloat* __restrict__ c_w2b = (cfloat*)(net + net_off_w2b(W));
    cfloat* __restrict__ c_b2b = (cfloat*)(net + net_off_b2b(W));
    // Per-node rows: moments (paper order, [27] = 1); per wavefront dL/dm
    // and the vectors of the current group element for the parameter-
    // gradient reduction: h1, dz2 and dz1 (at depth 3 the last two rows hold
    // h2 and dz3 first, for the third layer's reduction).
    __shared__ float s_m[64][28];
    __shared__ float s_dm[SPLIT][64][27];
    __shared__ float s_h1[SPLIT][64][W];
    __shared__ float s_d1[SPLIT][64][W];
    __shared__ float s_d2[SPLIT][64][W];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int idx = blockIdx.x * 64 + lane;
    const bool live = idx < a.n;
    // Forward quantities of the node: pulled populations and moments (one
    // wavefront pulls; the others read the moments back).
    float m[Q];
    const NodeIdx p = node_of(live ? idx : 0, a.nx, a.ny);
    if (wave == 0) {
        float f[Q];
        if (live) {
            pull<S>(xin, a, p, f);
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i) f[i] = (float)weight_of(i);
        }
        to_moments(f, m);
#pragma unroll
        for (int k = 0; k < Q; ++k) s_m[lane][k] = m[row_tensor(k)];
        s_m[lane][27] = 1.0f;
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) s_dm[wave][lane][k] = 0.0f;
    __syncthreads();
    if (wave != 0) {
#pragma unroll
        for (int k = 0; k < Q; ++k) m[row_tensor(k)] = s_m[lane][k];
    }

    // Pass 1: network forward for the rates; sum over g of act(z2), this
    // wavefront's share first.
    float S2[W];
#pragma unroll
    for (int o = 0; o < W; ++o) S2[o] = 0.0f;
#pragma unroll 1
    for (int g = g0; g < (MODE == ADJ_MAIN ? g0 : g0 + G); ++g) {
        const int* __restrict__ gs = gsrc + g * 27;
        float h[W];
#pragma unroll
        for (int j = 0; j < W; ++j) h[j] = c_b1[j];
#pragma unroll 3
        for (int k = 0; k < Q; ++k) {
            const int e = gs[k];
            const float xk = __int_as_float(__float_as_int(s_m[lane][e & 31]) ^ (e & (int)0x80000000));
#pragma unroll
            for (int j = 0; j < W; ++j) h[j] = fmaf(c_w1[k * W + j], xk, h[j]);
        }
        float z[W];
#pragma unroll
        for (int o = 0; o < W; ++o) z[o] = c_b2[o];
#pragma unroll 4
        for (int j = 0; j < W; ++j) {
            const float hj = act_f<ACT>(h[j]);
#pragma unroll
            for (int o = 0; o < W; ++o) z[o] = fmaf(c_w2[j * W + o], hj, z[o]);
        }
        if constexpr (DEPTH == 2) {
#pragma unroll
            for (int o = 0; o < W; ++o) S2[o] += act_f<ACT>(z[o]);
        } else {
            float z3[W];
#pragma unroll
            for (int o = 0; o < W; ++o) z3[o] = c_b2b[o];
#pragma unroll 4
            for (int j = 0; j < W; ++j) {
                const float hj = act_f<ACT>(z[j]);
#pragma unroll
                for (int o = 0; o < W; ++o) z3[o] = fmaf(c_w2b[j * W + o], hj, z3[o]);
            }
#pragma unroll
            for (int o = 0; o < W; ++o) S2[o] += act_f<ACT>(z3[o]);
        }
    }
    if constexpr (SPLIT > 1 && MODE != ADJ_MAIN) {
        // The block's group sum, in wavefront order (every wavefront the same).
#pragma unroll
        for (int o = 0; o < W; ++o) s_h1[wave][lane][o] = S2[o];
        __syncthreads();
#pragma unroll
        for (int o = 0; o < W; ++o) {
            float t = s_h1[0][lane][o];
#pragma unroll
            for (int w = 1; w < SPLIT; ++w) t += s_h1[w][lane][o];
            S2[o] = t;
        }
        __syncthreads();
    }
    if constexpr (MODE == ADJ_SUMS) {
        if (wave == 0 && live)
#pragma unroll
            for (int o = 0; o < W; ++o) xwork[((size_t)gy * a.n + idx) * W + o] = S2[o];
        return;
    }
    if constexpr (MODE == ADJ_MAIN) {
        // The full group sum: the blocks' shares in block order.
        if (live)
            for (int y = 0; y < GY; ++y)
#pragma unroll
                for (int o = 0; o < W; ++o) S2[o] += xwork[((size_t)y * a.n + idx) * W + o];
    }
    float tt[4], omega[4], tau[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        float t = 0.0f;
#pragma unroll
        for (int o = 0; o < W; ++o) t = fmaf(c_w3[o * 4 + n], S2[o], t);
        tt[n] = t * (1.0f / NGROUP) + c_b3[n];
        tau[n] = 0.5f + 0.5f / (1.0f + expf(tt[n]));
        omega[n] = 1.0f / tau[n];
    }

    // Adjoint of dm: nu = dL/d(dm) = -M^{-T} lambda.
    float lam[Q], nu[Q];
    if (live) {
#pragma unroll
        for (int i = 0; i < Q; ++i) lam[i] = lam_in[(size_t)i * a.n + idx];
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) lam[i] = 0.0f;
    }
    inverse_T(lam, nu);
    float gm[Q];
    float domega[4];
    float F[3] = {0.0f, 0.0f, 0.0f};
    if (a.n_modes > 0 && live) read_force(a, idx, F[0], F[1], F[2]);
    collision_vjp_local(m, nu, a.omega_nu_f, omega, a.n_modes > 0, F, gm, domega);
    // Through the squashing: omega = 1 / tau, tau = 1/2 + 1/(2 (1 + e^t)).
    float dtt[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const float e = expf(tt[n]);
        dtt[n] = domega[n] * 0.5f * e / ((1.0f + e) * (1.0f + e) * tau[n] * tau[n]);
    }
    // The output layer's adjoint is the same for every group element.
    float dh2[W];
#pragma unroll
    for (int o = 0; o < W; ++o) {
        float s = 0.0f;
#pragma unroll
        for (int n = 0; n < 4; ++n) s = fmaf(c_w3[o * 4 + n], dtt[n], s);
        dh2[o] = s * (1.0f / NGROUP);
    }

    // Gradient accumulators owned by this lane.
    const int r1 = 7 * (lane >> 4), c1 = 2 * (lane & 15);        // W1 rows r1..r1+6 (27 = b1), cols c1, c1+1
    const int r2 = 4 * (lane >> 3), c2 = 4 * (lane & 7);         // W2 rows r2..r2+3, cols c2..c2+3
    float acc1[7][2], acc2[4][4], accb2 = 0.0f;
    // Depth 3: W2b rows r2..r2+3, cols c2..c2+3 in acc3; lanes 32..63 own b2b.
    float acc3[4][4], accb2b = 0.0f;
#pragma unroll
    for (int i = 0; i < 7; ++i) acc1[i][0] = acc1[i][1] = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc2[i][j] = acc3[i][j] = 0.0f;

    // Pass 2: per group element, recompute, back-propagate, reduce.
#pragma unroll 1
    for (int g = g0; g < g0 + G; ++g) {
        const int* __restrict__ gs = gsrc + g * 27;
        float h1[W];
#pragma unroll
        for (int j = 0; j < W; ++j) h1[j] = c_b1[j];
#pragma unroll 3
        for (int k = 0; k < Q; ++k) {
            const int e = gs[k];
            const float xk = __int_as_float(__float_as_int(s_m[lane][e & 31]) ^ (e & (int)0x80000000));
#pragma unroll
            for (int j = 0; j < W; ++j) h1[j] = fmaf(c_w1[k * W + j], xk, h1[j]);
        }
#pragma unroll
        for (int j = 0; j < W; ++j) {
            h1[j] = act_f<ACT>(h1[j]);
            s_h1[wave][lane][j] = h1[j];
        }
        float dz2[W];
#pragma unroll
        for (int o = 0; o < W; ++o) dz2[o] = c_b2[o];
#pragma unroll 4
        for (int j = 0; j < W; ++j)
#pragma unroll
            for (int o = 0; o < W; ++o) dz2[o] = fmaf(c_w2[j * W + o], h1[j], dz2[o]);
        if constexpr (DEPTH == 2) {
#pragma unroll
            for (int o = 0; o < W; ++o) {
                dz2[o] = dh2[o] * act_d<ACT>(act_f<ACT>(dz2[o]));
                s_d2[wave][lane][o] = dz2[o];
            }
        } else {
            // h2 = act(z2); z3 = W2b^T h2 + b2b; dz3 = dh3 act'(z3) with dh3
            // the output layer's adjoint (dh2 above); dz2 = (W2b dz3) act'(z2).
            // h2 and dz3 go through the dz2 and dz1 rows, reduced into the
            // third layer's gradient before dz2 and dz1 take their place.
#pragma unroll
            for (int o = 0; o < W; ++o) {
                dz2[o] = act_f<ACT>(dz2[o]);
                s_d2[wave][lane][o] = dz2[o];
            }
            float dz3[W];
#pragma unroll
            for (int o = 0; o < W; ++o) dz3[o] = c_b2b[o];
#pragma unroll 4
            for (int j = 0; j < W; ++j)
#pragma unroll
                for (int o = 0; o < W; ++o) dz3[o] = fmaf(c_w2b[j * W + o], dz2[j], dz3[o]);
#pragma unroll
            for (int o = 0; o < W; ++o) {
                dz3[o] = dh2[o] * act_d<ACT>(act_f<ACT>(dz3[o]));
                s_d1[wave][lane][o] = dz3[o];
            }
            // Only this wavefront's rows are exchanged: a wavefront barrier.
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 4
            for (int nd = 0; nd < 64; ++nd) {
                float h2v[4], d3v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) h2v[i] = s_d2[wave][nd][r2 + i];
#pragma unroll
                for (int c = 0; c < 4; ++c) d3v[c] = s_d1[wave][nd][c2 + c];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc3[i][c] = fmaf(h2v[i], d3v[c], acc3[i][c]);
                if (lane >= 64 - W) accb2b += s_d1[wave][nd][lane - (64 - W)];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 4
            for (int j = 0; j < W; ++j) {
                float t = 0.0f;
#pragma unroll
                for (int o = 0; o < W; ++o) t = fmaf(c_w2b[j * W + o], dz3[o], t);
                dz2[j] = t * act_d<ACT>(dz2[j]);       // dz2[j] held h2[j]
                s_d2[wave][lane][j] = dz2[j];
            }
        }
        float dz1[W];
#pragma unroll 4
        for (int j = 0; j < W; ++j) {
            float s = 0.0f;
#pragma unroll
            for (int o = 0; o < W; ++o) s = fmaf(c_w2[j * W + o], dz2[o], s);
            dz1[j] = s * act_d<ACT>(s_h1[wave][lane][j]);
            s_d1[wave][lane][j] = dz1[j];
        }
        // dL/dm^(g) = W1 dz1, scattered back through the signed permutation.
#pragma unroll 3
        for (int k = 0; k < Q; ++k) {
            float s = 0.0f;
#pragma unroll
            for (int j = 0; j < W; ++j) s = fmaf(c_w1[k * W + j], dz1[j], s);
            const int e = gs[k];
            s_dm[wave][lane][e & 31] += __int_as_float(__float_as_int(s) ^ (e & (int)0x80000000));
        }
        // Only this wavefront's rows are exchanged: a wavefront barrier.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // Block reduction of this group element's parameter gradients.
        int er[7];
#pragma unroll
        for (int i = 0; i < 7; ++i) er[i] = r1 + i < 27 ? gs[r1 + i] : 27;
#pragma unroll 4
        for (int nd = 0; nd < 64; ++nd) {
            float xv[7], hv[4], d1v[2], d2v[4];
#pragma unroll
            for (int i = 0; i < 7; ++i)
                xv[i] = r1 + i < 28
                            ? __int_as_float(__float_as_int(s_m[nd][er[i] & 31]) ^ (er[i] & (int)0x80000000))
                            : 0.0f;
#pragma unroll
            for (int c = 0; c < 2; ++c) d1v[c] = s_d1[wave][nd][c1 + c];
#pragma unroll
            for (int i = 0; i < 4; ++i) hv[i] = s_h1[wave][nd][r2 + i];
#pragma unroll
            for (int c = 0; c < 4; ++c) d2v[c] = s_d2[wave][nd][c2 + c];
#pragma unroll
            for (int i = 0; i < 7; ++i)
#pragma unroll
                for (int c = 0; c < 2; ++c) acc1[i][c] = fmaf(xv[i], d1v[c], acc1[i][c]);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc2[i][c] = fmaf(hv[i], d2v[c], acc2[i][c]);
            if (lane < W) accb2 += s_d2[wave][nd][lane];
        }
        // Only this wavefront's rows are exchanged: a wavefront barrier.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    // dL/dy = lambda + M^T g_m, with the network's share of g_m from the
    // wavefronts' s_dm rows (in wavefront order); wavefront 0 scatters.
    __syncthreads();
    float* __restrict__ out = partial + (((size_t)gy * gridDim.x + blockIdx.x) * SPLIT + wave) * ROW;
    if (wave == 0) {
        if constexpr (MODE == ADJ_MAIN) {
            // This block's share of the network's dL/dm; the collision's part
            // of dL/dx before streaming from the first block of the node.
            if (live) {
                float* __restrict__ dmo = xwork + (size_t)GY * a.n * W + (size_t)gy * Q * a.n + idx;
#pragma unroll
                for (int k = 0; k < Q; ++k) {
                    float t = s_dm[0][lane][k];
#pragma unroll
                    for (int w = 1; w < SPLIT; ++w) t += s_dm[w][lane][k];
                    dmo[(size_t)k * a.n] = t;
                }
                if (gy == 0) {
                    float gf[Q];
                    moments_T(gm, gf);
                    float* __restrict__ v0 = xwork + (size_t)GY * a.n * (W + Q) + idx;
#pragma unroll
                    for (int i = 0; i < Q; ++i) v0[(size_t)i * a.n] = lam[i] + gf[i];
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                float t = s_dm[0][lane][k];
#pragma unroll
                for (int w = 1; w < SPLIT; ++w) t += s_dm[w][lane][k];
                gm[row_tensor(k)] += t;
            }
            float gf[Q];
            moments_T(gm, gf);
            // Scatter back along the streaming: the slot the pull read.
            if (live) {
                float v[Q];
#pragma unroll
                for (int i = 0; i < Q; ++i) v[i] = lam[i] + gf[i];
                scatter_to_sources(lam_out, a, p, v);
            }
        }
    }
    if (wave == 0 && gy == 0) {

        // Output-layer gradients: dW3 = sum (S2/48) dtt^T, db3 = sum dtt.
#pragma unroll
        for (int o = 0; o < W; ++o) s_h1[0][lane][o] = S2[o] * (1.0f / NGROUP);
#pragma unroll
        for (int n = 0; n < 4; ++n) s_d2[0][lane][n] = dtt[n];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float w3a = 0.0f, w3b = 0.0f, b3a = 0.0f;
        const int e0 = 2 * lane, e1 = 2 * lane + 1;              // W3 entries [o][n] = e / 4, e % 4
        for (int nd = 0; nd < 64; ++nd) {
            w3a = fmaf(s_h1[0][nd][e0 >> 2], s_d2[0][nd][e0 & 3], w3a);
            w3b = fmaf(s_h1[0][nd][e1 >> 2], s_d2[0][nd][e1 & 3], w3b);
            if (lane < 4) b3a += s_d2[0][nd][lane];
        }
        out[OFF_W3 + e0] = w3a;
        out[OFF_W3 + e1] = w3b;
        if (lane < 4) out[OFF_B3 + lane] = b3a;
    } else {
        // The output layer's gradient is that of wavefront 0 of the first block.
        out[OFF_W3 + 2 * lane] = 0.0f;
        out[OFF_W3 + 2 * lane + 1] = 0.0f;
        if (lane < 4) out[OFF_B3 + lane] = 0.0f;
    }
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        const int r = r1 + i;
        if (r < 27) {
            out[OFF_W1 + r * W + c1] = acc1[i][0];
            out[OFF_W1 + r * W + c1 + 1] = acc1[i][1];
        } else if (r == 27) {
            out[OFF_B1 + c1] = acc1[i][0];
            out[OFF_B1 + c1 + 1] = acc1[i][1];
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 4; ++c) out[OFF_W2 + (r2 + i) * W + c2 + c] = acc2[i][c];
    if (lane < W) out[OFF_B2 + lane] = accb2;
    if constexpr (DEPTH == 3) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int c = 0; c < 4; ++c) out[OFF_W2B + (r2 + i) * W + c2 + c] = acc3[i][c];
        if (lane >= 64 - W) out[OFF_B2B + lane - (64 - W)] = accb2b;
    }
}


// grad[p] += sum over blocks of partial[b][p] (rows of npar), in block
// order, in float64.
// The split reverse step's last part: dL/dx before streaming is the
// collision's part plus M^T of the network's dL/dm (the blocks' shares
// added in order), scattered back along the streaming.
__global__ __launch_bounds__(64) void k_adjoint_finish(float* __restrict__ lam_out, StepArgs a, int gy_count,
                                                        const float* __restrict__ xwork) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.n) return;
    const float* __restrict__ dm = xwork + (size_t)gy_count * a.n * AW + idx;     // [gy][27][n]
    const float* __restrict__ v0 = xwork + (size_t)gy_count * a.n * (AW + Q) + idx;  // [27][n]
    float gm[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        float t = dm[(size_t)k * a.n];
        for (int y = 1; y < gy_count; ++y) t += dm[((size_t)y * Q + k) * a.n];
        gm[row_tensor(k)] = t;
    }
    float gf[Q], v[Q];
    moments_T(gm, gf);
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = v0[(size_t)i * a.n] + gf[i];
    scatter_to_sources(lam_out, a, node_of(idx, a.nx, a.ny), v);
}

// grad[p] += sum over the rows of partial[row][p], in a fixed order: a block
// takes 8 parameters, its 32 row slices (rows s, s + 32, ...) are summed by
// 32 threads each, then the slices in order.  Many partial rows (the split
// reverse step of small lattices writes thousands) are spread over 256
// threads per 8 parameters instead of one thread per parameter.
__global__ __launch_bounds__(256) void k_grad_reduce(const float* __restrict__ partial, int nrows, int npar,
                                                     double* __restrict__ grad) {
    const int pl = threadIdx.x & 7, sl = threadIdx.x >> 3;
    const int pidx = blockIdx.x * 8 + pl;
    double s = 0.0;
    if (pidx < npar)
        for (int b = sl; b < nrows; b += 32) s += (double)partial[(size_t)b * npar + pidx];
    __shared__ double red[32][8];
    red[sl][pl] = s;
    __syncthreads();
    if (threadIdx.x < 8 && blockIdx.x * 8 + (int)threadIdx.x < npar) {
        double t = 0.0;
        for (int k = 0; k < 32; ++k) t += red[k][threadIdx.x];
        grad[blockIdx.x * 8 + threadIdx.x] += t;
    }
}

// stage[g][p] = sum of partial[64 g .. 64 g + 63][p] in row order.
__global__ __launch_bounds__(256) void k_grad_stage(const double* __restrict__ partial, int nblocks,
                                                    double* __restrict__ stage) {
    const int pidx = blockIdx.x * blockDim.x + threadIdx.x;
    if (pidx >= NPAR) return;
    const int g = blockIdx.y, b0 = 64 * g, b1 = min(nblocks, b0 + 64);
    double s = 0.0;
    for (int b = b0; b < b1; ++b) s += partial[(size_t)b * NPAR + pidx];
    stage[(size_t)g * NPAR + pidx] = s;
}

__global__ __launch_bounds__(256) void k_grad_final(const double* __restrict__ stage, int ngroups,
                                                    double* __restrict__ grad) {
    const int pidx = blockIdx.x * blockDim.x + threadIdx.x;
    if (pidx >= NPAR) return;
    double s = 0.0;
    for (int g = 0; g < ngroups; ++g) s += stage[(size_t)g * NPAR + pidx];
    grad[pidx] = s;
}

// lam_i(x) += coef (u . c_i - |u|^2) / rho: coef times the derivative of
// rho |u|^2 / (2 rho^2) summed over nodes, i.e. of N k with k = <|u|^2> / 2.
template <int S>
__global__ __launch_bounds__(256) void k_add_energy_grad(const typename Codec<S>::store_t* __restrict__ f,
                                                         float* __restrict__ lam, double coef, int n) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    double fv[Q], rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        fv[i] = Codec<S>::to_double(f[(size_t)i * n + idx], i);
        rho += fv[i];
        jx += cx_of(i) * fv[i];
        jy += cy_of(i) * fv[i];
        jz += cz_of(i) * fv[i];
    }
    const double ux = jx / rho, uy = jy / rho, uz = jz / rho, uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double uc = cx_of(i) * ux + cy_of(i) * uy + cz_of(i) * uz;
        lam[(size_t)i * n + idx] += (float)(coef * (uc - uu) / rho);
    }
}

// Reverse mode of the velocity-dependent forcing phase (Alvelius' rule,
// Sec. "Training Data - Forced Isotropic Turbulence").  The force of a step is
// F(x) = sum_m 2 Re(F_hat_m e^{i k_m.x}) with F_hat_m a function of the
// velocity modes u_hat_m of the state x_t the step starts from.  Given
// lambda = dL/dx_t+1, the extra term of dL/dx_t runs in three kernels.
//
// Stage 1, per collision node: g = dL/dF = (dS/dF)^T lambda for the exact-
// difference source S = f^eq(rho, j + F) - f^eq(rho, j) of the pulled
// populations (the forward adds the same source in moment form):
//     g_a = sum_i lambda_i w_i (3 c_ia + 9 (c_i . v) c_ia / rho) - 3 v_a / rho sum_i lambda_i w_i,
// v = j + F; then per block and forced mode the partial sums of
// (g cos(k.x), -g sin(k.x)), six doubles at partial[(6 m + q) nblocks + block].
// A thread takes FA_NPT nodes (256 apart) and the modes go in chunks of
// FA_CHUNK, one block reduction per chunk.
constexpr int FA_NPT = 4, FA_CHUNK = 8, FA_BLOCK_NODES = 256 * FA_NPT;

template <int S>
__global__ __launch_bounds__(256) void k_force_adj_partials(const typename Codec<S>::store_t* __restrict__ xin,
                                                            const float* __restrict__ lam, StepArgs a,
                                                            double* __restrict__ partial) {
    __shared__ double part[6 * FA_CHUNK][4];
    double g[FA_NPT][3];
    NodePhasors ph[FA_NPT];
#pragma unroll
    for (int j = 0; j < FA_NPT; ++j) {
        const int idx = blockIdx.x * FA_BLOCK_NODES + j * 256 + threadIdx.x;
        g[j][0] = g[j][1] = g[j][2] = 0.0;
        ph[j] = node_phasors(0, 0, 0, a.nx, a.ny, a.nz);
        if (idx < a.n) {
            const NodeIdx p = node_of(idx, a.nx, a.ny);
            ph[j] = node_phasors(p.x, p.y, p.z, a.nx, a.ny, a.nz);
            typename Codec<S>::real f[Q];
            pull<S>(xin, a, p, f);
            double rho = 0.0, jm[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const double v = (double)f[i];
                rho += v;
                jm[0] += cx_of(i) * v;
                jm[1] += cy_of(i) * v;
                jm[2] += cz_of(i) * v;
            }
            double F[3];
            read_force(a, idx, F[0], F[1], F[2]);
            const double v[3] = {jm[0] + F[0], jm[1] + F[1], jm[2] + F[2]};
            const double inv_rho = 1.0 / rho;
            double s0 = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const double lw = (double)lam[(size_t)i * a.n + idx] * weight_of(i);
                const double cv = cx_of(i) * v[0] + cy_of(i) * v[1] + cz_of(i) * v[2];
                const double t = lw * (3.0 + 9.0 * cv * inv_rho);
                g[j][0] += cx_of(i) * t;
                g[j][1] += cy_of(i) * t;
                g[j][2] += cz_of(i) * t;
                s0 += lw;
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) g[j][c] -= 3.0 * v[c] * inv_rho * s0;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int m0 = 0; m0 < a.n_modes; m0 += FA_CHUNK) {
        double q6[FA_CHUNK][6];
#pragma unroll
        for (int c = 0; c < FA_CHUNK; ++c) {
#pragma unroll
            for (int q = 0; q < 6; ++q) q6[c][q] = 0.0;
            const int m = m0 + c;
            if (m < a.n_modes) {
                const int* k = a.fk + 3 * m;
#pragma unroll
                for (int j = 0; j < FA_NPT; ++j) {
                    const Phasor e = mode_phase(k, ph[j]);
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        q6[c][2 * d] += g[j][d] * e.c;
                        q6[c][2 * d + 1] -= g[j][d] * e.s;
                    }
                }
            }
        }
#pragma unroll
        for (int c = 0; c < FA_CHUNK; ++c)
#pragma unroll
            for (int q = 0; q < 6; ++q)
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) q6[c][q] += __shfl_down(q6[c][q], off, 64);
        if (lane == 0)
#pragma unroll
            for (int c = 0; c < FA_CHUNK; ++c)
#pragma unroll
                for (int q = 0; q < 6; ++q) part[6 * c + q][wave] = q6[c][q];
        __syncthreads();
        if (threadIdx.x < 6 * FA_CHUNK) {
            const int e = threadIdx.x, m = m0 + e / 6;
            if (m < a.n_modes)
                partial[(size_t)(6 * m0 + e) * gridDim.x + blockIdx.x] =
                    part[e][0] + part[e][1] + part[e][2] + part[e][3];
        }
        __syncthreads();
    }
}

// Stage 2, one block per mode: dL/dF_hat = 2 x (sum of the partials, fixed
// order), then backwards through the phase rule with this step's F_hat and
// u_hat: dF_hat/d theta1 = i F_hat; theta1 = atan2(Re Z, Im Z) has gradient
// (Im Z, -Re Z) / |Z|^2 (zero where Z = 0); Z = g_A conj(xi1) + g_B e^{i psi}
// conj(xi2) and xi_i = u_hat . e_i are real-linear in u_hat.  Writes
// dL/du_hat / N as (Re, Im) of x, y, z to duhat[6 m ..].
__global__ __launch_bounds__(256) void k_force_phase_adj(const double* __restrict__ partial, int nblocks, double inv_n,
                                                         const double* __restrict__ basis,
                                                         const double* __restrict__ draw,
                                                         const double* __restrict__ fhat,
                                                         const double* __restrict__ uhat, double* __restrict__ duhat) {
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
    // dL/d Re F_hat_a and dL/d Im F_hat_a.
    double gr[3], gi[3];
    for (int c = 0; c < 3; ++c) {
        gr[c] = 2.0 * (part[2 * c][0] + part[2 * c][1] + part[2 * c][2] + part[2 * c][3]);
        gi[c] = 2.0 * (part[2 * c + 1][0] + part[2 * c + 1][1] + part[2 * c + 1][2] + part[2 * c + 1][3]);
    }
    const double* fh = fhat + 6 * m;
    const double* uh = uhat + 6 * m;
    double d_th1 = 0.0;
    for (int c = 0; c < 3; ++c) d_th1 += -gr[c] * fh[2 * c + 1] + gi[c] * fh[2 * c];
    const double* e1 = basis + 8 * m;
    const double* e2 = e1 + 3;
    const double x1r = uh[0] * e1[0] + uh[2] * e1[1] + uh[4] * e1[2];
    const double x1i = uh[1] * e1[0] + uh[3] * e1[1] + uh[5] * e1[2];
    const double x2r = uh[0] * e2[0] + uh[2] * e2[1] + uh[4] * e2[2];
    const double x2i = uh[1] * e2[0] + uh[3] * e2[1] + uh[5] * e2[2];
    const double phi = draw[2 * m], psi = draw[2 * m + 1];
    double sp, cp, s2, c2;
    sincos(psi, &sp, &cp);
    sincos(2.0 * phi, &s2, &c2);
    const double ga = s2, gb = c2;
    const double zr = ga * x1r + gb * (cp * x2r + sp * x2i);
    const double zi = -ga * x1i + gb * (sp * x2r - cp * x2i);
    const double z2 = zr * zr + zi * zi;
    double dzr = 0.0, dzi = 0.0;
    if (z2 > 0.0) {
        dzr = d_th1 * zi / z2;
        dzi = -d_th1 * zr / z2;
    }
    const double d1r = ga * dzr, d1i = -ga * dzi;
    const double d2r = gb * (cp * dzr + sp * dzi), d2i = gb * (sp * dzr - cp * dzi);
    for (int c = 0; c < 3; ++c) {
        duhat[6 * m + 2 * c] = (d1r * e1[c] + d2r * e2[c]) * inv_n;
        duhat[6 * m + 2 * c + 1] = (d1i * e1[c] + d2i * e2[c]) * inv_n;
    }
}

// Stage 3, per node of x_t: dL/du = sum_m (duhat_re cos(k.x) - duhat_im
// sin(k.x)), and through u = j / rho of the stored populations,
// lam_i += (c_i . dL/du - u . dL/du) / rho.
template <int S>
__global__ __launch_bounds__(256) void k_add_velocity_grad(const typename Codec<S>::store_t* __restrict__ x,
                                                           float* __restrict__ lam, StepArgs a,
                                                           const double* __restrict__ duhat) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.n) return;
    const NodeIdx p = node_of(idx, a.nx, a.ny);
    const NodePhasors ph = node_phasors(p.x, p.y, p.z, a.nx, a.ny, a.nz);
    double du[3] = {0.0, 0.0, 0.0};
    for (int m = 0; m < a.n_modes; ++m) {
        const Phasor e = mode_phase(a.fk + 3 * m, ph);
        const double* d = duhat + 6 * m;
        du[0] += d[0] * e.c - d[1] * e.s;
        du[1] += d[2] * e.c - d[3] * e.s;
        du[2] += d[4] * e.c - d[5] * e.s;
    }
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double v = Codec<S>::to_double(x[(size_t)i * a.n + idx], i);
        rho += v;
        j[0] += cx_of(i) * v;
        j[1] += cy_of(i) * v;
        j[2] += cz_of(i) * v;
    }
    const double inv_rho = 1.0 / rho;
    const double udu = (j[0] * du[0] + j[1] * du[1] + j[2] * du[2]) * inv_rho;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double cdu = cx_of(i) * du[0] + cy_of(i) * du[1] + cz_of(i) * du[2];
        lam[(size_t)i * a.n + idx] += (float)((cdu - udu) * inv_rho);
    }
}

__global__ __launch_bounds__(256) void k_fill_f32(float* __restrict__ p, size_t count, float v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

__global__ __launch_bounds__(256) void k_fill_f64(double* __restrict__ p, size_t count, double v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

__global__ __launch_bounds__(256) void k_add_f64_to_f32(float* __restrict__ dst, const double* __restrict__ src,
                                                       size_t count) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] += (float)src[i];
}

__global__ __launch_bounds__(256) void k_f32_to_f64(const float* __restrict__ src, double* __restrict__ dst,
                                                   size_t count) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = (double)src[i];
}

}  // namespace

int adjoint_param_count() { return NPAR; }
int adjoint_param_count_depth(int depth) { return depth == 3 ? NPAR3 : NPAR; }
// Wavefronts per 64-node block of the vector-unit adjoint: one per SIMD (each
// keeps three [64][32] rows and its dL/dm rows in LDS, 130 KiB for four),
// which shortens the serial chain of every lane.  Measured on the reduced
// Taylor-Green cubes and periodic boxes from 16^3 to 96^3, the split wins at
// every size at depth 3; at depth 2 it wins up to ~2000 blocks, breaks even
// at 4096 and loses at 13824, where one wavefront per block leaves room for
// more blocks per CU.
constexpr int ADJ_SPLIT_D3 = 4, ADJ_SPLIT_D2 = 4, ADJ_SPLIT_D2_MAX_BLOCKS = 2048;
static int adjoint_split(int n, int depth) {
    if (depth == 3) return ADJ_SPLIT_D3;
    return (n + 63) / 64 <= ADJ_SPLIT_D2_MAX_BLOCKS ? ADJ_SPLIT_D2 : 1;
}

// Blocks per 64 nodes (gridDim.y) of the depth-3 reverse step: the largest
// divisor of the 48 / SPLIT group elements per wavefront that keeps the grid
// within two blocks per compute unit (a block holds 130 KiB of LDS, so one
// runs per CU at a time), so that small lattices (the reduced Taylor-Green
// cubes) fill the device instead of running 12 elements per lane in series.
// Depth 2 keeps one block per 64 nodes.
static int device_cus() {
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cus[dev] && hipDeviceGetAttribute(&cus[dev], hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus[dev] = 256;
    return cus[dev] > 0 ? cus[dev] : 256;
}
static int adjoint_gsplit(int n, int depth) {
    if (depth != 3) return 1;
    const int nb = (n + 63) / 64;
    const int target = 2 * device_cus();
    int gy = 1;
    for (int d = 2; d <= NGROUP / ADJ_SPLIT_D3; ++d)
        if ((NGROUP / ADJ_SPLIT_D3) % d == 0 && nb * d <= target) gy = d;
    return gy;
}

int adjoint_blocks(int n, int depth) { return (n + 63) / 64 * adjoint_gsplit(n, depth) * adjoint_split(n, depth); }

size_t adjoint_xwork_floats(int n, int depth) {
    const int gy = adjoint_gsplit(n, depth);
    return gy > 1 ? (size_t)gy * n * (AW + Q) + (size_t)n * Q : 0;
}

hipError_t launch_adjoint(int storage, const void* xin, const float* lam_in, float* lam_out, const StepArgs& a,
                          const int* gsrc, float* partial, float* xwork, hipStream_t st) {
    const int split = adjoint_split(a.n, a.depth);
    const int gy = adjoint_gsplit(a.n, a.depth);
    if (gy > 1 && !xwork) return hipErrorInvalidValue;
    const dim3 grid((a.n + 63) / 64, gy), block(64 * split);
#define ADJ_LAUNCH_M(SS, ACT, DEPTH, SPLIT, MODE)                                                            \
    hipLaunchKernelGGL((k_adjoint<SS, ACT, DEPTH, SPLIT, MODE>), grid, block, 0, st,                          \
                       static_cast<const typename Codec<SS>::store_t*>(xin), lam_in, lam_out, a, gsrc, partial, \
                       xwork)
#define ADJ_LAUNCH(SS, ACT, DEPTH, SPLIT) ADJ_LAUNCH_M(SS, ACT, DEPTH, SPLIT, ADJ_WHOLE)
#define ADJ_LAUNCH_D3(SS, ACT)                                                                               \
    if (gy > 1) {                                                                                            \
        ADJ_LAUNCH_M(SS, ACT, 3, ADJ_SPLIT_D3, ADJ_SUMS);                                                    \
        ADJ_LAUNCH_M(SS, ACT, 3, ADJ_SPLIT_D3, ADJ_MAIN);                                                    \
        hipLaunchKernelGGL(k_adjoint_finish, dim3((a.n + 63) / 64), dim3(64), 0, st, lam_out, a, gy,         \
                           (const float*)xwork);                                                             \
    } else {                                                                                                 \
        ADJ_LAUNCH(SS, ACT, 3, ADJ_SPLIT_D3);                                                                \
    }
#define ADJ_CASE(SS)                                                                                         \
    case SS:                                                                                                 \
        if (a.depth == 3) {                                                                                  \
            if (a.act == ACT_TANH) {                                                                         \
                ADJ_LAUNCH_D3(SS, ACT_TANH)                                                                  \
            } else {                                                                                         \
                ADJ_LAUNCH_D3(SS, ACT_RELU)                                                                  \
            }                                                                                                \
        } else if (split > 1) {                                                                              \
            if (a.act == ACT_TANH)                                                                           \
                ADJ_LAUNCH(SS, ACT_TANH, 2, ADJ_SPLIT_D2);                                                   \
            else                                                                                             \
                ADJ_LAUNCH(SS, ACT_RELU, 2, ADJ_SPLIT_D2);                                                   \
        } else {                                                                                             \
            if (a.act == ACT_TANH)                                                                           \
                ADJ_LAUNCH(SS, ACT_TANH, 2, 1);                                                              \
            else                                                                                             \
                ADJ_LAUNCH(SS, ACT_RELU, 2, 1);                                                              \
        }                                                                                                    \
        return hipGetLastError();
    switch (storage) {
        ADJ_CASE(ST_F32)
        ADJ_CASE(ST_F16)
        ADJ_CASE(ST_BF16)
        default: return hipErrorInvalidValue;
    }
#undef ADJ_CASE
#undef ADJ_LAUNCH_D3
#undef ADJ_LAUNCH
#undef ADJ_LAUNCH_M
}

hipError_t launch_grad_reduce(const float* partial, int nblocks, int npar, double* grad, hipStream_t st) {
    hipLaunchKernelGGL(k_grad_reduce, dim3((npar + 7) / 8), dim3(256), 0, st, partial, nblocks, npar, grad);
    return hipGetLastError();
}

hipError_t launch_grad_reduce_f64(const double* partial, int nblocks, double* stage, double* grad, hipStream_t st) {
    const int groups = (nblocks + 63) / 64;
    hipLaunchKernelGGL(k_grad_stage, dim3((NPAR + 255) / 256, groups), dim3(256), 0, st, partial, nblocks, stage);
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(k_grad_final, dim3((NPAR + 255) / 256), dim3(256), 0, st, stage, groups, grad);
    return hipGetLastError();
}

hipError_t launch_add_energy_grad(int storage, const void* f, float* lam, double coef, int n, hipStream_t st) {
    const dim3 grid((n + 255) / 256), block(256);
#define AEG_CASE(SS)                                                                                           \
    case SS:                                                                                                   \
        hipLaunchKernelGGL(k_add_energy_grad<SS>, grid, block, 0, st,                                          \
                           static_cast<const typename Codec<SS>::store_t*>(f), lam, coef, n);                  \
        return hipGetLastError();
    switch (storage) {
        AEG_CASE(ST_F32)
        AEG_CASE(ST_F16)
        AEG_CASE(ST_BF16)
        default: return hipErrorInvalidValue;
    }
#undef AEG_CASE
}

hipError_t launch_force_phase_adjoint(int storage, const void* x, const float* lam_next, float* lam_out,
                                      const StepArgs& a, double* partial, const double* basis, const double* draw,
                                      const double* uhat, double* duhat, hipStream_t st) {
    if (a.n_modes < 1 || !a.fk || !a.fhat) return hipErrorInvalidValue;
    const dim3 grid((a.n + 255) / 256), pgrid((a.n + FA_BLOCK_NODES - 1) / FA_BLOCK_NODES), block(256);
#define FPA_CASE(SS)                                                                                           \
    case SS: {                                                                                                 \
        const auto* xs = static_cast<const typename Codec<SS>::store_t*>(x);                                   \
        hipLaunchKernelGGL(k_force_adj_partials<SS>, pgrid, block, 0, st, xs, lam_next, a, partial);           \
        if (hipError_t e = hipGetLastError()) return e;                                                        \
        hipLaunchKernelGGL(k_force_phase_adj, dim3(a.n_modes), block, 0, st, partial, (int)pgrid.x, 1.0 / a.n, \
                           basis, draw, a.fhat, uhat, duhat);                                                  \
        if (hipError_t e = hipGetLastError()) return e;                                                        \
        hipLaunchKernelGGL(k_add_velocity_grad<SS>, grid, block, 0, st, xs, lam_out, a,                        \
                           static_cast<const double*>(duhat));                                                 \
        return hipGetLastError();                                                                              \
    }
    switch (storage) {
        FPA_CASE(ST_F32)
        FPA_CASE(ST_F16)
        FPA_CASE(ST_BF16)
        default: return hipErrorInvalidValue;
    }
#undef FPA_CASE
}

hipError_t launch_fill_f32(float* p, size_t count, float v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, size_t count, double v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}

hipError_t launch_add_f64_to_f32(float* dst, const double* src, size_t count, hipStream_t st) {
    hipLaunchKernelGGL(k_add_f64_to_f32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, dst, src, count);
    return hipGetLastError();
}

hipError_t launch_f32_to_f64(const float* src, double* dst, size_t count, hipStream_t st) {
    hipLaunchKernelGGL(k_f32_to_f64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, src, dst, count);
    return hipGetLastError();
}

}  // namespace nco
