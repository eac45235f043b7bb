// Per-node collision operators (device side).
//
//  * BGK (Sec. II.A): f_i += (f_i^eq - f_i) / tau with the quadratic
//    equilibrium of Eq. EquilibriumDistribution.
//  * Moment relaxation (Eq. omegatheta): m = M f, relax m towards m^eq with
//    rate 1 for orders 0-1, 1/tau for order 2 and omega_n for the orders
//    n = 3..6, f = M^{-1} m*.  The equilibrium moments of the quadratic
//    equilibrium are rho, sqrt(3) j_a and m_a m_b / rho for second order, and
//    vanish for orders 3..6, so only second order needs m^eq.
//  * Kupershtokh exact-difference source (Sec. II.A): f^eq(rho, u + F/rho) -
//    f^eq(rho, u) only changes the first- and second-order equilibrium
//    moments, by sqrt(3) F_a and 3 (j_a F_b + j_b F_a + F_a F_b) / rho.
//  * The invariant network of Eq. gconv_m evaluated per node on the vector
//    units: tilde tau = (1/48) sum_g Phi(m^(g)), with the group action folded
//    into 48 stacked first-layer matrices (m^(g) = M Pi_g f is a signed
//    permutation of m, so W1^T m^(g) = W1_g^T m).  The last layer is affine,
//    so the mean of the outputs equals W3^T mean_g(h2_g) + b3.
#pragma once

#include "d3q27.h"

namespace nco {

enum Op { OP_BGK = 0, OP_MRT = 1, OP_NCO = 2, OP_NONE = 3 };
enum Act { ACT_TANH = 0, ACT_RELU = 1 };
// Matrix-core network arithmetic (values of nco_mlp_prec).
enum MlpPrec { MLP_PREC_F32 = 1, MLP_PREC_BF16 = 2, MLP_PREC_F32S = 3 };

constexpr int NGROUP = 48;

// Layout of the device network buffer for width W (floats):
// W1 stacked per group [48][27][W], b1[W], W2[W][W], b2[W], W3[W][4], b3[4].
__host__ __device__ constexpr int net_off_b1(int W) { return NGROUP * 27 * W; }
__host__ __device__ constexpr int net_off_w2(int W) { return net_off_b1(W) + W; }
__host__ __device__ constexpr int net_off_b2(int W) { return net_off_w2(W) + W * W; }
__host__ __device__ constexpr int net_off_w3(int W) { return net_off_b2(W) + W; }
__host__ __device__ constexpr int net_off_b3(int W) { return net_off_w3(W) + 4 * W; }
__host__ __device__ constexpr int net_floats(int W) { return net_off_b3(W) + 4; }
// A third hidden layer (depth 3) follows: W2b[W][W], b2b[W].
__host__ __device__ constexpr int net_off_w2b(int W) { return net_floats(W); }
__host__ __device__ constexpr int net_off_b2b(int W) { return net_off_w2b(W) + W * W; }
__host__ __device__ constexpr int net_floats_depth(int W, int depth) {
    return depth == 3 ? net_off_b2b(W) + W : net_floats(W);
}

template <int ACT, typename R>
__device__ __forceinline__ R activate(R x) {
    if constexpr (ACT == ACT_RELU) {
        return x > R(0) ? x : R(0);
    } else {
        return tanh(x);
    }
}

// Rate squashing of Sec. II.B: tau = 1/(2 (1 + e^t)) + 1/2, omega = 1/tau.
template <typename R>
__device__ __forceinline__ R squash_rate(R t) {
    const R tau = R(0.5) + R(0.5) / (R(1) + exp(t));
    return R(1) / tau;
}

// omega_3..omega_6 of one node from its moments (tensor order), with
// DEPTH = 2 or 3 hidden layers.
template <typename R, int W, int ACT, int DEPTH = 2>
__device__ __forceinline__ void net_rates(const R (&m)[Q], const float* __restrict__ net,
                                          R (&omega)[4]) {
    R x[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) x[k] = m[row_tensor(k)];
    const float* __restrict__ b1 = net + net_off_b1(W);
    const float* __restrict__ w2 = net + net_off_w2(W);
    const float* __restrict__ b2 = net + net_off_b2(W);
    const float* __restrict__ w3 = net + net_off_w3(W);
    const float* __restrict__ b3 = net + net_off_b3(W);
    R acc[W];
#pragma unroll
    for (int o = 0; o < W; ++o) acc[o] = R(0);
#pragma unroll 1
    for (int g = 0; g < NGROUP; ++g) {
        const float* __restrict__ wg = net + g * (27 * W);
        R h[W];
#pragma unroll
        for (int j = 0; j < W; ++j) h[j] = (R)b1[j];
#pragma unroll
        for (int k = 0; k < Q; ++k)
#pragma unroll
            for (int j = 0; j < W; ++j) h[j] = fma((R)wg[k * W + j], x[k], h[j]);
#pragma unroll
        for (int j = 0; j < W; ++j) h[j] = activate<ACT>(h[j]);
        if constexpr (DEPTH == 2) {
#pragma unroll
            for (int o = 0; o < W; ++o) {
                R s = (R)b2[o];
#pragma unroll
                for (int j = 0; j < W; ++j) s = fma((R)w2[j * W + o], h[j], s);
                acc[o] += activate<ACT>(s);
            }
        } else {
            const float* __restrict__ w2b = net + net_off_w2b(W);
            const float* __restrict__ b2b = net + net_off_b2b(W);
            R h2[W];
#pragma unroll
            for (int o = 0; o < W; ++o) {
                R s = (R)b2[o];
#pragma unroll
                for (int j = 0; j < W; ++j) s = fma((R)w2[j * W + o], h[j], s);
                h2[o] = activate<ACT>(s);
            }
#pragma unroll
            for (int o = 0; o < W; ++o) {
                R s = (R)b2b[o];
#pragma unroll
                for (int j = 0; j < W; ++j) s = fma((R)w2b[j * W + o], h2[j], s);
                acc[o] += activate<ACT>(s);
            }
        }
    }
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        R t = R(0);
#pragma unroll
        for (int o = 0; o < W; ++o) t = fma((R)w3[o * 4 + n], acc[o], t);
        omega[n] = squash_rate(t * R(1.0 / NGROUP) + (R)b3[n]);
    }
}

// Second-order equilibrium moment of tensor index t (order 2) from the
// first-order moments m_a = sqrt(3) j_a: 3 j_a j_b / rho = m_a m_b / rho.
template <typename R>
__device__ __forceinline__ R meq2(int t, const R (&m)[Q], R inv_rho) {
    const int nx = t % 3, ny = (t / 3) % 3, nz = t / 9;
    const R mx = m[1], my = m[3], mz = m[9];
    R a = nx == 2 ? mx * mx : ny == 2 ? my * my : nz == 2 ? mz * mz
        : (nx == 1 && ny == 1) ? mx * my : (nx == 1 && nz == 1) ? mx * mz : my * mz;
    return a * inv_rho;
}

// Moment-space change of one collision (with the optional Kupershtokh source):
// f_post = f - M^{-1} dm with dm = S (m - m^eq) - dm_source.  dm vanishes in
// the conserved moments (orders 0 and 1 relax with rate 1 onto themselves),
// so forming the update as a correction keeps mass and momentum to rounding
// of the (small) non-equilibrium part instead of the populations themselves.
template <typename R, bool FORCED>
__device__ __forceinline__ void collision_delta(const R (&m)[Q], R omega_nu, const R (&omega)[4],
                                                R Fx, R Fy, R Fz, R (&dm)[Q]) {
    const R inv_rho = R(1) / m[0];
#pragma unroll
    for (int t = 0; t < Q; ++t) {
        const int n = order_of(t);
        if (n <= 1) {
            dm[t] = R(0);
        } else if (n == 2) {
            dm[t] = omega_nu * (m[t] - meq2(t, m, inv_rho));
        } else {
            dm[t] = omega[n - 3] * m[t];
        }
    }
    if constexpr (FORCED) {
        const R is3 = R(1.0 / 1.7320508075688772);
        const R j[3] = {m[1] * is3, m[3] * is3, m[9] * is3}, F[3] = {Fx, Fy, Fz};
#pragma unroll
        for (int t = 0; t < Q; ++t) {
            if (order_of(t) == 2) {
                const int nx = t % 3, ny = (t / 3) % 3, nz = t / 9;
                int a, b;
                if (nx == 2) { a = 0; b = 0; } else if (ny == 2) { a = 1; b = 1; }
                else if (nz == 2) { a = 2; b = 2; } else if (nx == 1 && ny == 1) { a = 0; b = 1; }
                else if (nx == 1 && nz == 1) { a = 0; b = 2; } else { a = 1; b = 2; }
                dm[t] -= R(3) * (j[a] * F[b] + j[b] * F[a] + F[a] * F[b]) * inv_rho;
            }
        }
        dm[1] = -Sqrt3<R>::v * Fx;
        dm[3] = -Sqrt3<R>::v * Fy;
        dm[9] = -Sqrt3<R>::v * Fz;
    }
}

template <typename R, bool FORCED>
__device__ __forceinline__ void bgk(R (&f)[Q], R omega_nu, R Fx, R Fy, R Fz) {
    R rho = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        rho += f[i];
        if (cx_of(i)) jx += cx_of(i) > 0 ? f[i] : -f[i];
        if (cy_of(i)) jy += cy_of(i) > 0 ? f[i] : -f[i];
        if (cz_of(i)) jz += cz_of(i) > 0 ? f[i] : -f[i];
    }
    const R inv_rho = R(1) / rho;
    const R ux = jx * inv_rho, uy = jy * inv_rho, uz = jz * inv_rho;
    const R base = R(1) - R(1.5) * (ux * ux + uy * uy + uz * uz);
    R vx = ux, vy = uy, vz = uz, base2 = base;
    if constexpr (FORCED) {
        vx = ux + Fx * inv_rho;
        vy = uy + Fy * inv_rho;
        vz = uz + Fz * inv_rho;
        base2 = R(1) - R(1.5) * (vx * vx + vy * vy + vz * vz);
    }
    // The rest population's equilibrium is closed as rho minus the others, so
    // the rounded weights do not bias the mass of every step.
    R feq_sum = R(0), src_sum = R(0);
    R feq[Q], src[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (i == 13) continue;
        const R cu = R(cx_of(i)) * ux + R(cy_of(i)) * uy + R(cz_of(i)) * uz;
        const R wr = R(weight_of(i)) * rho;
        feq[i] = wr * (base + cu * (R(3) + R(4.5) * cu));
        feq_sum += feq[i];
        if constexpr (FORCED) {
            const R cv = R(cx_of(i)) * vx + R(cy_of(i)) * vy + R(cz_of(i)) * vz;
            src[i] = wr * (base2 + cv * (R(3) + R(4.5) * cv)) - feq[i];
            src_sum += src[i];
        }
    }
    feq[13] = rho - feq_sum;
    src[13] = -src_sum;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        f[i] += (feq[i] - f[i]) * omega_nu;
        if constexpr (FORCED) f[i] += src[i];
    }
}

}  // namespace nco
