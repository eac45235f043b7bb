// Device pieces of the reverse-mode step shared by the vector-unit and the
// matrix-core adjoint kernels: transposed moment transforms, activation
// derivatives and the vector-Jacobian product of the collision's
// node-local part (Eq. omegatheta with the quadratic equilibrium and the
// Kupershtokh source of Sec. II.A), everything except the network.
#pragma once

#include "collide.h"
#include "d3q27.h"

namespace nco {

inline constexpr int AW = 32;                    // network width of the adjoint path
inline constexpr int NPAR = AW * (27 + AW + 4) + 2 * AW + 4;
inline constexpr int OFF_W1 = 0, OFF_B1 = 27 * AW, OFF_W2 = OFF_B1 + AW, OFF_B2 = OFF_W2 + AW * AW;
inline constexpr int OFF_W3 = OFF_B2 + AW, OFF_B3 = OFF_W3 + 4 * AW;
// Depth 3 (vector-unit adjoint): the third hidden layer's gradient follows.
inline constexpr int OFF_W2B = NPAR, OFF_B2B = OFF_W2B + AW * AW, NPAR3 = OFF_B2B + AW;

// One-dimensional pieces of M^T (transpose of fwd3) and M^{-T} (transpose
// of inv3), applied along each axis like the transforms themselves.
template <typename R>
__device__ __forceinline__ void fwd3_t(R g0, R g1, R g2, R& fm, R& f0, R& fp) {
    const R s3 = Sqrt3<R>::v;
    fm = g0 - s3 * g1 + R(2) * g2;
    f0 = g0 - g2;
    fp = g0 + s3 * g1 + R(2) * g2;
}

template <typename R>
__device__ __forceinline__ void inv3_t(R lm, R l0, R lp, R& a0, R& a1, R& a2) {
    const R s3 = Sqrt3<R>::v;
    a0 = (lm + R(4) * l0 + lp) * R(1.0 / 6.0);
    a1 = s3 * (lp - lm) * R(1.0 / 6.0);
    a2 = (lm - R(2) * l0 + lp) * R(1.0 / 6.0);
}

// out = M^T g (g in tensor moment order, out in velocity order).
template <typename R>
__device__ __forceinline__ void moments_T(const R (&g)[Q], R (&out)[Q]) {
    R s[Q], t[Q];
#pragma unroll
    for (int p = 0; p < 9; ++p) fwd3_t(g[p], g[9 + p], g[18 + p], s[p], s[9 + p], s[18 + p]);
#pragma unroll
    for (int z = 0; z < 3; ++z)
#pragma unroll
        for (int n = 0; n < 3; ++n)
            fwd3_t(s[9 * z + n], s[9 * z + 3 + n], s[9 * z + 6 + n], t[9 * z + n], t[9 * z + 3 + n],
                   t[9 * z + 6 + n]);
#pragma unroll
    for (int r = 0; r < 9; ++r) fwd3_t(t[3 * r], t[3 * r + 1], t[3 * r + 2], out[3 * r], out[3 * r + 1], out[3 * r + 2]);
}

// mu = M^{-T} lam (lam in velocity order, mu in tensor moment order).
template <typename R>
__device__ __forceinline__ void inverse_T(const R (&lam)[Q], R (&mu)[Q]) {
    R t[Q], s[Q];
#pragma unroll
    for (int r = 0; r < 9; ++r) inv3_t(lam[3 * r], lam[3 * r + 1], lam[3 * r + 2], t[3 * r], t[3 * r + 1], t[3 * r + 2]);
#pragma unroll
    for (int z = 0; z < 3; ++z)
#pragma unroll
        for (int n = 0; n < 3; ++n)
            inv3_t(t[9 * z + n], t[9 * z + 3 + n], t[9 * z + 6 + n], s[9 * z + n], s[9 * z + 3 + n],
                   s[9 * z + 6 + n]);
#pragma unroll
    for (int p = 0; p < 9; ++p) inv3_t(s[p], s[9 + p], s[18 + p], mu[p], mu[9 + p], mu[18 + p]);
}

template <int ACT>
__device__ __forceinline__ float act_f(float z) {
    return ACT == ACT_RELU ? fmaxf(z, 0.0f) : tanhf(z);
}
// Derivative from the activation's output.
template <int ACT>
__device__ __forceinline__ float act_d(float h) {
    return ACT == ACT_RELU ? (h > 0.0f ? 1.0f : 0.0f) : 1.0f - h * h;
}

// Index of the two first-order factors of a second-order tensor index t
// (moment m_a m_b / rho): a, b in {0, 1, 2} as tensor indices 1, 3, 9.
__device__ __forceinline__ void pair_of(int t, int& ta, int& tb) {
    const int nx = t % 3, ny = (t / 3) % 3, nz = t / 9;
    const int idx[3] = {1, 3, 9};
    int k = 0, ab[2];
    for (int r = 0; r < 3; ++r) {
        const int n = r == 0 ? nx : r == 1 ? ny : nz;
        for (int c = 0; c < n; ++c) ab[k++] = idx[r];
    }
    ta = ab[0];
    tb = ab[1];
}

// g_m = (d dm / d m)^T nu for the node-local part of dm = S (m - m^eq) -
// dm_source (tensor moment order), and dL/d omega_n = sum over the moments of
// order n + 3 of nu_t m_t.  nu = -M^{-T} lambda; F is the body force when
// forced.  The network's share of g_m (through the rates) is added by the
// caller.
__device__ __forceinline__ void collision_vjp_local(const float (&m)[Q], const float (&nu)[Q], float wnu,
                                                    const float (&omega)[4], bool forced, const float (&F)[3],
                                                    float (&gm)[Q], float (&domega)[4]) {
    const float inv_rho = 1.0f / m[0];
#pragma unroll
    for (int t = 0; t < Q; ++t) gm[t] = 0.0f;
#pragma unroll
    for (int n = 0; n < 4; ++n) domega[n] = 0.0f;
#pragma unroll
    for (int t = 0; t < Q; ++t) {
        const int n = order_of(t);
        const float v = -nu[t];
        if (n == 2) {
            int ta, tb;
            pair_of(t, ta, tb);
            // dm_t = w_nu (m_t - m_a m_b / rho) - (sqrt3 (m_a F_b + m_b F_a) + 3 F_a F_b) / rho
            const int a_ = ta == 1 ? 0 : ta == 3 ? 1 : 2, b_ = tb == 1 ? 0 : tb == 3 ? 1 : 2;
            gm[t] += v * wnu;
            gm[ta] -= v * wnu * m[tb] * inv_rho;
            gm[tb] -= v * wnu * m[ta] * inv_rho;
            gm[0] += v * wnu * m[ta] * m[tb] * inv_rho * inv_rho;
            if (forced) {
                const float s3 = 1.7320508075688772f;
                const float src = (s3 * (m[ta] * F[b_] + m[tb] * F[a_]) + 3.0f * F[a_] * F[b_]) * inv_rho;
                gm[ta] -= v * s3 * F[b_] * inv_rho;
                gm[tb] -= v * s3 * F[a_] * inv_rho;
                gm[0] += v * src * inv_rho;
            }
        } else if (n >= 3) {
            gm[t] += v * omega[n - 3];
            domega[n - 3] += v * m[t];
        }
    }
}

}  // namespace nco
