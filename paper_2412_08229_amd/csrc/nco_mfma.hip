// NCO stream-collide with the invariant network on the matrix cores (gfx950).
//
// The network of Eq. gconv_m is evaluated for a tile of 16 nodes at a time as
// a chain of transposed GEMMs, hidden x nodes:
//     Z1 = W1^T X_g          (32 x 28) (28 x 16), X_g = m^(g) plus a 1 row
//     H1 = act(Z1)                                 (bias b1 rides on the 1 row)
//     Z2 = W2^T H1 + b2      (32 x 32) (32 x 16)
//     acc += act(Z2)         summed over the 48 group elements g
//     tilde tau = W3^T acc / 48 + b3               (vector units)
// With v_mfma_f32_16x16x4f32 the accumulator of one product is laid out as
// lane (q, c) = (lane / 16, lane % 16) holding rows 4q..4q+3 of column c,
// which is exactly the B-operand layout of the next product's K-step when the
// K index is ordered (t, r) -> hidden 16 t + 4 q + r.  Layer 1 therefore
// feeds layer 2 from registers, with no LDS round trip.
//
// The group action m^(g) = M Pi_g f is a signed permutation of the moment
// vector (the rows of M are products of one-dimensional Hermite polynomials,
// so a rotation/reflection of the velocities permutes the rows and flips the
// sign of odd ones).  It is applied while gathering the B operand from the
// LDS moment tile: a per-group table gives, for each lane group q and K-step,
// the source row and the sign bit.  W1, W2, b2 and W3 stay in registers for
// the whole kernel.
//
// Block = 256 threads = 256 nodes.  Phase A: each thread pulls its 27
// populations and writes its moments to LDS.  Phase B: each wavefront runs the
// network for its 64 nodes (4 tiles of 16) and writes the four rates per node
// to LDS.  Phase C: each thread pulls its populations again (the kernel is
// compute bound; the second read is cheap), relaxes in moment space with the
// rates and stores.
#include "kernels.h"
#include "stream.h"

namespace nco {

namespace {

constexpr int MW = 32;             // network width on this path
constexpr int NODE_STRIDE = 29;    // LDS floats per node: 27 moments, 1.0, pad
constexpr int GT_ENTRIES = NGROUP * 4 * 8;

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Offsets in the per-lane weight table (floats per lane: LANE_FLOATS).
constexpr int LT_A1 = 0;           // [t 2][s 7]      W1/b1 rows as A operand
constexpr int LT_A2 = 14;          // [u 2][t 2][r 4] W2 as A operand
constexpr int LT_B2 = 30;          // [u 2][r 4]      b2 as accumulator init
constexpr int LT_W3 = 38;          // [u 2][r 4][n 4] W3 / 48
constexpr int LT_B3 = 70;          // [n 4]
constexpr int LANE_FLOATS = 76;

// Activation of a pre-activation that was scaled by kappa = 2 log2(e) for
// tanh: tanh(z) = 1 - 2 / (1 + 2^(kappa z)); saturates correctly at +-inf.
template <int ACT>
__device__ __forceinline__ float act_scaled(float x) {
    if constexpr (ACT == ACT_RELU) {
        return fmaxf(x, 0.0f);
    } else {
        const float t = __builtin_amdgcn_exp2f(x);
        return fmaf(-2.0f, __builtin_amdgcn_rcpf(1.0f + t), 1.0f);
    }
}

// RATES = true: no streaming, the rates of the stored state are written to
// omega_out [4][n] instead of a step (readout and tests of the network alone).
template <int S, int ACT, bool RATES>
__global__ __launch_bounds__(256) void k_nco_mfma_f32(const typename Codec<S>::store_t* __restrict__ fin,
                                                      typename Codec<S>::store_t* __restrict__ fout,
                                                      StepArgs a, const float* __restrict__ lane_tab,
                                                      const int* __restrict__ gtab,
                                                      double* __restrict__ omega_out) {
    __shared__ float sm[256 * NODE_STRIDE];
    __shared__ int sg[GT_ENTRIES];
    __shared__ float sw[256 * 4];
    const int tid = threadIdx.x;
    const int idx = blockIdx.x * 256 + tid;
    const bool live = idx < a.n;

    for (int e = tid; e < GT_ENTRIES; e += 256) sg[e] = gtab[e];

    // Phase A: pull and transform to moments.
    {
        float f[Q];
        if (live) {
            if constexpr (RATES)
                load_local<S>(fin, a.n, idx, f);
            else
                pull<S>(fin, a, node_of(idx, a.nx, a.ny), f);
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i) f[i] = (float)weight_of(i);
        }
        float m[Q];
        to_moments(f, m);
        float* row = sm + tid * NODE_STRIDE;
#pragma unroll
        for (int k = 0; k < Q; ++k) row[k] = m[row_tensor(k)];
        row[27] = 1.0f;
        row[28] = 0.0f;
    }
    __syncthreads();

    // Phase B: the network on the matrix cores, one wavefront per 64 nodes.
    {
        const int lane = tid & 63, wave = tid >> 6, q = lane >> 4, c = lane & 15;
        const float* __restrict__ lt = lane_tab + lane * LANE_FLOATS;
        float A1[2][7], A2[2][2][4], B2[2][4];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int s = 0; s < 7; ++s) A1[t][s] = lt[LT_A1 + t * 7 + s];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) A2[u][t][r] = lt[LT_A2 + u * 8 + t * 4 + r];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) B2[u][r] = lt[LT_B2 + u * 4 + r];

#pragma unroll 1
        for (int j = 0; j < 4; ++j) {
            const int node = wave * 64 + j * 16 + c;
            const float* __restrict__ mrow = sm + node * NODE_STRIDE;
            f32x4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll 1
            for (int g = 0; g < NGROUP; ++g) {
                const int* __restrict__ ge = sg + (g * 4 + q) * 8;
                float b[7];
#pragma unroll
                for (int s = 0; s < 7; ++s) {
                    const int e = ge[s];
                    b[s] = __int_as_float(__float_as_int(mrow[e & 31]) ^ (e & (int)0x80000000));
                }
                f32x4 c1[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
                for (int s = 0; s < 7; ++s)
#pragma unroll
                    for (int t = 0; t < 2; ++t)
                        c1[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(A1[t][s], b[s], c1[t], 0, 0, 0);
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) c1[t][r] = act_scaled<ACT>(c1[t][r]);
                f32x4 c2[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) c2[u] = f32x4{B2[u][0], B2[u][1], B2[u][2], B2[u][3]};
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int u = 0; u < 2; ++u)
                            c2[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(A2[u][t][r], c1[t][r], c2[u], 0, 0, 0);
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[u][r] += act_scaled<ACT>(c2[u][r]);
            }
            // Output layer on the group mean, reduced over the 4 lane groups.
            float p[4];
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                float v = 0.0f;
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int r = 0; r < 4; ++r) v = fmaf(lt[LT_W3 + (u * 4 + r) * 4 + n], acc[u][r], v);
                v += __shfl_xor(v, 16, 64);
                v += __shfl_xor(v, 32, 64);
                p[n] = v;
            }
            if (q == 0) {
#pragma unroll
                for (int n = 0; n < 4; ++n) {
                    const float t = p[n] + lt[LT_B3 + n];
                    sw[node * 4 + n] = 1.0f / (0.5f + 0.5f / (1.0f + expf(t)));
                }
            }
        }
    }
    __syncthreads();

    if constexpr (RATES) {
        if (live)
#pragma unroll
            for (int n = 0; n < 4; ++n) omega_out[(size_t)n * a.n + idx] = (double)sw[tid * 4 + n];
        return;
    }

    // Phase C: relax with the rates and store.
    if (live) {
        float f[Q], m[Q];
        pull<S>(fin, a, node_of(idx, a.nx, a.ny), f);
        const float* row = sm + tid * NODE_STRIDE;
#pragma unroll
        for (int k = 0; k < Q; ++k) m[row_tensor(k)] = row[k];
        float omega[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) omega[n] = sw[tid * 4 + n];
        float dm[Q], df[Q];
        collision_delta<float, false>(m, a.omega_nu_f, omega, 0.f, 0.f, 0.f, dm);
        from_moments(dm, df);
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] -= df[i];
        store_local<S>(fout, a.n, idx, f);
    }
}

}  // namespace

size_t mfma_lane_table_floats() { return 64 * LANE_FLOATS; }
size_t mfma_group_table_ints() { return GT_ENTRIES; }

// Host-side preparation of the per-lane operand tables from the flat
// parameters (W1[27][W], b1, W2[W][W], b2, W3[W][4], b3) and of the group
// gather table from (src, sign) of every group element and row.
void mfma_prepare_tables(const float* params, int act, const int (*gsrc)[27], const float (*gsign)[27],
                         float* lane_tab, int* gtab) {
    const int W = MW;
    const float* W1 = params;
    const float* b1 = W1 + 27 * W;
    const float* W2 = b1 + W;
    const float* b2 = W2 + W * W;
    const float* W3 = b2 + W;
    const float* b3 = W3 + 4 * W;
    const float kappa = act == ACT_TANH ? (float)(2.0 / 0.69314718055994530942) : 1.0f;
    for (int lane = 0; lane < 64; ++lane) {
        const int q = lane >> 4, c = lane & 15;
        float* lt = lane_tab + lane * LANE_FLOATS;
        for (int i = 0; i < LANE_FLOATS; ++i) lt[i] = 0.0f;
        for (int t = 0; t < 2; ++t)
            for (int s = 0; s < 7; ++s) {
                const int k = 4 * s + q, h = 16 * t + c;
                lt[LT_A1 + t * 7 + s] = kappa * (k < 27 ? W1[k * W + h] : b1[h]);
            }
        for (int u = 0; u < 2; ++u)
            for (int t = 0; t < 2; ++t)
                for (int r = 0; r < 4; ++r)
                    lt[LT_A2 + u * 8 + t * 4 + r] = kappa * W2[(16 * t + 4 * q + r) * W + 16 * u + c];
        for (int u = 0; u < 2; ++u)
            for (int r = 0; r < 4; ++r) lt[LT_B2 + u * 4 + r] = kappa * b2[16 * u + 4 * q + r];
        for (int u = 0; u < 2; ++u)
            for (int r = 0; r < 4; ++r)
                for (int n = 0; n < 4; ++n)
                    lt[LT_W3 + (u * 4 + r) * 4 + n] = W3[(16 * u + 4 * q + r) * 4 + n] / (float)NGROUP;
        for (int n = 0; n < 4; ++n) lt[LT_B3 + n] = b3[n];
    }
    for (int g = 0; g < NGROUP; ++g)
        for (int q = 0; q < 4; ++q)
            for (int s = 0; s < 8; ++s) {
                const int k = 4 * s + q;
                int e;
                if (k < 27) {
                    e = gsrc[g][k] | (gsign[g][k] < 0.0f ? (int)0x80000000 : 0);
                } else if (k == 27) {
                    e = 27;          // the constant-1 row carrying b1
                } else {
                    e = 28;          // zero pad (unused K slot)
                }
                gtab[(g * 4 + q) * 8 + s] = e;
            }
}

// omega_out == nullptr: one stream-collide step fin -> fout.  Otherwise the
// rates of the state in fin are written to omega_out and fout is untouched.
hipError_t launch_nco_mfma(int storage, const void* fin, void* fout, const StepArgs& a,
                           const float* lane_tab, const int* gtab, double* omega_out, hipStream_t st) {
    const dim3 grid((a.n + 255) / 256), block(256);
#define MFMA_LAUNCH(SS, AA, RR)                                                                       \
    hipLaunchKernelGGL((k_nco_mfma_f32<SS, AA, RR>), grid, block, 0, st, static_cast<const T*>(fin), \
                       static_cast<T*>(fout), a, lane_tab, gtab, omega_out)
#define MFMA_CASE(SS)                                                         \
    case SS: {                                                                \
        using T = typename Codec<SS>::store_t;                                \
        if (omega_out) {                                                      \
            if (a.act == ACT_TANH) MFMA_LAUNCH(SS, ACT_TANH, true);           \
            else MFMA_LAUNCH(SS, ACT_RELU, true);                             \
        } else {                                                              \
            if (a.act == ACT_TANH) MFMA_LAUNCH(SS, ACT_TANH, false);          \
            else MFMA_LAUNCH(SS, ACT_RELU, false);                            \
        }                                                                     \
        return hipGetLastError();                                             \
    }
    switch (storage) {
        MFMA_CASE(ST_F32)
        MFMA_CASE(ST_F16)
        MFMA_CASE(ST_BF16)
        default: return hipErrorInvalidValue;
    }
#undef MFMA_CASE
#undef MFMA_LAUNCH
}

}  // namespace nco
