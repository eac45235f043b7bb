// NCO stream-collide with the invariant network on the matrix cores (gfx950).
//
// Network of Eq. gconv_m, evaluated for tiles of 16 nodes as transposed
// GEMMs (hidden x nodes):
//     Z1_g = W1^T m^(g) + b1     (32 x 28) (28 x 16)
//     H1   = act(Z1_g)
//     Z2_g = W2^T H1 + b2        (32 x 32) (32 x 16)
//     acc += act(Z2_g)           summed over the 48 elements g of O_h
//     tilde tau = W3^T acc / 48 + b3
// in one of two arithmetics:
//   PREC_F32  v_mfma_f32_16x16x4f32 (float32 operands and accumulation);
//   PREC_BF16 v_mfma_f32_16x16x32_bf16 (bf16 operands, float32 accumulation,
//             activations and group sum in float32).
//
// Group structure.  An element g of O_h is an axis permutation pi followed by
// axis reflections s in {+-1}^3.  Every row of M is a product of
// one-dimensional Hermite polynomials, so m^(g) = M Pi_g f is the permuted
// moment vector (Q_pi m) with row k multiplied by prod_r s_r^(n_kr): the sign
// depends only on the parity class c(k) = (n_kx, n_ky, n_kz) mod 2 of the row.
//  * float32: Z1_(pi,s) = sum_c chi_s(c) Y_(pi,c) with Y_(pi,c) =
//    W1_c^T (Q_pi m)_c and chi_s(c) = prod_r s_r^(c_r), i.e. the eight
//    reflections of one permutation are a 3-point Walsh-Hadamard transform of
//    eight class partial products (10 K-steps of 4 instead of 8 x 7).
//  * bf16: one K = 32 product covers all 28 rows, so each element is one
//    product per output tile; the reflection is applied to the packed bf16
//    operand by flipping sign bits with per-lane class masks.
// The moment operand is gathered from LDS once per permutation.
//
// Register chaining.  The accumulator of a 16x16 product holds, in lane
// (q, c) = (lane / 16, lane % 16), rows 4q..4q+3 of column c.  Ordering the K
// index of the next product as (t, r) -> hidden 16 t + 4 q + r (float32,
// K = 4 per step) or (j / 4, j % 4) -> hidden 16 (j / 4) + 4 q + j % 4 for the
// 8 K values j of a lane (bf16, K = 32) makes that exactly its B operand, so
// layer 2 consumes act(Z1) straight from registers.
//
// Block = 256 threads = 256 nodes.  Phase A: each thread pulls its 27
// populations and writes its 27 moments (plus the constant 1 of the bias row)
// to LDS.  Phase B: each wavefront runs the network for its 64 nodes, 16 at a
// time, and writes the four rates per node to LDS.  Phase C: each thread pulls
// its populations again (the kernel is compute bound; the second read is
// cheap), relaxes with the rates and stores.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "adjoint.h"
#include "kernels.h"
#include "stream.h"

namespace nco {

namespace {

constexpr int MW = 32;              // network width on this path
constexpr int NODE_STRIDE = 29;     // LDS floats per node: 27 moments, 1.0, 0.0
constexpr int KSTEPS = 10;          // K-steps of the eight parity-class products
constexpr int GT_STRIDE = 12;       // ints per (pi, q) in the gather table
constexpr int GT_ENTRIES = 6 * 4 * GT_STRIDE;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

// K-step -> parity class ci = cx + 2 cy + 4 cz of the W1 rows it holds.
__host__ __device__ constexpr int step_class(int st) {
    constexpr int c[KSTEPS] = {0, 0, 0, 1, 2, 4, 3, 5, 6, 7};
    return c[st];
}

// Offsets in the per-lane table (4-byte words per lane: LANE_WORDS).
// float32 path:
constexpr int LT_A1 = 0;            // [t 2][st 10]    W1 rows / b1 as A operand
constexpr int LT_A2 = 20;           // [u 2][t 2][r 4] W2 as A operand
constexpr int LT_B2 = 36;           // [u 2][r 4]      b2 as accumulator init
constexpr int LT_W3 = 44;           // [u 2][r 4][n 4] W3 / 48
constexpr int LT_B3 = 76;           // [n 4]
constexpr int LT_A2B = 80;          // [v 2][t 2][r 4] W2b as A operand (depth 3)
constexpr int LT_B2B = 96;          // [v 2][r 4]      b2b as accumulator init (depth 3)
// Split arithmetic (network_split): per layer the parts of its A operand as
// packed pairs in the K slots of the 16x16x32 product ([t or u 2][part 3][4
// words]: f16 head and remainder for tanh, bf16 head, middle and tail for
// ReLU; layer 1 of tanh in the slots of the bf16 path, K slot j of lane
// group q holding input row 8 q + j, layer 1 of ReLU as LT_A1 on the
// float32 matrix cores), the accumulator inits of the hidden-to-hidden
// layers, the scales that return each product to the pre-activation, the
// sign masks of the reflections and the output layer.
constexpr int LS_A1 = 0;
constexpr int LS_A2 = 24;
constexpr int LS_A3 = 48;
constexpr int LS_B2 = 72;           // [u 2][r 4]
constexpr int LS_B3 = 80;           // [u 2][r 4]
constexpr int LS_BACK = 88;         // [layer 1, 2, 3]
constexpr int LS_NEG1 = 91;         // -1.0 (see residual_f16)
constexpr int LS_SM = 92;           // [bit 3][4 words] as LB_SM
constexpr int LS_W3 = 104;          // [u 2][r 4][n 4] W3 / 48
constexpr int LS_B3O = 136;         // [n 4]
// bf16 path (A operands as packed bf16 pairs, two per word):
constexpr int LB_A1 = 0;            // [t 2][4 words]  W1 rows 8q..8q+7 / b1
constexpr int LB_A2 = 8;            // [u 2][4 words]  W2
constexpr int LB_B2 = 16;           // [u 2][r 4]
constexpr int LB_W3 = 24;           // [u 2][r 4][n 4]
constexpr int LB_B3 = 56;           // [n 4]
constexpr int LB_SM = 60;           // [bit 3][4 words] sign masks of classes with that bit
constexpr int LB_A2B = 72;          // [v 2][4 words]  W2b (depth 3)
constexpr int LB_B2B = 80;          // [v 2][r 4]      b2b (depth 3)
constexpr int LANE_WORDS = 144;

// Activation as evaluated on this path.  For tanh the pre-activation arrives
// scaled by kappa = 2 log2(e) and the function returns r = 1 / (1 + 2^(kappa z)),
// so that tanh(z) = 1 - 2 r; the affine map 1 - 2 r is folded into the next
// layer's weights and bias on the host (and into W3, b3 for the group sum),
// which leaves exp2, add and reciprocal per value.  r saturates correctly
// (2^+inf = inf gives 0).
template <int ACT>
__device__ __forceinline__ float act_scaled(float x) {
    if constexpr (ACT == ACT_RELU) {
        return fmaxf(x, 0.0f);
    } else {
        return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(x));
    }
}

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 mfma32(u32x4 a, u32x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// Two floats to a packed bf16 pair (round to nearest even), low half first.
__device__ __forceinline__ unsigned pack_bf16(float lo, float hi) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{lo, hi}, bf16x2));
}

__device__ __forceinline__ f32x4 mfma32h(u32x4 a, u32x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                  0, 0);
}

// Two floats to a packed f16 pair (round to nearest even), low half first.
__device__ __forceinline__ unsigned pack_f16(float lo, float hi) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{lo, hi}, f16x2));
}

// The f16 pair (round to nearest even) of the remainders x0 - h0, x1 - h1,
// h0 and h1 being the two halves of hw (the differences are exact in
// float32).  neg1 = -1 arrives as data: with it the compiler emits one
// mixed-precision multiply-add per value that reads the f16 half in place
// (a literal -1 turns into a subtraction after a separate conversion), and,
// unlike hand-written assembly, it sees the write and keeps the wait
// states a matrix-core read of the result needs.
__device__ __forceinline__ unsigned residual_f16(unsigned hw, float x0, float x1, float neg1) {
    const f16x2 h = __builtin_bit_cast(f16x2, hw);
    return pack_f16(fmaf((float)h[0], neg1, x0), fmaf((float)h[1], neg1, x1));
}

// Three-part bf16 split of a float32 pair into head, middle and tail words
// (low half: x0's part), each part the nearest bf16 of what the previous
// parts leave (those differences are exact in float32): |x - head| <=
// 2^-8 |x|, |x - head - middle| <= 2^-16 |x|, |x - head - middle - tail| <=
// 2^-24 |x|.  bf16 has float32's exponent range, so no part overflows or
// leaves the normal range before float32 itself would.
__device__ __forceinline__ void split3_bf16(float x0, float x1, unsigned& h, unsigned& m, unsigned& t) {
    h = pack_bf16(x0, x1);
    const float r0 = x0 - __uint_as_float(h << 16), r1 = x1 - __uint_as_float(h & 0xffff0000u);
    m = pack_bf16(r0, r1);
    const float s0 = r0 - __uint_as_float(m << 16), s1 = r1 - __uint_as_float(m & 0xffff0000u);
    t = pack_bf16(s0, s1);
}

// tanh activation of the split arithmetic: 2^11 r with r as in act_scaled,
// from (1 + 2^x) 2^-11 in one fused multiply-add (exact scaling by a power
// of two), so that the head and the remainder of 2^11 r in (0, 2048] are
// both normal f16 numbers down to r ~ 3e-8.
__device__ __forceinline__ float act_split(float x) {
    constexpr float S = 0x1p-11f;
    return __builtin_amdgcn_rcpf(fmaf(__builtin_amdgcn_exp2f(x), S, S));
}

// Output layer on the group sum of one node tile and the rate squashing;
// lanes of group q = 0 write the four rates of node (tile, c) to LDS, or with
// RAW the pre-squash outputs tilde tau_n (for the adjoint).
template <bool RAW = false>
__device__ __forceinline__ void output_layer(const f32x4 (&acc)[2], const float* __restrict__ w3,
                                             const float* __restrict__ b3, int q, float* __restrict__ sw_node,
                                             float* __restrict__ tt_node = nullptr) {
    float pn[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        float v = 0.0f;
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) v = fmaf(w3[(u * 4 + r) * 4 + n], acc[u][r], v);
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        pn[n] = v;
    }
    if (q == 0) {
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const float t = pn[n] + b3[n];
            sw_node[n] = RAW ? t : 1.0f / (0.5f + 0.5f / (1.0f + expf(t)));
            if (tt_node) tt_node[n] = t;
        }
    }
}

// Layer 1 of one axis permutation on the float32 matrix cores for lane group
// q of a node tile (mrow: the node's moment row, ge: the permutation's gather
// slots of the group): the eight parity-class partial products over 10
// K-steps, then their Walsh-Hadamard transform over the class index, after
// which Y[s][t] is the pre-activation of reflection pattern s (hidden rows
// 16 t + 4 q + r).
__device__ __forceinline__ void layer1_reflections(const float (&A1)[2][KSTEPS], const float* __restrict__ mrow,
                                                   const int* __restrict__ ge, f32x4 (&Y)[8][2]) {
    // Moment operand of this permutation, one K-step per register.
    float b[KSTEPS];
#pragma unroll
    for (int st = 0; st < KSTEPS; ++st) b[st] = mrow[ge[st]];
#pragma unroll
    for (int ci = 0; ci < 8; ++ci) {
        Y[ci][0] = f32x4{0.f, 0.f, 0.f, 0.f};
        Y[ci][1] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int st = 0; st < KSTEPS; ++st)
#pragma unroll
        for (int t = 0; t < 2; ++t) Y[step_class(st)][t] = mfma4(A1[t][st], b[st], Y[step_class(st)][t]);
#pragma unroll
    for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
        for (int ci = 0; ci < 8; ++ci)
            if (!(ci & bit))
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const f32x4 u0 = Y[ci][t], u1 = Y[ci | bit][t];
                    Y[ci][t] = u0 + u1;
                    Y[ci | bit][t] = u0 - u1;
                }
}

// One axis permutation p of a node tile on the float32 matrix cores (ge:
// the permutation's gather slots of lane group q), the arithmetic of one
// pass of network_f32's permutation loop: layer 1 of the 8 reflections, the
// hidden layers (DEPTH 2 or 3), and each activation of the last hidden layer
// handed to sink(s, u, r, value) (reflection s, hidden row 16 u + 4 q + r)
// in the order network_f32 adds it to the group sum.
template <int ACT, int DEPTH, typename Sink>
__device__ __forceinline__ void permutation_f32(const float (&A1)[2][KSTEPS], const float (&A2)[2][2][4],
                                                const float (&B2)[2][4], const float* __restrict__ lt,
                                                const float* __restrict__ mrow, const int* __restrict__ ge,
                                                Sink&& sink) {
    f32x4 Y[8][2];
    layer1_reflections(A1, mrow, ge, Y);
    if constexpr (DEPTH == 3) {
        // Unrolled: Y[s] must stay in registers.
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            float h1v[2][4];
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) h1v[t][r] = act_scaled<ACT>(Y[s][t][r]);
            f32x4 c2[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) c2[u] = f32x4{B2[u][0], B2[u][1], B2[u][2], B2[u][3]};
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int u = 0; u < 2; ++u) c2[u] = mfma4(A2[u][t][r], h1v[t][r], c2[u]);
            float h2v[2][4];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int r = 0; r < 4; ++r) h2v[u][r] = act_scaled<ACT>(c2[u][r]);
            f32x4 c3[2];
#pragma unroll
            for (int v = 0; v < 2; ++v)
                c3[v] = f32x4{lt[LT_B2B + v * 4], lt[LT_B2B + v * 4 + 1], lt[LT_B2B + v * 4 + 2],
                              lt[LT_B2B + v * 4 + 3]};
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int v = 0; v < 2; ++v) c3[v] = mfma4(lt[LT_A2B + v * 8 + t * 4 + r], h2v[t][r], c3[v]);
#pragma unroll
            for (int v = 0; v < 2; ++v)
#pragma unroll
                for (int r = 0; r < 4; ++r) sink(s, v, r, act_scaled<ACT>(c3[v][r]));
        }
        return;
    }
    // Layer 2 and the two activations, software-pipelined over the
    // reflections: while the 16 products of reflection s run on the matrix
    // cores, the vector units activate layer 1 of reflection s + 1 and layer
    // 2 of reflection s - 1 (independent of them).
    f32x4 h1[2], c2p[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) h1[t][r] = act_scaled<ACT>(Y[0][t][r]);
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        f32x4 c2[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) c2[u] = f32x4{B2[u][0], B2[u][1], B2[u][2], B2[u][3]};
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int u = 0; u < 2; ++u) c2[u] = mfma4(A2[u][t][r], h1[t][r], c2[u]);
        if (s > 0) {
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int r = 0; r < 4; ++r) sink(s - 1, u, r, act_scaled<ACT>(c2p[u][r]));
        }
        if (s < 7) {
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) h1[t][r] = act_scaled<ACT>(Y[s + 1][t][r]);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) c2p[u] = c2[u];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) sink(7, u, r, act_scaled<ACT>(c2p[u][r]));
}

// The float32 network's weights in registers, from the lane table.
struct NetF32Regs {
    float A1[2][KSTEPS], A2[2][2][4], B2[2][4];
    __device__ __forceinline__ explicit NetF32Regs(const float* __restrict__ lt) {
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int st = 0; st < KSTEPS; ++st) A1[t][st] = lt[LT_A1 + t * KSTEPS + st];
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
    }
};

// The group sum of a node tile and what follows it: with sums (a step
// whose adjoint follows) the sum and tilde tau into sums[node]
// [NET_SUMS_PER_NODE] and the rates into sw, else the rates into sw; as at
// the end of network_f32's tile loop.
__device__ __forceinline__ void finish_tile(const f32x4 (&acc)[2], const float* __restrict__ lt, int q, int node,
                                            float* __restrict__ sw, float* __restrict__ sums) {
    if (sums) {
        float* __restrict__ row = sums + (size_t)node * NET_SUMS_PER_NODE;
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) row[16 * u + 4 * q + r] = acc[u][r];
        output_layer(acc, lt + LT_W3, lt + LT_B3, q, sw + node * 4, row + 32);
    } else {
        output_layer(acc, lt + LT_W3, lt + LT_B3, q, sw + node * 4);
    }
}

// s2 != nullptr (adjoint): sw receives tilde tau instead of the rates and
// s2[node][32] the group sum of the folded second-layer activations (row
// 16 u + 4 q + r in lane (q, c)).  sums != nullptr (a step whose adjoint
// follows): sw receives the rates, and sums[node][NET_SUMS_PER_NODE] (global
// memory, the block's nodes) the same group sums and tilde tau.
//
// DEPTH = 3: a third hidden layer (W2b, b2b) between the second layer and
// the group sum, one more product per group element whose B operand is the
// second layer's accumulator, like the second layer's is the first's.
// TPW: 16-node tiles per wavefront; wavefront w serves nodes
// [16 TPW w, 16 TPW (w + 1)) of the block.
template <int ACT, int DEPTH = 2, int TPW = 4>
__device__ __forceinline__ void network_f32(const float* __restrict__ sm, const int* __restrict__ sg,
                                            float* __restrict__ sw, const float* __restrict__ lt, int wave,
                                            int q, int c, float* __restrict__ s2 = nullptr,
                                            float* __restrict__ sums = nullptr) {
    float A1[2][KSTEPS], A2[2][2][4], B2[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int st = 0; st < KSTEPS; ++st) A1[t][st] = lt[LT_A1 + t * KSTEPS + st];
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
    for (int j = 0; j < TPW; ++j) {
        const int node = wave * 16 * TPW + j * 16 + c;
        const float* __restrict__ mrow = sm + node * NODE_STRIDE;
        f32x4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll 1
        for (int p = 0; p < 6; ++p) {
            f32x4 Y[8][2];
            layer1_reflections(A1, mrow, sg + (p * 4 + q) * GT_STRIDE, Y);
            if constexpr (DEPTH == 3) {
                // Unrolled: Y[s] must stay in registers.
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    float h1v[2][4];
#pragma unroll
                    for (int t = 0; t < 2; ++t)
#pragma unroll
                        for (int r = 0; r < 4; ++r) h1v[t][r] = act_scaled<ACT>(Y[s][t][r]);
                    f32x4 c2[2];
#pragma unroll
                    for (int u = 0; u < 2; ++u) c2[u] = f32x4{B2[u][0], B2[u][1], B2[u][2], B2[u][3]};
#pragma unroll
                    for (int t = 0; t < 2; ++t)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
#pragma unroll
                            for (int u = 0; u < 2; ++u) c2[u] = mfma4(A2[u][t][r], h1v[t][r], c2[u]);
                    float h2v[2][4];
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int r = 0; r < 4; ++r) h2v[u][r] = act_scaled<ACT>(c2[u][r]);
                    f32x4 c3[2];
#pragma unroll
                    for (int v = 0; v < 2; ++v)
                        c3[v] = f32x4{lt[LT_B2B + v * 4], lt[LT_B2B + v * 4 + 1], lt[LT_B2B + v * 4 + 2],
                                      lt[LT_B2B + v * 4 + 3]};
#pragma unroll
                    for (int t = 0; t < 2; ++t)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
#pragma unroll
                            for (int v = 0; v < 2; ++v)
                                c3[v] = mfma4(lt[LT_A2B + v * 8 + t * 4 + r], h2v[t][r], c3[v]);
#pragma unroll
                    for (int v = 0; v < 2; ++v)
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[v][r] += act_scaled<ACT>(c3[v][r]);
                }
                continue;
            }
            // Layer 2 and the two activations, software-pipelined over the
            // reflections: while the 16 products of reflection s run on the
            // matrix cores, the vector units activate layer 1 of reflection
            // s + 1 and layer 2 of reflection s - 1 (independent of them).
            f32x4 h1[2], c2p[2];
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) h1[t][r] = act_scaled<ACT>(Y[0][t][r]);
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                f32x4 c2[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) c2[u] = f32x4{B2[u][0], B2[u][1], B2[u][2], B2[u][3]};
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int u = 0; u < 2; ++u) c2[u] = mfma4(A2[u][t][r], h1[t][r], c2[u]);
                if (s > 0) {
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[u][r] += act_scaled<ACT>(c2p[u][r]);
                }
                if (s < 7) {
#pragma unroll
                    for (int t = 0; t < 2; ++t)
#pragma unroll
                        for (int r = 0; r < 4; ++r) h1[t][r] = act_scaled<ACT>(Y[s + 1][t][r]);
                }
#pragma unroll
                for (int u = 0; u < 2; ++u) c2p[u] = c2[u];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[u][r] += act_scaled<ACT>(c2p[u][r]);
        }
        if (s2) {
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int r = 0; r < 4; ++r) s2[node * 32 + 16 * u + 4 * q + r] = acc[u][r];
            output_layer<true>(acc, lt + LT_W3, lt + LT_B3, q, sw + node * 4);
        } else if (sums) {
            float* __restrict__ row = sums + (size_t)node * NET_SUMS_PER_NODE;
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int r = 0; r < 4; ++r) row[16 * u + 4 * q + r] = acc[u][r];
            output_layer(acc, lt + LT_W3, lt + LT_B3, q, sw + node * 4, row + 32);
        } else {
            output_layer(acc, lt + LT_W3, lt + LT_B3, q, sw + node * 4);
        }
    }
}

// Small lattices: one 16-node tile per block and its six axis permutations
// on six wavefronts (wavefront p takes permutation p), where blocks of one
// tile per wavefront leave most SIMDs idle and run the 48 group elements of
// a tile in series.  Each wavefront writes the last-layer activations of its
// permutation to vals[p][s][node][hidden] in LDS; wavefront 0 adds them in
// the order (permutation, reflection) of network_f32, so the group sums, the
// rates and the step equal those of the other block shapes bit for bit.
constexpr int PSPLIT_ROW = 36;      // floats per (p, s, node) row of vals: 32 hidden, 16-byte aligned rows
constexpr int PSPLIT_VALS = 6 * 8 * 16 * PSPLIT_ROW;
constexpr int PSPLIT_FROW = 28;     // floats per node of the pulled populations, after vals in LDS
constexpr int PSPLIT_LDS = PSPLIT_VALS + 16 * PSPLIT_FROW;

template <int ACT, int DEPTH>
__device__ __forceinline__ void network_f32_psplit(const float* __restrict__ sm, const int* __restrict__ sg,
                                                   float* __restrict__ sw, const float* __restrict__ lt, int wave,
                                                   int q, int c, float* __restrict__ vals,
                                                   float* __restrict__ sums) {
    const NetF32Regs w(lt);
    permutation_f32<ACT, DEPTH>(w.A1, w.A2, w.B2, lt, sm + c * NODE_STRIDE, sg + (wave * 4 + q) * GT_STRIDE,
                                [&](int s, int u, int r, float v) {
                                    vals[((wave * 8 + s) * 16 + c) * PSPLIT_ROW + 16 * u + 4 * q + r] = v;
                                });
    __syncthreads();
    if (wave == 0) {
        f32x4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll 4
        for (int ps = 0; ps < 48; ++ps) {
            const float* __restrict__ row = vals + (ps * 16 + c) * PSPLIT_ROW + 4 * q;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const f32x4 v = *reinterpret_cast<const f32x4*>(row + 16 * u);
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[u][r] += v[r];
            }
        }
        finish_tile(acc, lt, q, c, sw, sums);
    }
}

// Activation feeding a split layer: 2^11 r for tanh (act_split), max(x, 0)
// for ReLU.
template <int ACT>
__device__ __forceinline__ float act_into_split(float x) {
    if constexpr (ACT == ACT_TANH)
        return act_split(x);
    else
        return fmaxf(x, 0.0f);
}

// The parts of the moment operand of one axis permutation (K slot 2 w + e
// holding x[2 w + e]): f16 head and remainder for tanh, three bf16 parts
// for ReLU.
template <int ACT>
__device__ __forceinline__ void split_input(const float (&x)[8], float neg1, u32x4 (&bp)[3]) {
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        if constexpr (ACT == ACT_TANH) {
            bp[0][w] = pack_f16(x[2 * w], x[2 * w + 1]);
            bp[1][w] = residual_f16(bp[0][w], x[2 * w], x[2 * w + 1], neg1);
            bp[2][w] = 0u;
        } else {
            unsigned h, m, t;
            split3_bf16(x[2 * w], x[2 * w + 1], h, m, t);
            bp[0][w] = h;
            bp[1][w] = m;
            bp[2][w] = t;
        }
    }
}

// The split products of one 16-row tile of A with the parts bp of B,
// accumulated from c: Ah Bh + Ah Bl + Al Bh (f16, tanh) or the six bf16
// products whose parts' orders sum to at most 2 (ReLU).
template <int ACT>
__device__ __forceinline__ f32x4 split_product(const u32x4 (&A)[3], const u32x4 (&bp)[3], f32x4 c) {
    if constexpr (ACT == ACT_TANH) {
        c = mfma32h(A[0], bp[0], c);
        c = mfma32h(A[0], bp[1], c);
        return mfma32h(A[1], bp[0], c);
    } else {
        c = mfma32(A[0], bp[0], c);
        c = mfma32(A[0], bp[1], c);
        c = mfma32(A[1], bp[0], c);
        c = mfma32(A[0], bp[2], c);
        c = mfma32(A[2], bp[0], c);
        return mfma32(A[1], bp[1], c);
    }
}

// One split layer: the pre-activations c[u] (rows 16 u + 4 q + r, f32x4 over
// r) of A h + b for the activations h[t][r] (hidden unit 16 t + 4 q + r) of
// the previous layer, K slot 2 w + e of the products holding
// h[w / 2][2 (w % 2) + e].
//   tanh: h = 2^11 r (act_split), A = sigma W (sigma a power of two putting
//     max |A| in [128, 256)); each split into an f16 head and the f16
//     remainder, A h = Ah hh + Ah hl + Al hh (the dropped Al hl is below
//     2^-22 |A h|), three f16 products accumulated in float32 from
//     sigma 2^11 b, times back = 1 / (sigma 2^11).
//   ReLU: h unbounded, so three bf16 parts of each (split3_bf16), unscaled,
//     and the six products whose parts' orders sum to at most 2 (the dropped
//     ones are below 2^-23 |A h|), accumulated from b.
// A[u][part]: the operand parts of the layer (A[u][2] unused for tanh).
template <int ACT>
__device__ __forceinline__ void split_layer(const u32x4 (&A)[2][3], const float (&b)[2][4], float back, float neg1,
                                            const float (&h)[2][4], f32x4 (&c)[2]) {
    float x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = h[i >> 2][i & 3];
    u32x4 bp[3];
    split_input<ACT>(x, neg1, bp);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        c[u] = split_product<ACT>(A[u], bp, f32x4{b[u][0], b[u][1], b[u][2], b[u][3]});
        if constexpr (ACT == ACT_TANH) c[u] *= back;
    }
}

// Float32-class network on the f16 / bf16 matrix cores, the products equal
// to float32's to a few units of its rounding.  tanh: every layer but the
// output one as split f16 products, layer 1 per group element like the
// bf16 network (the reflections as sign flips of the moment operand's
// parts, in Gray-code order) and scaled back by 1 / sigma_1; 12 products of
// 16x16x32 per group element and 16-node tile at depth 2.  ReLU: layer 1 on
// the float32 matrix cores with the Walsh-Hadamard fold (layer1_reflections;
// split into three bf16 parts it would take 12 more products, and these
// kernels are bound by the matrix cores), the hidden-to-hidden layers as 12
// split bf16 products each.
template <int ACT, int DEPTH = 2, int TPW = 4>
__device__ __forceinline__ void network_split(const float* __restrict__ sm, const int* __restrict__ sg,
                                              float* __restrict__ sw, const float* __restrict__ lt, int wave, int q,
                                              int c) {
    const unsigned* __restrict__ lw = reinterpret_cast<const unsigned*>(lt);
    constexpr int NP = ACT == ACT_TANH ? 2 : 3;
    float B2[2][4], B3[2][4], A1[2][KSTEPS];
    u32x4 AS1[2][3], AS2[2][3], AS3[2][3], SM[3];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const unsigned* w1 = lw + LS_A1 + 12 * u + 4 * k;
            const unsigned* w2 = lw + LS_A2 + 12 * u + 4 * k;
            if constexpr (ACT == ACT_TANH)
                AS1[u][k] = k < NP ? u32x4{w1[0], w1[1], w1[2], w1[3]} : u32x4{0u, 0u, 0u, 0u};
            AS2[u][k] = k < NP ? u32x4{w2[0], w2[1], w2[2], w2[3]} : u32x4{0u, 0u, 0u, 0u};
            if constexpr (DEPTH == 3) {
                const unsigned* w3 = lw + LS_A3 + 12 * u + 4 * k;
                AS3[u][k] = k < NP ? u32x4{w3[0], w3[1], w3[2], w3[3]} : u32x4{0u, 0u, 0u, 0u};
            }
        }
    if constexpr (ACT == ACT_TANH) {
#pragma unroll
        for (int b = 0; b < 3; ++b)
            SM[b] = u32x4{lw[LS_SM + 4 * b], lw[LS_SM + 4 * b + 1], lw[LS_SM + 4 * b + 2], lw[LS_SM + 4 * b + 3]};
    } else {
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int st = 0; st < KSTEPS; ++st) A1[t][st] = lt[LT_A1 + t * KSTEPS + st];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            B2[u][r] = lt[LS_B2 + u * 4 + r];
            B3[u][r] = DEPTH == 3 ? lt[LS_B3 + u * 4 + r] : 0.0f;
        }
    const float back1 = lt[LS_BACK], back2 = lt[LS_BACK + 1], back3 = lt[LS_BACK + 2], neg1 = lt[LS_NEG1];

#pragma unroll 1
    for (int j = 0; j < TPW; ++j) {
        const int node = wave * 16 * TPW + j * 16 + c;
        const float* __restrict__ mrow = sm + node * NODE_STRIDE;
        f32x4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll 1
        for (int p = 0; p < 6; ++p) {
            const int* __restrict__ ge = sg + (p * 4 + q) * GT_STRIDE;
            u32x4 bp[3];
            f32x4 Y[8][2];
            if constexpr (ACT == ACT_TANH) {
                float x[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) x[i] = mrow[ge[i]];
                split_input<ACT>(x, neg1, bp);
            } else {
                layer1_reflections(A1, mrow, ge, Y);
            }
            // tanh: the 8 reflections in Gray-code order, consecutive ones
            // differing in one reflection bit: one mask XOR per word and part.
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                float h1[2][4];
                if constexpr (ACT == ACT_TANH) {
                    if (k > 0)
#pragma unroll
                        for (int e = 0; e < NP; ++e) bp[e] ^= SM[__builtin_ctz(k)];
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        const f32x4 c1 = split_product<ACT>(AS1[t], bp, f32x4{0.f, 0.f, 0.f, 0.f}) * back1;
#pragma unroll
                        for (int r = 0; r < 4; ++r) h1[t][r] = act_into_split<ACT>(c1[r]);
                    }
                } else {
#pragma unroll
                    for (int t = 0; t < 2; ++t)
#pragma unroll
                        for (int r = 0; r < 4; ++r) h1[t][r] = act_into_split<ACT>(Y[k][t][r]);
                }
                f32x4 cz[2];
                split_layer<ACT>(AS2, B2, back2, neg1, h1, cz);
                if constexpr (DEPTH == 3) {
                    float h2[2][4];
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int r = 0; r < 4; ++r) h2[u][r] = act_into_split<ACT>(cz[u][r]);
                    split_layer<ACT>(AS3, B3, back3, neg1, h2, cz);
                }
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[u][r] += act_scaled<ACT>(cz[u][r]);
            }
        }
        output_layer(acc, lt + LS_W3, lt + LS_B3O, q, sw + node * 4);
    }
}

// DEPTH 3: the third hidden layer as one more bf16 product per group
// element, fed by the second layer's activations packed like the first's.
template <int ACT, int DEPTH = 2, int TPW = 4>
__device__ __forceinline__ void network_bf16(const float* __restrict__ sm, const int* __restrict__ sg,
                                             float* __restrict__ sw, const float* __restrict__ lt, int wave,
                                             int q, int c) {
    const unsigned* __restrict__ lw = reinterpret_cast<const unsigned*>(lt);
    u32x4 A1[2], A2[2], SM[3], A3[2];
    float B2[2][4], B3[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
        A1[t] = u32x4{lw[LB_A1 + 4 * t], lw[LB_A1 + 4 * t + 1], lw[LB_A1 + 4 * t + 2], lw[LB_A1 + 4 * t + 3]};
#pragma unroll
    for (int u = 0; u < 2; ++u)
        A2[u] = u32x4{lw[LB_A2 + 4 * u], lw[LB_A2 + 4 * u + 1], lw[LB_A2 + 4 * u + 2], lw[LB_A2 + 4 * u + 3]};
#pragma unroll
    for (int b = 0; b < 3; ++b)
        SM[b] = u32x4{lw[LB_SM + 4 * b], lw[LB_SM + 4 * b + 1], lw[LB_SM + 4 * b + 2], lw[LB_SM + 4 * b + 3]};
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) B2[u][r] = lt[LB_B2 + u * 4 + r];
    if constexpr (DEPTH == 3) {
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            A3[v] = u32x4{lw[LB_A2B + 4 * v], lw[LB_A2B + 4 * v + 1], lw[LB_A2B + 4 * v + 2], lw[LB_A2B + 4 * v + 3]};
#pragma unroll
            for (int r = 0; r < 4; ++r) B3[v][r] = lt[LB_B2B + v * 4 + r];
        }
    }

#pragma unroll 1
    for (int j = 0; j < TPW; ++j) {
        const int node = wave * 16 * TPW + j * 16 + c;
        const float* __restrict__ mrow = sm + node * NODE_STRIDE;
        f32x4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll 1
        for (int p = 0; p < 6; ++p) {
            const int* __restrict__ ge = sg + (p * 4 + q) * GT_STRIDE;
            float x[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = mrow[ge[i]];
            const u32x4 xb = {pack_bf16(x[0], x[1]), pack_bf16(x[2], x[3]), pack_bf16(x[4], x[5]),
                              pack_bf16(x[6], x[7])};
            // The 8 reflections in Gray-code order k ^ (k >> 1): consecutive
            // ones differ in one reflection bit (bit ctz(k)), so one mask XOR
            // per word moves to the next instead of one per set bit.
            u32x4 bs = xb;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (k > 0) bs ^= SM[__builtin_ctz(k)];
                f32x4 c1[2];
#pragma unroll
                for (int t = 0; t < 2; ++t) c1[t] = mfma32(A1[t], bs, f32x4{0.f, 0.f, 0.f, 0.f});
                float h[2][4];
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) h[t][r] = act_scaled<ACT>(c1[t][r]);
                const u32x4 hb = {pack_bf16(h[0][0], h[0][1]), pack_bf16(h[0][2], h[0][3]),
                                  pack_bf16(h[1][0], h[1][1]), pack_bf16(h[1][2], h[1][3])};
                f32x4 c2[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) c2[u] = mfma32(A2[u], hb, f32x4{B2[u][0], B2[u][1], B2[u][2], B2[u][3]});
                if constexpr (DEPTH == 3) {
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int r = 0; r < 4; ++r) h[u][r] = act_scaled<ACT>(c2[u][r]);
                    const u32x4 h2b = {pack_bf16(h[0][0], h[0][1]), pack_bf16(h[0][2], h[0][3]),
                                       pack_bf16(h[1][0], h[1][1]), pack_bf16(h[1][2], h[1][3])};
#pragma unroll
                    for (int v = 0; v < 2; ++v)
                        c2[v] = mfma32(A3[v], h2b, f32x4{B3[v][0], B3[v][1], B3[v][2], B3[v][3]});
                }
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[u][r] += act_scaled<ACT>(c2[u][r]);
            }
        }
        output_layer(acc, lt + LB_W3, lt + LB_B3, q, sw + node * 4);
    }
}

// RATES = true: no streaming, the rates of the stored state are written to
// omega_out [4][n] instead of a step (readout and tests of the network alone).
// Work space of one block in LDS, declared by each kernel.  A block serves
// NODES = 256 or 64 nodes with TPW 16-node tiles per wavefront, so
// 64 NODES / (16 TPW) threads: 256 nodes on 4 wavefronts (TPW 4), 64 nodes on
// one wavefront (TPW 4) or on 4 wavefronts of one tile each (TPW 1, the
// shortest serial chain per wavefront, for small lattices).  The wavefronts
// of a block share only the gather table; every variant does the same
// arithmetic per node.
struct BlockLds {
    float* sm;      // [NODES][NODE_STRIDE] moments, then hidden activations
    int* sg;        // [GT_ENTRIES] gather table
    float* sw;      // [NODES][4] rates
    float* vals = nullptr;  // [PSPLIT_VALS] last-layer activations (six-wavefront tiles)
};

template <int S, int ACT, bool RATES, int PREC, int NODES, int DEPTH = 2, int TPW = 4, bool SUMS = false>
__device__ __forceinline__ void nco_mfma_block(const typename Codec<S>::store_t* __restrict__ fin,
                                               typename Codec<S>::store_t* __restrict__ fout, const StepArgs& a,
                                               const float* __restrict__ lane_tab, const int* __restrict__ gtab,
                                               double* __restrict__ omega_out, int blk, BlockLds lds);

#define NCO_BLOCK_LDS(NODES)                         \
    __shared__ float lds_sm[(NODES) * NODE_STRIDE];  \
    __shared__ int lds_sg[GT_ENTRIES];               \
    __shared__ float lds_sw[(NODES) * 4];            \
    const BlockLds lds{lds_sm, lds_sg, lds_sw};

// TPW = 0: the six-wavefront tile of network_f32_psplit (16 nodes).
constexpr int mfma_block_threads(int nodes, int tpw) { return tpw == 0 ? 6 * 64 : nodes / (16 * tpw) * 64; }

// XCD-aware block order: workgroups are dispatched to the 8 XCDs in turn
// (workgroup b to XCD b mod 8), each XCD with its own L2.  Block b takes
// the logical block that makes the blocks of one XCD a contiguous run of
// the lattice (XCD x: its i-th block is the i-th of the x-th run), so the
// halo rows that neighbouring blocks share, and the second pull after the
// network, meet in that XCD's L2.  A bijection of [0, n): the results do
// not depend on it.
__device__ __forceinline__ int xcd_block(int b, int n) {
    constexpr int XCDS = 8;
    const int x = b % XCDS, i = b / XCDS, q = n / XCDS, r = n % XCDS;
    return x * q + min(x, r) + i;
}

// Waves per SIMD the register allocation must leave room for: 3 for the
// split networks (156 VGPRs for tanh at depth 2; the others spill 12-57
// registers into scratch and still run 1-7 % faster than at 2 waves, the
// third wave keeping their vector instructions issuing) and for the float32
// depth-3 steps (the instantiation with the network-value branch, 177
// VGPRs unconstrained; at 168, 0-17 spilled, 4 % faster at 128^3 and 8 % on
// a 16^3 lattice), 4 for the bf16 depth-3 steps (ReLU 132 VGPRs
// unconstrained, 128 without spills at 4 waves, 2 % faster), no constraint
// otherwise.
constexpr int mfma_min_waves(int prec, int depth, bool sums) {
    return prec == MLP_PREC_BF16 && depth == 3 ? 4
           : prec == MLP_PREC_F32S || (prec == MLP_PREC_F32 && depth == 3 && sums) ? 3
                                                                                     : 1;
}

template <int S, int ACT, bool RATES, int PREC, int NODES, int DEPTH, int TPW, bool SUMS = false>
__global__ __launch_bounds__(mfma_block_threads(NODES, TPW))
__attribute__((amdgpu_waves_per_eu(mfma_min_waves(PREC, DEPTH, SUMS)))) void k_nco_mfma(
    const typename Codec<S>::store_t* __restrict__ fin, typename Codec<S>::store_t* __restrict__ fout,
    StepArgs a, const float* __restrict__ lane_tab, const int* __restrict__ gtab, double* __restrict__ omega_out) {
    NCO_BLOCK_LDS(NODES)
    if constexpr (TPW == 0) {
        __shared__ __align__(16) float lds_vals[PSPLIT_LDS];
        BlockLds lv = lds;
        lv.vals = lds_vals;
        nco_mfma_block<S, ACT, RATES, PREC, NODES, DEPTH, TPW, SUMS>(fin, fout, a, lane_tab, gtab, omega_out,
                                                               xcd_block(blockIdx.x, gridDim.x), lv);
    } else {
        nco_mfma_block<S, ACT, RATES, PREC, NODES, DEPTH, TPW, SUMS>(fin, fout, a, lane_tab, gtab, omega_out,
                                                               xcd_block(blockIdx.x, gridDim.x), lds);
    }
}

template <int S, int ACT, int PREC>
__device__ __forceinline__ void grouped_block(const GroupDesc& d, int blk, BlockLds lds) {
    using T = typename Codec<S>::store_t;
    // The float32 network through the instantiation with the (here unused)
    // network-value branch, for its register allocation (see
    // launch_mfma_kind).
    nco_mfma_block<S, ACT, false, PREC, 256, 2, 4, PREC == MLP_PREC_F32>(
        static_cast<const T*>(d.fin), static_cast<T*>(d.fout), d.a, d.lane_tab, d.gtab, nullptr, blk, lds);
}

// One step of several lattices with the same storage, activation and
// network arithmetic.
template <int S, int ACT, int PREC>
__global__ __launch_bounds__(256) void k_nco_mfma_grouped(LaunchGroup g) {
    NCO_BLOCK_LDS(256)
    const int i = group_member(g, blockIdx.x);
    grouped_block<S, ACT, PREC>(g.d[i], blockIdx.x - g.prefix[i], lds);
}

template <int S, int ACT, bool RATES, int PREC, int NODES, int DEPTH, int TPW, bool SUMS>
__device__ __forceinline__ void nco_mfma_block(const typename Codec<S>::store_t* __restrict__ fin,
                                               typename Codec<S>::store_t* __restrict__ fout, const StepArgs& a,
                                               const float* __restrict__ lane_tab, const int* __restrict__ gtab,
                                               double* __restrict__ omega_out, int blk, BlockLds lds) {
    constexpr int THREADS = mfma_block_threads(NODES, TPW);
    float* __restrict__ sm = lds.sm;
    int* __restrict__ sg = lds.sg;
    float* __restrict__ sw = lds.sw;
    const int tid = threadIdx.x;
    const int idx = blk * NODES + tid;
    const bool live = (THREADS == NODES || tid < NODES) && idx < a.n;

    for (int e = tid; e < GT_ENTRIES; e += THREADS) sg[e] = gtab[e];

    // Phase A: pull and transform to moments.
    if constexpr (TPW == 0) {
        // Six-wavefront tiles: the tile's 16 x 27 pulls spread over the
        // block's threads (each a load or a folded one at the faces of the
        // reduced cube), kept in LDS for the relaxation as well.
        static_assert(!RATES, "six-wavefront tiles run steps");
        float* __restrict__ fl = lds.vals + PSPLIT_VALS;
        for (int e = tid; e < NODES * Q; e += THREADS) {
            const int nd = e % NODES, i = e / NODES, id = blk * NODES + nd;
            fl[nd * PSPLIT_FROW + i] =
                id < a.n ? pull_one<S>(fin, a, node_of(id, a.nx, a.ny), i) : (float)weight_of(i);
        }
        __syncthreads();
        if (tid < NODES) {
            float f[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) f[i] = fl[tid * PSPLIT_FROW + i];
            float m[Q];
            to_moments(f, m);
            float* row = sm + tid * NODE_STRIDE;
#pragma unroll
            for (int k = 0; k < Q; ++k) row[k] = m[row_tensor(k)];
            row[27] = 1.0f;
            row[28] = 0.0f;
        }
    } else if (THREADS == NODES || tid < NODES) {
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

    // Phase B: the network, one wavefront per 64 nodes.
    {
        const int lane = tid & 63;
        const float* __restrict__ lt = lane_tab + lane * LANE_WORDS;
        if constexpr (TPW == 0) {
            static_assert(PREC == MLP_PREC_F32 && NODES == 16, "six-wavefront tiles: the float32 network");
            float* sums = SUMS && a.net_sums ? a.net_sums + (size_t)blk * NODES * NET_SUMS_PER_NODE : nullptr;
            network_f32_psplit<ACT, DEPTH>(sm, sg, sw, lt, tid >> 6, lane >> 4, lane & 15, lds.vals, sums);
        } else if constexpr (PREC == MLP_PREC_BF16) {
            network_bf16<ACT, DEPTH, TPW>(sm, sg, sw, lt, tid >> 6, lane >> 4, lane & 15);
        } else if constexpr (PREC == MLP_PREC_F32S) {
            static_assert(!SUMS, "the split arithmetic keeps no network values");
            network_split<ACT, DEPTH, TPW>(sm, sg, sw, lt, tid >> 6, lane >> 4, lane & 15);
        } else if constexpr (SUMS) {
            // Keeps the network values when a.net_sums is set, else a plain
            // step (a uniform branch after each tile).
            float* sums = a.net_sums ? a.net_sums + (size_t)blk * NODES * NET_SUMS_PER_NODE : nullptr;
            network_f32<ACT, DEPTH, TPW>(sm, sg, sw, lt, tid >> 6, lane >> 4, lane & 15, nullptr, sums);
        } else {
            network_f32<ACT, DEPTH, TPW>(sm, sg, sw, lt, tid >> 6, lane >> 4, lane & 15);
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
        if constexpr (TPW == 0) {
#pragma unroll
            for (int i = 0; i < Q; ++i) f[i] = lds.vals[PSPLIT_VALS + tid * PSPLIT_FROW + i];
        } else {
            pull<S>(fin, a, node_of(idx, a.nx, a.ny), f);
        }
        const float* row = sm + tid * NODE_STRIDE;
#pragma unroll
        for (int k = 0; k < Q; ++k) m[row_tensor(k)] = row[k];
        float omega[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) omega[n] = sw[tid * 4 + n];
        float dm[Q], df[Q];
        if (a.n_modes > 0) {
            float Fx, Fy, Fz;
            read_force(a, idx, Fx, Fy, Fz);
            collision_delta<float, true>(m, a.omega_nu_f, omega, Fx, Fy, Fz, dm);
        } else {
            collision_delta<float, false>(m, a.omega_nu_f, omega, 0.f, 0.f, 0.f, dm);
        }
        from_moments(dm, df);
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] -= df[i];
        store_local<S>(fout, a.n, idx, f, a.sr_key);
    }
}

// ---------------------------------------------------------------- adjoint --
//
// Reverse mode of one step on the matrix cores (float32), the same
// computation as the vector-unit adjoint (adjoint.hip): given lambda =
// dL/dx_t+1, the pre-collision adjoint M^T g_m + lambda is scattered back
// along the streaming, and the parameter gradient of this step is added to
// the block's row of `partial` (float64, one row per block, each row touched
// by its block only, so the sum over steps is in a fixed order).
//
// Per node tile of 16 and group element g = (pi, s), in the layout of the
// forward network (hidden x nodes, lane (q, c) holding rows 4q..4q+3 of
// node c):
//   forward recompute   r1 = act(Z1), r2 = act(Z2)          (forward tables)
//   dz2 = dh2 (.) act'(z2),   dh2 = W3 dtt / 48 (the same for every g)
//   dh1 = W2 dz2,   dz1 = dh1 (.) act'(z1)                 (products whose
//         B operands are the previous accumulators, as in the forward)
//   Z_cl = sum_s chi_s(cl) dz1_s over the 8 reflections s of the
//         permutation (Walsh-Hadamard transform), for the 8 parity classes
//   dL/dm[src_pi(k)] += (W1 Z_class(k))[k]                   (through LDS)
//   dW2 += h1 dz2^T per element, dW1 += x_pi Z_class^T per class (the bias
//   row of x_pi gives db1), db2 += dz2                       (products over
//         the 16 nodes of the tile: h1, dz2 and Z are transposed through
//         a per-wave LDS buffer so that the node index becomes K)
// For tanh, with r = 1 / (1 + 2^(kappa z)): h = 1 - 2 r, act' = 4 r (1 - r).

// Per-lane table of the adjoint (4-byte words per lane).
// The reverse step's input-row tiles hold the moment rows (and the bias row
// 27) grouped by parity class, four classes per 16-row tile, so that the
// products through the first layer run once per class (see k_adjoint_mfma):
// positions 0-15 hold the classes 0 (with row 27), 1, 3, 7; positions 16-27
// the classes 2, 4, 5, 6; positions 28-31 are empty (row 28, zero).
__host__ __device__ constexpr int adj_tile_class(int kt, int i) {
    constexpr int c[2][4] = {{0, 1, 3, 7}, {2, 4, 5, 6}};
    return c[kt][i];
}
__host__ __device__ constexpr int moment_class(int k) {
    return k >= 27 ? 0 : (row_tensor(k) % 3) % 2 + 2 * (((row_tensor(k) / 3) % 3) % 2) + 4 * ((row_tensor(k) / 9) % 2);
}
// Row of M (27 = bias row, 28 = empty) at tile position p.
__host__ __device__ constexpr int adj_row(int p) {
    for (int kt = 0; kt < 2; ++kt) {
        int pos = 16 * kt;
        for (int i = 0; i < 4; ++i)
            for (int k = 0; k < 28; ++k)
                if (moment_class(k) == adj_tile_class(kt, i)) {
                    if (pos == p) return k;
                    ++pos;
                }
        if (p < 16 * (kt + 1)) return 28;
    }
    return 28;
}

constexpr int AT_W2T = 0;           // [t 2][u 2][r 4]  W2[16 t + c][16 u + 4 q + r]
constexpr int AT_W1T = 16;          // [kt 2][t 2][r 4] W1[adj_row(16 kt + c)][16 t + 4 q + r] (rows >= 27: 0)
constexpr int AT_W3 = 32;           // [u 2][r 4][n 4]  W3[16 u + 4 q + r][n] / 48
constexpr int AT_CLS = 64;          // [kt 2][r 4]      class of position 16 kt + 4 q + r (-1: empty) (int)
constexpr int AT_CLSC = 72;         // [kt 2]           class of position 16 kt + c (-1: empty) (int)
constexpr int AT_ROWO = 74;         // [kt 2][r 4]      adj_row(16 kt + 4 q + r) (int)
constexpr int AT_ROWC = 82;         // [kt 2]           adj_row(16 kt + c) (int)
constexpr int ADJ_WORDS = 84;
constexpr int ADJ_ROWS_AT = 64 * ADJ_WORDS;   // then [32] adj_row(p) (int), shared by all lanes
constexpr int TB = 32;              // row stride of the per-wave transpose buffers

// Column swizzle of row n of a per-wave transpose buffer: element (n, h) is
// kept at n TB + (h ^ tr_swz(n)).  The buffers are written as (node c,
// hidden 16 t + 4 q + r) and read as (node 4 st + q, hidden 16 x + c) by
// the lanes (q, c); with node bits 0, 1, 2, 3 sent to column bits 4, 0, 1, 3
// both patterns reach 32 distinct banks in each half-wavefront.
__device__ __forceinline__ int tr_swz(int n) {
    return ((n & 1) << 4) | ((n >> 1) & 1) | (((n >> 2) & 1) << 1) | (((n >> 3) & 1) << 3);
}


template <int ACT>
__device__ __forceinline__ float act_grad(float r) {
    if constexpr (ACT == ACT_RELU)
        return r > 0.0f ? 1.0f : 0.0f;
    else
        return 4.0f * r * (1.0f - r);
}

template <int ACT>
__device__ __forceinline__ float act_value(float r) {
    if constexpr (ACT == ACT_RELU)
        return r;
    else
        return 1.0f - 2.0f * r;
}

// TPW = 4: 256 nodes per block, 4 tiles per wavefront; TPW = 1: 64 nodes
// per block, one tile per wavefront (a 4x shorter serial chain for lattices
// too small to fill the device with 256-node blocks).
template <int S, int ACT, int TPW>
__global__ __launch_bounds__(256) void k_adjoint_mfma(const typename Codec<S>::store_t* __restrict__ xin,
                                                      const float* __restrict__ lam_in, float* __restrict__ lam_out,
                                                      StepArgs a, const float* __restrict__ lane_tab,
                                                      const int* __restrict__ gtab, const float* __restrict__ adj_tab,
                                                      const int* __restrict__ gsrc, double* __restrict__ partial) {
    __shared__ float sm[256 * NODE_STRIDE];     // moments (row order of M; [27] = 1, [28] = 0)
    __shared__ int sg[GT_ENTRIES];              // forward gather table
    __shared__ int sgs[6 * 27];                 // source rows of the reflection-free elements g = 8 pi
    __shared__ float sw[256 * 4];               // tilde tau, then dL/d tilde tau
    __shared__ float som[256 * 4];              // rates omega_3..omega_6
    __shared__ float sF[256 * 3];               // body force
    __shared__ float sdm[256 * 32];             // group sums of the second layer, then dL/dm (network part)
    __shared__ float sbuf[4][3][16 * TB];       // per-wave transposes
    const int tid = threadIdx.x;
    constexpr int NB = 64 * TPW;                // nodes of the block
    const int idx = blockIdx.x * NB + tid;
    const bool live = (NB == 256 || tid < NB) && idx < a.n;
    const NodeIdx p = node_of(live ? idx : 0, a.nx, a.ny);

    for (int e = tid; e < GT_ENTRIES; e += 256) sg[e] = gtab[e];
    for (int e = tid; e < 6 * 27; e += 256) sgs[e] = gsrc[(e / 27) * 8 * 27 + e % 27] & 31;
    // Phase A: moments of the pulled state, body force.
    {
        float f[Q], m[Q];
        if (live) {
            pull<S>(xin, a, p, f);
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i) f[i] = (float)weight_of(i);
        }
        to_moments(f, m);
        float* row = sm + tid * NODE_STRIDE;
#pragma unroll
        for (int k = 0; k < Q; ++k) row[k] = m[row_tensor(k)];
        row[27] = 1.0f;
        row[28] = 0.0f;
        float Fd[3] = {0.0f, 0.0f, 0.0f};
        if (a.n_modes > 0 && live) read_force(a, idx, Fd[0], Fd[1], Fd[2]);
#pragma unroll
        for (int d = 0; d < 3; ++d) sF[tid * 3 + d] = Fd[d];
    }
    __syncthreads();

    const int wave = tid >> 6, lane = tid & 63, q = lane >> 4, c = lane & 15;
    // Phase B1: the network forward for tilde tau and the group sums, or the
    // values the forward step of this state kept (the same arithmetic on the
    // same moments, so the same values).
    if (a.net_sums) {
        if (tid < NB) {
            const float* __restrict__ src = a.net_sums + ((size_t)blockIdx.x * NB + tid) * NET_SUMS_PER_NODE;
#pragma unroll
            for (int k = 0; k < 32; ++k) sdm[tid * 32 + k] = src[k];
#pragma unroll
            for (int n = 0; n < 4; ++n) sw[tid * 4 + n] = src[32 + n];
        }
    } else {
        network_f32<ACT, 2, TPW>(sm, sg, sw, lane_tab + lane * LANE_WORDS, wave, q, c, sdm);
    }
    __syncthreads();

    // Phase B2: per node, dL/d tilde tau from the node-local collision adjoint.
    {
        float m[Q], lam[Q], nu[Q], gm[Q], omega[4], tau[4], e[4], domega[4];
        const float* row = sm + tid * NODE_STRIDE;
#pragma unroll
        for (int k = 0; k < Q; ++k) m[row_tensor(k)] = row[k];
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            e[n] = expf(sw[tid * 4 + n]);
            tau[n] = 0.5f + 0.5f / (1.0f + e[n]);
            omega[n] = 1.0f / tau[n];
            som[tid * 4 + n] = omega[n];
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) lam[i] = live ? lam_in[(size_t)i * a.n + idx] : 0.0f;
        inverse_T(lam, nu);
        const float F[3] = {sF[tid * 3], sF[tid * 3 + 1], sF[tid * 3 + 2]};
        collision_vjp_local(m, nu, a.omega_nu_f, omega, a.n_modes > 0, F, gm, domega);
#pragma unroll
        for (int n = 0; n < 4; ++n)
            sw[tid * 4 + n] = domega[n] * 0.5f * e[n] / ((1.0f + e[n]) * (1.0f + e[n]) * tau[n] * tau[n]);
    }
    __syncthreads();

    // Output layer: dW3 = sum (H2 / 48) dtt^T with H2 the group sum of the
    // (unfolded) second-layer activations, db3 = sum dtt.
    double* __restrict__ out = partial + (size_t)blockIdx.x * NPAR;
    if (tid < 132) {
        double sacc = 0.0;
        if (tid < 128) {
            const int o = tid >> 2, n = tid & 3;
            float v = 0.0f;
            for (int nd = 0; nd < NB; ++nd) {
                const float acc = sdm[nd * 32 + o];
                const float h2 = ACT == ACT_RELU ? acc : (float)NGROUP - 2.0f * acc;
                v = fmaf(h2 * (1.0f / NGROUP), sw[nd * 4 + n], v);
            }
            sacc = v;
            out[OFF_W3 + o * 4 + n] += sacc;
        } else {
            const int n = tid - 128;
            float v = 0.0f;
            for (int nd = 0; nd < NB; ++nd) v += sw[nd * 4 + n];
            out[OFF_B3 + n] += (double)v;
        }
    }
    __syncthreads();
    for (int k = 0; k < 32; ++k) sdm[tid * 32 + k] = 0.0f;
    __syncthreads();

    // Phase B3: the network adjoint on the matrix cores.
    f32x4 gW2[2][2], gW1[2][2];
    float gb2[2][4];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            gW2[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};
            gW1[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) gb2[u][r] = 0.0f;
    {
        const float* __restrict__ lt = lane_tab + lane * LANE_WORDS;
        const float* __restrict__ at = adj_tab + lane * ADJ_WORDS;
        const int* __restrict__ ati = reinterpret_cast<const int*>(at);
        float A1[2][KSTEPS], A2[2][2][4], B2[2][4], W2T[2][2][4], W1T[2][2][4];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int st = 0; st < KSTEPS; ++st) A1[t][st] = lt[LT_A1 + t * KSTEPS + st];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    A2[u][t][r] = lt[LT_A2 + u * 8 + t * 4 + r];
                    W2T[t][u][r] = at[AT_W2T + t * 8 + u * 4 + r];
                    W1T[u][t][r] = at[AT_W1T + u * 8 + t * 4 + r];
                }
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) B2[u][r] = lt[LT_B2 + u * 4 + r];
        int cls[2][4], clsc[2], rowo[2][4], rowc[2];
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) {
            clsc[kt] = ati[AT_CLSC + kt];
            rowc[kt] = ati[AT_ROWC + kt];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                cls[kt][r] = ati[AT_CLS + kt * 4 + r];
                rowo[kt][r] = ati[AT_ROWO + kt * 4 + r];
            }
        }
        float* __restrict__ bh = sbuf[wave][0];
        float* __restrict__ bz2 = sbuf[wave][1];
        float* __restrict__ bz1 = sbuf[wave][2];
        const int swz_w = tr_swz(c);

#pragma unroll 1
        for (int j = 0; j < TPW; ++j) {
            const int base = wave * 16 * TPW + j * 16;
            const int node = base + c;
            const float* __restrict__ mrow = sm + node * NODE_STRIDE;
            // dh2 = W3 dtt / 48 for this lane's rows.
            float dh2[2][4];
            {
                float dt[4];
#pragma unroll
                for (int n = 0; n < 4; ++n) dt[n] = sw[node * 4 + n];
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        float v = 0.0f;
#pragma unroll
                        for (int n = 0; n < 4; ++n) v = fmaf(at[AT_W3 + (u * 4 + r) * 4 + n], dt[n], v);
                        dh2[u][r] = v;
                    }
            }
#pragma unroll 1
            for (int pi = 0; pi < 6; ++pi) {
                // Layer 1 of the eight reflections (as in the forward).
                const int* __restrict__ ge = sg + (pi * 4 + q) * GT_STRIDE;
                float b[KSTEPS];
#pragma unroll
                for (int st = 0; st < KSTEPS; ++st) b[st] = mrow[ge[st]];
                f32x4 Y[8][2];
#pragma unroll
                for (int ci = 0; ci < 8; ++ci) {
                    Y[ci][0] = f32x4{0.f, 0.f, 0.f, 0.f};
                    Y[ci][1] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
#pragma unroll
                for (int st = 0; st < KSTEPS; ++st)
#pragma unroll
                    for (int t = 0; t < 2; ++t) Y[step_class(st)][t] = mfma4(A1[t][st], b[st], Y[step_class(st)][t]);
#pragma unroll
                for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
                    for (int ci = 0; ci < 8; ++ci)
                        if (!(ci & bit))
#pragma unroll
                            for (int t = 0; t < 2; ++t) {
                                const f32x4 u0 = Y[ci][t], u1 = Y[ci | bit][t];
                                Y[ci][t] = u0 + u1;
                                Y[ci | bit][t] = u0 - u1;
                            }
                // x_pi (reflection-free input) in the A layout of the dW1
                // product: the row at position 16 kt + c, node 4 st + q of
                // the tile.
                float xa[2][4];
#pragma unroll
                for (int kt = 0; kt < 2; ++kt) {
                    const int k = rowc[kt];
                    const int src = k < 27 ? sgs[pi * 27 + k] : k;
#pragma unroll
                    for (int st = 0; st < 4; ++st) xa[kt][st] = sm[(base + 4 * st + q) * NODE_STRIDE + src];
                }
                f32x4 Z[8][2];                  // dz1 of reflection s, then its class transform

#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    float r1[2][4], d1[2][4];
#pragma unroll
                    for (int t = 0; t < 2; ++t)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            r1[t][r] = act_scaled<ACT>(Y[s][t][r]);
                            d1[t][r] = act_grad<ACT>(r1[t][r]);
                        }
                    f32x4 c2[2];
#pragma unroll
                    for (int u = 0; u < 2; ++u) c2[u] = f32x4{B2[u][0], B2[u][1], B2[u][2], B2[u][3]};
#pragma unroll
                    for (int t = 0; t < 2; ++t)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
#pragma unroll
                            for (int u = 0; u < 2; ++u) c2[u] = mfma4(A2[u][t][r], r1[t][r], c2[u]);
                    float dz2[2][4];
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            dz2[u][r] = dh2[u][r] * act_grad<ACT>(act_scaled<ACT>(c2[u][r]));
                            gb2[u][r] += dz2[u][r];
                        }
                    // dh1 = W2 dz2, dz1 = dh1 act'(z1).
                    f32x4 h[2];
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        h[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int u = 0; u < 2; ++u)
#pragma unroll
                            for (int r = 0; r < 4; ++r) h[t] = mfma4(W2T[t][u][r], dz2[u][r], h[t]);
                    }
#pragma unroll
                    for (int t = 0; t < 2; ++t)
#pragma unroll
                        for (int r = 0; r < 4; ++r) Z[s][t][r] = h[t][r] * d1[t][r];
                    // Transposes: [node c][hidden] from the accumulator layout.
#pragma unroll
                    for (int t = 0; t < 2; ++t)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int o = c * TB + ((16 * t + 4 * q + r) ^ swz_w);
                            bh[o] = act_value<ACT>(r1[t][r]);
                            bz2[o] = dz2[t][r];
                        }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    float ha[2][4], zb2[2][4];
#pragma unroll
                    for (int x = 0; x < 2; ++x)
#pragma unroll
                        for (int st = 0; st < 4; ++st) {
                            const int o = (4 * st + q) * TB + ((16 * x + c) ^ tr_swz(4 * st + q));
                            ha[x][st] = bh[o];
                            zb2[x][st] = bz2[o];
                        }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    // dW2[j][o] += sum over the tile's nodes h1[j] dz2[o].
#pragma unroll
                    for (int x = 0; x < 2; ++x)
#pragma unroll
                        for (int y = 0; y < 2; ++y)
#pragma unroll
                            for (int st = 0; st < 4; ++st) gW2[x][y] = mfma4(ha[x][st], zb2[y][st], gW2[x][y]);
                }
                // The first layer's input x_g = chi_s x_pi differs between
                // the reflections only by the sign chi_s(class k) of each
                // row, so dx_g and the dW1 terms of the 8 reflections need
                // dz1 only through Z_cl = sum_s chi_s(cl) dz1_s (the
                // Walsh-Hadamard transform over s, the same butterfly as
                // the forward's): dL/dm[k] = (W1 Z_class(k))[k] and
                // dW1[k][j] += x_pi[k] Z_class(k)[j].  With the rows grouped
                // by class, four classes per 16-row tile, each runs once
                // per class instead of once per reflection.
#pragma unroll
                for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
                    for (int ci = 0; ci < 8; ++ci)
                        if (!(ci & bit))
#pragma unroll
                            for (int t = 0; t < 2; ++t) {
                                const f32x4 u0 = Z[ci][t], u1 = Z[ci | bit][t];
                                Z[ci][t] = u0 + u1;
                                Z[ci | bit][t] = u0 - u1;
                            }
                // dL/dm of this permutation: the row at position
                // 16 kt + 4 q + r feeds from moment src_pi(row).
#pragma unroll
                for (int kt = 0; kt < 2; ++kt) {
                    float D[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int cl = adj_tile_class(kt, i);
                        f32x4 dx = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int t = 0; t < 2; ++t)
#pragma unroll
                            for (int r = 0; r < 4; ++r) dx = mfma4(W1T[kt][t][r], Z[cl][t][r], dx);
#pragma unroll
                        for (int r = 0; r < 4; ++r) D[r] = cls[kt][r] == cl ? dx[r] : D[r];
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (rowo[kt][r] < 27) sdm[node * 32 + sgs[pi * 27 + rowo[kt][r]]] += D[r];
                }
                // dW1 per class: A = the tile's x_pi rows of that class.
#pragma unroll
                for (int cl = 0; cl < 8; ++cl) {
                    const int x = (cl == 0 || cl == 1 || cl == 3 || cl == 7) ? 0 : 1;
#pragma unroll
                    for (int t = 0; t < 2; ++t)
#pragma unroll
                        for (int r = 0; r < 4; ++r) bz1[c * TB + ((16 * t + 4 * q + r) ^ swz_w)] = Z[cl][t][r];
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    float zb1[2][4];
#pragma unroll
                    for (int y = 0; y < 2; ++y)
#pragma unroll
                        for (int st = 0; st < 4; ++st)
                            zb1[y][st] = bz1[(4 * st + q) * TB + ((16 * y + c) ^ tr_swz(4 * st + q))];
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    const bool mine = clsc[x] == cl;
#pragma unroll
                    for (int y = 0; y < 2; ++y)
#pragma unroll
                        for (int st = 0; st < 4; ++st)
                            gW1[x][y] = mfma4(mine ? xa[x][st] : 0.0f, zb1[y][st], gW1[x][y]);
                }
            }
        }
    }
    __syncthreads();

    // Phase C: the full collision adjoint per node, scattered along the streaming.
    {
        float m[Q], lam[Q], nu[Q], gm[Q], omega[4], domega[4];
        const float* row = sm + tid * NODE_STRIDE;
#pragma unroll
        for (int k = 0; k < Q; ++k) m[row_tensor(k)] = row[k];
#pragma unroll
        for (int n = 0; n < 4; ++n) omega[n] = som[tid * 4 + n];
#pragma unroll
        for (int i = 0; i < Q; ++i) lam[i] = live ? lam_in[(size_t)i * a.n + idx] : 0.0f;
        inverse_T(lam, nu);
        const float F[3] = {sF[tid * 3], sF[tid * 3 + 1], sF[tid * 3 + 2]};
        collision_vjp_local(m, nu, a.omega_nu_f, omega, a.n_modes > 0, F, gm, domega);
#pragma unroll
        for (int k = 0; k < Q; ++k) gm[row_tensor(k)] += sdm[tid * 32 + k];
        float gf[Q];
        moments_T(gm, gf);
        if (live) {
            float v[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) v[i] = lam[i] + gf[i];
            scatter_to_sources(lam_out, a, p, v);
        }
    }
    __syncthreads();

    // Block sums of the waves' gradients, in wave order, added to the block's row.
    float* red = sm;                            // 4 waves x 1024 floats (reuses the moment tile)
    // dW2: lane (q, c) holds [j = 16 x + 4 q + r][o = 16 y + c].
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[wave * 1024 + (16 * x + 4 * q + r) * 32 + 16 * y + c] = gW2[x][y][r];
    __syncthreads();
    for (int e = tid; e < 1024; e += 256) {
        const float v = red[e] + red[1024 + e] + red[2048 + e] + red[3072 + e];
        out[OFF_W2 + e] += (double)v;
    }
    __syncthreads();
    // dW1 and db1: lane (q, c) holds [position 16 x + 4 q + r][j = 16 y + c];
    // the position's row is adj_row (27 is b1, 28 empty).
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[wave * 1024 + (16 * x + 4 * q + r) * 32 + 16 * y + c] = gW1[x][y][r];
    __syncthreads();
    // Rows are tile positions (class-grouped): back to the parameter order.
    const int* __restrict__ adj_rows = reinterpret_cast<const int*>(adj_tab + ADJ_ROWS_AT);
    for (int e = tid; e < 32 * 32; e += 256) {
        const int k = adj_rows[e >> 5], j = e & 31;
        if (k > 27) continue;
        const float v = red[e] + red[1024 + e] + red[2048 + e] + red[3072 + e];
        out[(k < 27 ? OFF_W1 + k * 32 + j : OFF_B1 + j)] += (double)v;
    }
    __syncthreads();
    // db2: lane (q, c) holds rows o = 16 u + 4 q + r summed over its nodes c.
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[(wave * 16 + c) * 32 + 16 * u + 4 * q + r] = gb2[u][r];
    __syncthreads();
    if (tid < 32) {
        float v = 0.0f;
        for (int w = 0; w < 64; ++w) v += red[w * 32 + tid];
        out[OFF_B2 + tid] += (double)v;
    }
}

// Parity class of row k of M (the bias row 27 and padding rows count as 0).
int row_class(int k) {
    if (k >= 27) return 0;
    const int t = row_tensor(k);
    return (t % 3) % 2 + 2 * (((t / 3) % 3) % 2) + 4 * ((t / 9) % 2);
}

// Canonical placement of the 28 K rows (27 moments + bias row 27) into the
// 10 K-steps x 4 slots, grouped by parity class; -1 marks an empty slot.
void class_slots(int slot_row[KSTEPS][4]) {
    int fill[KSTEPS] = {0};
    for (int st = 0; st < KSTEPS; ++st)
        for (int q = 0; q < 4; ++q) slot_row[st][q] = -1;
    for (int k = 0; k < 28; ++k) {
        const int ci = row_class(k);
        for (int st = 0; st < KSTEPS; ++st)
            if (step_class(st) == ci && fill[st] < 4) {
                slot_row[st][fill[st]++] = k;
                break;
            }
    }
}

unsigned bf16_bits(float v) {                 // round to nearest even
    unsigned u;
    std::memcpy(&u, &v, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

float bf16_value(unsigned bits) {
    const unsigned u = bits << 16;
    float v;
    std::memcpy(&v, &u, 4);
    return v;
}

unsigned f16_bits(float v) {                  // round to nearest even (the compiler's conversion)
    const _Float16 h = (_Float16)v;
    unsigned short u;
    std::memcpy(&u, &h, 2);
    return u;
}

}  // namespace

size_t mfma_lane_table_floats() { return 64 * LANE_WORDS; }
size_t mfma_group_table_ints() { return GT_ENTRIES; }

// Host-side preparation of the per-lane operand table from the flat
// parameters (W1[27][W], b1, W2[W][W], b2, W3[W][4], b3) and of the gather
// table: for axis permutation p and K slot holding W1 row k, the moment row
// that m^(g) places at k.  gsrc is indexed by group element g = 8 p +
// reflection mask; the reflection-free elements g = 8 p give Q_p.
void mfma_prepare_tables(const float* params, int act, int prec, const int (*gsrc)[27], float* lane_tab,
                         int* gtab, int depth) {
    const int W = MW;
    const float* W1 = params;
    const float* b1 = W1 + 27 * W;
    const float* W2 = b1 + W;
    const float* b2 = W2 + W * W;
    const float* W2b = b2 + W;                      // depth 3 only
    const float* b2b = W2b + W * W;
    const float* W3 = depth == 3 ? b2b + W : b2 + W;
    const float* b3 = W3 + 4 * W;
    const bool th = act == ACT_TANH;
    const float kappa = th ? (float)(2.0 / 0.69314718055994530942) : 1.0f;
    // tanh = 1 - 2 r folded into the consumer of each activation:
    // W2 -> -2 W2, b2 -> b2 + sum_h W2[h][:], W3 -> -2 W3, b3 -> b3 + sum_h W3[h][:]
    // (the group mean turns 1 into 48 / 48).
    const float fold = th ? -2.0f : 1.0f;
    float b2f[MW], b3f[4];
    for (int o = 0; o < W; ++o) {
        double s = b2[o];
        if (th)
            for (int h = 0; h < W; ++h) s += W2[h * W + o];
        b2f[o] = (float)s;
    }
    for (int n = 0; n < 4; ++n) {
        double s = b3[n];
        if (th)
            for (int h = 0; h < W; ++h) s += W3[h * 4 + n];
        b3f[n] = (float)s;
    }
    auto w1row = [&](int k, int h) { return k < 27 ? W1[k * W + h] : k == 27 ? b1[h] : 0.0f; };
    // Split arithmetic, tanh: per layer (first, second, third) the power of
    // two sigma that puts the largest |A| (kappa W1 with the bias row, kappa
    // fold W2, kappa fold W2b) into [128, 256), well inside the f16 range,
    // with the remainders of all but negligible weights normal; b2bf the
    // third layer's bias with the tanh fold.
    float split_sigma[3] = {1.0f, 1.0f, 1.0f};
    float b2bf[MW] = {};
    if (prec == MLP_PREC_F32S && th) {
        float amax[3] = {0.0f, 0.0f, 0.0f};
        for (int k = 0; k < 28; ++k)
            for (int h = 0; h < W; ++h) amax[0] = std::max(amax[0], std::fabs(kappa * w1row(k, h)));
        for (int i = 0; i < W * W; ++i) {
            amax[1] = std::max(amax[1], std::fabs(kappa * fold * W2[i]));
            if (depth == 3) amax[2] = std::max(amax[2], std::fabs(kappa * fold * W2b[i]));
        }
        for (int l = 0; l < 3; ++l)
            if (amax[l] > 0.0f) split_sigma[l] = std::ldexp(1.0f, 7 - std::ilogb(amax[l]));
    }
    if (depth == 3)
        for (int o = 0; o < W; ++o) {
            double sb = b2b[o];
            if (th)
                for (int h = 0; h < W; ++h) sb += W2b[h * W + o];
            b2bf[o] = (float)sb;
        }
    int slot_row[KSTEPS][4];
    class_slots(slot_row);
    for (int lane = 0; lane < 64; ++lane) {
        const int q = lane >> 4, c = lane & 15;
        float* lt = lane_tab + lane * LANE_WORDS;
        unsigned* lw = reinterpret_cast<unsigned*>(lt);
        for (int i = 0; i < LANE_WORDS; ++i) lt[i] = 0.0f;
        if (prec == MLP_PREC_F32S) {
            // Parts of each layer's A operand in the K slots of its product:
            // layer 1 slot j of lane group q holds input row 8 q + j, a
            // hidden-to-hidden layer's slot j hidden unit 16 (j / 4) + 4 q +
            // j % 4.
            auto hid = [&](int j) { return 16 * (j / 4) + 4 * q + j % 4; };
            auto put = [&](int off, int t, int w, int e, float a) {
                unsigned part[3];
                if (th) {
                    part[0] = f16_bits(a);
                    part[1] = f16_bits(a - (float)(_Float16)a);
                    part[2] = 0;
                } else {
                    part[0] = bf16_bits(a);
                    const float r = a - bf16_value(part[0]);
                    part[1] = bf16_bits(r);
                    part[2] = bf16_bits(r - bf16_value(part[1]));
                }
                for (int k = 0; k < 3; ++k) lw[off + 12 * t + 4 * k + w] |= part[k] << (16 * e);
            };
            if (th) {
                for (int t = 0; t < 2; ++t)
                    for (int w = 0; w < 4; ++w)
                        for (int e = 0; e < 2; ++e)
                            put(LS_A1, t, w, e, split_sigma[0] * (kappa * w1row(8 * q + 2 * w + e, 16 * t + c)));
                lt[LS_BACK] = 1.0f / split_sigma[0];
            } else {
                for (int t = 0; t < 2; ++t)
                    for (int st = 0; st < KSTEPS; ++st) {
                        const int k = slot_row[st][q];
                        lt[LT_A1 + t * KSTEPS + st] = k < 0 ? 0.0f : w1row(k, 16 * t + c);
                    }
            }
            auto fill = [&](const float* Wl, const float* bfold, float sigma, int offA, int offB, int slot) {
                for (int u = 0; u < 2; ++u)
                    for (int w = 0; w < 4; ++w)
                        for (int e = 0; e < 2; ++e)
                            put(offA, u, w, e, sigma * (kappa * fold * Wl[hid(2 * w + e) * W + 16 * u + c]));
                const float up = th ? sigma * 2048.0f : 1.0f;
                for (int u = 0; u < 2; ++u)
                    for (int r = 0; r < 4; ++r) lt[offB + u * 4 + r] = up * (kappa * bfold[16 * u + 4 * q + r]);
                lt[LS_BACK + slot] = 1.0f / up;
            };
            fill(W2, b2f, split_sigma[1], LS_A2, LS_B2, 1);
            if (depth == 3) fill(W2b, b2bf, split_sigma[2], LS_A3, LS_B3, 2);
            lt[LS_NEG1] = -1.0f;
            for (int b = 0; b < 3; ++b)
                for (int w = 0; w < 4; ++w) {
                    const int k0 = 8 * q + 2 * w, k1 = k0 + 1;
                    lw[LS_SM + 4 * b + w] = ((row_class(k0) >> b) & 1 ? 0x8000u : 0u) |
                                            ((row_class(k1) >> b) & 1 ? 0x80000000u : 0u);
                }
            for (int u = 0; u < 2; ++u)
                for (int r = 0; r < 4; ++r)
                    for (int n = 0; n < 4; ++n)
                        lt[LS_W3 + (u * 4 + r) * 4 + n] = fold * W3[(16 * u + 4 * q + r) * 4 + n] / (float)NGROUP;
            for (int n = 0; n < 4; ++n) lt[LS_B3O + n] = b3f[n];
        } else if (prec == MLP_PREC_F32) {
            for (int t = 0; t < 2; ++t)
                for (int st = 0; st < KSTEPS; ++st) {
                    const int k = slot_row[st][q];
                    lt[LT_A1 + t * KSTEPS + st] = k < 0 ? 0.0f : kappa * w1row(k, 16 * t + c);
                }
            for (int u = 0; u < 2; ++u)
                for (int t = 0; t < 2; ++t)
                    for (int r = 0; r < 4; ++r)
                        lt[LT_A2 + u * 8 + t * 4 + r] = kappa * fold * W2[(16 * t + 4 * q + r) * W + 16 * u + c];
            for (int u = 0; u < 2; ++u)
                for (int r = 0; r < 4; ++r) lt[LT_B2 + u * 4 + r] = kappa * b2f[16 * u + 4 * q + r];
            for (int u = 0; u < 2; ++u)
                for (int r = 0; r < 4; ++r)
                    for (int n = 0; n < 4; ++n)
                        lt[LT_W3 + (u * 4 + r) * 4 + n] = fold * W3[(16 * u + 4 * q + r) * 4 + n] / (float)NGROUP;
            for (int n = 0; n < 4; ++n) lt[LT_B3 + n] = b3f[n];
            if (depth == 3) {
                // Third layer: tanh of the second folded in as for W2 above.
                for (int v = 0; v < 2; ++v)
                    for (int t = 0; t < 2; ++t)
                        for (int r = 0; r < 4; ++r)
                            lt[LT_A2B + v * 8 + t * 4 + r] = kappa * fold * W2b[(16 * t + 4 * q + r) * W + 16 * v + c];
                for (int v = 0; v < 2; ++v)
                    for (int r = 0; r < 4; ++r) {
                        const int o = 16 * v + 4 * q + r;
                        double sb = b2b[o];
                        if (th)
                            for (int h = 0; h < W; ++h) sb += W2b[h * W + o];
                        lt[LT_B2B + v * 4 + r] = kappa * (float)sb;
                    }
            }
        } else {
            // K slot j of lane group q is row k = 8 q + j (layer 1) and hidden
            // unit 16 (j / 4) + 4 q + j % 4 (layer 2).
            for (int t = 0; t < 2; ++t)
                for (int w = 0; w < 4; ++w) {
                    const int k0 = 8 * q + 2 * w, k1 = k0 + 1;
                    lw[LB_A1 + 4 * t + w] = bf16_bits(kappa * w1row(k0, 16 * t + c)) |
                                            (bf16_bits(kappa * w1row(k1, 16 * t + c)) << 16);
                }
            auto hid = [&](int j) { return 16 * (j / 4) + 4 * q + j % 4; };
            for (int u = 0; u < 2; ++u)
                for (int w = 0; w < 4; ++w)
                    lw[LB_A2 + 4 * u + w] =
                        bf16_bits(kappa * fold * W2[hid(2 * w) * W + 16 * u + c]) |
                        (bf16_bits(kappa * fold * W2[hid(2 * w + 1) * W + 16 * u + c]) << 16);
            for (int u = 0; u < 2; ++u)
                for (int r = 0; r < 4; ++r) lt[LB_B2 + u * 4 + r] = kappa * b2f[16 * u + 4 * q + r];
            if (depth == 3) {
                // Third layer, in the second's layout, tanh of the second
                // folded in as for W2.
                for (int v = 0; v < 2; ++v)
                    for (int w = 0; w < 4; ++w)
                        lw[LB_A2B + 4 * v + w] =
                            bf16_bits(kappa * fold * W2b[hid(2 * w) * W + 16 * v + c]) |
                            (bf16_bits(kappa * fold * W2b[hid(2 * w + 1) * W + 16 * v + c]) << 16);
                for (int v = 0; v < 2; ++v)
                    for (int r = 0; r < 4; ++r) lt[LB_B2B + v * 4 + r] = kappa * b2bf[16 * v + 4 * q + r];
            }
            for (int u = 0; u < 2; ++u)
                for (int r = 0; r < 4; ++r)
                    for (int n = 0; n < 4; ++n)
                        lt[LB_W3 + (u * 4 + r) * 4 + n] = fold * W3[(16 * u + 4 * q + r) * 4 + n] / (float)NGROUP;
            for (int n = 0; n < 4; ++n) lt[LB_B3 + n] = b3f[n];
            for (int b = 0; b < 3; ++b)
                for (int w = 0; w < 4; ++w) {
                    const int k0 = 8 * q + 2 * w, k1 = k0 + 1;
                    lw[LB_SM + 4 * b + w] = ((row_class(k0) >> b) & 1 ? 0x8000u : 0u) |
                                            ((row_class(k1) >> b) & 1 ? 0x80000000u : 0u);
                }
        }
    }
    for (int p = 0; p < 6; ++p)
        for (int q = 0; q < 4; ++q)
            for (int i = 0; i < GT_STRIDE; ++i) {
                // Row k placed in this slot; 27 is the constant-1 row, 28 zero.
                int k = -1;
                if (prec == MLP_PREC_F32 || (prec == MLP_PREC_F32S && !th)) {
                    if (i < KSTEPS) k = slot_row[i][q];
                } else if (i < 8) {
                    k = 8 * q + i;
                }
                int e = 28;
                if (k >= 0 && k < 27) e = gsrc[8 * p][k];
                if (k == 27) e = 27;
                gtab[(p * 4 + q) * GT_STRIDE + i] = e;
            }
}

size_t mfma_adjoint_table_floats() { return 64 * ADJ_WORDS + 32; }

// Per-lane table of the matrix-core adjoint from the flat parameters of a
// width-32 network (unfolded weights: the adjoint works with h = tanh(z)).
void mfma_prepare_adjoint_table(const float* params, float* tab) {
    const int W = MW;
    const float* W1 = params;
    const float* W2 = W1 + 27 * W + W;
    const float* W3 = W2 + W * W + W;
    for (int lane = 0; lane < 64; ++lane) {
        const int q = lane >> 4, c = lane & 15;
        float* at = tab + lane * ADJ_WORDS;
        int* ai = reinterpret_cast<int*>(at);
        for (int t = 0; t < 2; ++t)
            for (int u = 0; u < 2; ++u)
                for (int r = 0; r < 4; ++r) at[AT_W2T + t * 8 + u * 4 + r] = W2[(16 * t + c) * W + 16 * u + 4 * q + r];
        for (int kt = 0; kt < 2; ++kt)
            for (int t = 0; t < 2; ++t)
                for (int r = 0; r < 4; ++r) {
                    const int k = adj_row(16 * kt + c);
                    at[AT_W1T + kt * 8 + t * 4 + r] = k < 27 ? W1[k * W + 16 * t + 4 * q + r] : 0.0f;
                }
        for (int u = 0; u < 2; ++u)
            for (int r = 0; r < 4; ++r)
                for (int n = 0; n < 4; ++n)
                    at[AT_W3 + (u * 4 + r) * 4 + n] = W3[(16 * u + 4 * q + r) * 4 + n] / (float)NGROUP;
        for (int kt = 0; kt < 2; ++kt) {
            for (int r = 0; r < 4; ++r) {
                const int k = adj_row(16 * kt + 4 * q + r);
                ai[AT_CLS + kt * 4 + r] = k < 28 ? moment_class(k) : -1;
                ai[AT_ROWO + kt * 4 + r] = k;
            }
            const int k = adj_row(16 * kt + c);
            ai[AT_CLSC + kt] = k < 28 ? moment_class(k) : -1;
            ai[AT_ROWC + kt] = k;
        }
    }
    int* rows = reinterpret_cast<int*>(tab + ADJ_ROWS_AT);
    for (int p = 0; p < 32; ++p) rows[p] = adj_row(p);
}

// One 4-wavefront block per CU (the kernel's registers): with 256-node
// blocks each wavefront runs 4 tiles per round, with 64-node blocks one tile
// and 4x the blocks, so below 256 CUs x 256 nodes the small blocks finish in
// fewer tile-rounds (4x fewer up to 16384 nodes) and above it they tie.
constexpr int ADJM_SMALL_NODES = 65536;
int adjoint_mfma_blocks(int n) { return n < ADJM_SMALL_NODES ? (n + 63) / 64 : (n + 255) / 256; }

hipError_t launch_adjoint_mfma(int storage, int act, const void* xin, const float* lam_in, float* lam_out,
                               const StepArgs& a, const float* lane_tab, const int* gtab, const float* adj_tab,
                               const int* gsrc, double* partial, hipStream_t st) {
    const bool small = a.n < ADJM_SMALL_NODES;
    const dim3 grid(adjoint_mfma_blocks(a.n)), block(256);
#define ADJM_LAUNCH(SS, ACT, TPW)                                                                                \
    hipLaunchKernelGGL((k_adjoint_mfma<SS, ACT, TPW>), grid, block, 0, st,                                      \
                       static_cast<const typename Codec<SS>::store_t*>(xin), lam_in, lam_out, a, lane_tab, gtab,  \
                       adj_tab, gsrc, partial)
#define ADJM_CASE(SS)                                                                                            \
    case SS:                                                                                                     \
        if (act == ACT_TANH) {                                                                                   \
            if (small)                                                                                           \
                ADJM_LAUNCH(SS, ACT_TANH, 1);                                                                    \
            else                                                                                                 \
                ADJM_LAUNCH(SS, ACT_TANH, 4);                                                                    \
        } else {                                                                                                 \
            if (small)                                                                                           \
                ADJM_LAUNCH(SS, ACT_RELU, 1);                                                                    \
            else                                                                                                 \
                ADJM_LAUNCH(SS, ACT_RELU, 4);                                                                    \
        }                                                                                                        \
        return hipGetLastError();
    switch (storage) {
        ADJM_CASE(ST_F32)
        ADJM_CASE(ST_F16)
        ADJM_CASE(ST_BF16)
        default: return hipErrorInvalidValue;
    }
#undef ADJM_CASE
#undef ADJM_LAUNCH
}

// omega_out == nullptr: one stream-collide step fin -> fout.  Otherwise the
// rates of the state in fin are written to omega_out and fout is untouched.
hipError_t launch_nco_mfma_grouped(int storage, int prec, int act, const LaunchGroup& g, hipStream_t st) {
    const dim3 grid(g.prefix[g.count]), block(256);
#define GRP_LAUNCH(SS, AA, PP) hipLaunchKernelGGL((k_nco_mfma_grouped<SS, AA, PP>), grid, block, 0, st, g)
#define GRP_CASE(SS)                                                      \
    case SS:                                                              \
        if (prec == MLP_PREC_BF16) {                                      \
            if (act == ACT_TANH) GRP_LAUNCH(SS, ACT_TANH, MLP_PREC_BF16); \
            else GRP_LAUNCH(SS, ACT_RELU, MLP_PREC_BF16);                 \
        } else if (prec == MLP_PREC_F32S) {                               \
            if (act == ACT_TANH) GRP_LAUNCH(SS, ACT_TANH, MLP_PREC_F32S); \
            else GRP_LAUNCH(SS, ACT_RELU, MLP_PREC_F32S);                 \
        } else {                                                          \
            if (act == ACT_TANH) GRP_LAUNCH(SS, ACT_TANH, MLP_PREC_F32);  \
            else GRP_LAUNCH(SS, ACT_RELU, MLP_PREC_F32);                  \
        }                                                                 \
        return hipGetLastError();
    switch (storage) {
        GRP_CASE(ST_F32)
        GRP_CASE(ST_F16)
        GRP_CASE(ST_BF16)
        default: return hipErrorInvalidValue;
    }
#undef GRP_CASE
#undef GRP_LAUNCH
}

// Block shape of the single-lattice kernel (the results are bit-identical
// for all three).  About 2 wavefronts per SIMD are resident (8 per CU).
// Below 65536 nodes, 64-node blocks with one tile per wavefront finish in
// fewer rounds of tiles (4x fewer up to 32768 nodes).  Up to 131072 nodes,
// one-wavefront 64-node blocks (measured 10 % faster than 256-node blocks at
// 32^3 before the one-tile blocks existed, equal from 64^3 up).  Above, the
// 256-node blocks.
enum MfmaBlock { MFMA_BLOCK_256 = 0, MFMA_BLOCK_64 = 1, MFMA_BLOCK_64_TILE = 2 };
// Float32-network steps of lattices up to this many nodes run six-wavefront
// tiles (network_f32_psplit): 256 blocks, one round over the 256 CUs.  A
// block holds 111 KB of LDS, one per CU, so beyond that the blocks run in
// rounds and the one-tile-per-wavefront blocks are faster (16^3: 15 against
// 30 us per step; 24^3: 53 against 31).
constexpr int PSPLIT_MAX_NODES = 4096;
int mfma_block_kind(int n) {
    return n < 65536 ? MFMA_BLOCK_64_TILE : n < 2 * 256 * 256 ? MFMA_BLOCK_64 : MFMA_BLOCK_256;
}

template <int S, int ACT, bool RR, int PP, int DD>
hipError_t launch_mfma_kind(int kind, const void* fin, void* fout, const StepArgs& a, const float* lane_tab,
                            const int* gtab, double* omega_out, hipStream_t st) {
    using T = typename Codec<S>::store_t;
    const int nodes = kind == MFMA_BLOCK_256 ? 256 : 64;
    const dim3 grid((a.n + nodes - 1) / nodes);
    if constexpr (!RR && PP == MLP_PREC_F32) {
        // The instantiation that can keep the network values for the adjoint
        // (when a.net_sums is set; depth 2) runs the plain steps too: with
        // that branch the compiler allocates 154-161 VGPRs at depth 2, 3
        // waves per SIMD, where the instantiation without it takes 230 and 2
        // waves and runs 3 % slower; at depth 3, 177 against 254 (with
        // mfma_min_waves, 3 waves).  Steps of lattices up to
        // PSPLIT_MAX_NODES run six-wavefront tiles.
        if (a.n <= PSPLIT_MAX_NODES)
            hipLaunchKernelGGL((k_nco_mfma<S, ACT, RR, PP, 16, DD, 0, true>), dim3((a.n + 15) / 16),
                               dim3(mfma_block_threads(16, 0)), 0, st, static_cast<const T*>(fin),
                               static_cast<T*>(fout), a, lane_tab, gtab, omega_out);
        else if (kind == MFMA_BLOCK_64_TILE)
            hipLaunchKernelGGL((k_nco_mfma<S, ACT, RR, PP, 64, DD, 1, true>), dim3(grid), dim3(mfma_block_threads(64, 1)),
                               0, st, static_cast<const T*>(fin), static_cast<T*>(fout), a, lane_tab, gtab, omega_out);
        else if (kind == MFMA_BLOCK_64)
            hipLaunchKernelGGL((k_nco_mfma<S, ACT, RR, PP, 64, DD, 4, true>), dim3(grid), dim3(mfma_block_threads(64, 4)),
                               0, st, static_cast<const T*>(fin), static_cast<T*>(fout), a, lane_tab, gtab, omega_out);
        else
            hipLaunchKernelGGL((k_nco_mfma<S, ACT, RR, PP, 256, DD, 4, true>), dim3(grid),
                               dim3(mfma_block_threads(256, 4)), 0, st, static_cast<const T*>(fin),
                               static_cast<T*>(fout), a, lane_tab, gtab, omega_out);
        return hipGetLastError();
    }
    if (a.net_sums) return hipErrorInvalidValue;
    if (kind == MFMA_BLOCK_64_TILE)
        hipLaunchKernelGGL((k_nco_mfma<S, ACT, RR, PP, 64, DD, 1>), dim3(grid), dim3(mfma_block_threads(64, 1)), 0,
                           st, static_cast<const T*>(fin), static_cast<T*>(fout), a, lane_tab, gtab, omega_out);
    else if (kind == MFMA_BLOCK_64)
        hipLaunchKernelGGL((k_nco_mfma<S, ACT, RR, PP, 64, DD, 4>), dim3(grid), dim3(mfma_block_threads(64, 4)), 0,
                           st, static_cast<const T*>(fin), static_cast<T*>(fout), a, lane_tab, gtab, omega_out);
    else
        hipLaunchKernelGGL((k_nco_mfma<S, ACT, RR, PP, 256, DD, 4>), dim3(grid), dim3(mfma_block_threads(256, 4)),
                           0, st, static_cast<const T*>(fin), static_cast<T*>(fout), a, lane_tab, gtab, omega_out);
    return hipGetLastError();
}

template <int S, int ACT, bool RR>
hipError_t launch_mfma_prec(int prec, const void* fin, void* fout, const StepArgs& a, const float* lane_tab,
                            const int* gtab, double* omega_out, hipStream_t st) {
    const int kind = mfma_block_kind(a.n);
    if (prec == MLP_PREC_BF16) {
        if (a.depth == 3)
            return launch_mfma_kind<S, ACT, RR, MLP_PREC_BF16, 3>(kind, fin, fout, a, lane_tab, gtab, omega_out, st);
        return launch_mfma_kind<S, ACT, RR, MLP_PREC_BF16, 2>(kind, fin, fout, a, lane_tab, gtab, omega_out, st);
    }
    if (prec == MLP_PREC_F32S) {
        if (a.depth == 3)
            return launch_mfma_kind<S, ACT, RR, MLP_PREC_F32S, 3>(kind, fin, fout, a, lane_tab, gtab, omega_out, st);
        return launch_mfma_kind<S, ACT, RR, MLP_PREC_F32S, 2>(kind, fin, fout, a, lane_tab, gtab, omega_out, st);
    }
    if (a.depth == 3)
        return launch_mfma_kind<S, ACT, RR, MLP_PREC_F32, 3>(kind, fin, fout, a, lane_tab, gtab, omega_out, st);
    return launch_mfma_kind<S, ACT, RR, MLP_PREC_F32, 2>(kind, fin, fout, a, lane_tab, gtab, omega_out, st);
}

template <int S>
hipError_t launch_mfma_storage(int prec, const void* fin, void* fout, const StepArgs& a, const float* lane_tab,
                               const int* gtab, double* omega_out, hipStream_t st) {
    if (omega_out)
        return a.act == ACT_TANH ? launch_mfma_prec<S, ACT_TANH, true>(prec, fin, fout, a, lane_tab, gtab, omega_out, st)
                                 : launch_mfma_prec<S, ACT_RELU, true>(prec, fin, fout, a, lane_tab, gtab, omega_out, st);
    return a.act == ACT_TANH ? launch_mfma_prec<S, ACT_TANH, false>(prec, fin, fout, a, lane_tab, gtab, omega_out, st)
                             : launch_mfma_prec<S, ACT_RELU, false>(prec, fin, fout, a, lane_tab, gtab, omega_out, st);
}

hipError_t launch_nco_mfma(int storage, int prec, const void* fin, void* fout, const StepArgs& a,
                           const float* lane_tab, const int* gtab, double* omega_out, hipStream_t st) {
    switch (storage) {
        case ST_F32: return launch_mfma_storage<ST_F32>(prec, fin, fout, a, lane_tab, gtab, omega_out, st);
        case ST_F16: return launch_mfma_storage<ST_F16>(prec, fin, fout, a, lane_tab, gtab, omega_out, st);
        case ST_BF16: return launch_mfma_storage<ST_BF16>(prec, fin, fout, a, lane_tab, gtab, omega_out, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace nco
