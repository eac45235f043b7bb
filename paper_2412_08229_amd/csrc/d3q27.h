// D3Q27 lattice, Hermite moment transform and population storage codecs for
// gfx950 kernels.
//
// Velocity index i = 9 (c_z + 1) + 3 (c_y + 1) + (c_x + 1); weights are the
// tensor product of the D1Q3 weights (1/6, 2/3, 1/6) and cs^2 = 1/3.
//
// Moments are held in tensor order t = 9 n_z + 3 n_y + n_x, where
// (n_x, n_y, n_z) in {0,1,2}^3 is the Hermite multi-index.  The Hermite
// moment matrix of Sec. II.B is a tensor product of the one-dimensional
// polynomials h0 = 1, h1 = xi, h2 = xi^2 - 1 at xi = sqrt(3) c, so M f is
// three passes of a 3-point transform, one per axis, instead of a dense
// 27 x 27 product.  Its rows are w-orthogonal with norms 1, 1, 2 per factor,
// which gives the inverse in closed form, again one pass per axis.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace nco {

constexpr int Q = 27;

__host__ __device__ constexpr int cx_of(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int cy_of(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int cz_of(int i) { return i / 9 - 1; }
__host__ __device__ constexpr int csq_of(int i) {
    return cx_of(i) * cx_of(i) + cy_of(i) * cy_of(i) + cz_of(i) * cz_of(i);
}
__host__ __device__ constexpr double w1_of(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
__host__ __device__ constexpr double weight_of(int i) {
    return w1_of(cx_of(i)) * w1_of(cy_of(i)) * w1_of(cz_of(i));
}
// Moment order of tensor index t.
__host__ __device__ constexpr int order_of(int t) { return t % 3 + (t / 3) % 3 + t / 9; }

// Tensor index of each row of M in the order printed in Sec. II.B:
// 1, x, y, z, xx, xy, xz, yy, yz, zz, xxy, xxz, xyy, xyz, xzz, yyz, yzz,
// xxyy, xxyz, xxzz, xyyz, xyzz, yyzz, xxyyz, xxyzz, xyyzz, xxyyzz.
__host__ __device__ constexpr int row_tensor(int k) {
    constexpr int t[27] = {0, 1, 3, 9, 2, 4, 10, 6, 12, 18, 5, 11, 7, 13, 19, 15, 21,
                           8, 14, 20, 16, 22, 24, 17, 23, 25, 26};
    return t[k];
}

// Power-of-two scale of the 16-bit deviation storage, by velocity class:
// 2^2, 2^4, 2^6, 2^8 for |c|^2 = 0, 1, 2, 3 (about 1/w_i).
__host__ __device__ constexpr float dev_scale(int i) {
    return csq_of(i) == 0 ? 4.0f : csq_of(i) == 1 ? 16.0f : csq_of(i) == 2 ? 64.0f : 256.0f;
}

template <typename R> struct Sqrt3;
template <> struct Sqrt3<float> { static constexpr float v = 1.7320508075688772f; };
template <> struct Sqrt3<double> { static constexpr double v = 1.7320508075688772; };

// One-dimensional forward transform of (f(-1), f(0), f(+1)).
template <typename R>
__device__ __forceinline__ void fwd3(R fm, R f0, R fp, R& a0, R& a1, R& a2) {
    a0 = fm + f0 + fp;
    a1 = Sqrt3<R>::v * (fp - fm);
    a2 = R(2) * (fm + fp) - f0;
}

// Inverse of fwd3: f(c) = w1(c) sum_n h_n(c) a_n / norm_n.  The rest value
// is formed as a0 - (f(-1) + f(+1)) (algebraically (2/3)(a0 - a2/2)), so the
// zeroth moment of the three outputs is a0 up to one unbiased rounding; the
// rounded constant 1/6 would otherwise scale the mass of every pass.
template <typename R>
__device__ __forceinline__ void inv3(R a0, R a1, R a2, R& fm, R& f0, R& fp) {
    const R s = a0 + a2;
    const R d = Sqrt3<R>::v * a1;
    fm = (s - d) * R(1.0 / 6.0);
    fp = (s + d) * R(1.0 / 6.0);
    f0 = a0 - (fm + fp);
}

// m = M f in tensor order (f in velocity order).
template <typename R>
__device__ __forceinline__ void to_moments(const R (&f)[Q], R (&m)[Q]) {
    R t[Q];
#pragma unroll
    for (int r = 0; r < 9; ++r)          // along x: rows (cz, cy)
        fwd3(f[3 * r], f[3 * r + 1], f[3 * r + 2], t[3 * r], t[3 * r + 1], t[3 * r + 2]);
    R s[Q];
#pragma unroll
    for (int z = 0; z < 3; ++z)          // along y
#pragma unroll
        for (int n = 0; n < 3; ++n)
            fwd3(t[9 * z + n], t[9 * z + 3 + n], t[9 * z + 6 + n], s[9 * z + n], s[9 * z + 3 + n],
                 s[9 * z + 6 + n]);
#pragma unroll
    for (int p = 0; p < 9; ++p)          // along z
        fwd3(s[p], s[9 + p], s[18 + p], m[p], m[9 + p], m[18 + p]);
}

// f = M^{-1} m.
template <typename R>
__device__ __forceinline__ void from_moments(const R (&m)[Q], R (&f)[Q]) {
    R s[Q];
#pragma unroll
    for (int p = 0; p < 9; ++p)
        inv3(m[p], m[9 + p], m[18 + p], s[p], s[9 + p], s[18 + p]);
    R t[Q];
#pragma unroll
    for (int z = 0; z < 3; ++z)
#pragma unroll
        for (int n = 0; n < 3; ++n)
            inv3(s[9 * z + n], s[9 * z + 3 + n], s[9 * z + 6 + n], t[9 * z + n], t[9 * z + 3 + n],
                 t[9 * z + 6 + n]);
#pragma unroll
    for (int r = 0; r < 9; ++r)
        inv3(t[3 * r], t[3 * r + 1], t[3 * r + 2], f[3 * r], f[3 * r + 1], f[3 * r + 2]);
}

// ---------------------------------------------------------------- storage --

enum Storage { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2, ST_F64 = 3 };

template <int S> struct Codec;

// float32 populations are written with non-temporal stores: the buffer
// just written is read only in the next step, after the whole lattice has
// streamed through the caches, so keeping it there only evicts the lines the
// current step still reads (measured: BGK at 256^3 moves 5.73 instead of
// 5.43 TB/s).  16-bit lattices of serving and test sizes fit the 256 MB
// last-level cache, where ordinary stores are faster.
template <> struct Codec<ST_F32> {
    using store_t = float;
    using real = float;
    static __device__ __forceinline__ real load(const store_t* p, int) { return *p; }
    static __device__ __forceinline__ void store(store_t* p, int, real v) { __builtin_nontemporal_store(v, p); }
    // Ordinary store, for a buffer that is read again while it stays cached.
    static __device__ __forceinline__ void store_cached(store_t* p, int, real v) { *p = v; }
    static __device__ __forceinline__ real from_double(double v, int) { return (float)v; }
    static __device__ __forceinline__ double to_double(store_t v, int) { return (double)v; }
};

template <> struct Codec<ST_F64> {
    using store_t = double;
    using real = double;
    static __device__ __forceinline__ real load(const store_t* p, int) { return *p; }
    static __device__ __forceinline__ void store(store_t* p, int, real v) { *p = v; }
    static __device__ __forceinline__ void store_cached(store_t* p, int i, real v) { store(p, i, v); }
    static __device__ __forceinline__ store_t from_double(double v, int) { return v; }
    static __device__ __forceinline__ double to_double(store_t v, int) { return v; }
};

template <> struct Codec<ST_F16> {
    using store_t = __half;
    using real = float;
    static __device__ __forceinline__ real load(const store_t* p, int i) {
        return (float)weight_of(i) + __half2float(*p) * (1.0f / dev_scale(i));
    }
    static __device__ __forceinline__ void store(store_t* p, int i, real v) {
        *p = __float2half_rn((v - (float)weight_of(i)) * dev_scale(i));
    }
    static __device__ __forceinline__ void store_cached(store_t* p, int i, real v) { store(p, i, v); }
    // Stochastic rounding with 16 random bits r: |x| rounded toward zero to
    // the half value lo, then up to the next half value (gap above lo, a
    // power of two) when r / 2^16 < (|x| - lo) / gap.  The largest finite
    // half has gap infinity and never rounds up.
    static __device__ __forceinline__ void store_sr(store_t* p, int i, real v, unsigned r) {
        const float x = (v - (float)weight_of(i)) * dev_scale(i);
        const float ax = fabsf(x);
        const unsigned short bz = __half_as_ushort(__float2half_rz(ax));
        const float lo = __half2float(__ushort_as_half(bz));
        const float gap = __half2float(__ushort_as_half((unsigned short)(bz + 1))) - lo;
        const bool up = (float)(r & 0xffffu) * (1.0f / 65536.0f) * gap < ax - lo;
        const unsigned short b = (unsigned short)((bz + (up ? 1 : 0)) | (x < 0.0f ? 0x8000u : 0u));
        *reinterpret_cast<unsigned short*>(p) = b;
    }
    static __device__ __forceinline__ store_t from_double(double v, int i) {
        return __float2half_rn((float)((v - weight_of(i)) * dev_scale(i)));
    }
    static __device__ __forceinline__ double to_double(store_t v, int i) {
        return weight_of(i) + (double)__half2float(v) / dev_scale(i);
    }
};

// Random bits of the stochastic rounding of 16-bit deviations (Codec
// store_sr): a counter-based hash of (step key, node, population), C.
// Wellons' "lowbias32" integer hash (xor-shift / multiply rounds, constants
// 0x7feb352d and 0x846ca68b).  For bfloat16 the float32 value's low 16 bits
// plus 16 random bits, truncated, rounds up with probability equal to the
// dropped fraction, so the stored value is unbiased; float16 compares the
// random fraction with the position of |x| between its two half neighbours.
__host__ __device__ __forceinline__ unsigned lowbias32(unsigned x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__device__ __forceinline__ unsigned sr_bits(unsigned key, int node, int i) {
    return lowbias32(key ^ lowbias32((unsigned)node * 27u + (unsigned)i));
}

template <> struct Codec<ST_BF16> {
    using store_t = __hip_bfloat16;
    using real = float;
    static __device__ __forceinline__ real load(const store_t* p, int i) {
        return (float)weight_of(i) + __bfloat162float(*p) * (1.0f / dev_scale(i));
    }
    static __device__ __forceinline__ void store(store_t* p, int i, real v) {
        *p = __float2bfloat16((v - (float)weight_of(i)) * dev_scale(i));
    }
    static __device__ __forceinline__ void store_cached(store_t* p, int i, real v) { store(p, i, v); }
    // Stochastic rounding with 16 random bits r (finite values; a value
    // within one bfloat16 step of the largest may round to infinity).
    static __device__ __forceinline__ void store_sr(store_t* p, int i, real v, unsigned r) {
        const unsigned bits = __float_as_uint((v - (float)weight_of(i)) * dev_scale(i)) + (r & 0xffffu);
        *reinterpret_cast<unsigned short*>(p) = (unsigned short)(bits >> 16);
    }
    static __device__ __forceinline__ store_t from_double(double v, int i) {
        return __float2bfloat16((float)((v - weight_of(i)) * dev_scale(i)));
    }
    static __device__ __forceinline__ double to_double(store_t v, int i) {
        return weight_of(i) + (double)__bfloat162float(v) / dev_scale(i);
    }
};

}  // namespace nco
