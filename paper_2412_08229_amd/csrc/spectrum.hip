// Energy spectrum E(k) of the velocity field, in float64.
//
// The loss of Sec. "Learning Task" compares shell-summed kinetic energy
// spectra.  Here u_hat = DFT(u) / n^3 over a cubic periodic lattice and
// E(k) = 1/2 sum |u_hat|^2 over the integer wavevectors in [-n/2, n/2)^3 with
// round(|k|) = k.  Lattice sizes such as 96 and 192 are not powers of two,
// so the transform is a sum-factorised direct DFT: one O(n) dot product per
// output element and axis (x, then y, then z), register-blocked over 64 or
// 128 frequencies and 16 lines per wavefront, with a float64 twiddle table.
// The velocity is real, so the spectrum readout transforms only the half
// k_x <= n / 2 and counts the conjugate partners twice.
// The shell sums are deterministic: for each (k_z, k_y) row the k_x values
// are visited in order of |k_x|, so the shell index never decreases and each
// (shell, row) partial is written exactly once; a second kernel adds the
// rows of each shell in a fixed order.
#include <mutex>
#include <type_traits>

#include "kernels.h"

namespace nco {

namespace {

template <int S>
__global__ __launch_bounds__(256) void k_velocity(const typename Codec<S>::store_t* __restrict__ f,
                                                  double* __restrict__ u, int n) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    double r = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double v = Codec<S>::to_double(f[(size_t)i * n + idx], i);
        r += v;
        jx += cx_of(i) * v;
        jy += cy_of(i) * v;
        jz += cz_of(i) * v;
    }
    u[idx] = jx / r;
    u[(size_t)n + idx] = jy / r;
    u[2 * (size_t)n + idx] = jz / r;
}

// One axis of the DFT over a [3][n][n][n] field, out[k] = sum_j w^(j k) in[j]
// along AXIS (0 = x, stride 1; 1 = y, stride n; 2 = z, stride n^2) for every
// line ("column") of the field, w = exp(-2 pi i / n), or its conjugate with
// CONJ (the unnormalised inverse).  REAL_IN reads a real field (float64) and
// skips the products with its zero imaginary part.  The x pass computes the
// frequencies k < kout; the y and z passes take only the lines with x < xk
// (kout = xk = n // 2 + 1 for the half spectrum of a real field, n
// otherwise).
//
// Register-blocked: a block of 4 wavefronts takes 4 C columns and 64 KL
// frequencies; lane l of wavefront v accumulates the frequencies
// k0 + l + 64 q (q < KL) for the columns C v .. C v + C - 1 (C = 16, 16, 8
// for KL = 1, 2, 4).  The inputs come
// through LDS in chunks of 32 along the axis (loaded once per block, read by
// every lane of a wavefront at the same address, each read feeding KL
// frequencies), and a lane's twiddle w^(j k) starts each chunk from the
// table and is advanced by w^k from one j to the next.
constexpr int DB_JC = 32, DB_THREADS = 256;
// Columns per wavefront and per block for KL frequency groups per lane: the
// lane keeps 16 (KL = 1) or 32 (KL = 2, 4) accumulators.
template <int KL> constexpr int db_cpw() { return KL == 1 ? 16 : 32 / KL; }
template <int KL> constexpr int db_cols() { return 4 * db_cpw<KL>(); }

template <int AXIS>
__device__ __forceinline__ size_t dft_stride(int n) {
    return AXIS == 0 ? 1 : AXIS == 1 ? (size_t)n : (size_t)n * n;
}

// Offset of the first element of compact column c (see above): for the x
// pass every x line (c = (comp n + z) n + y); for the y and z passes the
// lines with x < xk, c = (comp n + outer) xk + x, outer = z (y pass) or y
// (z pass).  Column counts stay below 2^32.
template <int AXIS>
__device__ __forceinline__ size_t dft_base(unsigned c, int n, int xk) {
    if constexpr (AXIS == 0) return (size_t)c * n;
    const unsigned q = c / (unsigned)xk, x = c - q * (unsigned)xk;    // q = comp n + outer
    if constexpr (AXIS == 1) return (size_t)q * n * n + x;            // [comp][z][.][x]
    const unsigned comp = q / (unsigned)n, y = q - comp * (unsigned)n;
    return (size_t)comp * n * n * n + (size_t)y * n + x;              // [comp][.][y][x]
}

template <bool REAL_IN>
using dft_elem = typename std::conditional<REAL_IN, double, double2>::type;

// The j loop of one chunk.
template <int AXIS, bool REAL_IN, int KL>
__device__ __forceinline__ void dft_chunk(const dft_elem<REAL_IN>* __restrict__ tile, int jn, int wave,
                                          double2 (&w)[KL], const double2 (&wk)[KL],
                                          double2 (&acc)[KL][db_cpw<KL>()]) {
    constexpr int DB_CPW = db_cpw<KL>(), DB_COLS = db_cols<KL>();
#pragma unroll 1
    for (int j = 0; j < jn; ++j) {
#pragma unroll
        for (int c = 0; c < DB_CPW; ++c) {
            const int col = wave * DB_CPW + c;
            const dft_elem<REAL_IN> v = tile[AXIS == 0 ? col * DB_JC + j : j * DB_COLS + col];
#pragma unroll
            for (int q = 0; q < KL; ++q) {
                if constexpr (REAL_IN) {
                    acc[q][c].x = fma(w[q].x, v, acc[q][c].x);
                    acc[q][c].y = fma(w[q].y, v, acc[q][c].y);
                } else {
                    acc[q][c].x = fma(w[q].x, v.x, fma(-w[q].y, v.y, acc[q][c].x));
                    acc[q][c].y = fma(w[q].x, v.y, fma(w[q].y, v.x, acc[q][c].y));
                }
            }
        }
#pragma unroll
        for (int q = 0; q < KL; ++q) {
            const double t = w[q].x * wk[q].x - w[q].y * wk[q].y;
            w[q].y = w[q].x * wk[q].y + w[q].y * wk[q].x;
            w[q].x = t;
        }
    }
}

// Two wavefronts per SIMD at two frequency groups per lane (the 128
// accumulator registers and a column's 16 values in flight), four at one.
template <int AXIS, bool REAL_IN, bool CONJ, int KL>
__global__ __launch_bounds__(DB_THREADS, KL == 1 ? 4 : 2) void k_dft_axis(
    const void* __restrict__ in_, double2* __restrict__ out, const double2* __restrict__ tw, int n, int kout,
    int xk) {
    // x: [column][j], so that the loads along a line write consecutive LDS
    // words; y, z: [j][column].  Either way a wavefront reads one word.
    constexpr int DB_CPW = db_cpw<KL>(), DB_COLS = db_cols<KL>();
    __shared__ dft_elem<REAL_IN> tile[DB_JC * DB_COLS];
    const dft_elem<REAL_IN>* __restrict__ in = static_cast<const dft_elem<REAL_IN>*>(in_);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int k0 = blockIdx.y * 64 * KL;
    const unsigned ncol = AXIS == 0 ? 3u * n * n : 3u * n * xk;
    const unsigned c0 = blockIdx.x * DB_COLS;
    const size_t S = dft_stride<AXIS>(n);
    // The loads: x pass, thread t takes j = t % 32 of the columns t / 32 + 8 i;
    // y, z passes, column t % 64 at j = t / 64 + 4 i.
    constexpr int LOADS = DB_JC * DB_COLS / DB_THREADS;
    const int lj = AXIS == 0 ? (int)threadIdx.x % DB_JC : (int)threadIdx.x / DB_COLS;
    const int lc = AXIS == 0 ? (int)threadIdx.x / DB_JC : (int)threadIdx.x % DB_COLS;
    const bool lcol_ok = c0 + lc < ncol;
    const size_t lbase = lcol_ok ? dft_base<AXIS>(c0 + lc, n, xk) : 0;
    double2 acc[KL][DB_CPW];
    double2 w[KL], wk[KL];
    int kq[KL];
#pragma unroll
    for (int q = 0; q < KL; ++q) {
        kq[q] = k0 + lane + 64 * q;
        wk[q] = kq[q] < kout ? tw[kq[q]] : make_double2(1.0, 0.0);
        if constexpr (CONJ) wk[q].y = -wk[q].y;
#pragma unroll
        for (int c = 0; c < DB_CPW; ++c) acc[q][c] = make_double2(0.0, 0.0);
    }
    for (int j0 = 0; j0 < n; j0 += DB_JC) {
        const int jn = min(DB_JC, n - j0);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < LOADS; ++i) {
            dft_elem<REAL_IN> v{};
            if constexpr (AXIS == 0) {
                const int c = lc + (DB_THREADS / DB_JC) * i;
                if (lj < jn && c0 + c < ncol) v = in[(size_t)(c0 + c) * n + j0 + lj];
                tile[c * DB_JC + lj] = v;
            } else {
                const int j = lj + (DB_THREADS / DB_COLS) * i;
                if (j < jn && lcol_ok) v = in[lbase + (size_t)(j0 + j) * S];
                tile[j * DB_COLS + lc] = v;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < KL; ++q) {
            w[q] = tw[(int)(((long)j0 * (kq[q] < kout ? kq[q] : 0)) % n)];
            if constexpr (CONJ) w[q].y = -w[q].y;
        }
        dft_chunk<AXIS, REAL_IN, KL>(tile, jn, wave, w, wk, acc);
    }
    // Output: the wavefront's 16 columns are consecutive compact columns;
    // their offsets are block-uniform and advance by one line at a time.
    const unsigned cw = c0 + wave * DB_CPW;
    size_t base = cw < ncol ? dft_base<AXIS>(cw, n, xk) : 0;
    unsigned xr = AXIS == 0 ? 0 : cw % (unsigned)xk;       // x of the current line (y, z passes)
    unsigned yr = AXIS == 2 ? (cw / (unsigned)xk) % (unsigned)n : 0;
#pragma unroll
    for (int c = 0; c < DB_CPW; ++c) {
        if (cw + c < ncol)
#pragma unroll
            for (int q = 0; q < KL; ++q)
                if (kq[q] < kout) out[base + (size_t)kq[q] * S] = acc[q][c];
        // Next compact column.
        if constexpr (AXIS == 0) {
            base += n;
        } else {
            if (++xr < (unsigned)xk) {
                base += 1;
            } else if constexpr (AXIS == 1) {
                xr = 0;
                base += (size_t)n * n - (xk - 1);                 // next z (or component)
            } else {
                xr = 0;
                if (++yr < (unsigned)n) {
                    base += (size_t)n - (xk - 1);                 // next y
                } else {
                    yr = 0;
                    base += (size_t)n * n * n - (size_t)(n - 1) * n - (xk - 1);   // next component
                }
            }
        }
    }
}

template <int AXIS, bool REAL_IN, bool CONJ, int KL>
void dft_launch(const void* in, double2* out, const double2* tw, int n, int kspan, int xk, size_t ncol,
                hipStream_t st) {
    const dim3 grid((unsigned)((ncol + db_cols<KL>() - 1) / db_cols<KL>()), (unsigned)((kspan + 64 * KL - 1) / (64 * KL)));
    hipLaunchKernelGGL((k_dft_axis<AXIS, REAL_IN, CONJ, KL>), grid, dim3(DB_THREADS), 0, st, in, out, tw, n, kspan, xk);
}

// Launch of one axis pass over the [3][n][n][n] field (kout, xk as above).
// Above 64 a lane takes two frequency groups, above 128 four (with 16 and 8
// columns per wavefront): each LDS read then feeds 2 or 4 frequencies, so
// the reads stop limiting the FMAs, and the 129 frequencies of the 256^3
// half spectrum's x pass take one 256-frequency block.
template <int AXIS, bool REAL_IN, bool CONJ = false>
void dft_pass(const void* in, double2* out, const double2* tw, int n, int kout, int xk, hipStream_t st) {
    const size_t ncol = AXIS == 0 ? 3 * (size_t)n * n : 3 * (size_t)n * xk;
    const int kspan = AXIS == 0 ? kout : n;
    if (n > 128)
        dft_launch<AXIS, REAL_IN, CONJ, 4>(in, out, tw, n, kspan, xk, ncol, st);
    else if (n > 64)
        dft_launch<AXIS, REAL_IN, CONJ, 2>(in, out, tw, n, kspan, xk, ncol, st);
    else
        dft_launch<AXIS, REAL_IN, CONJ, 1>(in, out, tw, n, kspan, xk, ncol, st);
}

// The three forward passes: full (every frequency) or the half spectrum
// k_x <= n / 2 of the real velocity field.
void dft_forward(const double* u, double2* A, double2* B, const double2* tw, int n, bool half, hipStream_t st) {
    const int xk = half ? n / 2 + 1 : n;
    dft_pass<0, true>(u, A, tw, n, xk, xk, st);
    dft_pass<1, false>(A, B, tw, n, n, xk, st);
    dft_pass<2, false>(B, A, tw, n, n, xk, st);
}

__device__ __forceinline__ int wavenumber(int idx, int n) { return idx < n - n / 2 ? idx : idx - n; }

// Partial shell sums of one (kz, ky) row; partial is [nbins][n*n], zeroed.
// uh holds k_x = 0 .. n / 2 only (the half spectrum of a real field):
// |u_hat(-k_x, k_y, k_z)| = |u_hat(k_x, -k_y, -k_z)| lies in the same shell,
// so each k_x whose conjugate partner is another k_x counts twice (k_x = 0,
// and -n/2 for even n, once).  The k_x are visited in order of |k_x|, so the
// shell index never decreases along a row.
__global__ __launch_bounds__(256) void k_shell_rows(const double2* __restrict__ uh, int n,
                                                    double* __restrict__ partial, int nbins) {
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    const int nn = n * n;
    if (row >= nn) return;
    const int kz = wavenumber(row / n, n), ky = wavenumber(row % n, n);
    const size_t n3 = (size_t)n * nn;
    const double scale = 0.5 / ((double)n3 * (double)n3);
    const int c2 = kz * kz + ky * ky;
    int cur = -1;
    double acc = 0.0;
    for (int a = 0; a <= n / 2; ++a) {
        const int b = (int)floor(sqrt((double)(c2 + a * a)) + 0.5);
        if (b != cur) {
            if (cur >= 0 && cur < nbins) partial[(size_t)cur * nn + row] = acc;
            cur = b;
            acc = 0.0;
        }
        const size_t e = (size_t)row * n + a;
        double t = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double2 v = uh[(size_t)c * n3 + e];
            t += (v.x * v.x + v.y * v.y) * scale;
        }
        acc += (a == 0 || 2 * a == n) ? t : 2.0 * t;
    }
    if (cur >= 0 && cur < nbins) partial[(size_t)cur * nn + row] = acc;
}

__global__ __launch_bounds__(256) void k_fill_zero(double* __restrict__ p, size_t count) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.0;
}

// One block per shell: fixed-order strided sums, a wavefront shuffle
// reduction, then the four wavefront sums in order.
__global__ __launch_bounds__(256) void k_shell_final(const double* __restrict__ partial, int rows,
                                                     double* __restrict__ E) {
    const int b = blockIdx.x;
    double s = 0.0;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) s += partial[(size_t)b * rows + r];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    __shared__ double part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) E[b] = (part[0] + part[1]) + (part[2] + part[3]);
}

// dL/dE at every wavevector: A[c][e] *= dL/dE(shell of e).
__global__ __launch_bounds__(256) void k_scale_shells(double2* __restrict__ A, int n,
                                                      const double* __restrict__ dE, int nbins) {
    const size_t n3 = (size_t)n * n * n;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n3) return;
    const int kx = wavenumber((int)(e % n), n), ky = wavenumber((int)((e / n) % n), n),
              kz = wavenumber((int)(e / ((size_t)n * n)), n);
    const int b = (int)floor(sqrt((double)(kx * kx + ky * ky + kz * kz)) + 0.5);
    const double s = b < nbins ? dE[b] : 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double2 v = A[(size_t)c * n3 + e];
        v.x *= s;
        v.y *= s;
        A[(size_t)c * n3 + e] = v;
    }
}

// rho and u = j / rho of every node (float64).
template <int S>
__global__ __launch_bounds__(256) void k_rho_u(const typename Codec<S>::store_t* __restrict__ f, double* __restrict__ u,
                                               double* __restrict__ rho, int n) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    double r = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double v = Codec<S>::to_double(f[(size_t)i * n + idx], i);
        r += v;
        jx += cx_of(i) * v;
        jy += cy_of(i) * v;
        jz += cz_of(i) * v;
    }
    u[idx] = jx / r;
    u[(size_t)n + idx] = jy / r;
    u[2 * (size_t)n + idx] = jz / r;
    rho[idx] = r;
}

// lambda_f = lambda_rho + c . lambda_j with lambda_u = Re(B) / n^6 (B the
// unnormalised inverse DFT of the shell-weighted spectrum), lambda_j =
// lambda_u / rho, lambda_rho = -lambda_u . u / rho.
__global__ __launch_bounds__(256) void k_lambda_from_u(const double2* __restrict__ B, const double* __restrict__ u,
                                                       const double* __restrict__ rho, int n3, double scale,
                                                       float* __restrict__ lam) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n3) return;
    double lu[3], lr = 0.0;
    const double ir = 1.0 / rho[idx];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        lu[c] = B[(size_t)c * n3 + idx].x * scale;
        lr -= lu[c] * u[(size_t)c * n3 + idx];
    }
    lr *= ir;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        lam[(size_t)i * n3 + idx] = (float)(lr + (cx_of(i) * lu[0] + cy_of(i) * lu[1] + cz_of(i) * lu[2]) * ir);
}

struct SpecLayout {
    size_t u, a, b, part, tw, rho, total;
};

SpecLayout spec_layout(int n, int nbins) {
    const size_t n3 = (size_t)n * n * n;
    SpecLayout L;
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    L.u = 0;
    L.a = up(L.u + 3 * n3 * sizeof(double));
    L.b = up(L.a + 3 * n3 * sizeof(double2));
    L.part = up(L.b + 3 * n3 * sizeof(double2));
    L.tw = up(L.part + (size_t)nbins * n * n * sizeof(double));
    L.rho = up(L.tw + (size_t)n * sizeof(double2));
    L.total = up(L.rho + n3 * sizeof(double));
    return L;
}

// Twiddles exp(-2 pi i m / n), m = 0 .. n-1, in float64 on the device.
__global__ __launch_bounds__(256) void k_twiddles(double2* __restrict__ tw, int n) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    double s, c;
    sincospi(2.0 * (double)m / (double)n, &s, &c);
    tw[m] = make_double2(c, -s);
}

hipError_t upload_twiddles(double2* tw, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_twiddles, dim3((n + 255) / 256), dim3(256), 0, st, tw, n);
    return hipGetLastError();
}

// Scratch of the allocation-free spectrum (nco_energy_spectrum_noalloc):
// one array per device, held until the process ends.  Host code never
// passes the array's name to a kernel (on the host it stands for a host-side
// symbol, not a device address); it uses the device address that
// hipGetSymbolAddress gives, taken once per device with that device current.
constexpr size_t SCRATCH_BYTES = (size_t)36 << 20;
__device__ __align__(256) char scratch[SCRATCH_BYTES];

constexpr int SCRATCH_DEVICES = 64;
void* g_scratch_ptr[SCRATCH_DEVICES] = {};
std::mutex g_scratch_mutex;

}  // namespace

int spectrum_bins(int n) { return (int)floor(sqrt(3.0) * (n / 2) + 0.5) + 1; }

// lam (float [27][n^3]) = (dE/df)^T dL/dE for the spectrum of f; dE lives on
// the device (nbins doubles).  Forward DFT, weight each wavevector by the
// derivative of its shell, inverse DFT, then the chain rule through u = j/rho.
hipError_t launch_spectrum_adjoint(int storage, const void* f, int n, void* work, const double* dE,
                                   int nbins, float* lam, hipStream_t st) {
    const SpecLayout L = spec_layout(n, nbins);
    char* w = static_cast<char*>(work);
    double* u = reinterpret_cast<double*>(w + L.u);
    double2* A = reinterpret_cast<double2*>(w + L.a);
    double2* B = reinterpret_cast<double2*>(w + L.b);
    double2* tw = reinterpret_cast<double2*>(w + L.tw);
    double* rho = reinterpret_cast<double*>(w + L.rho);
    const int n3 = n * n * n;
    if (hipError_t e = upload_twiddles(tw, n, st); e != hipSuccess) return e;
    const int nb = (n3 + 255) / 256;
    switch (storage) {
        case ST_F32: hipLaunchKernelGGL(k_rho_u<ST_F32>, dim3(nb), dim3(256), 0, st, static_cast<const float*>(f), u, rho, n3); break;
        case ST_F16: hipLaunchKernelGGL(k_rho_u<ST_F16>, dim3(nb), dim3(256), 0, st, static_cast<const __half*>(f), u, rho, n3); break;
        case ST_BF16: hipLaunchKernelGGL(k_rho_u<ST_BF16>, dim3(nb), dim3(256), 0, st, static_cast<const __hip_bfloat16*>(f), u, rho, n3); break;
        case ST_F64: hipLaunchKernelGGL(k_rho_u<ST_F64>, dim3(nb), dim3(256), 0, st, static_cast<const double*>(f), u, rho, n3); break;
        default: return hipErrorInvalidValue;
    }
    dft_forward(u, A, B, tw, n, false, st);
    hipLaunchKernelGGL(k_scale_shells, dim3(nb), dim3(256), 0, st, A, n, dE, nbins);
    dft_pass<0, false, true>(A, B, tw, n, n, n, st);
    dft_pass<1, false, true>(B, A, tw, n, n, n, st);
    dft_pass<2, false, true>(A, B, tw, n, n, n, st);
    const double scale = 1.0 / ((double)n3 * (double)n3);
    hipLaunchKernelGGL(k_lambda_from_u, dim3(nb), dim3(256), 0, st, B, u, rho, n3, scale, lam);
    return hipGetLastError();
}

size_t spectrum_workspace_bytes(int n) { return spec_layout(n, spectrum_bins(n)).total; }

// Bytes of the work space the forward spectrum uses (everything before the
// density array, which only the adjoint needs).
size_t spectrum_forward_bytes(int n) { return spec_layout(n, spectrum_bins(n)).rho; }

size_t spectrum_scratch_bytes() { return SCRATCH_BYTES; }

// Device address of the scratch array on `device` (the current device),
// looked up on the first call per device and kept.
hipError_t spectrum_scratch(int device, void** ptr) {
    if (device < 0 || device >= SCRATCH_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        if (hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)); e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

hipError_t launch_energy_spectrum(int storage, const void* f, int n, void* work, double* E_dev,
                                  int nbins, hipStream_t st) {
    const SpecLayout L = spec_layout(n, nbins);
    char* w = static_cast<char*>(work);
    double* u = reinterpret_cast<double*>(w + L.u);
    double2* A = reinterpret_cast<double2*>(w + L.a);
    double2* B = reinterpret_cast<double2*>(w + L.b);
    double* part = reinterpret_cast<double*>(w + L.part);
    double2* tw = reinterpret_cast<double2*>(w + L.tw);
    const int n3 = n * n * n;
    if (hipError_t e = upload_twiddles(tw, n, st); e != hipSuccess) return e;
    const int nb = (n3 + 255) / 256;
    switch (storage) {
        case ST_F32: hipLaunchKernelGGL(k_velocity<ST_F32>, dim3(nb), dim3(256), 0, st, static_cast<const float*>(f), u, n3); break;
        case ST_F16: hipLaunchKernelGGL(k_velocity<ST_F16>, dim3(nb), dim3(256), 0, st, static_cast<const __half*>(f), u, n3); break;
        case ST_BF16: hipLaunchKernelGGL(k_velocity<ST_BF16>, dim3(nb), dim3(256), 0, st, static_cast<const __hip_bfloat16*>(f), u, n3); break;
        case ST_F64: hipLaunchKernelGGL(k_velocity<ST_F64>, dim3(nb), dim3(256), 0, st, static_cast<const double*>(f), u, n3); break;
        default: return hipErrorInvalidValue;
    }
    dft_forward(u, A, B, tw, n, true, st);
    const size_t pc = (size_t)nbins * n * n;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((pc + 255) / 256)), dim3(256), 0, st, part, pc);
    hipLaunchKernelGGL(k_shell_rows, dim3((n * n + 255) / 256), dim3(256), 0, st, A, n, part, nbins);
    hipLaunchKernelGGL(k_shell_final, dim3(nbins), dim3(256), 0, st, part, n * n, E_dev);
    return hipGetLastError();
}

}  // namespace nco
