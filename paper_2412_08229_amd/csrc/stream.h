// Pull streaming and local load/store of the structure-of-arrays population
// buffers [27][z][y][x] (x fastest), shared by the stream-collide kernels.
#pragma once

#include "d3q27.h"
#include "kernels.h"

namespace nco {

struct NodeIdx {
    int x, y, z;
};

__device__ __forceinline__ NodeIdx node_of(int idx, int nx, int ny) {
    const int nxy = nx * ny;
    NodeIdx r;
    r.z = idx / nxy;
    const int rem = idx - r.z * nxy;
    r.y = rem / nx;
    r.x = rem - r.y * nx;
    return r;
}

// Pull the 27 populations of node (x, y, z): f_i(x) <- f_i(x - c_i), periodic.
template <int S>
__device__ __forceinline__ void pull(const typename Codec<S>::store_t* __restrict__ fin,
                                     const StepArgs& a, NodeIdx p,
                                     typename Codec<S>::real (&f)[Q]) {
    // Source coordinate for c = -1, 0, +1 is x + 1, x, x - 1.
    const int xs[3] = {p.x == a.nx - 1 ? 0 : p.x + 1, p.x, p.x == 0 ? a.nx - 1 : p.x - 1};
    const int ys[3] = {(p.y == a.ny - 1 ? 0 : p.y + 1) * a.nx, p.y * a.nx,
                       (p.y == 0 ? a.ny - 1 : p.y - 1) * a.nx};
    const int nxy = a.nx * a.ny;
    const int zs[3] = {(p.z == a.nz - 1 ? 0 : p.z + 1) * nxy, p.z * nxy,
                       (p.z == 0 ? a.nz - 1 : p.z - 1) * nxy};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int src = zs[cz_of(i) + 1] + ys[cy_of(i) + 1] + xs[cx_of(i) + 1];
        f[i] = Codec<S>::load(fin + (size_t)i * a.n + src, i);
    }
}

template <int S>
__device__ __forceinline__ void load_local(const typename Codec<S>::store_t* __restrict__ fin,
                                           int n, int idx, typename Codec<S>::real (&f)[Q]) {
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = Codec<S>::load(fin + (size_t)i * n + idx, i);
}

template <int S>
__device__ __forceinline__ void store_local(typename Codec<S>::store_t* __restrict__ fout, int n,
                                            int idx, const typename Codec<S>::real (&f)[Q]) {
#pragma unroll
    for (int i = 0; i < Q; ++i) Codec<S>::store(fout + (size_t)i * n + idx, i, f[i]);
}

}  // namespace nco
