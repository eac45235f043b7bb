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

// Reduced Taylor-Green domain (Appendix A): the lattice is the cube
// [0, pi/2]^3 of the vortex with n nodes per edge, half a spacing from the
// faces, and stands for the whole 2 pi box, which the vortex's symmetries
// fill with images of the cube.  A streaming source outside the cube is
// mapped inside by one of those symmetries, and the population's velocity is
// mapped with it:
//   coordinate < 0 (the planes through the origin): mirror, that velocity
//     component reversed (S_x, S_y, S_z);
//   z > pi/2: half turn about the line x = y, z = pi/2,
//     (x, y, z) -> (y, x, pi - z), c -> (c_y, c_x, -c_z);
//   x > pi/2: quarter turn about the vortex axis x = y = pi/2,
//     (x, y) -> (y, pi - x), c -> (c_y, -c_x);
//   y > pi/2: the opposite quarter turn, (x, y) -> (pi - y, x), c -> (-c_y, c_x).
// In node indices pi - x is 2n - 1 - j.  Two rounds bring every source with
// coordinates in [-1, n] inside (checked exhaustively against the unfolded
// periodic streaming for n = 1..7); the map is a bijection of population
// slots, so its adjoint is the scatter to the same slot.  The clamp only
// keeps an impossible input in bounds.
struct Slot {
    int plane, node;
};

__device__ __forceinline__ Slot fold_octant(int n, int sx, int sy, int sz, int cx, int cy, int cz) {
#pragma unroll
    for (int round = 0; round < 2; ++round) {
        if (sx < 0) { sx = -1 - sx; cx = -cx; }
        if (sy < 0) { sy = -1 - sy; cy = -cy; }
        if (sz < 0) { sz = -1 - sz; cz = -cz; }
        if (sz >= n) {
            int t = sx; sx = sy; sy = t; sz = 2 * n - 1 - sz;
            t = cx; cx = cy; cy = t; cz = -cz;
        }
        if (sx >= n) {
            int t = sx; sx = sy; sy = 2 * n - 1 - t;
            t = cx; cx = cy; cy = -t;
        }
        if (sy >= n) {
            int t = sy; sy = sx; sx = 2 * n - 1 - t;
            t = cy; cy = cx; cx = -t;
        }
    }
    sx = min(max(sx, 0), n - 1);
    sy = min(max(sy, 0), n - 1);
    sz = min(max(sz, 0), n - 1);
    return {9 * (cz + 1) + 3 * (cy + 1) + (cx + 1), (sz * n + sy) * n + sx};
}

__device__ __forceinline__ bool on_octant_face(const StepArgs& a, NodeIdx p) {
    return a.domain == DOMAIN_TGV_OCTANT &&
           (p.x == 0 || p.y == 0 || p.z == 0 || p.x == a.nx - 1 || p.y == a.nx - 1 || p.z == a.nx - 1);
}

// Pull the 27 populations of node (x, y, z): f_i(x) <- f_i(x - c_i), periodic,
// or folded into the reduced Taylor-Green cube at its faces.
template <int S>
__device__ __forceinline__ void pull(const typename Codec<S>::store_t* __restrict__ fin,
                                     const StepArgs& a, NodeIdx p,
                                     typename Codec<S>::real (&f)[Q]) {
    if (on_octant_face(a, p)) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const Slot s = fold_octant(a.nx, p.x - cx_of(i), p.y - cy_of(i), p.z - cz_of(i), cx_of(i), cy_of(i),
                                       cz_of(i));
            f[i] = Codec<S>::load(fin + (size_t)s.plane * a.n + s.node, i);
        }
        return;
    }
    // Interior nodes of the reduced cube never wrap, so the periodic code
    // serves them too.
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

// Population i of node (x, y, z) as pull reads it: one of its 27 loads.
template <int S>
__device__ __forceinline__ typename Codec<S>::real pull_one(const typename Codec<S>::store_t* __restrict__ fin,
                                                            const StepArgs& a, NodeIdx p, int i) {
    const int cx = cx_of(i), cy = cy_of(i), cz = cz_of(i);
    if (on_octant_face(a, p)) {
        const Slot s = fold_octant(a.nx, p.x - cx, p.y - cy, p.z - cz, cx, cy, cz);
        return Codec<S>::load(fin + (size_t)s.plane * a.n + s.node, i);
    }
    const int x = cx < 0 ? (p.x == a.nx - 1 ? 0 : p.x + 1) : cx > 0 ? (p.x == 0 ? a.nx - 1 : p.x - 1) : p.x;
    const int y = cy < 0 ? (p.y == a.ny - 1 ? 0 : p.y + 1) : cy > 0 ? (p.y == 0 ? a.ny - 1 : p.y - 1) : p.y;
    const int z = cz < 0 ? (p.z == a.nz - 1 ? 0 : p.z + 1) : cz > 0 ? (p.z == 0 ? a.nz - 1 : p.z - 1) : p.z;
    return Codec<S>::load(fin + (size_t)i * a.n + ((size_t)z * a.ny + y) * a.nx + x, i);
}

// Adjoint of pull: v_i(x) goes to the slot the pull of population i at x
// read, dL/df_i(x - c_i) = v_i(x) (periodic) or its folded slot.
__device__ __forceinline__ void scatter_to_sources(float* __restrict__ out, const StepArgs& a, NodeIdx p,
                                                   const float (&v)[Q]) {
    if (on_octant_face(a, p)) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const Slot s = fold_octant(a.nx, p.x - cx_of(i), p.y - cy_of(i), p.z - cz_of(i), cx_of(i), cy_of(i),
                                       cz_of(i));
            out[(size_t)s.plane * a.n + s.node] = v[i];
        }
        return;
    }
    const int xs[3] = {p.x == a.nx - 1 ? 0 : p.x + 1, p.x, p.x == 0 ? a.nx - 1 : p.x - 1};
    const int ys[3] = {(p.y == a.ny - 1 ? 0 : p.y + 1) * a.nx, p.y * a.nx, (p.y == 0 ? a.ny - 1 : p.y - 1) * a.nx};
    const int nxy = a.nx * a.ny;
    const int zs[3] = {(p.z == a.nz - 1 ? 0 : p.z + 1) * nxy, p.z * nxy, (p.z == 0 ? a.nz - 1 : p.z - 1) * nxy};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int dst = zs[cz_of(i) + 1] + ys[cy_of(i) + 1] + xs[cx_of(i) + 1];
        out[(size_t)i * a.n + dst] = v[i];
    }
}

template <int S>
__device__ __forceinline__ void load_local(const typename Codec<S>::store_t* __restrict__ fin,
                                           int n, int idx, typename Codec<S>::real (&f)[Q]) {
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = Codec<S>::load(fin + (size_t)i * n + idx, i);
}

// Store the 27 post-collision populations of node idx; with 16-bit
// deviation storage and sr_key != 0 by stochastic rounding.
template <int S>
__device__ __forceinline__ void store_local(typename Codec<S>::store_t* __restrict__ fout, int n,
                                            int idx, const typename Codec<S>::real (&f)[Q], unsigned sr_key = 0) {
    if constexpr (S == ST_BF16 || S == ST_F16) {
        if (sr_key) {
#pragma unroll
            for (int i = 0; i < Q; ++i) Codec<S>::store_sr(fout + (size_t)i * n + idx, i, f[i], sr_bits(sr_key, idx, i));
            return;
        }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) Codec<S>::store(fout + (size_t)i * n + idx, i, f[i]);
}

// One population of node idx to slot p (cached store; stochastic rounding
// as in store_local).
template <int S>
__device__ __forceinline__ void store_one_cached(typename Codec<S>::store_t* p, int idx, int i,
                                                 typename Codec<S>::real v, unsigned sr_key) {
    if constexpr (S == ST_BF16 || S == ST_F16) {
        if (sr_key) {
            Codec<S>::store_sr(p, i, v, sr_bits(sr_key, idx, i));
            return;
        }
    }
    Codec<S>::store_cached(p, i, v);
}

}  // namespace nco
