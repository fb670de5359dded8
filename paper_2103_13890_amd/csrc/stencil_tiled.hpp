// z-marching LDS-tiled evaluation for large 3D levels of the scalar kinds.
//
// A block owns a TTX x TTY column of nodes (one 64-wide wavefront per x row,
// so every global access is a coalesced row) and TZC consecutive node
// planes.  It marches up in z keeping two node planes of the state (and
// direction, coefficient) in LDS with a one-node halo.  For each element
// layer it evaluates every element of the tile (plus the one-element halo)
// exactly once, writes the element's eight corner contributions to LDS, and
// each node then sums the four contributions from below (carried in a
// register from the previous layer) and the four from above.  The element
// work, which dominates the arithmetic, is therefore done once per element
// instead of once per adjacent node.
//
// Workgroup ids are remapped so that the blocks dispatched to one XCD
// (ids are dealt round-robin over the 8 XCDs) own a contiguous range of
// tiles, keeping shared halo rows in that XCD's L2.
#pragma once
#include "stencil.hpp"

namespace jfnk {

constexpr int TTX = 64, TTY = 4, TZC = 16;

__device__ __forceinline__ int xcd_tile(int id, int nb) {
    const int q = nb / 8, r = nb % 8;
    const int xcd = id % 8, loc = id / 8;
    return xcd < r ? xcd * (q + 1) + loc : r * (q + 1) + (xcd - r) * q + loc;
}

inline int tiled_blocks(const Grid &g) {
    return ((g.NX + TTX - 1) / TTX) * ((g.NY + TTY - 1) / TTY) * ((g.NZ + TZC - 1) / TZC);
}

template <int KIND, int MODE, typename T, typename TV, class Epi>
__global__ __launch_bounds__(TTX *TTY) void k_tiled(Grid g, Phys ph, const T *kap, const T *x, const TV *v,
                                                    const T *Ax, FdStep fd, Epi epi, Red red) {
    constexpr int HX = TTX + 2, HY = TTY + 2, EX = TTX + 1, EY = TTY + 1;
    constexpr int NT = TTX * TTY;
    constexpr bool FD = MODE != M_RESID;
    constexpr bool INV = KIND == JFNK_INVCOEF;
    __shared__ T sx[2][HY * HX];
    __shared__ T sv[FD ? 2 : 1][FD ? HY * HX : 1];
    __shared__ T sk[INV ? 2 : 1][INV ? HY * HX : 1];
    __shared__ T se[8][EY * EX];

    const int ntx = (g.NX + TTX - 1) / TTX, nty = (g.NY + TTY - 1) / TTY;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tix = tile % ntx, rest = tile / ntx;
    const int tiy = rest % nty, tiz = rest / nty;
    const int x0 = tix * TTX, y0 = tiy * TTY, z0 = tiz * TZC;
    const int z1 = min(z0 + TZC, g.NZ);
    const int tx = threadIdx.x % TTX, ty = threadIdx.x / TTX;
    const double eps = fd.eps();
    const bool zero_fd = FD && eps == 0.0;
    const T e = (T)eps;
    const T ie = eps > 0.0 ? (T)(1.0 / eps) : T(0);
    const T h = (T)g.h;
    double sums[Epi::NS > 0 ? Epi::NS : 1];
#pragma unroll
    for (int k = 0; k < (Epi::NS > 0 ? Epi::NS : 1); ++k) sums[k] = 0.0;

    auto load_plane = [&](int pz) {
        const int sl = pz & 1;
        for (int k = threadIdx.x; k < HX * HY; k += NT) {
            const int lx = k % HX, ly = k / HX;
            const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
            const bool in = gx >= 0 && gx < g.NX && gy >= 0 && gy < g.NY && pz >= 0 && pz < g.NZ;
            const long long j = in ? node_index(g, gx, gy, pz) : 0;
            sx[sl][k] = in ? x[j] : T(0);
            if constexpr (FD) sv[sl][k] = (in && !is_dirichlet(g, gx, gy, pz)) ? (T)v[j] : T(0);
            if constexpr (INV) sk[sl][k] = in ? kap[j] : T(0);
        }
    };
    auto elem_layer = [&](int ez) {
        const int p0 = ez & 1, p1 = (ez + 1) & 1;
        for (int k = threadIdx.x; k < EX * EY; k += NT) {
            const int lx = k % EX, ly = k / EX;
            const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
            const bool valid = !zero_fd && gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny && ez >= 0 && ez < g.nz;
            T r[1][8];
            if (valid) {
                T xe[1][8], ve[1][8], kp[8];
#pragma unroll
                for (int a = 0; a < 8; ++a) {
                    const int o = (ly + ((a >> 1) & 1)) * HX + lx + (a & 1);
                    const int ps = (a >> 2) ? p1 : p0;
                    xe[0][a] = sx[ps][o];
                    ve[0][a] = FD ? sv[FD ? ps : 0][FD ? o : 0] : T(0);
                    kp[a] = INV ? sk[INV ? ps : 0][INV ? o : 0] : T(0);
                }
                elem_eval<3, KIND, MODE, T, 1, 8>(xe, ve, kp, e, ph, h, r);
            } else {
#pragma unroll
                for (int a = 0; a < 8; ++a) r[0][a] = T(0);
            }
#pragma unroll
            for (int a = 0; a < 8; ++a) se[a][k] = r[0][a];
        }
    };
    // contributions of the element layer in se to the node (tx, ty) below
    // (corners with a_z = 1 ... of the layer under the plane) and above
    auto gather = [&](bool upper_corners) -> T {
        T acc = T(0);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int c = upper_corners ? a + 4 : a;
            const int idx = (ty + 1 - ((c >> 1) & 1)) * EX + (tx + 1 - (c & 1));
            acc += se[c][idx];
        }
        return acc;
    };

    load_plane(z0 - 1);
    load_plane(z0);
    __syncthreads();
    elem_layer(z0 - 1);
    __syncthreads();
    T carry = gather(true);        // element layer z0-1, corners on plane z0
    for (int z = z0; z < z1; ++z) {
        __syncthreads();
        load_plane(z + 1);
        __syncthreads();
        elem_layer(z);
        __syncthreads();
        const T below = carry;
        const T above = gather(false);   // element layer z, corners on plane z
        carry = gather(true);            // element layer z, corners on plane z+1
        const int gx = x0 + tx, gy = y0 + ty;
        if (gx < g.NX && gy < g.NY) {
            const long long i = node_index(g, gx, gy, z);
            const bool dir = is_dirichlet(g, gx, gy, z);
            T val[1] = {T(0)};
            if (!dir && !zero_fd) {
                T acc = below + above;
                if constexpr (MODE == M_FD_PLAIN) acc = (acc - Ax[i]) * ie;
                val[0] = acc;
            }
            epi.node(i, val, dir, sums);
        }
    }
    if constexpr (Epi::NS > 0) block_partials<Epi::NS>(sums, red);
}

}  // namespace jfnk
