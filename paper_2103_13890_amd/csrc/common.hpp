// Shared device/host definitions of libjfnk: level grids and physics
// parameters passed by value to every kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/libjfnk.h"

namespace jfnk {

// One multigrid level (Sec. 2: nested meshes T_l).  Nodes are stored
// C-order [NZ][NY][NX] with x fastest; NZ = 1 for 2D grids.
struct Grid {
    int dim;
    int nx, ny, nz;        // elements per axis (nz = 0 in 2D)
    int NX, NY, NZ;        // nodes per axis
    long long nn;          // nodes (< 2^31, checked at context creation)
    double h;              // element edge
    unsigned dir;          // Dirichlet faces (JFNK_FACE_* bits)
    double rNX, rNY;       // 1/NX, 1/NY for index decoding
};

// Residual kind and its constants (Sec. 3 problem statements).
struct Phys {
    int kind;
    int ncomp;
    double a0, a1;         // BRATU lam | PLAP p, delta | NEOHOOKE mu, lambda (Lame)
};

__host__ __device__ inline bool is_dirichlet(const Grid &g, int x, int y, int z) {
    return ((g.dir & JFNK_FACE_XLO) && x == 0) || ((g.dir & JFNK_FACE_XHI) && x == g.nx) ||
           ((g.dir & JFNK_FACE_YLO) && y == 0) || ((g.dir & JFNK_FACE_YHI) && y == g.ny) ||
           (g.dim == 3 && (((g.dir & JFNK_FACE_ZLO) && z == 0) ||
                           ((g.dir & JFNK_FACE_ZHI) && z == g.nz)));
}

__host__ __device__ inline long long node_index(const Grid &g, int x, int y, int z) {
    return ((long long)z * g.NY + y) * g.NX + x;
}

// (x, y, z) of node i.  The quotients come from a double-precision
// reciprocal: for i < 2^31 its error is below 2^-21, so the truncated
// quotient is off by at most one and a single correction makes it exact
// (64-bit integer division has no hardware instruction and costs ~10x more).
__device__ __forceinline__ void udivmod(unsigned n, unsigned d, double rd, unsigned &q, unsigned &r) {
    q = (unsigned)((double)n * rd);
    int rr = (int)(n - q * d);
    if (rr < 0) { --q; rr += (int)d; }
    else if (rr >= (int)d) { ++q; rr -= (int)d; }
    r = (unsigned)rr;
}

__device__ __forceinline__ void node_coords(const Grid &g, long long i, int &x, int &y, int &z) {
    unsigned q, r, q2, r2;
    udivmod((unsigned)i, (unsigned)g.NX, g.rNX, q, r);
    udivmod(q, (unsigned)g.NY, g.rNY, q2, r2);
    x = (int)r;
    y = (int)r2;
    z = (int)q2;
}

// Evaluation modes of the stencil kernels: the residual A(x), the FD
// quotient from two residual evaluations, or its element difference form.
enum { M_RESID = 0, M_FD_PLAIN = 1, M_FD_DIFF = 2 };

template <typename T> struct Prec;
template <> struct Prec<double> {
    // sqrt(2^-52): root of the finite-difference step (Sec. 1)
    static constexpr double root_eps = 1.4901161193847656e-08;
};
template <> struct Prec<float> {
    // sqrt(2^-23)
    static constexpr double root_eps = 3.4526698300124393e-04;
};

}  // namespace jfnk
