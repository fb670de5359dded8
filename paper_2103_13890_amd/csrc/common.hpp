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
    long long nn;          // nodes
    double h;              // element edge
    unsigned dir;          // Dirichlet faces (JFNK_FACE_* bits)
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

__device__ inline void node_coords(const Grid &g, long long i, int &x, int &y, int &z) {
    long long q = i / g.NX;
    x = (int)(i - q * g.NX);
    z = (int)(q / g.NY);
    y = (int)(q - (long long)z * g.NY);
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
