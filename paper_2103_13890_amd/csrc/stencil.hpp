// Evaluation of A(w) = sum_e r_e(w_e) at nodes, and of the finite-difference
// Jacobian action (Sec. 1), with fused epilogues.  A kernel instance is
// (grid dimension, residual kind, mode, precision, epilogue):
//
//   mode M_RESID    val = A(x)
//        M_FD_PLAIN val = (A(x + eps v) - A(x)) / eps, A(x) read from a cache
//        M_FD_DIFF  val = the same quotient summed from per-element
//                   difference forms (elem_*_fd), no cache read
//   epilogue        consumes val at node i: store F = val - b, store J v,
//                   a fused Chebyshev step, a power-method step, ...
//
// The step eps = num / ||v|| is read from device scalars at kernel start
// (num: the level's root (1 + ||x||) or the paper's variant; ||v||^2 written
// by the kernel that produced v), so no host round trip is needed.  The
// direction v is taken as 0 on Dirichlet nodes (J acts on the DoF space).
//
// This header holds the node-centric form (one thread per node, the
// elements around it evaluated in registers); stencil_tiled.hpp holds the
// z-marching LDS-tiled form for large 3D levels.  Both share the element
// routines and the epilogues.
#pragma once
#include <type_traits>

#include "access.hpp"
#include "elem.hpp"
#include "reduce.hpp"

namespace jfnk {

// ---- epilogues ---------------------------------------------------------------
// NS: number of grid sums; NCOMP: components; NIN: values read per node and
// component; VIN: the index of the input that is the FD direction itself
// (-1: none).  load(at, in) reads them (issued ahead of the element work by
// the tiled kernel, which passes SKIPV and takes input VIN from the direction
// plane it holds in LDS), node(at, val, dir, sums, in) consumes val at the node;
// at addresses the node (PtrAt or BufAt, access.hpp), the component c being
// c * nn further on.  operator()(totals) runs in the reduction's finishing
// kernel.

// F = val - b (b nullable); Aout (nullable) receives val; ||F||^2 -> out
template <typename T, int NC> struct EpiResidual {
    static constexpr int NS = 1;
    static constexpr int NCOMP = NC;
    static constexpr int NIN = 1;
    static constexpr int VIN = -1;
    const T *b;
    T *F;
    T *Aout;
    long long nn;
    double *out;
    template <bool SKIPV = false, class At> __device__ __forceinline__ void load(const At &at, T *in) const {
#pragma unroll
        for (int c = 0; c < NC; ++c) in[c] = b ? at.ld(b, c * nn) : T(0);
    }
    template <class At>
    __device__ __forceinline__ void node(const At &at, const T *val, bool dir, double *s, const T *in) const {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            T f = dir ? T(0) : val[c] - in[c];
            at.st(F, c * nn, f);
            if (Aout) at.st(Aout, c * nn, dir ? T(0) : val[c]);
            s[0] += (double)f * (double)f;
        }
    }
    __device__ void operator()(const double *t) const { if (out) out[0] = t[0]; }
    double *slot() const { return out; }
};

// J v
template <typename T, int NC> struct EpiJv {
    static constexpr int NS = 0;
    static constexpr int NCOMP = NC;
    static constexpr int NIN = 0;
    static constexpr int VIN = -1;
    T *Jv;
    long long nn;
    template <bool SKIPV = false, class At> __device__ __forceinline__ void load(const At &, T *) const {}
    template <class At>
    __device__ __forceinline__ void node(const At &at, const T *val, bool dir, double *, const T *) const {
#pragma unroll
        for (int c = 0; c < NC; ++c) at.st(Jv, c * nn, dir ? T(0) : val[c]);
    }
    __device__ void operator()(const double *) const {}
    double *slot() const { return nullptr; }
};

// Chebyshev step k (three-term recurrence), q = J d_k:
// s <- s + d_k;  r <- r - q;  d_{k+1} = c1 d_k + c2 r;  ||d_{k+1}||^2 -> out
template <typename T, int NC> struct EpiCheb {
    static constexpr int NS = 1;
    static constexpr int NCOMP = NC;
    static constexpr int NIN = 3;
    static constexpr int VIN = 0;
    const T *d;
    T *r, *s, *dn;
    T c1, c2;
    long long nn;
    double *out;
    template <bool SKIPV = false, class At> __device__ __forceinline__ void load(const At &at, T *in) const {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (!SKIPV) in[3 * c] = at.ld(d, c * nn);
            in[3 * c + 1] = at.ld((const T *)r, c * nn);
            in[3 * c + 2] = at.ld((const T *)s, c * nn);
        }
    }
    template <class At>
    __device__ __forceinline__ void node(const At &at, const T *val, bool dir, double *sm, const T *in) const {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const long long k = c * nn;
            const T dk = in[3 * c];
            const T rk = in[3 * c + 1] - val[c];
            const T dnew = c1 * dk + c2 * rk;
            at.st(s, k, dir ? T(0) : in[3 * c + 2] + dk);
            at.st(r, k, dir ? T(0) : rk);
            at.st(dn, k, dir ? T(0) : dnew);
            if (!dir) sm[0] += (double)dnew * (double)dnew;
        }
    }
    __device__ void operator()(const double *t) const { out[0] = t[0]; }
    double *slot() const { return out; }
};

// First Chebyshev step from s = 0, with the direction b instead of
// d_0 = b / theta: the FD quotient is homogeneous in its direction (the step
// eps = num / ||v|| makes eps v the same vector), so J d_0 = (J b) / theta.
// val = J b;  s_1 = b / theta;  r_1 = b - val / theta;  d_1 = c1 s_1 + c2 r_1;
// ||d_1||^2 -> out
template <typename T, int NC> struct EpiChebFirst {
    static constexpr int NS = 1;
    static constexpr int NCOMP = NC;
    static constexpr int NIN = 1;
    static constexpr int VIN = 0;
    const T *b;
    T *r, *s, *dn;
    T inv_theta, c1, c2;
    long long nn;
    double *out;
    template <bool SKIPV = false, class At> __device__ __forceinline__ void load(const At &at, T *in) const {
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (!SKIPV) in[c] = at.ld(b, c * nn);
    }
    template <class At>
    __device__ __forceinline__ void node(const At &at, const T *val, bool dir, double *sm, const T *in) const {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const long long k = c * nn;
            const T d0 = in[c] * inv_theta;
            const T rk = in[c] - val[c] * inv_theta;
            const T dnew = c1 * d0 + c2 * rk;
            at.st(s, k, dir ? T(0) : d0);
            at.st(r, k, dir ? T(0) : rk);
            at.st(dn, k, dir ? T(0) : dnew);
            if (!dir) sm[0] += (double)dnew * (double)dnew;
        }
    }
    __device__ void operator()(const double *t) const { out[0] = t[0]; }
    double *slot() const { return out; }
};

// Last Chebyshev step k, q = J d_k: r' = r - q, d_{k+1} = c1 d_k + c2 r',
// and the polynomial's final update s_out = s + d_k + d_{k+1} (r' and
// d_{k+1} are not kept); ||s_out||^2 -> out (nullable)
template <typename T, int NC> struct EpiChebLast {
    static constexpr int NS = 1;
    static constexpr int NCOMP = NC;
    static constexpr int NIN = 3;
    static constexpr int VIN = 0;
    const T *d, *r, *s;
    T *sout;
    T c1, c2;
    long long nn;
    double *out;
    template <bool SKIPV = false, class At> __device__ __forceinline__ void load(const At &at, T *in) const {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (!SKIPV) in[3 * c] = at.ld(d, c * nn);
            in[3 * c + 1] = at.ld(r, c * nn);
            in[3 * c + 2] = at.ld(s, c * nn);
        }
    }
    template <class At>
    __device__ __forceinline__ void node(const At &at, const T *val, bool dir, double *sm, const T *in) const {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const T dk = in[3 * c];
            const T rk = in[3 * c + 1] - val[c];
            const T dnew = c1 * dk + c2 * rk;
            const T so = dir ? T(0) : (in[3 * c + 2] + dk) + dnew;
            at.st(sout, c * nn, so);
            sm[0] += (double)so * (double)so;
        }
    }
    __device__ void operator()(const double *t) const { if (out) out[0] = t[0]; }
    double *slot() const { return out; }
};

// t = b - J s  (the residual restricted in Algorithm 1)
template <typename T, int NC> struct EpiResidJv {
    static constexpr int NS = 0;
    static constexpr int NCOMP = NC;
    static constexpr int NIN = 1;
    static constexpr int VIN = -1;
    const T *b;
    T *t;
    long long nn;
    template <bool SKIPV = false, class At> __device__ __forceinline__ void load(const At &at, T *in) const {
#pragma unroll
        for (int c = 0; c < NC; ++c) in[c] = at.ld(b, c * nn);
    }
    template <class At>
    __device__ __forceinline__ void node(const At &at, const T *val, bool dir, double *, const T *in) const {
#pragma unroll
        for (int c = 0; c < NC; ++c) at.st(t, c * nn, dir ? T(0) : in[c] - val[c]);
    }
    __device__ void operator()(const double *) const {}
    double *slot() const { return nullptr; }
};

// Chebyshev start from s != 0: r = b - J s, d = r / theta; ||d||^2 -> out
template <typename T, int NC> struct EpiChebInit {
    static constexpr int NS = 1;
    static constexpr int NCOMP = NC;
    static constexpr int NIN = 1;
    static constexpr int VIN = -1;
    const T *b;
    T *r, *d;
    T inv_theta;
    long long nn;
    double *out;
    template <bool SKIPV = false, class At> __device__ __forceinline__ void load(const At &at, T *in) const {
#pragma unroll
        for (int c = 0; c < NC; ++c) in[c] = at.ld(b, c * nn);
    }
    template <class At>
    __device__ __forceinline__ void node(const At &at, const T *val, bool dir, double *sm, const T *in) const {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const long long k = c * nn;
            const T rk = dir ? T(0) : in[c] - val[c];
            const T dk = rk * inv_theta;
            at.st(r, k, rk);
            at.st(d, k, dk);
            sm[0] += (double)dk * (double)dk;
        }
    }
    __device__ void operator()(const double *t) const { out[0] = t[0]; }
    double *slot() const { return out; }
};

// Power step on an unnormalized direction v (Sec. 2, smoothers: the power
// method).  With s = 1/||v||, the FD quotient is homogeneous in its
// direction (the step scales as 1/||v||, so the perturbed state is the same),
// J(s v) = s J(v): q = s J(v) is the image of the unit vector s v, and
// s v^T q and ||q||^2 are its Rayleigh quotient and squared norm.  The
// normalisation of the previous image thus needs no pass of its own.
template <typename T, int NC> struct EpiPower {
    static constexpr int NS = 2;
    static constexpr int NCOMP = NC;
    static constexpr int NIN = 1;
    static constexpr int VIN = 0;
    const T *v;
    T *q;
    long long nn;
    double *out;
    double sc = 0.0;     // 1/||v||, set on the device from the step's norm
    __device__ __forceinline__ void prepare(double n2) { sc = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0; }
    template <bool SKIPV = false, class At> __device__ __forceinline__ void load(const At &at, T *in) const {
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (!SKIPV) in[c] = at.ld(v, c * nn);
    }
    template <class At>
    __device__ __forceinline__ void node(const At &at, const T *val, bool dir, double *sm, const T *in) const {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const T qk = dir ? T(0) : (T)(sc * (double)val[c]);
            at.st(q, c * nn, qk);
            sm[0] += ((double)in[c] * sc) * (double)qk;
            sm[1] += (double)qk * (double)qk;
        }
    }
    __device__ void operator()(const double *t) const { out[0] = t[0]; out[1] = t[1]; }
    double *slot() const { return out; }
};

// epilogues that scale by 1/||v|| define prepare(||v||^2); the step and the
// norm come from the same (possibly block-summed) value
template <class E, class = void> struct EpiPrepares : std::false_type {};
template <class E> struct EpiPrepares<E, std::void_t<decltype(&E::prepare)>> : std::true_type {};
template <class E> __device__ __forceinline__ double fd_eps_prepare(const FdStep &fd, E &epi) {
    if constexpr (EpiPrepares<E>::value) {
        double n2 = 0.0;
        const double e = fd.eps(&n2);
        epi.prepare(n2);
        return e;
    } else {
        return fd.eps();
    }
}

// ---- one element in any mode ------------------------------------------------------
// xe: state corners; ve: direction corners (FD modes); r: output contributions
// m (scalar kinds): multiplies the element vector; 0 switches the element off
template <int DIM, int KIND, int MODE, typename T, int NC, int NV, int PF = 0>
__device__ __forceinline__ void elem_eval(const T (*xe)[NV], const T (*ve)[NV], const T *kp, T eps,
                                          const Phys &ph, T h, T (*r)[NV], T m = T(1)) {
    if constexpr (KIND == JFNK_NEOHOOKE) {
        if constexpr (MODE == M_FD_DIFF) {
            elem_neohooke_fd<T>(xe, ve, eps, ph, h, r);
        } else if constexpr (MODE == M_FD_PLAIN) {
            T w[3][8];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int a = 0; a < 8; ++a) w[c][a] = xe[c][a] + eps * ve[c][a];
            elem_neohooke<T>(w, ph, h, r);
        } else {
            elem_neohooke<T>(xe, ph, h, r);
        }
    } else {
        if constexpr (MODE == M_FD_DIFF) {
            elem_scalar_fd<DIM, KIND, T, PF>(xe[0], ve[0], kp, eps, ph, h, r[0], m);
        } else if constexpr (MODE == M_FD_PLAIN) {
            T w[NV];
#pragma unroll
            for (int a = 0; a < NV; ++a) w[a] = xe[0][a] + eps * ve[0][a];
            elem_scalar<DIM, KIND, T, PF>(w, kp, ph, h, r[0], m);
        } else {
            elem_scalar<DIM, KIND, T, PF>(xe[0], kp, ph, h, r[0], m);
        }
    }
}

// ---- node-centric value ---------------------------------------------------------------
// Sum of the contributions of the elements around node (X, Y, Z).
// Scalar kinds: the 3^DIM neighbourhood of x, v (and e^m) is loaded into
// registers first (clamped indices, all loads in flight together), then the
// 2^DIM elements around the node are evaluated from registers.
template <int DIM, int KIND, int MODE, typename T, typename TV>
__device__ __forceinline__ void node_value_scalar(const Grid &g, const Phys &ph, const T *kap, const T *x,
                                                  const TV *v, const T *Ax, double eps, int X, int Y, int Z,
                                                  long long i, T *val) {
    constexpr int NV = Cell<DIM>::NV;
    constexpr int NZ3 = DIM == 3 ? 3 : 1;
    constexpr int NB = 9 * NZ3;
    constexpr bool FD = MODE != M_RESID;
    constexpr bool INV = KIND == JFNK_INVCOEF;
    val[0] = T(0);
    if (FD && eps == 0.0) return;
    const T h = (T)g.h;
    const T e = (T)eps;
    T nx[NB], nv[NB], nk[NB];
    bool ok[3][3];     // [axis][offset]: neighbour index inside the grid
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ok[0][d] = X + d - 1 >= 0 && X + d - 1 < g.NX;
        ok[1][d] = Y + d - 1 >= 0 && Y + d - 1 < g.NY;
        ok[2][d] = DIM == 3 ? (Z + d - 1 >= 0 && Z + d - 1 < g.NZ) : d == 1;
    }
#pragma unroll
    for (int dz = 0; dz < NZ3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int k = (dz * 3 + dy) * 3 + dx;
                const int ax = min(max(X + dx - 1, 0), g.NX - 1), ay = min(max(Y + dy - 1, 0), g.NY - 1);
                const int az = DIM == 3 ? min(max(Z + dz - 1, 0), g.NZ - 1) : 0;
                const long long j = node_index(g, ax, ay, az);
                const bool in = ok[0][dx] && ok[1][dy] && ok[2][DIM == 3 ? dz : 1];
                nx[k] = x[j];
                nv[k] = FD ? (T)v[j] : T(0);
                nk[k] = INV ? kap[j] : T(0);
                if (FD && (!in || is_dirichlet(g, ax, ay, az))) nv[k] = T(0);
                if (!in) { nx[k] = T(0); nk[k] = T(0); }
            }
#pragma unroll
    for (int el = 0; el < NV; ++el) {
        const int ox = 1 - (el & 1), oy = 1 - ((el >> 1) & 1), oz = DIM == 3 ? 1 - ((el >> 2) & 1) : 0;
        const bool inside = ok[0][ox] && ok[1][oy] && (DIM == 2 || ok[2][oz]) &&
                            X - (el & 1) < g.nx && Y - ((el >> 1) & 1) < g.ny &&
                            (DIM == 2 || Z - ((el >> 2) & 1) < g.nz);
        if (!inside) continue;
        T xe[1][NV], ve[1][NV], kp[NV], r[1][NV];
#pragma unroll
        for (int a = 0; a < NV; ++a) {
            const int k = ((oz + ((a >> 2) & 1)) * 3 + oy + ((a >> 1) & 1)) * 3 + ox + (a & 1);
            xe[0][a] = nx[k];
            ve[0][a] = nv[k];
            kp[a] = nk[k];
        }
        elem_eval<DIM, KIND, MODE, T, 1, NV>(xe, ve, kp, e, ph, h, r);
        val[0] += r[0][el];
    }
    if constexpr (MODE == M_FD_PLAIN) val[0] = (val[0] - Ax[i]) * (T)(1.0 / eps);
}

template <int DIM, int KIND, int MODE, typename T, typename TV>
__device__ __forceinline__ void node_value(const Grid &g, const Phys &ph, const T *kap, const T *x, const TV *v,
                                           const T *Ax, double eps, int X, int Y, int Z, long long i, T *val) {
    constexpr int NV = Cell<DIM>::NV;
    constexpr int NC = (KIND == JFNK_NEOHOOKE) ? 3 : 1;
    if constexpr (NC == 1) {
        node_value_scalar<DIM, KIND, MODE, T, TV>(g, ph, kap, x, v, Ax, eps, X, Y, Z, i, val);
        return;
    }
    const long long nn = g.nn;
#pragma unroll
    for (int c = 0; c < NC; ++c) val[c] = T(0);
    if (MODE != M_RESID && eps == 0.0) return;
    const T h = (T)g.h;
    const T e = (T)eps;
    for (int el = 0; el < NV; ++el) {
        const int ex = X - (el & 1), ey = Y - ((el >> 1) & 1), ez = (DIM == 3) ? Z - ((el >> 2) & 1) : 0;
        if (ex < 0 || ex >= g.nx || ey < 0 || ey >= g.ny) continue;
        if (DIM == 3 && (ez < 0 || ez >= g.nz)) continue;
        T xe[NC][NV], ve[NC][NV], kp[NV], r[NC][NV];
#pragma unroll
        for (int a = 0; a < NV; ++a) {
            const int ax = ex + (a & 1), ay = ey + ((a >> 1) & 1), az = ez + ((a >> 2) & 1);
            const long long j = node_index(g, ax, ay, az);
            const bool dj = (MODE != M_RESID) && is_dirichlet(g, ax, ay, az);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                xe[c][a] = x[c * nn + j];
                ve[c][a] = (MODE == M_RESID || dj) ? T(0) : (T)v[c * nn + j];
            }
            kp[a] = (KIND == JFNK_INVCOEF) ? kap[j] : T(0);
        }
        elem_eval<DIM, KIND, MODE, T, NC, NV>(xe, ve, kp, e, ph, h, r);
#pragma unroll
        for (int c = 0; c < NC; ++c) val[c] += r[c][el];
    }
    if constexpr (MODE == M_FD_PLAIN) {
        const T ie = (T)(1.0 / eps);
#pragma unroll
        for (int c = 0; c < NC; ++c) val[c] = (val[c] - Ax[c * nn + i]) * ie;
    }
}

template <int DIM, int KIND, int MODE, typename T, typename TV, class Epi>
__global__ __launch_bounds__(BLOCK) void k_node(Grid g, Phys ph, const T *kap, const T *x, const TV *v, const T *Ax,
                                                FdStep fd, Epi epi, Red red) {
    constexpr int NC = (KIND == JFNK_NEOHOOKE) ? 3 : 1;
    const double eps = fd_eps_prepare(fd, epi);
    double sums[Epi::NS > 0 ? Epi::NS : 1];
#pragma unroll
    for (int k = 0; k < (Epi::NS > 0 ? Epi::NS : 1); ++k) sums[k] = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.nn; i += stride) {
        int X, Y, Z;
        node_coords(g, i, X, Y, Z);
        const bool dir = is_dirichlet(g, X, Y, Z);
        T val[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) val[c] = T(0);
        if (!dir) node_value<DIM, KIND, MODE, T, TV>(g, ph, kap, x, v, Ax, eps, X, Y, Z, i, val);
        T in[Epi::NIN * NC > 0 ? Epi::NIN * NC : 1];
        const PtrAt at{i};
        epi.load(at, in);
        epi.node(at, val, dir, sums, in);
    }
    if constexpr (Epi::NS > 0) block_partials<Epi::NS>(sums, red);
}

// Contribution to node (X, Y, Z) of element el around it (the element whose
// corner el the node is), for the scalar kinds; 0 outside the grid.
template <int DIM, int KIND, int MODE, typename T, typename TV>
__device__ __forceinline__ T node_elem_scalar(const Grid &g, const Phys &ph, const T *kap, const T *x, const TV *v,
                                              double eps, int X, int Y, int Z, int el) {
    constexpr int NV = Cell<DIM>::NV;
    constexpr bool FD = MODE != M_RESID;
    constexpr bool INV = KIND == JFNK_INVCOEF;
    const int ex = X - (el & 1), ey = Y - ((el >> 1) & 1), ez = DIM == 3 ? Z - ((el >> 2) & 1) : 0;
    if (ex < 0 || ex >= g.nx || ey < 0 || ey >= g.ny) return T(0);
    if (DIM == 3 && (ez < 0 || ez >= g.nz)) return T(0);
    T xe[1][NV], ve[1][NV], kp[NV], r[1][NV];
#pragma unroll
    for (int a = 0; a < NV; ++a) {
        const int ax = ex + (a & 1), ay = ey + ((a >> 1) & 1), az = ez + ((a >> 2) & 1);
        const long long j = node_index(g, ax, ay, az);
        xe[0][a] = x[j];
        ve[0][a] = (FD && !is_dirichlet(g, ax, ay, az)) ? (T)v[j] : T(0);
        kp[a] = INV ? kap[j] : T(0);
    }
    elem_eval<DIM, KIND, MODE, T, 1, NV>(xe, ve, kp, (T)eps, ph, (T)g.h, r);
    T out = T(0);
#pragma unroll
    for (int a = 0; a < NV; ++a)
        if (a == el) out = r[0][a];
    return out;
}

// Node-centric evaluation for the scalar kinds on small levels with 2^d
// lanes per node: lane el of a node's group evaluates element el around
// it, and the group sums the contributions by a fixed butterfly, so a
// node's 2^d element evaluations run in parallel (on small levels one
// thread's chain of them bounds the launch).  Every lane runs the same
// number of rounds, so the exchanges are wave-uniform; lane 0 of a group
// applies the epilogue.
template <int DIM, int KIND, int MODE, typename T, typename TV, class Epi>
__global__ __launch_bounds__(BLOCK) void k_node_split(Grid g, Phys ph, const T *kap, const T *x, const TV *v,
                                                      const T *Ax, FdStep fd, Epi epi, Red red) {
    constexpr int NV = Cell<DIM>::NV;
    static_assert(BLOCK % NV == 0, "a node's lanes share one block");
    const double eps = fd_eps_prepare(fd, epi);
    double sums[Epi::NS > 0 ? Epi::NS : 1];
#pragma unroll
    for (int k = 0; k < (Epi::NS > 0 ? Epi::NS : 1); ++k) sums[k] = 0.0;
    const long long total = g.nn * NV;
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long rounds = (total + stride - 1) / stride;
    const int el = threadIdx.x & (NV - 1);
    for (long long k = 0; k < rounds; ++k) {
        const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x + k * stride;
        const bool live = t < total;
        const long long i = live ? t / NV : 0;
        int X = 0, Y = 0, Z = 0;
        bool dir = true;
        if (live) {
            node_coords(g, i, X, Y, Z);
            dir = is_dirichlet(g, X, Y, Z);
        }
        const bool eval = live && !dir && !(MODE != M_RESID && eps == 0.0);
        T c = T(0);
        if (eval) c = node_elem_scalar<DIM, KIND, MODE, T, TV>(g, ph, kap, x, v, eps, X, Y, Z, el);
#pragma unroll
        for (int o = 1; o < NV; o <<= 1) c += __shfl_xor(c, o);
        if (live && el == 0) {
            T val[1] = {c};
            if constexpr (MODE == M_FD_PLAIN) {
                if (eval) val[0] = (val[0] - Ax[i]) * (T)(1.0 / eps);
            }
            T in[Epi::NIN > 0 ? Epi::NIN : 1];
            const PtrAt at{i};
            epi.load(at, in);
            epi.node(at, val, dir, sums, in);
        }
    }
    if constexpr (Epi::NS > 0) block_partials<Epi::NS>(sums, red);
}

// Node values of the Neo-Hookean kind with one wavefront per node: lane l
// evaluates Gauss point l & 7 of element l >> 3 around the node (the
// element whose corner l >> 3 the node is), and the wave sums the 64 parts
// by DPP in a fixed order.  A node's 8 elements x 8 points run in parallel
// instead of in one lane's sequence, which bounded every level of the
// node-centric Neo-Hookean hierarchy by one thread's latency.  Every lane of
// a wave walks the same nodes, so the sums are wave-uniform; lane 0 applies
// the epilogue.
template <int MODE, typename T, typename TV, class Epi>
__global__ __launch_bounds__(BLOCK) void k_node_nh(Grid g, Phys ph, const T *x, const TV *v, const T *Ax,
                                                   FdStep fd, Epi epi, Red red) {
    constexpr int NC = 3;
    const double eps = fd_eps_prepare(fd, epi);
    double sums[Epi::NS > 0 ? Epi::NS : 1];
#pragma unroll
    for (int k = 0; k < (Epi::NS > 0 ? Epi::NS : 1); ++k) sums[k] = 0.0;
    const long long nn = g.nn;
    const int lane = threadIdx.x & 63;
    const int el = lane >> 3, gq = lane & 7;
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
    const T h = (T)g.h, e = (T)eps;
    for (long long i = wave; i < nn; i += nwaves) {
        int X, Y, Z;
        node_coords(g, i, X, Y, Z);
        const bool dir = is_dirichlet(g, X, Y, Z);
        const bool eval = !dir && !(MODE != M_RESID && eps == 0.0);
        const int ex = X - (el & 1), ey = Y - ((el >> 1) & 1), ez = Z - ((el >> 2) & 1);
        const bool inside = eval && ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny && ez >= 0 && ez < g.nz;
        T c3[NC] = {T(0), T(0), T(0)};
        if (inside) {
            T xe[NC][8], ve[NC][8], r8[NC][8];
#pragma unroll
            for (int a = 0; a < 8; ++a) {
                const int ax = ex + (a & 1), ay = ey + ((a >> 1) & 1), az = ez + ((a >> 2) & 1);
                const long long j = node_index(g, ax, ay, az);
                const bool dj = (MODE != M_RESID) && is_dirichlet(g, ax, ay, az);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    xe[c][a] = x[c * nn + j];
                    ve[c][a] = (MODE == M_RESID || dj) ? T(0) : (T)v[c * nn + j];
                    r8[c][a] = T(0);
                }
            }
            if constexpr (MODE == M_FD_DIFF) {
                nh_point_fd<T>(xe, ve, e, ph, h, gq, r8);
            } else if constexpr (MODE == M_FD_PLAIN) {
                T w[NC][8];
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int a = 0; a < 8; ++a) w[c][a] = xe[c][a] + e * ve[c][a];
                nh_point<T>(w, ph, h, gq, r8);
            } else {
                nh_point<T>(xe, ph, h, gq, r8);
            }
#pragma unroll
            for (int a = 0; a < 8; ++a)
                if (a == el) {
#pragma unroll
                    for (int c = 0; c < NC; ++c) c3[c] = r8[c][a];
                }
        }
        T val[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) val[c] = (T)wave_sum((double)c3[c]);
        if (lane == 0) {
            if constexpr (MODE == M_FD_PLAIN) {
                if (eval) {
                    const T ie = (T)(1.0 / eps);
#pragma unroll
                    for (int c = 0; c < NC; ++c) val[c] = (val[c] - Ax[c * nn + i]) * ie;
                }
            }
            T in[Epi::NIN * NC > 0 ? Epi::NIN * NC : 1];
            const PtrAt at{i};
            epi.load(at, in);
            epi.node(at, val, dir, sums, in);
        }
    }
    if constexpr (Epi::NS > 0) block_partials<Epi::NS>(sums, red);
}

}  // namespace jfnk
