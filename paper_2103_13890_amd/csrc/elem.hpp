// Element routines of the first-order finite-element residuals (Sec. 3) on
// cubic cells of edge h.  Corners are numbered a = a_x + 2 a_y + 4 a_z; the
// Q1 basis is the tensor product of 1 - t and t.  Every routine takes the
// corner values of one element and returns that element's contribution to
// each corner; the node kernels sum the contributions of adjacent elements.
//
//   BRATU    r_a = (K u)_a - lam sum_q w_q exp(u_h(x_q)) phi_a(x_q)
//   PLAP     r_a = (delta^2 + s)^((p-2)/2) (K u)_a,   s = u^T K u / |e|
//   PLAP_GAUSS  r_a = sum_q w_q k_q grad phi_a(x_q) . g_q,  g_q = grad u_h(x_q),
//               k_q = (delta^2 + |g_q|^2)^((p-2)/2)
//   INVCOEF  r_a = kbar (1 + ubar^2) (K u)_a,          kbar = mean e^{m}, ubar = mean u
//   NEOHOOKE r_{i,a} = sum_q w_q P_ij(F_q) d_j phi_a(x_q),
//            P = mu (F - F^-T) + lam ln J F^-T,  F = I + grad u
//
// K is the exact Q1 stiffness: its entry between corners a and b depends
// only on the number c of coordinates in which they differ,
// 2D: (2/3, -1/6, -1/3)[c];  3D: h (1/3, 0, -1/12, -1/12)[c].
// Gauss points are the tensor points 1/2 -+ 1/(2 sqrt 3), weights |e|/2^d.
#pragma once
#include "common.hpp"

namespace jfnk {

constexpr double GL0 = 0.21132486540518711775;   // 1/2 - 1/(2 sqrt 3)
constexpr double GL1 = 0.78867513459481288225;   // 1/2 + 1/(2 sqrt 3)

template <int DIM> struct Cell { static constexpr int NV = 1 << DIM; };

// phi_b at Gauss point q: GL1^(DIM-c) GL0^c with c = popcount(b ^ q).
template <int DIM, typename T>
__device__ __forceinline__ T phi_gauss(int c) {
    if (DIM == 2) {
        return c == 0 ? T(GL1 * GL1) : (c == 1 ? T(GL1 * GL0) : T(GL0 * GL0));
    } else {
        return c == 0 ? T(GL1 * GL1 * GL1)
                      : (c == 1 ? T(GL1 * GL1 * GL0) : (c == 2 ? T(GL1 * GL0 * GL0) : T(GL0 * GL0 * GL0)));
    }
}

// (K u)_a for all corners (without the h^(d-2) factor).
template <int DIM, typename T>
__device__ __forceinline__ void stiff_apply(const T *u, T *Ku) {
    if (DIM == 2) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
            Ku[a] = T(2.0 / 3.0) * u[a] - T(1.0 / 6.0) * (u[a ^ 1] + u[a ^ 2]) - T(1.0 / 3.0) * u[a ^ 3];
    } else {
        // (K u)_a = u_a / 3 - (sum of the four corners differing in >= 2 coordinates) / 12
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            T far = (u[a ^ 3] + u[a ^ 5]) + (u[a ^ 6] + u[a ^ 7]);
            Ku[a] = T(1.0 / 3.0) * u[a] - T(1.0 / 12.0) * far;
        }
    }
}

// KS (K u) with KS = 12 in 3D, where 12 K has integer entries (4 on the
// diagonal, -1 between corners that differ in two or three coordinates, 0
// between edge neighbours), so each entry is one multiply-add; KS = 1 in 2D.
template <int DIM> struct KScale { static constexpr double value = DIM == 3 ? 12.0 : 1.0; };
template <int DIM, typename T>
__device__ __forceinline__ void stiff_apply_s(const T *u, T *Ku) {
    if (DIM == 2) {
        stiff_apply<2, T>(u, Ku);
    } else {
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const T far = (u[a ^ 3] + u[a ^ 5]) + (u[a ^ 6] + u[a ^ 7]);
            Ku[a] = T(4) * u[a] - far;
        }
    }
}

// Square root and quotient: IEEE-rounded in FP64; in FP32 the hardware
// approximations (about 1 ulp), which the FP32 multigrid levels tolerate.
template <typename T> __device__ __forceinline__ T hw_sqrt(T x) { return sqrt(x); }
template <> __device__ __forceinline__ float hw_sqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <typename T> __device__ __forceinline__ T hw_div(T a, T b) { return a / b; }
template <> __device__ __forceinline__ float hw_div<float>(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// (delta^2 + s)^e for the exponents the p-Laplacian needs
// PF = 3: the exponent p = 3 is known at compile time; PF = 0: read p.
template <typename T, int PF = 0>
__device__ __forceinline__ T plap_pow(T base, double p, int which) {
    // which 0: (p-2)/2, 1: p/2, 2: (p-4)/2
    if (PF == 3 || p == 3.0) {
        T r = hw_sqrt(base);
        return which == 0 ? r : (which == 1 ? base * r : hw_div(T(1), r));
    }
    if (p == 2.0) return which == 0 ? T(1) : (which == 1 ? base : hw_div(T(1), base));
    if (p == 1.0) {     // the minimal-surface energy: exponents -1/2, 1/2, -3/2
        T r = hw_sqrt(base);
        return which == 1 ? r : hw_div(T(1), which == 0 ? r : base * r);
    }
    double e = which == 0 ? 0.5 * (p - 2.0) : (which == 1 ? 0.5 * p : 0.5 * (p - 4.0));
    return (T)pow(base, (T)e);
}

// ---------------------------------------------------------------------------
// Gradients at the Gauss points (PLAP_GAUSS).  In reference units G = h g.
// Inside a Q1 cell the derivative along axis i does not vary along i, so G_i
// takes 2^(d-1) values: the tensor interpolation of the 2^(d-1) edge
// differences along i, with weights W(b, q) = GL1 if b == q else GL0 on each
// other axis.  W is symmetric, so the same interpolation maps per-point
// fluxes back to the corners.  Index j of the other axes: lower axis first.
// ---------------------------------------------------------------------------
template <int DIM> __device__ __forceinline__ constexpr int gq_corner(int i, int b, int j) {
    if (DIM == 2) return (b << i) | (j << (1 - i));
    return (b << i) | ((j & 1) << (i == 0 ? 1 : 0)) | (((j >> 1) & 1) << (i == 2 ? 1 : 2));
}
template <int DIM> __device__ __forceinline__ constexpr int gq_other(int i, int q) {
    if (DIM == 2) return (q >> (1 - i)) & 1;
    return ((q >> (i == 0 ? 1 : 0)) & 1) | (((q >> (i == 2 ? 1 : 2)) & 1) << 1);
}
template <int DIM, typename T> __device__ __forceinline__ void gq_interp(const T *in, T *out) {
    const T A = T(GL1), B = T(GL0);
    if (DIM == 2) {
        out[0] = A * in[0] + B * in[1];
        out[1] = B * in[0] + A * in[1];
    } else {
        const T t0 = A * in[0] + B * in[1], t1 = B * in[0] + A * in[1];
        const T t2 = A * in[2] + B * in[3], t3 = B * in[2] + A * in[3];
        out[0] = A * t0 + B * t2;
        out[1] = A * t1 + B * t3;
        out[2] = B * t0 + A * t2;
        out[3] = B * t1 + A * t3;
    }
}
template <int DIM, typename T> __device__ __forceinline__ void gq_grad(const T *u, T (*G)[1 << (DIM - 1)]) {
    constexpr int NH = 1 << (DIM - 1);
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        T e[NH];
#pragma unroll
        for (int j = 0; j < NH; ++j) e[j] = u[gq_corner<DIM>(i, 1, j)] - u[gq_corner<DIM>(i, 0, j)];
        gq_interp<DIM, T>(e, G[i]);
    }
}
// |G_q|^2 and G_q . H_q at Gauss point q
template <int DIM, typename T>
__device__ __forceinline__ T gq_dot(const T (*G)[1 << (DIM - 1)], const T (*H)[1 << (DIM - 1)], int q) {
    T d = T(0);
#pragma unroll
    for (int i = 0; i < DIM; ++i) d += G[i][gq_other<DIM>(i, q)] * H[i][gq_other<DIM>(i, q)];
    return d;
}
// r_a = c sum_i s_i(a) (interp F_i)[j(a)], s_i(a) = +1 if corner a has bit i, else -1;
// F_i[j] is the flux along i summed over the two Gauss points that share j
template <int DIM, typename T>
__device__ __forceinline__ void gq_scatter(T (*F)[1 << (DIM - 1)], T c, T *r) {
    constexpr int NH = 1 << (DIM - 1);
    T E[DIM][NH];
#pragma unroll
    for (int i = 0; i < DIM; ++i) gq_interp<DIM, T>(F[i], E[i]);
#pragma unroll
    for (int a = 0; a < (1 << DIM); ++a) {
        T acc = T(0);
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            const T e = E[i][gq_other<DIM>(i, a)];
            acc += ((a >> i) & 1) ? e : -e;
        }
        r[a] = c * acc;
    }
}
// Sum over the pair of Gauss points that differ only along axis i.
template <int DIM, typename T> __device__ __forceinline__ T gq_pair(const T *k, int i, int j) {
    return k[gq_corner<DIM>(i, 0, j)] + k[gq_corner<DIM>(i, 1, j)];
}

// PLAP_GAUSS element vector; c = m |e| / (2^d h^2) (= m h^(d-2) / 2^d)
template <int DIM, typename T, int PF>
__device__ __forceinline__ void elem_plap_gauss(const T *w, const Phys &ph, T h, T *r, T m) {
    constexpr int NV = Cell<DIM>::NV, NH = NV / 2;
    T G[DIM][NH];
    gq_grad<DIM, T>(w, G);
    const T ih2 = T(1) / (h * h), d2 = T(ph.a1) * T(ph.a1);
    T k[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) k[q] = plap_pow<T, PF>(d2 + gq_dot<DIM, T>(G, G, q) * ih2, ph.a0, 0);
    T F[DIM][NH];
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < NH; ++j) F[i][j] = G[i][j] * gq_pair<DIM, T>(k, i, j);
    const T hs = (DIM == 3) ? h : T(1);
    const bool on = m != T(0);
    gq_scatter<DIM, T>(F, on ? m * hs * T(1.0 / NV) : T(0), r);
}

// PLAP_GAUSS FD quotient in difference form: per Gauss point
// k_w - k_x from s_w - s_x = eps (2 g_x . g_v + eps |g_v|^2), as for PLAP
template <int DIM, typename T, int PF>
__device__ __forceinline__ void elem_plap_gauss_fd(const T *x, const T *v, T eps, const Phys &ph, T h, T *q_out,
                                                   T m) {
    constexpr int NV = Cell<DIM>::NV, NH = NV / 2;
    T Gx[DIM][NH], Gv[DIM][NH];
    gq_grad<DIM, T>(x, Gx);
    gq_grad<DIM, T>(v, Gv);
    const T ih2 = T(1) / (h * h), d2 = T(ph.a1) * T(ph.a1);
    T kw[NV], dk[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const T bx = d2 + gq_dot<DIM, T>(Gx, Gx, q) * ih2;
        const T dsq = (T(2) * gq_dot<DIM, T>(Gx, Gv, q) + eps * gq_dot<DIM, T>(Gv, Gv, q)) * ih2;
        const T bw = bx + eps * dsq;
        if (PF == 3 || ph.a0 == 3.0) {
            const T kx = hw_sqrt(bx);
            kw[q] = hw_sqrt(bw);
            dk[q] = hw_div(dsq, kw[q] + kx);
        } else if (ph.a0 == 2.0) {
            kw[q] = T(1);
            dk[q] = T(0);
        } else if (ph.a0 == 1.0) {   // k = b^(-1/2): (k_w - k_x)/eps = -dsq / (s_x s_w (s_x + s_w))
            const T sx = hw_sqrt(bx), sw = hw_sqrt(bw);
            kw[q] = hw_div(T(1), sw);
            dk[q] = -hw_div(dsq, sx * sw * (sx + sw));
        } else {
            const T al = T(0.5 * (ph.a0 - 2.0));
            const T kx = (T)pow(bx, al);
            const T em = expm1(al * log1p(eps * dsq / bx));
            kw[q] = kx * (T(1) + em);
            dk[q] = kx * em / eps;
        }
    }
    T F[DIM][NH];
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < NH; ++j)
            F[i][j] = Gv[i][j] * gq_pair<DIM, T>(kw, i, j) + Gx[i][j] * gq_pair<DIM, T>(dk, i, j);
    const T hs = (DIM == 3) ? h : T(1);
    const bool on = m != T(0);
    gq_scatter<DIM, T>(F, on ? m * hs * T(1.0 / NV) : T(0), q_out);
}

// PLAP_GAUSS exact J_e lam (symmetric): per Gauss point
// k_q g_lam + (p - 2) (delta^2 + |g|^2)^((p-4)/2) (g . g_lam) g
template <int DIM, typename T>
__device__ __forceinline__ void elem_plap_gauss_vjp(const T *w, const T *lam, const Phys &ph, T h, T *r) {
    constexpr int NV = Cell<DIM>::NV, NH = NV / 2;
    T G[DIM][NH], L[DIM][NH];
    gq_grad<DIM, T>(w, G);
    gq_grad<DIM, T>(lam, L);
    const T ih2 = T(1) / (h * h), d2 = T(ph.a1) * T(ph.a1);
    T k[NV], cm[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const T b = d2 + gq_dot<DIM, T>(G, G, q) * ih2;
        k[q] = plap_pow<T>(b, ph.a0, 0);
        cm[q] = T(ph.a0 - 2.0) * plap_pow<T>(b, ph.a0, 2) * gq_dot<DIM, T>(G, L, q) * ih2;
    }
    T F[DIM][NH];
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < NH; ++j)
            F[i][j] = L[i][j] * gq_pair<DIM, T>(k, i, j) + G[i][j] * gq_pair<DIM, T>(cm, i, j);
    const T hs = (DIM == 3) ? h : T(1);
    gq_scatter<DIM, T>(F, hs * T(1.0 / NV), r);
}

// ---------------------------------------------------------------------------
// scalar kinds: r[a] for one element.  w: state corners, kap: e^{m} corners
// ---------------------------------------------------------------------------
// m multiplies the whole element vector (0 switches an element off without
// a branch).  A switched-off element may have a degenerate state (no
// gradient at delta = 0), so its nonlinear coefficient is selected away
// rather than multiplied by 0.
template <int DIM, int KIND, typename T, int PF = 0>
__device__ __forceinline__ void elem_scalar(const T *w, const T *kap, const Phys &ph, T h, T *r, T m = T(1)) {
    if constexpr (KIND == JFNK_PLAP_GAUSS) {
        elem_plap_gauss<DIM, T, PF>(w, ph, h, r, m);
        return;
    }
    constexpr int NV = Cell<DIM>::NV;
    constexpr double KS = KScale<DIM>::value;
    T Ku[NV];
    stiff_apply_s<DIM, T>(w, Ku);                 // KS K u
    const T hs = (DIM == 3) ? h : T(1);          // h^(d-2)
    const T hk = hs * T(1.0 / KS) * m;
    if (KIND == JFNK_BRATU) {
        T vol = (DIM == 3) ? h * h * h : h * h;
        T wq = vol / T(NV);
        T src[NV];
#pragma unroll
        for (int a = 0; a < NV; ++a) src[a] = T(0);
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            T uq = T(0);
#pragma unroll
            for (int b = 0; b < NV; ++b) uq += phi_gauss<DIM, T>(__builtin_popcount(b ^ q)) * w[b];
            T e = exp(uq);
#pragma unroll
            for (int a = 0; a < NV; ++a) src[a] += e * phi_gauss<DIM, T>(__builtin_popcount(a ^ q));
        }
        T lw = T(ph.a0) * wq * m;
#pragma unroll
        for (int a = 0; a < NV; ++a) r[a] = hk * Ku[a] - lw * src[a];
    } else if (KIND == JFNK_PLAP) {
        T quad = T(0);
#pragma unroll
        for (int a = 0; a < NV; ++a) quad += w[a] * Ku[a];
        // s = u^T K_e u / |e| = quad * h^(d-2) / h^d = quad / h^2  (quad carries KS)
        T s = quad * (T(1) / (T(KS) * h * h));
        T d2 = T(ph.a1) * T(ph.a1);
        T k = plap_pow<T, PF>(d2 + s, ph.a0, 0) * hk;
        if (!(m != T(0))) k = T(0);
#pragma unroll
        for (int a = 0; a < NV; ++a) r[a] = k * Ku[a];
    } else {  // INVCOEF
        T ks = T(0), us = T(0);
#pragma unroll
        for (int a = 0; a < NV; ++a) { ks += kap[a]; us += w[a]; }
        T kb = ks / T(NV), ub = us / T(NV);
        T k = kb * (T(1) + ub * ub) * hk;
        if (!(m != T(0))) k = T(0);
#pragma unroll
        for (int a = 0; a < NV; ++a) r[a] = k * Ku[a];
    }
}

// Element energy (variational scalar kinds).
template <int DIM, int KIND, typename T>
__device__ __forceinline__ T elem_scalar_energy(const T *w, const Phys &ph, T h) {
    constexpr int NV = Cell<DIM>::NV;
    if constexpr (KIND == JFNK_PLAP_GAUSS) {   // sum_q |e|/2^d (delta^2 + |g_q|^2)^(p/2) / p
        T G[DIM][NV / 2];
        gq_grad<DIM, T>(w, G);
        const T ih2 = T(1) / (h * h), d2 = T(ph.a1) * T(ph.a1);
        T acc = T(0);
#pragma unroll
        for (int q = 0; q < NV; ++q) acc += plap_pow<T>(d2 + gq_dot<DIM, T>(G, G, q) * ih2, ph.a0, 1);
        const T vol = (DIM == 3) ? h * h * h : h * h;
        return vol / (T(NV) * T(ph.a0)) * acc;
    }
    T Ku[NV];
    stiff_apply<DIM, T>(w, Ku);
    const T hs = (DIM == 3) ? h : T(1);
    T quad = T(0);
#pragma unroll
    for (int a = 0; a < NV; ++a) quad += w[a] * Ku[a];
    T vol = (DIM == 3) ? h * h * h : h * h;
    if (KIND == JFNK_BRATU) {
        T acc = T(0);
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            T uq = T(0);
#pragma unroll
            for (int b = 0; b < NV; ++b) uq += phi_gauss<DIM, T>(__builtin_popcount(b ^ q)) * w[b];
            acc += exp(uq);
        }
        return T(0.5) * hs * quad - T(ph.a0) * (vol / T(NV)) * acc;
    }
    // PLAP: |e|/p (delta^2 + s)^(p/2)
    T s = quad / (h * h);
    T d2 = T(ph.a1) * T(ph.a1);
    return vol / T(ph.a0) * plap_pow<T>(d2 + s, ph.a0, 1);
}

// Finite-difference quotient (r_e(x + eps v) - r_e(x)) / eps of the
// element vector, evaluated without subtracting two nearly equal element
// vectors: with w = x + eps v,
//   K w = K x + eps K v,   s_w - s_x = eps (2 x^T K v + eps v^T K v) / h^2,
//   k_w - k_x from that difference (quotients for p = 3 and p = 1,
//   expm1/log1p else),
// so  q = k_w K v + ((k_w - k_x) / eps) K x  (scaled by h^(d-2)).  Algebraically
// the same quotient as Sec. 1 with the same eps; only the rounding differs
// (no cancellation between the two residual evaluations, which in FP32
// destroys the action on smooth directions).
template <int DIM, int KIND, typename T, int PF = 0>
__device__ __forceinline__ void elem_scalar_fd(const T *x, const T *v, const T *kap, T eps, const Phys &ph,
                                               T h, T *q, T m = T(1)) {
    if constexpr (KIND == JFNK_PLAP_GAUSS) {
        elem_plap_gauss_fd<DIM, T, PF>(x, v, eps, ph, h, q, m);
        return;
    }
    constexpr int NV = Cell<DIM>::NV;
    constexpr double KS = KScale<DIM>::value;
    const T hs = (DIM == 3) ? h : T(1);
    const T hk = hs * T(1.0 / KS) * m;            // undoes KS; m switches the element off
    T Kv[NV];
    stiff_apply_s<DIM, T>(v, Kv);
    if (KIND == JFNK_BRATU) {
        // sum_q w_q (e^{w_q} - e^{x_q}) phi_a / eps = sum_q w_q e^{x_q} expm1(eps v_q) / eps phi_a
        T vol = (DIM == 3) ? h * h * h : h * h;
        T wq = vol / T(NV);
        T src[NV];
#pragma unroll
        for (int a = 0; a < NV; ++a) src[a] = T(0);
        const T ie = T(1) / eps;
#pragma unroll
        for (int qq = 0; qq < NV; ++qq) {
            T xq = T(0), vq = T(0);
#pragma unroll
            for (int b = 0; b < NV; ++b) {
                const T f = phi_gauss<DIM, T>(__builtin_popcount(b ^ qq));
                xq += f * x[b];
                vq += f * v[b];
            }
            const T e = exp(xq) * (expm1(eps * vq) * ie);
#pragma unroll
            for (int a = 0; a < NV; ++a) src[a] += e * phi_gauss<DIM, T>(__builtin_popcount(a ^ qq));
        }
        const T lw = T(ph.a0) * wq * m;
#pragma unroll
        for (int a = 0; a < NV; ++a) q[a] = hk * Kv[a] - lw * src[a];
        return;
    }
    T Kx[NV];
    stiff_apply_s<DIM, T>(x, Kx);
    T kw, dk;
    if (KIND == JFNK_PLAP) {
        T qxx = T(0), qxv = T(0), qvv = T(0);
#pragma unroll
        for (int a = 0; a < NV; ++a) {
            qxx += x[a] * Kx[a];
            qxv += x[a] * Kv[a];
            qvv += v[a] * Kv[a];
        }
        const T ih2 = T(1) / (T(KS) * h * h);
        const T bx = T(ph.a1) * T(ph.a1) + qxx * ih2;
        const T dsq = (T(2) * qxv + eps * qvv) * ih2;        // (s_w - s_x) / eps
        const T bw = bx + eps * dsq;
        if (PF == 3 || ph.a0 == 3.0) {
            const T kx = hw_sqrt(bx);
            kw = hw_sqrt(bw);
            dk = hw_div(dsq, kw + kx);
        } else if (ph.a0 == 2.0) {
            kw = T(1);
            dk = T(0);
        } else if (ph.a0 == 1.0) {   // the minimal surface, k = b^(-1/2):
            // (k_w - k_x) / eps = -dsq / (s_x s_w (s_x + s_w)), s = sqrt(b)
            const T sx = hw_sqrt(bx), sw = hw_sqrt(bw);
            kw = hw_div(T(1), sw);
            dk = -hw_div(dsq, sx * sw * (sx + sw));
        } else {
            const T al = T(0.5 * (ph.a0 - 2.0));
            const T kx = (T)pow(bx, al);
            const T t = eps * dsq / bx;
            const T em = expm1(al * log1p(t));
            kw = kx * (T(1) + em);
            dk = kx * em / eps;
        }
    } else {   // INVCOEF: k = kbar (1 + ubar^2)
        T ks = T(0), xs = T(0), vs = T(0);
#pragma unroll
        for (int a = 0; a < NV; ++a) { ks += kap[a]; xs += x[a]; vs += v[a]; }
        const T kb = ks / T(NV), xb = xs / T(NV), vb = vs / T(NV);
        const T wb = xb + eps * vb;
        kw = kb * (T(1) + wb * wb);
        dk = kb * vb * (T(2) * xb + eps * vb);
    }
    const bool on = m != T(0);
    const T cv = on ? hk * kw : T(0), cx = on ? hk * dk : T(0);
#pragma unroll
    for (int a = 0; a < NV; ++a) q[a] = cv * Kv[a] + cx * Kx[a];
}

// Exact J_e^T lam (= J_e lam for the symmetric kinds), FP64 use.
template <int DIM, int KIND, typename T>
__device__ __forceinline__ void elem_scalar_vjp(const T *w, const T *kap, const T *lam, const Phys &ph,
                                                T h, T *r) {
    if constexpr (KIND == JFNK_PLAP_GAUSS) {
        elem_plap_gauss_vjp<DIM, T>(w, lam, ph, h, r);
        return;
    }
    constexpr int NV = Cell<DIM>::NV;
    const T hs = (DIM == 3) ? h : T(1);
    T Kl[NV];
    stiff_apply<DIM, T>(lam, Kl);
    if (KIND == JFNK_BRATU) {
        T vol = (DIM == 3) ? h * h * h : h * h;
        T wq = vol / T(NV);
        T src[NV];
#pragma unroll
        for (int a = 0; a < NV; ++a) src[a] = T(0);
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            T uq = T(0), lq = T(0);
#pragma unroll
            for (int b = 0; b < NV; ++b) {
                T f = phi_gauss<DIM, T>(__builtin_popcount(b ^ q));
                uq += f * w[b];
                lq += f * lam[b];
            }
            T e = exp(uq) * lq;
#pragma unroll
            for (int a = 0; a < NV; ++a) src[a] += e * phi_gauss<DIM, T>(__builtin_popcount(a ^ q));
        }
        T lw = T(ph.a0) * wq;
#pragma unroll
        for (int a = 0; a < NV; ++a) r[a] = hs * Kl[a] - lw * src[a];
        return;
    }
    T Ku[NV];
    stiff_apply<DIM, T>(w, Ku);
    if (KIND == JFNK_PLAP) {
        T quad = T(0), kul = T(0);
#pragma unroll
        for (int a = 0; a < NV; ++a) { quad += w[a] * Ku[a]; kul += lam[a] * Ku[a]; }
        T s = quad / (h * h);
        T d2 = T(ph.a1) * T(ph.a1);
        T k = plap_pow<T>(d2 + s, ph.a0, 0) * hs;
        // (p-2)(delta^2+s)^((p-4)/2) / |e| * (K_e u)(K_e u)^T lam, K_e = hs K
        T vol = (DIM == 3) ? h * h * h : h * h;
        T dk = T(ph.a0 - 2.0) * plap_pow<T>(d2 + s, ph.a0, 2) / vol * hs * hs * kul;
#pragma unroll
        for (int a = 0; a < NV; ++a) r[a] = k * Kl[a] + dk * Ku[a];
        return;
    }
    // INVCOEF transpose: k K lam + (kbar * 2 ubar / NV) (lam^T K_e u) 1
    T ks = T(0), us = T(0), kul = T(0);
#pragma unroll
    for (int a = 0; a < NV; ++a) { ks += kap[a]; us += w[a]; kul += lam[a] * Ku[a]; }
    T kb = ks / T(NV), ub = us / T(NV);
    T k = kb * (T(1) + ub * ub) * hs;
    T c = kb * T(2) * ub / T(NV) * hs * kul;
#pragma unroll
    for (int a = 0; a < NV; ++a) r[a] = k * Kl[a] + c;
}

// INVCOEF coefficient VJP: the element's common factor
// (1 + ubar^2) (lam^T K_e u) / NV; node a multiplies it by e^{m_a}.
template <int DIM, typename T>
__device__ __forceinline__ T elem_coef_factor(const T *w, const T *lam, T h) {
    constexpr int NV = Cell<DIM>::NV;
    const T hs = (DIM == 3) ? h : T(1);
    T Ku[NV];
    stiff_apply<DIM, T>(w, Ku);
    T us = T(0), kul = T(0);
#pragma unroll
    for (int a = 0; a < NV; ++a) { us += w[a]; kul += lam[a] * Ku[a]; }
    T ub = us / T(NV);
    return (T(1) + ub * ub) * hs * kul / T(NV);
}

// ---------------------------------------------------------------------------
// Neo-Hookean (3D, 3 components, SoA corners w[3][8])
// ---------------------------------------------------------------------------
// reference gradient of phi_a at Gauss point q, component k (times h)
__device__ __forceinline__ double nh_dphi(int a, int q, int k) {
    double g = ((a >> k) & 1) ? 1.0 : -1.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        if (j == k) continue;
        g *= (((a >> j) & 1) == ((q >> j) & 1)) ? GL1 : GL0;
    }
    return g;
}

// F = I + grad w at Gauss point q (ident = false: grad w alone)
template <typename T>
__device__ __forceinline__ void nh_grad(const T (*w)[8], int q, T h, T F[3][3], bool ident = true) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) F[i][j] = (ident && i == j) ? T(1) : T(0);
    const T ih = T(1) / h;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        T d0 = T(nh_dphi(a, q, 0)) * ih, d1 = T(nh_dphi(a, q, 1)) * ih, d2 = T(nh_dphi(a, q, 2)) * ih;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            F[i][0] += w[i][a] * d0;
            F[i][1] += w[i][a] * d1;
            F[i][2] += w[i][a] * d2;
        }
    }
}

// cofactor matrix C (F^-T = C / J) and J = det F
template <typename T>
__device__ __forceinline__ T nh_cof(const T F[3][3], T C[3][3]) {
    C[0][0] = F[1][1] * F[2][2] - F[1][2] * F[2][1];
    C[0][1] = F[1][2] * F[2][0] - F[1][0] * F[2][2];
    C[0][2] = F[1][0] * F[2][1] - F[1][1] * F[2][0];
    C[1][0] = F[0][2] * F[2][1] - F[0][1] * F[2][2];
    C[1][1] = F[0][0] * F[2][2] - F[0][2] * F[2][0];
    C[1][2] = F[0][1] * F[2][0] - F[0][0] * F[2][1];
    C[2][0] = F[0][1] * F[1][2] - F[0][2] * F[1][1];
    C[2][1] = F[0][2] * F[1][0] - F[0][0] * F[1][2];
    C[2][2] = F[0][0] * F[1][1] - F[0][1] * F[1][0];
    return F[0][0] * C[0][0] + F[0][1] * C[0][1] + F[0][2] * C[0][2];
}

// Gauss point q's part of the element vector, added to r
template <typename T>
__device__ __forceinline__ void nh_point(const T (*w)[8], const Phys &ph, T h, int q, T (*r)[8]) {
    const T mu = T(ph.a0), lam = T(ph.a1);
    const T wq = h * h * h / T(8);
    const T ih = T(1) / h;
    {
        T F[3][3], C[3][3];
        nh_grad<T>(w, q, h, F);
        T J = nh_cof<T>(F, C);
        T lnJ = J > T(0) ? log(J) : T(NAN);
        T iJ = T(1) / J;
        T P[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                T fit = C[i][j] * iJ;   // (F^-T)_ij
                P[i][j] = wq * (mu * (F[i][j] - fit) + lam * lnJ * fit);
            }
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            T d0 = T(nh_dphi(a, q, 0)) * ih, d1 = T(nh_dphi(a, q, 1)) * ih, d2 = T(nh_dphi(a, q, 2)) * ih;
#pragma unroll
            for (int i = 0; i < 3; ++i) r[i][a] += P[i][0] * d0 + P[i][1] * d1 + P[i][2] * d2;
        }
    }
}

template <typename T>
__device__ __forceinline__ void elem_neohooke(const T (*w)[8], const Phys &ph, T h, T (*r)[8]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int a = 0; a < 8; ++a) r[i][a] = T(0);
    for (int q = 0; q < 8; ++q) nh_point<T>(w, ph, h, q, r);
}

template <typename T>
__device__ __forceinline__ T elem_neohooke_energy(const T (*w)[8], const Phys &ph, T h) {
    const T mu = T(ph.a0), lam = T(ph.a1);
    const T wq = h * h * h / T(8);
    T acc = T(0);
    for (int q = 0; q < 8; ++q) {
        T F[3][3], C[3][3];
        nh_grad<T>(w, q, h, F);
        T J = nh_cof<T>(F, C);
        if (!(J > T(0))) return T(INFINITY);
        T lnJ = log(J);
        T IC = T(0);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) IC += F[i][j] * F[i][j];
        acc += T(0.5) * mu * (IC - T(3)) - mu * lnJ + T(0.5) * lam * lnJ * lnJ;
    }
    return wq * acc;
}

// Difference form of the Neo-Hookean element quotient (P(F_w) - P(F_x)) / eps
// with F_w = F_x + eps G, G = grad v:
//   F_w^-T - F_x^-T = -eps F_w^-T G^T F_x^-T
//   J_w - J_x = eps tr(adj(F_x) G) + eps^2 tr(F_x adj(G)) + eps^3 det G
//   (P_w - P_x)/eps = mu G + (mu - lam ln J_x) F_w^-T G^T F_x^-T
//                     + lam log1p((J_w - J_x)/J_x)/eps F_w^-T
// Gauss point q's part, added to r
template <typename T>
__device__ __forceinline__ void nh_point_fd(const T (*x)[8], const T (*v)[8], T eps, const Phys &ph, T h, int q,
                                            T (*r)[8]) {
    const T mu = T(ph.a0), lam = T(ph.a1);
    const T wq = h * h * h / T(8);
    const T ih = T(1) / h;
    {
        T F[3][3], C[3][3], G[3][3], Cg[3][3];
        nh_grad<T>(x, q, h, F);
        nh_grad<T>(v, q, h, G, false);
        const T Jx = nh_cof<T>(F, C);       // C = cof(F_x) = adj(F_x)^T
        const T dG = nh_cof<T>(G, Cg);      // Cg = cof(G)
        // tr(adj(F) G) = sum_ij C_ij G_ij ; tr(F adj(G)) = sum_ij F_ij Cg_ij
        T t1 = T(0), t2 = T(0);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) { t1 += C[i][j] * G[i][j]; t2 += F[i][j] * Cg[i][j]; }
        const T dJ = eps * (t1 + eps * (t2 + eps * dG));
        T Fw[3][3], Cw[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Fw[i][j] = F[i][j] + eps * G[i][j];
        const T Jw = nh_cof<T>(Fw, Cw);
        const T iJx = T(1) / Jx, iJw = T(1) / Jw;
        T Fxit[3][3], Fwit[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) { Fxit[i][j] = C[i][j] * iJx; Fwit[i][j] = Cw[i][j] * iJw; }
        // X = G^T F_x^-T : X_kj = sum_l G_lk Fxit_lj
        T X[3][3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) X[k][j] = G[0][k] * Fxit[0][j] + G[1][k] * Fxit[1][j] + G[2][k] * Fxit[2][j];
        const T lnJx = Jx > T(0) ? log(Jx) : T(NAN);
        const T c1 = mu - lam * lnJx;
        const T c2 = (Jw > T(0) && Jx > T(0)) ? lam * log1p(dJ * iJx) / eps : T(NAN);
        T P[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const T M = Fwit[i][0] * X[0][j] + Fwit[i][1] * X[1][j] + Fwit[i][2] * X[2][j];
                P[i][j] = wq * (mu * G[i][j] + c1 * M + c2 * Fwit[i][j]);
            }
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            T d0 = T(nh_dphi(a, q, 0)) * ih, d1 = T(nh_dphi(a, q, 1)) * ih, d2 = T(nh_dphi(a, q, 2)) * ih;
#pragma unroll
            for (int i = 0; i < 3; ++i) r[i][a] += P[i][0] * d0 + P[i][1] * d1 + P[i][2] * d2;
        }
    }
}

template <typename T>
__device__ __forceinline__ void elem_neohooke_fd(const T (*x)[8], const T (*v)[8], T eps, const Phys &ph, T h,
                                                 T (*r)[8]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int a = 0; a < 8; ++a) r[i][a] = T(0);
    for (int q = 0; q < 8; ++q) nh_point_fd<T>(x, v, eps, ph, h, q, r);
}

// dP = mu dF + (mu - lam ln J) F^-T dF^T F^-T + lam tr(F^-1 dF) F^-T ; r = sum_q w_q dP grad phi
template <typename T>
__device__ __forceinline__ void elem_neohooke_jvp(const T (*w)[8], const T (*v)[8], const Phys &ph, T h,
                                                  T (*r)[8]) {
    const T mu = T(ph.a0), lam = T(ph.a1);
    const T wq = h * h * h / T(8);
    const T ih = T(1) / h;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int a = 0; a < 8; ++a) r[i][a] = T(0);
    for (int q = 0; q < 8; ++q) {
        T F[3][3], C[3][3], dF[3][3];
        nh_grad<T>(w, q, h, F);
        nh_grad<T>(v, q, h, dF, false);
        T J = nh_cof<T>(F, C);
        T iJ = T(1) / J;
        T lnJ = log(J);
        T Fit[3][3];   // F^-T
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Fit[i][j] = C[i][j] * iJ;
        // tr(F^-1 dF) = sum_ij (F^-1)_ji dF_ij = sum_ij Fit_ij dF_ij
        T tr = T(0);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) tr += Fit[i][j] * dF[i][j];
        // M = F^-T dF^T F^-T : M_ij = sum_kl Fit_ik dF_lk Fit_lj
        T X[3][3];   // X = dF^T F^-T : X_kj = sum_l dF_lk Fit_lj
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) X[k][j] = dF[0][k] * Fit[0][j] + dF[1][k] * Fit[1][j] + dF[2][k] * Fit[2][j];
        T P[3][3];
        const T c1 = mu - lam * lnJ, c2 = lam * tr;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                T M = Fit[i][0] * X[0][j] + Fit[i][1] * X[1][j] + Fit[i][2] * X[2][j];
                P[i][j] = wq * (mu * dF[i][j] + c1 * M + c2 * Fit[i][j]);
            }
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            T d0 = T(nh_dphi(a, q, 0)) * ih, d1 = T(nh_dphi(a, q, 1)) * ih, d2 = T(nh_dphi(a, q, 2)) * ih;
#pragma unroll
            for (int i = 0; i < 3; ++i) r[i][a] += P[i][0] * d0 + P[i][1] * d1 + P[i][2] * d2;
        }
    }
}

}  // namespace jfnk
