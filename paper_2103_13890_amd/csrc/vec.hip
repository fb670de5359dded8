// Vector kernels: masked casts and scalings with fused norms, Chebyshev
// start/finish, FD-step numerators, SplitMix64 start vectors, Gram-Schmidt
// passes of flexible GMRES, and load-vector assembly.
#include <algorithm>
#include <array>
#include <utility>

#include "elem.hpp"
#include "ops.hpp"

namespace jfnk {

static inline int vblocks(long long n, int cap = 2048) {
    long long b = (n + BLOCK - 1) / BLOCK;
    if (b > cap) b = cap;
    return (int)(b < 1 ? 1 : b);
}

__device__ __forceinline__ bool dir_at(const Grid &g, long long i) {
    int x, y, z;
    node_coords(g, i, x, y, z);
    return is_dirichlet(g, x, y, z);
}

// two FP64 (or FP32) entries per lane access: one 16-byte (8-byte) load
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));

#define GRID_STRIDE(i, n) \
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long long)gridDim.x * blockDim.x)

// ---------------------------------------------------------------------------
template <typename T> __global__ void k_fill(T *x, long long n, T v) {
    GRID_STRIDE(i, n) x[i] = v;
}
template <typename T> void vec_fill(const Exec &ex, T *x, long long n, T val) {
    k_fill<T><<<vblocks(n), BLOCK, 0, ex.st>>>(x, n, val);
}
template void vec_fill<float>(const Exec &, float *, long long, float);
template void vec_fill<double>(const Exec &, double *, long long, double);

// y = a x on DoFs; a = scale (* 1/sqrt(*rs))
template <typename TI, typename TO>
__global__ void k_scale(Grid g, int nc, const TI *x, TO *y, double scale, const double *rs, Red red, double *out) {
    double a = scale;
    if (rs) a = (*rs > 0.0) ? scale / sqrt(*rs) : 0.0;
    double s[1] = {0.0};
    GRID_STRIDE(i, g.nn) {
        const bool d = dir_at(g, i);
        for (int c = 0; c < nc; ++c) {
            const long long k = c * g.nn + i;
            TO v = d ? TO(0) : (TO)(a * (double)x[k]);
            y[k] = v;
            s[0] += (double)v * (double)v;
        }
    }
    if (out) block_partials<1>(s, red);
}

template <typename TI, typename TO>
void vec_cast(const Exec &ex, const Grid &g, int nc, const TI *x, TO *y, double *nrm2) {
    const int nb = vblocks(g.nn);
    const Red r = red_for(ex, nrm2, nb);
    k_scale<TI, TO><<<nb, BLOCK, 0, ex.st>>>(g, nc, x, y, 1.0, nullptr, r, nrm2);
    if (nrm2) finish_to<1>(ex, nrm2, r, nb, FinStore<1>{nrm2});
}
template void vec_cast<double, double>(const Exec &, const Grid &, int, const double *, double *, double *);
template void vec_cast<double, float>(const Exec &, const Grid &, int, const double *, float *, double *);
template void vec_cast<float, double>(const Exec &, const Grid &, int, const float *, double *, double *);
template void vec_cast<float, float>(const Exec &, const Grid &, int, const float *, float *, double *);

template <typename TI, typename TO>
void vec_scale_cast(const Exec &ex, const Grid &g, int nc, const TI *x, TO *y, double scale, const double *rs,
                    double *nrm2) {
    const int nb = vblocks(g.nn);
    materialize(ex, const_cast<double *>(rs));
    const Red r = red_for(ex, nrm2, nb);
    k_scale<TI, TO><<<nb, BLOCK, 0, ex.st>>>(g, nc, x, y, scale, rs, r, nrm2);
    if (nrm2) finish_to<1>(ex, nrm2, r, nb, FinStore<1>{nrm2});
}
template void vec_scale_cast<double, double>(const Exec &, const Grid &, int, const double *, double *, double,
                                             const double *, double *);
template void vec_scale_cast<double, float>(const Exec &, const Grid &, int, const double *, float *, double,
                                            const double *, double *);

template <typename T>
void vec_scale(const Exec &ex, const Grid &g, int nc, const T *x, T *y, double scale, const double *rs,
               double *nrm2) {
    const int nb = vblocks(g.nn);
    materialize(ex, const_cast<double *>(rs));
    const Red r = red_for(ex, nrm2, nb);
    k_scale<T, T><<<nb, BLOCK, 0, ex.st>>>(g, nc, x, y, scale, rs, r, nrm2);
    if (nrm2) finish_to<1>(ex, nrm2, r, nb, FinStore<1>{nrm2});
}
template void vec_scale<float>(const Exec &, const Grid &, int, const float *, float *, double, const double *, double *);
template void vec_scale<double>(const Exec &, const Grid &, int, const double *, double *, double, const double *, double *);

// FD step numerator (Sec. 1): mode 0 root (1 + ||x||), mode 1 root mean(1 + |x_i|)
struct FinEpsNum {
    double *out;
    double root, ndof;
    int mode;
    __device__ void operator()(const double *t) const {
        out[0] = mode == 0 ? root * (1.0 + sqrt(t[0])) : root * ((ndof + t[1]) / ndof);
    }
};
template <typename T>
__global__ void k_eps_num(Grid g, int nc, const T *x, Red red) {
    double s[2] = {0.0, 0.0};
    GRID_STRIDE(i, g.nn) {
        if (dir_at(g, i)) continue;
        for (int c = 0; c < nc; ++c) {
            const double v = (double)x[c * g.nn + i];
            s[0] += v * v;
            s[1] += fabs(v);
        }
    }
    block_partials<2>(s, red);
}
static double count_dofs(const Grid &g, int nc) {
    // DoFs = nodes off the Dirichlet faces
    long long nx = g.NX, ny = g.NY, nz = g.NZ;
    if (g.dir & JFNK_FACE_XLO) nx--;
    if (g.dir & JFNK_FACE_XHI) nx--;
    if (g.dir & JFNK_FACE_YLO) ny--;
    if (g.dir & JFNK_FACE_YHI) ny--;
    if (g.dim == 3) {
        if (g.dir & JFNK_FACE_ZLO) nz--;
        if (g.dir & JFNK_FACE_ZHI) nz--;
    }
    long long n = (nx > 0 ? nx : 0) * (ny > 0 ? ny : 0) * (nz > 0 ? nz : 0);
    return (double)n * nc;
}
template <typename T>
void vec_eps_num(const Exec &ex, const Grid &g, int nc, const T *x, double root, int mode, double *num) {
    double nd = count_dofs(g, nc);
    const int nb = vblocks(g.nn);
    k_eps_num<T><<<nb, BLOCK, 0, ex.st>>>(g, nc, x, ex.red);
    finish<2>(ex.st, ex.red, nb, FinEpsNum{num, root, nd > 0 ? nd : 1.0, mode});
}
template void vec_eps_num<float>(const Exec &, const Grid &, int, const float *, double, int, double *);
template void vec_eps_num<double>(const Exec &, const Grid &, int, const double *, double, int, double *);

// Chebyshev from s = 0: r = b, d = b / theta, s = 0
template <typename T>
__global__ void k_cheb_zero(Grid g, int nc, const T *b, T *r, T *d, T *s, T inv_theta, Red red, double *out) {
    double sm[1] = {0.0};
    GRID_STRIDE(i, g.nn) {
        const bool dd = dir_at(g, i);
        for (int c = 0; c < nc; ++c) {
            const long long k = c * g.nn + i;
            T bk = dd ? T(0) : b[k];
            r[k] = bk;
            T dk = bk * inv_theta;
            d[k] = dk;
            s[k] = T(0);
            sm[0] += (double)dk * (double)dk;
        }
    }
    block_partials<1>(sm, red);
}
template <typename T>
void vec_cheb_zero(const Exec &ex, const Grid &g, int nc, const T *b, T *r, T *d, T *s, double inv_theta,
                   double *d_nrm2) {
    const int nb = vblocks(g.nn);
    const Red rr = red_for(ex, d_nrm2, nb);
    k_cheb_zero<T><<<nb, BLOCK, 0, ex.st>>>(g, nc, b, r, d, s, (T)inv_theta, rr, d_nrm2);
    finish_to<1>(ex, d_nrm2, rr, nb, FinStore<1>{d_nrm2});
}
template void vec_cheb_zero<float>(const Exec &, const Grid &, int, const float *, float *, float *, float *, double, double *);
template void vec_cheb_zero<double>(const Exec &, const Grid &, int, const double *, double *, double *, double *, double, double *);

template <typename T>
__global__ void k_add(Grid g, int nc, const T *s, const T *d, T *o, Red red, double *out) {
    double sm[1] = {0.0};
    GRID_STRIDE(i, g.nn) {
        const bool dd = dir_at(g, i);
        for (int c = 0; c < nc; ++c) {
            const long long k = c * g.nn + i;
            T v = dd ? T(0) : s[k] + d[k];
            o[k] = v;
            sm[0] += (double)v * (double)v;
        }
    }
    if (out) block_partials<1>(sm, red);
}
template <typename T>
void vec_add(const Exec &ex, const Grid &g, int nc, const T *s, const T *d, T *o, double *nrm2) {
    const int nb = vblocks(g.nn);
    const Red r = red_for(ex, nrm2, nb);
    k_add<T><<<nb, BLOCK, 0, ex.st>>>(g, nc, s, d, o, r, nrm2);
    if (nrm2) finish_to<1>(ex, nrm2, r, nb, FinStore<1>{nrm2});
}
template void vec_add<float>(const Exec &, const Grid &, int, const float *, const float *, float *, double *);
template void vec_add<double>(const Exec &, const Grid &, int, const double *, const double *, double *, double *);

// SplitMix64 (Steele, Lea, Flood 2014) as a counter-based generator: value
// at flat index k of level l is the (k+1)-th output of the sequence whose
// state starts at seed + l 2^32, mapped to [-1, 1).
__device__ __forceinline__ double splitmix_uniform(unsigned long long s0, unsigned long long k) {
    unsigned long long z = s0 + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * 0x1.0p-52 - 1.0;
}
template <typename T>
__global__ void k_random(Grid g, int nc, unsigned long long s0, T *v, Red red, double *out) {
    double sm[1] = {0.0};
    GRID_STRIDE(i, g.nn) {
        const bool dd = dir_at(g, i);
        for (int c = 0; c < nc; ++c) {
            const long long k = c * g.nn + i;
            T val = dd ? T(0) : (T)splitmix_uniform(s0, (unsigned long long)k);
            v[k] = val;
            sm[0] += (double)val * (double)val;
        }
    }
    block_partials<1>(sm, red);
}
template <typename T>
void vec_random(const Exec &ex, const Grid &g, int nc, unsigned long long seed, int level, T *v, double *nrm2) {
    unsigned long long s0 = seed + ((unsigned long long)level << 32);
    const int nb = vblocks(g.nn);
    const Red r = red_for(ex, nrm2, nb);
    k_random<T><<<nb, BLOCK, 0, ex.st>>>(g, nc, s0, v, r, nrm2);
    finish_to<1>(ex, nrm2, r, nb, FinStore<1>{nrm2});
}
template void vec_random<float>(const Exec &, const Grid &, int, unsigned long long, int, float *, double *);
template void vec_random<double>(const Exec &, const Grid &, int, unsigned long long, int, double *, double *);

template <typename T> __global__ void k_exp(long long n, const double *m, T *kap) {
    GRID_STRIDE(i, n) kap[i] = (T)exp(m[i]);
}
template <typename T> void vec_exp(const Exec &ex, long long n, const double *m, T *kap) {
    k_exp<T><<<vblocks(n), BLOCK, 0, ex.st>>>(n, m, kap);
}
template void vec_exp<float>(const Exec &, long long, const double *, float *);
template void vec_exp<double>(const Exec &, long long, const double *, double *);

template <typename TA, typename TB>
__global__ void k_dot(long long n, const TA *x, const TB *y, Red red, double *out) {
    double sm[1] = {0.0};
    GRID_STRIDE(i, n) sm[0] += (double)x[i] * (double)y[i];
    block_partials<1>(sm, red);
}
template <typename TA, typename TB>
void vec_dot(const Exec &ex, long long n, const TA *x, const TB *y, double *out) {
    const int nb = vblocks(n);
    const Red r = red_for(ex, out, nb);
    k_dot<TA, TB><<<nb, BLOCK, 0, ex.st>>>(n, x, y, r, out);
    finish_to<1>(ex, out, r, nb, FinStore<1>{out});
}
template void vec_dot<double, double>(const Exec &, long long, const double *, const double *, double *);
template void vec_dot<float, float>(const Exec &, long long, const float *, const float *, double *);

template void vec_dot<double, float>(const Exec &, long long, const double *, const float *, double *);

// ---- preconditioned CG steps --------------------------------------------------------
// x += a p, r -= a q with a = rz / pq, ||r||^2 -> rn2; nothing is updated
// unless pq > 0 (the negative-curvature exit keeps x and r)
__global__ void k_cg_update(long long n, const double *p, const double *q, double *x, double *r, const double *rz,
                            const double *pq, Red red) {
    const double c = *pq;
    const bool go = c > 0.0;
    const double a = go ? *rz / c : 0.0;
    double sm[1] = {0.0};
    if (go) {
        GRID_STRIDE(i, n) {
            x[i] += a * p[i];
            const double ri = r[i] - a * q[i];
            r[i] = ri;
            sm[0] += ri * ri;
        }
    }
    block_partials<1>(sm, red);
}
void vec_cg_update(const Exec &ex, long long n, const double *p, const double *q, double *x, double *r,
                   const double *rz, const double *pq, double *rn2) {
    materialize(ex, const_cast<double *>(rz));
    materialize(ex, const_cast<double *>(pq));
    const int nb = vblocks(n);
    const Red rd = red_for(ex, rn2, nb);
    k_cg_update<<<nb, BLOCK, 0, ex.st>>>(n, p, q, x, r, rz, pq, rd);
    finish_to<1>(ex, rn2, rd, nb, FinStore<1>{rn2});
}

// p = z + b p with b = rz / rz_prev (rz_prev null: p = z), ||p||^2 -> pn2
template <typename TZ>
__global__ void k_cg_dir(long long n, const TZ *z, double *p, const double *rz, const double *rz_prev, Red red) {
    const double b = rz_prev ? *rz / *rz_prev : 0.0;
    double sm[1] = {0.0};
    GRID_STRIDE(i, n) {
        const double v = rz_prev ? (double)z[i] + b * p[i] : (double)z[i];
        p[i] = v;
        sm[0] += v * v;
    }
    block_partials<1>(sm, red);
}
template <typename TZ>
void vec_cg_dir(const Exec &ex, long long n, const TZ *z, double *p, const double *rz, const double *rz_prev,
                double *pn2) {
    materialize(ex, const_cast<double *>(rz));
    if (rz_prev) materialize(ex, const_cast<double *>(rz_prev));
    const int nb = vblocks(n);
    const Red rd = red_for(ex, pn2, nb);
    k_cg_dir<TZ><<<nb, BLOCK, 0, ex.st>>>(n, z, p, rz, rz_prev, rd);
    finish_to<1>(ex, pn2, rd, nb, FinStore<1>{pn2});
}
template void vec_cg_dir<float>(const Exec &, long long, const float *, double *, const double *, const double *,
                                double *);
template void vec_cg_dir<double>(const Exec &, long long, const double *, double *, const double *, const double *,
                                 double *);

__global__ void k_axpy(long long n, const double *x, double a, const double *d, double *y) {
    GRID_STRIDE(i, n) y[i] = x[i] + a * d[i];
}
void vec_axpy(const Exec &ex, long long n, const double *x, double a, const double *d, double *y) {
    k_axpy<<<vblocks(n), BLOCK, 0, ex.st>>>(n, x, a, d, y);
}

// ---- Gram-Schmidt passes ----------------------------------------------------------
// Classical Gram-Schmidt with delayed reorthogonalisation (DCGS2: Swirydowicz,
// Langou, Ananthan, Yang, Thomas, "Low synchronization Gram-Schmidt and
// generalized minimal residual algorithms", Numer. Linear Algebra Appl. 2021;
// Bielich et al., Parallel Computing 2022).  Iteration j holds the final
// orthonormal columns V_0..V_{J-1} (J = j), the candidate u = column J,
// projected once, and the new image w.  One reading pass forms
//   a = V^T u,  b = V^T w,  c = u.u,  d = u.w;
// then s = a (the delayed second projection of u), r = sqrt(c - s.s),
// v_J = (u - V s) / r, and the coefficient of w on v_J is (d - s.b) / r.  One
// update pass writes v_J over u and the next candidate
//   u' = w - V b - ((d - s.b) / r) v_J
// into column J + 1, with ||u'||^2.  In exact arithmetic this is CGS2 with
// the second projection of each vector one iteration late; per iteration it
// reads the basis twice instead of three times.
// The number of basis vectors J is a template parameter, so the loads of a
// pass issue back to back (the compiler places one wait in front of each
// use); up to J = 12 a thread also takes two elements per trip.  When the
// columns start on 16-byte boundaries (an even leading dimension) those two
// elements are adjacent and each column is read with one 16-byte load per
// lane (PAIR); the last element of an odd length goes to the first thread.
constexpr int ARN_MAX = 32;

template <int J> struct ArnUnroll { static constexpr int U = J <= 12 ? 2 : 1; };

template <int J, bool PAIR>
__global__ __launch_bounds__(BLOCK) void k_dcgs_dots(long long n, const double *V, long long ld, const double *w,
                                                     Red red) {
    constexpr int U = ArnUnroll<J>::U;
    constexpr int NS = 2 * J + 2;
    const double *u = V + J * ld;
    double s[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) s[k] = 0.0;
    auto acc = [&](double ui, double wi, const double *vk) {
#pragma unroll
        for (int k = 0; k < J; ++k) {
            s[k] += vk[k] * ui;
            s[J + k] += vk[k] * wi;
        }
        s[2 * J] += ui * ui;
        s[2 * J + 1] += ui * wi;
    };
    const long long stride = (long long)gridDim.x * BLOCK;
    long long i = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if constexpr (PAIR) {
        const long long n2 = n >> 1;
        for (long long q = i; q < n2; q += stride) {
            const long long e = 2 * q;
            const d2v uu = *(const d2v *)(u + e), ww = *(const d2v *)(w + e);
            double v0[J > 0 ? J : 1], v1[J > 0 ? J : 1];
#pragma unroll
            for (int k = 0; k < J; ++k) {
                const d2v vv = *(const d2v *)(V + k * ld + e);
                v0[k] = vv.x;
                v1[k] = vv.y;
            }
            acc(uu.x, ww.x, v0);
            acc(uu.y, ww.y, v1);
        }
        if ((n & 1) && i == 0) {
            double vk[J > 0 ? J : 1];
#pragma unroll
            for (int k = 0; k < J; ++k) vk[k] = V[k * ld + n - 1];
            acc(u[n - 1], w[n - 1], vk);
        }
    } else {
        for (; i + (U - 1) * stride < n; i += U * stride) {
            double ui[U], wi[U], vk[U][J > 0 ? J : 1];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                ui[q] = u[i + q * stride];
                wi[q] = w[i + q * stride];
#pragma unroll
                for (int k = 0; k < J; ++k) vk[q][k] = V[k * ld + i + q * stride];
            }
#pragma unroll
            for (int q = 0; q < U; ++q) acc(ui[q], wi[q], vk[q]);
        }
        if (U > 1 && i < n) {
            double vk[J > 0 ? J : 1];
#pragma unroll
            for (int k = 0; k < J; ++k) vk[k] = V[k * ld + i];
            acc(u[i], w[i], vk);
        }
    }
    block_partials<NS>(s, red);
}

// coefficients of the update pass from the dot products t[0..2J+1]:
// out[0..J) = s, out[J..2J) = b, out[2J] = 1/r, out[2J+1] = (d - s.b)/r,
// out[2J+2] = r
struct FinDcgs {
    double *out;
    int J;
    __device__ void operator()(const double *t) const {
        double ss = 0.0, sb = 0.0;
        for (int k = 0; k < J; ++k) {
            out[k] = t[k];
            out[J + k] = t[J + k];
            ss += t[k] * t[k];
            sb += t[k] * t[J + k];
        }
        const double rr = t[2 * J] - ss;
        const double r = rr > 0.0 ? sqrt(rr) : 0.0;
        const double ir = r > 0.0 ? 1.0 / r : 0.0;
        out[2 * J] = ir;
        out[2 * J + 1] = (t[2 * J + 1] - sb) * ir;
        out[2 * J + 2] = r;
    }
};

template <int J, bool PAIR>
__global__ __launch_bounds__(BLOCK) void k_dcgs_update(long long n, double *V, long long ld, const double *coef,
                                                       const double *w, Red red) {
    constexpr int U = ArnUnroll<J>::U;
    __shared__ double cs[2 * J + 2];
    if (threadIdx.x < 2 * J + 2) cs[threadIdx.x] = coef[threadIdx.x];
    __syncthreads();
    double sk[J > 0 ? J : 1], bk[J > 0 ? J : 1];
#pragma unroll
    for (int k = 0; k < J; ++k) { sk[k] = cs[k]; bk[k] = cs[J + k]; }
    const double ir = cs[2 * J], hj = cs[2 * J + 1];
    double *u = V + J * ld, *un = V + (J + 1) * ld;
    double nrm[1] = {0.0};
    // the new column entry and the next candidate's, from u, w and the basis
    auto entry = [&](double ui, double wi, const double *vk, double &vj, double &x) {
#pragma unroll
        for (int k = 0; k < J; ++k) {
            ui -= sk[k] * vk[k];
            wi -= bk[k] * vk[k];
        }
        vj = ui * ir;
        x = wi - hj * vj;
        nrm[0] += x * x;
    };
    auto one = [&](long long idx, double ui, double wi, const double *vk) {
        double vj, x;
        entry(ui, wi, vk, vj, x);
        u[idx] = vj;
        un[idx] = x;
    };
    const long long stride = (long long)gridDim.x * BLOCK;
    long long i = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if constexpr (PAIR) {
        const long long n2 = n >> 1;
        for (long long q = i; q < n2; q += stride) {
            const long long e = 2 * q;
            const d2v uu = *(const d2v *)(u + e), ww = *(const d2v *)(w + e);
            double v0[J > 0 ? J : 1], v1[J > 0 ? J : 1];
#pragma unroll
            for (int k = 0; k < J; ++k) {
                const d2v vv = *(const d2v *)(V + k * ld + e);
                v0[k] = vv.x;
                v1[k] = vv.y;
            }
            double vj0, x0, vj1, x1;
            entry(uu.x, ww.x, v0, vj0, x0);
            entry(uu.y, ww.y, v1, vj1, x1);
            *(d2v *)(u + e) = d2v{vj0, vj1};
            *(d2v *)(un + e) = d2v{x0, x1};
        }
        if ((n & 1) && i == 0) {
            double vk[J > 0 ? J : 1];
#pragma unroll
            for (int k = 0; k < J; ++k) vk[k] = V[k * ld + n - 1];
            one(n - 1, u[n - 1], w[n - 1], vk);
        }
        block_partials<1>(nrm, red);
        return;
    }
    for (; i + (U - 1) * stride < n; i += U * stride) {
        double ui[U], wi[U], vk[U][J > 0 ? J : 1];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            ui[q] = u[i + q * stride];
            wi[q] = w[i + q * stride];
#pragma unroll
            for (int k = 0; k < J; ++k) vk[q][k] = V[k * ld + i + q * stride];
        }
#pragma unroll
        for (int q = 0; q < U; ++q) one(i + q * stride, ui[q], wi[q], vk[q]);
    }
    if (U > 1 && i < n) {
        double vk[J > 0 ? J : 1];
#pragma unroll
        for (int k = 0; k < J; ++k) vk[k] = V[k * ld + i];
        one(i, u[i], w[i], vk);
    }
    block_partials<1>(nrm, red);
}

static inline int arn_blocks(long long n) { return vblocks(n, 2048); }

// the 16-byte form while a thread takes two elements per trip and the
// columns and w start on 16-byte boundaries
static inline bool arn_pair(const double *V, long long ld, const double *w) {
    return (ld % 2) == 0 && ((size_t)V % 16) == 0 && ((size_t)w % 16) == 0;
}
template <int J> void dcgs_dots_k(const Exec &ex, long long n, const double *V, long long ld, const double *w,
                                  double *coef) {
    const int nb = arn_blocks(n);
    bool pair = false;
    if constexpr (ArnUnroll<J>::U == 2) {
        pair = arn_pair(V, ld, w);
        if (pair) k_dcgs_dots<J, true><<<nb, BLOCK, 0, ex.st>>>(n, V, ld, w, ex.red);
    }
    if (!pair) k_dcgs_dots<J, false><<<nb, BLOCK, 0, ex.st>>>(n, V, ld, w, ex.red);
    finish<2 * J + 2>(ex.st, ex.red, nb, FinDcgs{coef, J});
}
template <int J> void dcgs_update_k(const Exec &ex, long long n, double *V, long long ld, const double *coef,
                                    const double *w, double *nrm2) {
    const int nb = arn_blocks(n);
    bool pair = false;
    if constexpr (ArnUnroll<J>::U == 2) {
        pair = arn_pair(V, ld, w);
        if (pair) k_dcgs_update<J, true><<<nb, BLOCK, 0, ex.st>>>(n, V, ld, coef, w, ex.red);
    }
    if (!pair) k_dcgs_update<J, false><<<nb, BLOCK, 0, ex.st>>>(n, V, ld, coef, w, ex.red);
    finish<1>(ex.st, ex.red, nb, FinStore<1>{nrm2});
}

using DotsFn = void (*)(const Exec &, long long, const double *, long long, const double *, double *);
using UpdFn = void (*)(const Exec &, long long, double *, long long, const double *, const double *, double *);
template <int... Js> constexpr std::array<DotsFn, sizeof...(Js)> dots_table(std::integer_sequence<int, Js...>) {
    return {&dcgs_dots_k<Js>...};
}
template <int... Js> constexpr std::array<UpdFn, sizeof...(Js)> upd_table(std::integer_sequence<int, Js...>) {
    return {&dcgs_update_k<Js>...};
}
static constexpr auto kDots = dots_table(std::make_integer_sequence<int, ARN_MAX - 1>{});
static constexpr auto kUpd = upd_table(std::make_integer_sequence<int, ARN_MAX - 1>{});

void dcgs_dots(const Exec &ex, long long n, const double *V, long long ld, int J, const double *w, double *coef) {
    if (J < 0 || J >= ARN_MAX - 1) return;
    kDots[J](ex, n, V, ld, w, coef);
}
void dcgs_update(const Exec &ex, long long n, double *V, long long ld, int J, const double *coef, const double *w,
                 double *nrm2) {
    if (J < 0 || J >= ARN_MAX - 1) return;
    kUpd[J](ex, n, V, ld, coef, w, nrm2);
}

// x += Z y  (y passed by value)
struct CombineArgs {
    double y[ARN_MAX];
};
// PAIR: two adjacent entries per lane (x by 16-byte, Z by 16- or 8-byte
// accesses) when x and the columns of Z start on such boundaries; the same
// sum per entry, in the same order
template <typename TZ, int K, bool PAIR>
__global__ __launch_bounds__(BLOCK) void k_arn_combine(long long n, const TZ *Z, long long ld, CombineArgs ya,
                                                       double *x) {
    if constexpr (PAIR) {
        typedef TZ z2v __attribute__((ext_vector_type(2)));
        const long long n2 = n >> 1;
        GRID_STRIDE(q, n2) {
            const long long e = 2 * q;
            z2v zj[K];
#pragma unroll
            for (int j = 0; j < K; ++j) zj[j] = *(const z2v *)(Z + j * ld + e);
            d2v acc = *(const d2v *)(x + e);
#pragma unroll
            for (int j = 0; j < K; ++j) {
                acc.x += ya.y[j] * (double)zj[j].x;
                acc.y += ya.y[j] * (double)zj[j].y;
            }
            *(d2v *)(x + e) = acc;
        }
        if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
            double acc = x[n - 1];
#pragma unroll
            for (int j = 0; j < K; ++j) acc += ya.y[j] * (double)Z[j * ld + n - 1];
            x[n - 1] = acc;
        }
        return;
    }
    GRID_STRIDE(i, n) {
        TZ zj[K];
#pragma unroll
        for (int j = 0; j < K; ++j) zj[j] = Z[j * ld + i];
        double acc = x[i];
#pragma unroll
        for (int j = 0; j < K; ++j) acc += ya.y[j] * (double)zj[j];
        x[i] = acc;
    }
}
template <typename TZ, int K>
void arn_combine_k(const Exec &ex, long long n, const TZ *Z, long long ld, const CombineArgs &a, double *x) {
    const bool pair = (ld % 2) == 0 && ((size_t)Z % (2 * sizeof(TZ))) == 0 && ((size_t)x % 16) == 0;
    if (pair) k_arn_combine<TZ, K, true><<<vblocks(n / 2), BLOCK, 0, ex.st>>>(n, Z, ld, a, x);
    else k_arn_combine<TZ, K, false><<<vblocks(n), BLOCK, 0, ex.st>>>(n, Z, ld, a, x);
}
template <typename TZ> using CombFn = void (*)(const Exec &, long long, const TZ *, long long, const CombineArgs &,
                                               double *);
template <typename TZ, int... Ks>
constexpr std::array<CombFn<TZ>, sizeof...(Ks)> comb_table(std::integer_sequence<int, Ks...>) {
    return {&arn_combine_k<TZ, Ks + 1>...};
}

// y: host array of k coefficients
template <typename TZ>
void arn_combine(const Exec &ex, long long n, const TZ *Z, long long ld, int k, const double *y, double *x) {
    static constexpr auto tab = comb_table<TZ>(std::make_integer_sequence<int, ARN_MAX>{});
    if (k < 1 || k > ARN_MAX) return;
    CombineArgs a;
    for (int j = 0; j < ARN_MAX; ++j) a.y[j] = j < k ? y[j] : 0.0;
    tab[k - 1](ex, n, Z, ld, a, x);
}
template void arn_combine<float>(const Exec &, long long, const float *, long long, int, const double *, double *);
template void arn_combine<double>(const Exec &, long long, const double *, long long, int, const double *, double *);

// ---- transfers (Sec. 2) ------------------------------------------------------------
// 1D weights of I^T: fine index f contributes to coarse c with 1 (f = 2c) or
// 1/2 (f = 2c +- 1).
template <typename TI, typename TO>
__global__ void k_project(Grid gf, Grid gc, int nc, const TI *xf, TO *xc) {
    GRID_STRIDE(i, gc.nn) {
        int cx, cy, cz;
        node_coords(gc, i, cx, cy, cz);
        if (is_dirichlet(gc, cx, cy, cz)) {
            const long long j = node_index(gf, 2 * cx, 2 * cy, 2 * cz);
            for (int c = 0; c < nc; ++c) xc[c * gc.nn + i] = (TO)xf[c * gf.nn + j];
            continue;
        }
        const int zlo = gc.dim == 3 ? -1 : 0, zhi = gc.dim == 3 ? 1 : 0;
        for (int c = 0; c < nc; ++c) {
            double acc = 0.0, wsum = 0.0;
            for (int dz = zlo; dz <= zhi; ++dz) {
                const int fz = 2 * cz + dz;
                if (fz < 0 || fz >= gf.NZ) continue;
                const double wz = dz == 0 ? 1.0 : 0.5;
                for (int dy = -1; dy <= 1; ++dy) {
                    const int fy = 2 * cy + dy;
                    if (fy < 0 || fy >= gf.NY) continue;
                    const double wy = wz * (dy == 0 ? 1.0 : 0.5);
                    for (int dx = -1; dx <= 1; ++dx) {
                        const int fx = 2 * cx + dx;
                        if (fx < 0 || fx >= gf.NX) continue;
                        const double w = wy * (dx == 0 ? 1.0 : 0.5);
                        acc += w * (double)xf[c * gf.nn + node_index(gf, fx, fy, fz)];
                        wsum += w;
                    }
                }
            }
            xc[c * gc.nn + i] = (TO)(acc / wsum);
        }
    }
}
template <typename TI, typename TO>
void tr_project(const Exec &ex, const Grid &gf, const Grid &gc, int nc, const TI *xf, TO *xc) {
    k_project<TI, TO><<<vblocks(gc.nn), BLOCK, 0, ex.st>>>(gf, gc, nc, xf, xc);
}
template void tr_project<double, double>(const Exec &, const Grid &, const Grid &, int, const double *, double *);
template void tr_project<double, float>(const Exec &, const Grid &, const Grid &, int, const double *, float *);
template void tr_project<float, float>(const Exec &, const Grid &, const Grid &, int, const float *, float *);

// R = I^T with zero rows at coarse Dirichlet nodes
template <typename T>
__global__ void k_restrict(Grid gf, Grid gc, int nc, const T *rf, T *rc, Red red, double *out) {
    double sm[1] = {0.0};
    GRID_STRIDE(i, gc.nn) {
        int cx, cy, cz;
        node_coords(gc, i, cx, cy, cz);
        const bool dd = is_dirichlet(gc, cx, cy, cz);
        const int zlo = gc.dim == 3 ? -1 : 0, zhi = gc.dim == 3 ? 1 : 0;
        for (int c = 0; c < nc; ++c) {
            T acc = T(0);
            if (!dd) {
                for (int dz = zlo; dz <= zhi; ++dz) {
                    const int fz = 2 * cz + dz;
                    if (fz < 0 || fz >= gf.NZ) continue;
                    const T wz = dz == 0 ? T(1) : T(0.5);
                    for (int dy = -1; dy <= 1; ++dy) {
                        const int fy = 2 * cy + dy;
                        if (fy < 0 || fy >= gf.NY) continue;
                        const T wy = wz * (dy == 0 ? T(1) : T(0.5));
                        for (int dx = -1; dx <= 1; ++dx) {
                            const int fx = 2 * cx + dx;
                            if (fx < 0 || fx >= gf.NX) continue;
                            acc += wy * (dx == 0 ? T(1) : T(0.5)) * rf[c * gf.nn + node_index(gf, fx, fy, fz)];
                        }
                    }
                }
            }
            rc[c * gc.nn + i] = acc;
            sm[0] += (double)acc * (double)acc;
        }
    }
    if (out) block_partials<1>(sm, red);
}
// 3D, one component: the 27 fine neighbours of a coarse node with weights
// (1/2, 1, 1/2) per axis, as straight-line code; indices are clamped into the
// grid and the weight of a clamped neighbour is 0.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_restrict3(Grid gf, Grid gc, const T *rf, T *rc, Red red, double *out) {
    double sm[1] = {0.0};
    GRID_STRIDE(i, gc.nn) {
        int cx, cy, cz;
        node_coords(gc, i, cx, cy, cz);
        T acc = T(0);
        if (!is_dirichlet(gc, cx, cy, cz)) {
            int ix[3], iy[3], iz[3];
            T wx[3], wy[3], wz[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int fx = 2 * cx + d - 1, fy = 2 * cy + d - 1, fz = 2 * cz + d - 1;
                const T w = d == 1 ? T(1) : T(0.5);
                wx[d] = (fx >= 0 && fx < gf.NX) ? w : T(0);
                wy[d] = (fy >= 0 && fy < gf.NY) ? w : T(0);
                wz[d] = (fz >= 0 && fz < gf.NZ) ? w : T(0);
                ix[d] = min(max(fx, 0), gf.NX - 1);
                iy[d] = min(max(fy, 0), gf.NY - 1);
                iz[d] = min(max(fz, 0), gf.NZ - 1);
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                T pz = T(0);
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const T *row = rf + ((long long)iz[a] * gf.NY + iy[b]) * gf.NX;
                    const T px = wx[0] * row[ix[0]] + wx[1] * row[ix[1]] + wx[2] * row[ix[2]];
                    pz += wy[b] * px;
                }
                acc += wz[a] * pz;
            }
        }
        rc[i] = acc;
        sm[0] += (double)acc * (double)acc;
    }
    if (out) block_partials<1>(sm, red);
}

template <typename T>
void tr_restrict(const Exec &ex, const Grid &gf, const Grid &gc, int nc, const T *rf, T *rc, double *nrm2) {
    const int nb = vblocks(gc.nn);
    const Red r = red_for(ex, nrm2, nb);
    if (gf.dim == 3 && nc == 1) k_restrict3<T><<<nb, BLOCK, 0, ex.st>>>(gf, gc, rf, rc, r, nrm2);
    else k_restrict<T><<<nb, BLOCK, 0, ex.st>>>(gf, gc, nc, rf, rc, r, nrm2);
    if (nrm2) finish_to<1>(ex, nrm2, r, nb, FinStore<1>{nrm2});
}
template void tr_restrict<float>(const Exec &, const Grid &, const Grid &, int, const float *, float *, double *);
template void tr_restrict<double>(const Exec &, const Grid &, const Grid &, int, const double *, double *, double *);

// s_f += I c: even fine index -> coarse f/2 (weight 1), odd -> both neighbours (1/2)
template <typename T>
__global__ void k_prolong_add(Grid gf, Grid gc, int nc, const T *cc, T *sf, Red red, double *out) {
    double sm[1] = {0.0};
    GRID_STRIDE(i, gf.nn) {
        int fx, fy, fz;
        node_coords(gf, i, fx, fy, fz);
        const bool dd = is_dirichlet(gf, fx, fy, fz);
        const int x0 = fx >> 1, x1 = (fx + 1) >> 1, y0 = fy >> 1, y1 = (fy + 1) >> 1;
        const int z0 = fz >> 1, z1 = (fz + 1) >> 1;
        const T wx = (fx & 1) ? T(0.5) : T(1), wy = (fy & 1) ? T(0.5) : T(1), wz = (fz & 1) ? T(0.5) : T(1);
        for (int c = 0; c < nc; ++c) {
            const long long k = c * gf.nn + i;
            if (dd) {
                sf[k] = T(0);
                continue;
            }
            const T *cb = cc + c * gc.nn;
            T v = T(0);
            // (x0,x1) coincide for even fx: count the node once with weight 1
            const int nxs = (fx & 1) ? 2 : 1, nys = (fy & 1) ? 2 : 1, nzs = (gf.dim == 3 && (fz & 1)) ? 2 : 1;
            for (int a = 0; a < nzs; ++a)
                for (int b = 0; b < nys; ++b)
                    for (int d = 0; d < nxs; ++d) {
                        const int X = d ? x1 : x0, Y = b ? y1 : y0, Z = a ? z1 : z0;
                        v += wx * wy * wz * cb[node_index(gc, X, Y, Z)];
                    }
            T s = sf[k] + v;
            sf[k] = s;
            sm[0] += (double)s * (double)s;
        }
    }
    if (out) block_partials<1>(sm, red);
}
// 3D, one component: the (up to) 8 coarse corners of the fine node's
// coarse cell as straight-line code.  On an even fine coordinate both coarse
// indices coincide and the weights are (1, 0); on an odd one (1/2, 1/2).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_prolong_add3(Grid gf, Grid gc, const T *cc, T *sf, Red red,
                                                        double *out) {
    double sm[1] = {0.0};
    GRID_STRIDE(i, gf.nn) {
        int fx, fy, fz;
        node_coords(gf, i, fx, fy, fz);
        T sv = T(0);
        if (!is_dirichlet(gf, fx, fy, fz)) {
            const int X[2] = {fx >> 1, (fx + 1) >> 1}, Y[2] = {fy >> 1, (fy + 1) >> 1}, Z[2] = {fz >> 1, (fz + 1) >> 1};
            const T wx[2] = {(fx & 1) ? T(0.5) : T(1), (fx & 1) ? T(0.5) : T(0)};
            const T wy[2] = {(fy & 1) ? T(0.5) : T(1), (fy & 1) ? T(0.5) : T(0)};
            const T wz[2] = {(fz & 1) ? T(0.5) : T(1), (fz & 1) ? T(0.5) : T(0)};
            T v = T(0);
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                T py = T(0);
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const T *row = cc + ((long long)Z[a] * gc.NY + Y[b]) * gc.NX;
                    py += wy[b] * (wx[0] * row[X[0]] + wx[1] * row[X[1]]);
                }
                v += wz[a] * py;
            }
            sv = sf[i] + v;
        }
        sf[i] = sv;
        sm[0] += (double)sv * (double)sv;
    }
    if (out) block_partials<1>(sm, red);
}

template <typename T>
void tr_prolong_add(const Exec &ex, const Grid &gf, const Grid &gc, int nc, const T *cc, T *sf, double *nrm2) {
    const int nb = vblocks(gf.nn);
    const Red r = red_for(ex, nrm2, nb);
    if (gf.dim == 3 && nc == 1) k_prolong_add3<T><<<nb, BLOCK, 0, ex.st>>>(gf, gc, cc, sf, r, nrm2);
    else k_prolong_add<T><<<nb, BLOCK, 0, ex.st>>>(gf, gc, nc, cc, sf, r, nrm2);
    if (nrm2) finish_to<1>(ex, nrm2, r, nb, FinStore<1>{nrm2});
}
template void tr_prolong_add<float>(const Exec &, const Grid &, const Grid &, int, const float *, float *, double *);
template void tr_prolong_add<double>(const Exec &, const Grid &, const Grid &, int, const double *, double *, double *);

// ---- loads ---------------------------------------------------------------------------
// b_i = sum over adjacent elements e, Gauss points q: w_q f(x_q) phi_i(x_q).
// Each Gaussian of f factors over the axes, and along an axis the Gauss
// points of the elements on either side of node i take 4 coordinates, so a
// source costs 4 one-dimensional exponentials per axis instead of one per
// (element, Gauss point) pair.  The element and Gauss-point loops are
// unrolled, so the factor table stays in registers.
template <int D>
__global__ void k_load_gauss(Grid g, const double *prm, int count, double *b) {
    constexpr int NV = 1 << D;
    const double w = (D == 3 ? g.h * g.h * g.h : g.h * g.h) / NV;
    GRID_STRIDE(i, g.nn) {
        int x, y, z;
        node_coords(g, i, x, y, z);
        if (is_dirichlet(g, x, y, z)) {
            b[i] = 0.0;
            continue;
        }
        const int X[3] = {x, y, z};
        const int NE[3] = {g.nx, g.ny, g.nz};
        unsigned valid = 0;     // bit e: element e (e = sx + 2 sy + 4 sz steps below) inside the grid
#pragma unroll
        for (int e = 0; e < NV; ++e) {
            bool ok = true;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const int c = X[a] - ((e >> a) & 1);
                ok = ok && c >= 0 && c < NE[a];
            }
            if (ok) valid |= 1u << e;
        }
        double acc = 0.0;
        for (int k = 0; k < count; ++k) {
            const double *pk = prm + k * (D + 2);
            const double s2 = 2.0 * pk[D] * pk[D];
            // E[a][2 s + j]: the factor of axis a at Gauss coordinate j of
            // the element s steps below the node
            double E[D][4];
#pragma unroll
            for (int a = 0; a < D; ++a) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const double t = (X[a] - (j >> 1) + ((j & 1) ? GL1 : GL0)) * g.h;
                    E[a][j] = exp(-(t - pk[a]) * (t - pk[a]) / s2);
                }
            }
            double sk = 0.0;
#pragma unroll
            for (int e = 0; e < NV; ++e) {
                double se = 0.0;
#pragma unroll
                for (int q = 0; q < NV; ++q) {
                    double f = 1.0;
#pragma unroll
                    for (int a = 0; a < D; ++a) f *= E[a][2 * ((e >> a) & 1) + ((q >> a) & 1)];
                    // phi at corner e (local index of node i) evaluated at q
                    const int c = __builtin_popcount((unsigned)(e ^ q));
                    double ph = 1.0;
#pragma unroll
                    for (int a = 0; a < D; ++a) ph *= (a < D - c) ? GL1 : GL0;
                    se += f * ph;
                }
                if ((valid >> e) & 1u) sk += se;
            }
            acc += w * pk[D + 1] * sk;
        }
        b[i] = acc;
    }
}
void load_gaussians(const Exec &ex, const Grid &g, const double *prm, int count, double *b) {
    if (g.dim == 3) k_load_gauss<3><<<vblocks(g.nn), BLOCK, 0, ex.st>>>(g, prm, count, b);
    else k_load_gauss<2><<<vblocks(g.nn), BLOCK, 0, ex.st>>>(g, prm, count, b);
}

// traction t on the x = x_max face: each face cell gives t h^2 / 4 to its corners
__global__ void k_load_traction(Grid g, double tx, double ty, double tz, double *b) {
    GRID_STRIDE(i, g.nn) {
        int x, y, z;
        node_coords(g, i, x, y, z);
        double w = 0.0;
        if (x == g.nx && !is_dirichlet(g, x, y, z)) {
            const int cy = (y > 0) + (y < g.ny), cz = (z > 0) + (z < g.nz);
            w = g.h * g.h / 4.0 * cy * cz;
        }
        b[i] = w * tx;
        b[g.nn + i] = w * ty;
        b[2 * g.nn + i] = w * tz;
    }
}
void load_traction(const Exec &ex, const Grid &g, const double *t, double *b) {
    k_load_traction<<<vblocks(g.nn), BLOCK, 0, ex.st>>>(g, t[0], t[1], t[2], b);
}

// ---- streaming calibration: c = a + s b, 16 bytes per lane and array, with
// the non-temporal hint (every element is touched once); a dense sweep of
// the whole arrays by the grid, the access pattern HBM serves best
__global__ __launch_bounds__(256) void k_triad(const d2v *a, const d2v *b, d2v *c, long long n2, double s) {
    const long long st = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += st) {
        const d2v x = __builtin_nontemporal_load(&a[i]);
        const d2v y = __builtin_nontemporal_load(&b[i]);
        __builtin_nontemporal_store(x + s * y, &c[i]);
    }
}
__global__ void k_triad_tail(const double *a, const double *b, double *c, long long n, double s) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && (n & 1)) c[n - 1] = a[n - 1] + s * b[n - 1];
}
void stream_triad(hipStream_t st, const double *a, const double *b, double *c, long long n, double s) {
    int ncu = 256, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const long long n2 = n / 2;
    const long long want = (n2 + 255) / 256;
    const int nb = (int)std::max(1LL, std::min<long long>(4LL * ncu, want));
    if (n2 > 0) k_triad<<<nb, 256, 0, st>>>((const d2v *)a, (const d2v *)b, (d2v *)c, n2, s);
    if (n & 1) k_triad_tail<<<1, 64, 0, st>>>(a, b, c, n, s);
}

}  // namespace jfnk
