// Coarse-level solver of Algorithm 1 as one persistent workgroup: CG on the
// finite-difference Jacobian of the coarsest level, stopped at negative
// curvature with the Rayleigh quotient lambda_c = p^T A_s p / p^T p, and the
// shift loop lambda_c+ <- gamma min(lambda_c, lambda_c+), A_s = J - lambda_c+ I,
// rerun from the current correction while lambda_c < 0 (Sec. 2, coarse
// level solver).  The whole loop runs on the device: one launch per coarse
// solve, no host round trip.
#include "stencil.hpp"
#include "ops.hpp"

namespace jfnk {

constexpr int CBLOCK = 1024;

__device__ __forceinline__ double cg_bsum(double v) {
    __shared__ double scratch[MAX_WAVES];
    __shared__ double tot[1];
    double a[1] = {v};
    block_sum<1>(a, scratch, tot);
    return tot[0];
}

#define NODE_LOOP(i, n) for (long long i = threadIdx.x; i < (n); i += blockDim.x)

template <int DIM, int KIND, int MODE, typename T>
__global__ __launch_bounds__(CBLOCK) void k_coarse(Grid g, Phys ph, const T *kap, const T *x, const T *Ax,
                                                   const double *num, const T *b, T *s, T *work, CoarseArgs ca) {
    constexpr int NC = (KIND == JFNK_NEOHOOKE) ? 3 : 1;
    const long long nn = g.nn, n = nn * NC;
    T *r = work, *p = work + n, *q = work + 2 * n;
    const double epsn = *num;

    // q = (J - shift I) v via the FD quotient; returns v.v
    auto apply = [&](const T *v, double shift) -> double {
        double vv = 0.0;
        NODE_LOOP(i, n) vv += (double)v[i] * (double)v[i];
        vv = cg_bsum(vv);
        const double eps = vv > 0.0 ? epsn / sqrt(vv) : 0.0;
        NODE_LOOP(i, nn) {
            int X, Y, Z;
            node_coords(g, i, X, Y, Z);
            T val[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) val[c] = T(0);
            const bool dir = is_dirichlet(g, X, Y, Z);
            if (!dir) node_value<DIM, KIND, MODE, T, T>(g, ph, kap, x, v, Ax, eps, X, Y, Z, i, val);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const long long k = c * nn + i;
                q[k] = dir ? T(0) : val[c] - (T)shift * v[k];
            }
        }
        __syncthreads();
        return vv;
    };

    double bb = 0.0;
    NODE_LOOP(i, n) {
        bb += (double)b[i] * (double)b[i];
        s[i] = T(0);
    }
    bb = cg_bsum(bb);
    const double tol = fmax(ca.atol, ca.rtol * sqrt(bb));
    long long fd = 0, iters = 0;
    bool s_nonzero = false;

    auto cg = [&](double shift) -> double {
        if (s_nonzero) {
            apply(s, shift);
            ++fd;
            NODE_LOOP(i, n) r[i] = b[i] - q[i];
        } else {
            NODE_LOOP(i, n) r[i] = b[i];
        }
        double rr = 0.0;
        NODE_LOOP(i, n) {
            p[i] = r[i];
            rr += (double)r[i] * (double)r[i];
        }
        rr = cg_bsum(rr);
        if (sqrt(rr) <= tol) return 0.0;
        for (int it = 1; it <= ca.maxit; ++it) {
            const double pp = apply(p, shift);
            ++fd;
            ++iters;
            double pq = 0.0;
            NODE_LOOP(i, n) pq += (double)p[i] * (double)q[i];
            pq = cg_bsum(pq);
            if (pq <= 0.0) return pq / pp;
            const double alpha = rr / pq;
            const T a = (T)alpha;
            double rn = 0.0;
            NODE_LOOP(i, n) {
                s[i] += a * p[i];
                T ri = r[i] - a * q[i];
                r[i] = ri;
                rn += (double)ri * (double)ri;
            }
            s_nonzero = true;
            rn = cg_bsum(rn);
            if (sqrt(rn) <= tol) return 0.0;
            const T beta = (T)(rn / rr);
            NODE_LOOP(i, n) p[i] = r[i] + beta * p[i];
            __syncthreads();
            rr = rn;
        }
        return 0.0;
    };

    double shift = 0.0;
    double lam_c = cg(shift);
    int rounds = 0;
    int negc = lam_c < 0.0 ? 1 : 0;
    while (lam_c < 0.0 && rounds < ca.shift_max) {
        shift = ca.gamma * fmin(lam_c, shift);
        lam_c = cg(shift);
        if (lam_c < 0.0) ++negc;
        ++rounds;
    }
    if (threadIdx.x == 0) {
        ca.stats[0] = shift;
        ca.stats[1] += (double)iters;
        ca.stats[2] = rounds;
        ca.stats[3] += (double)fd;
        ca.stats[4] += (double)negc;
        ca.stats[5] += 1.0;
    }
}

template <int DIM, int KIND, typename T>
static void launch_coarse(const Exec &ex, int mode, const Grid &g, const Phys &ph, const T *kap, const T *x,
                          const T *Ax, const double *num, const T *b, T *s, T *work, const CoarseArgs &ca) {
    if (mode == M_FD_DIFF)
        k_coarse<DIM, KIND, M_FD_DIFF, T><<<1, CBLOCK, 0, ex.st>>>(g, ph, kap, x, Ax, num, b, s, work, ca);
    else
        k_coarse<DIM, KIND, M_FD_PLAIN, T><<<1, CBLOCK, 0, ex.st>>>(g, ph, kap, x, Ax, num, b, s, work, ca);
}

template <typename T>
void coarse_solve(const Exec &ex, int mode, const Grid &g, const Phys &ph, const T *kap, const T *x, const T *Ax,
                  const double *num, const T *b, T *s, T *work, const CoarseArgs &ca) {
    switch (ph.kind) {
    case JFNK_BRATU:
        if (g.dim == 2) launch_coarse<2, JFNK_BRATU, T>(ex, mode, g, ph, kap, x, Ax, num, b, s, work, ca);
        else launch_coarse<3, JFNK_BRATU, T>(ex, mode, g, ph, kap, x, Ax, num, b, s, work, ca);
        break;
    case JFNK_PLAP:
        if (g.dim == 2) launch_coarse<2, JFNK_PLAP, T>(ex, mode, g, ph, kap, x, Ax, num, b, s, work, ca);
        else launch_coarse<3, JFNK_PLAP, T>(ex, mode, g, ph, kap, x, Ax, num, b, s, work, ca);
        break;
    case JFNK_INVCOEF:
        if (g.dim == 2) launch_coarse<2, JFNK_INVCOEF, T>(ex, mode, g, ph, kap, x, Ax, num, b, s, work, ca);
        else launch_coarse<3, JFNK_INVCOEF, T>(ex, mode, g, ph, kap, x, Ax, num, b, s, work, ca);
        break;
    case JFNK_NEOHOOKE:
        launch_coarse<3, JFNK_NEOHOOKE, T>(ex, mode, g, ph, kap, x, Ax, num, b, s, work, ca);
        break;
    }
}
template void coarse_solve<float>(const Exec &, int, const Grid &, const Phys &, const float *, const float *,
                                  const float *, const double *, const float *, float *, float *, const CoarseArgs &);
template void coarse_solve<double>(const Exec &, int, const Grid &, const Phys &, const double *, const double *,
                                   const double *, const double *, const double *, double *, double *,
                                   const CoarseArgs &);

int coarse_max_nodes() { return 1 << 16; }

}  // namespace jfnk
