// Coarse-level solver of Algorithm 1 as one persistent workgroup: CG on the
// finite-difference Jacobian of the coarsest level, stopped at negative
// curvature with the Rayleigh quotient lambda_c = p^T A_s p / p^T p, and the
// shift loop lambda_c+ <- gamma min(lambda_c, lambda_c+), A_s = J - lambda_c+ I,
// rerun from the current correction while lambda_c < 0 (Sec. 2, coarse
// level solver).  The whole loop runs on the device: one launch per coarse
// solve, no host round trip.
#include <map>
#include <mutex>

#include "stencil.hpp"
#include "ops.hpp"

namespace jfnk {

constexpr int CBLOCK = 1024;

// Block sum for the solver loops: one barrier per call, the wave totals in
// one of two LDS arrays taken in turn (see block_sum1).  Every thread calls
// it the same number of times, so the parity is uniform.
struct CgSum {
    int parity = 0;
    __device__ __forceinline__ double operator()(double v) {
        __shared__ double scratch[2][MAX_WAVES];
        const double s = block_sum1(v, scratch[parity]);
        parity ^= 1;
        return s;
    }
};

#define NODE_LOOP(i, n) for (long long i = threadIdx.x; i < (n); i += blockDim.x)

// ---- CG-QN: the L-BFGS two-loop recursion in compact form -------------------
// H r (Nocedal and Wright, Alg. 7.4, H_0 = gamma I) for the kept pairs
// (s_k, y_k), oldest first, written with their Gram entries s_a.y_b (a < b)
// and y_a.y_b: the first loop's coefficients are
//   alpha_k = rho_k (s_k.r - sum_{j>k} alpha_j s_k.y_j),
// the second loop's
//   beta_k = rho_k (gamma (y_k.r - sum_j alpha_j y_k.y_j)
//                   + sum_{j<k} (alpha_j - beta_j) s_j.y_k),
// and H r = gamma (r - sum_k alpha_k y_k) + sum_k (alpha_k - beta_k) s_k.
// The same terms as the two loops, summed in another order: an application
// needs one batched reduction of the 2m products s_k.r, y_k.r instead of 2m
// block sums in sequence.  The Gram entries are formed once, when the pairs
// are kept, and stored after rho in the state.

struct QnLds {
    double scr[MAX_WAVES][2 * QN_MAX];   // wave totals of a batched sum
    double tot[2 * QN_MAX];              // its block totals
    double rho[QN_MAX], cs[QN_MAX], cy[QN_MAX];
    double sy[QN_MAX * QN_MAX], yy[QN_MAX * QN_MAX];
};

// L.tot[k] = the block sum of v(k) for k < cnt <= 2 QN_MAX, each wave's part
// by DPP and the waves in order; two barriers, all threads must call.
template <class F> __device__ __forceinline__ void qn_sums(QnLds &L, int cnt, F v) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    for (int k = 0; k < cnt; ++k) {
        const double w = wave_sum(v(k));
        if (lane == 0) L.scr[wid][k] = w;
    }
    __syncthreads();
    if (threadIdx.x < cnt) {
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += L.scr[w][threadIdx.x];
        L.tot[threadIdx.x] = t;
    }
    __syncthreads();
}

// Coefficients of H r from L.tot[2k] = s_k.r, L.tot[2k+1] = y_k.r, by the
// first wave (lane k owns pair k; the recurrences broadcast each new
// coefficient by a lane read and update the open sums of the other lanes):
// H r = gamma r + sum_k (cs_k s_k + cy_k y_k).
__device__ __forceinline__ void qn_coeffs(QnLds &L, int np, double gam) {
    const int l = threadIdx.x;
    const bool on = l < np;
    // first loop, k = np-1 .. 0: t_l = s_l.r - sum_{j>l} alpha_j s_l.y_j
    double t = on ? L.tot[2 * l] : 0.0, al = 0.0;
    for (int k = np - 1; k >= 0; --k) {
        const double ak = L.rho[k] * read_lane(t, k);
        if (l == k) al = ak;
        if (on && l < k) t -= ak * L.sy[l * QN_MAX + k];
    }
    // y_l.q with q = r - sum_j alpha_j y_j
    double yq = on ? L.tot[2 * l + 1] : 0.0;
    for (int j = 0; j < np; ++j) {
        const double aj = read_lane(al, j);
        if (on) yq -= aj * L.yy[l * QN_MAX + j];
    }
    // second loop, k = 0 .. np-1: u_l = gamma y_l.q + sum_{j<l} (alpha_j - beta_j) s_j.y_l
    double u = gam * yq, be = 0.0;
    for (int k = 0; k < np; ++k) {
        const double bk = L.rho[k] * read_lane(u, k);
        const double dk = read_lane(al, k) - bk;
        if (l == k) be = bk;
        if (on && l > k) u += dk * L.sy[k * QN_MAX + l];
    }
    if (on) {
        L.cs[l] = al - be;
        L.cy[l] = -gam * al;
    }
}

// Load rho and the Gram entries of np kept pairs from the state into LDS.
__device__ __forceinline__ void qn_load(QnLds &L, const double *st, int np) {
    if ((int)threadIdx.x < np) L.rho[threadIdx.x] = st[3 + threadIdx.x];
    for (int t = threadIdx.x; t < np * np; t += blockDim.x) {
        const int a = t / np, b = t % np;
        L.sy[a * QN_MAX + b] = st[QN_OFF_SY + a * QN_MAX + b];
        L.yy[a * QN_MAX + b] = st[QN_OFF_YY + a * QN_MAX + b];
    }
}

// Gram entries of the np pairs just kept, to LDS and the state; dot(k, a, b)
// returns this thread's part of y_a.y_b (k = 0) or s_a.y_b (k = 1).
template <class D> __device__ __forceinline__ void qn_gram(QnLds &L, double *st, int np, D dot) {
    for (int a = 0; a < np; ++a) {
        const int cnt = 2 * (np - a);
        qn_sums(L, cnt, [&](int k) -> double { return dot(k & 1, a, a + (k >> 1)); });
        if ((int)threadIdx.x < cnt) {
            const int b = a + ((int)threadIdx.x >> 1);
            const double v = L.tot[threadIdx.x];
            if (threadIdx.x & 1) {
                L.sy[a * QN_MAX + b] = v;
                st[QN_OFF_SY + a * QN_MAX + b] = v;
            } else {
                L.yy[a * QN_MAX + b] = v;
                L.yy[b * QN_MAX + a] = v;
                st[QN_OFF_YY + a * QN_MAX + b] = v;
                st[QN_OFF_YY + b * QN_MAX + a] = v;
            }
        }
    }
    __syncthreads();
}

template <int DIM, int KIND, int MODE, typename T>
__global__ __launch_bounds__(CBLOCK) void k_coarse(Grid g, Phys ph, const T *kap, const T *x, const T *Ax,
                                                   const double *num, const T *b, T *s, T *work, CoarseArgs ca) {
    constexpr int NC = (KIND == JFNK_NEOHOOKE) ? 3 : 1;
    constexpr int NV = Cell<DIM>::NV;
    const long long nn = g.nn, n = nn * NC;
    const long long ne = (long long)g.nx * g.ny * (DIM == 3 ? g.nz : 1);
    // r, p, q, z, then the element contributions ew[(c * ne + e) * NV + a]
    T *r = work, *p = work + n, *q = work + 2 * n, *z = work + 3 * n, *ew = work + 4 * n;
    CgSum cg_bsum;
    const double epsn = *num;
    const T h = (T)g.h;
    const double rnx = 1.0 / g.nx, rny = 1.0 / g.ny;

    // q = (J - shift I) v via the FD quotient, given vv = v.v.  Every element
    // is evaluated once (its corner contributions go to ew); each node then
    // sums the contributions of its adjacent elements in a fixed order.
    auto apply = [&](const T *v, double vv, double shift) __attribute__((always_inline)) {
        const double eps = vv > 0.0 ? epsn / sqrt(vv) : 0.0;
        const T e = (T)eps;
        const bool zero_fd = eps == 0.0;
        if constexpr (KIND == JFNK_NEOHOOKE) {
            // eight lanes per element, one per Gauss point, summed by a fixed
            // butterfly; every lane runs the same rounds (wave-uniform exchanges)
            const long long tot = ne * 8;
            const long long rounds = (tot + blockDim.x - 1) / blockDim.x;
            for (long long k = 0; k < rounds; ++k) {
                const long long t = threadIdx.x + k * blockDim.x;
                const bool live = t < tot && !zero_fd;
                const long long el = t < tot ? (t >> 3) : 0;
                const int gq = (int)(t & 7);
                T r8[NC][NV];
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int a = 0; a < NV; ++a) r8[c][a] = T(0);
                if (live) {
                    unsigned qq, rr, q2, r2;
                    udivmod((unsigned)el, (unsigned)g.nx, rnx, qq, rr);
                    udivmod(qq, (unsigned)g.ny, rny, q2, r2);
                    const int ex = (int)rr, ey = (int)r2, ez = (int)q2;
                    T xe[NC][NV], ve[NC][NV];
#pragma unroll
                    for (int a = 0; a < NV; ++a) {
                        const int ax = ex + (a & 1), ay = ey + ((a >> 1) & 1), az = ez + ((a >> 2) & 1);
                        const long long j = node_index(g, ax, ay, az);
                        const bool dj = is_dirichlet(g, ax, ay, az);
#pragma unroll
                        for (int c = 0; c < NC; ++c) {
                            xe[c][a] = x[c * nn + j];
                            ve[c][a] = dj ? T(0) : v[c * nn + j];
                        }
                    }
                    if constexpr (MODE == M_FD_DIFF) {
                        nh_point_fd<T>(xe, ve, e, ph, h, gq, r8);
                    } else {
                        T w[NC][NV];
#pragma unroll
                        for (int c = 0; c < NC; ++c)
#pragma unroll
                            for (int a = 0; a < NV; ++a) w[c][a] = xe[c][a] + e * ve[c][a];
                        nh_point<T>(w, ph, h, gq, r8);
                    }
                }
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int a = 0; a < NV; ++a) {
                        T val = r8[c][a];
                        val += __shfl_xor(val, 1);
                        val += __shfl_xor(val, 2);
                        val += __shfl_xor(val, 4);
                        r8[c][a] = val;
                    }
                if (t < tot && gq == 0) {
#pragma unroll
                    for (int c = 0; c < NC; ++c)
#pragma unroll
                        for (int a = 0; a < NV; ++a) ew[(c * ne + el) * NV + a] = zero_fd ? T(0) : r8[c][a];
                }
            }
        } else NODE_LOOP(el, ne) {
            unsigned qq, rr, q2, r2;
            udivmod((unsigned)el, (unsigned)g.nx, rnx, qq, rr);
            udivmod(qq, (unsigned)g.ny, rny, q2, r2);
            const int ex = (int)rr, ey = DIM == 3 ? (int)r2 : (int)qq, ez = DIM == 3 ? (int)q2 : 0;
            T xe[NC][NV], ve[NC][NV], kp[NV], r8[NC][NV];
#pragma unroll
            for (int a = 0; a < NV; ++a) {
                const int ax = ex + (a & 1), ay = ey + ((a >> 1) & 1), az = ez + ((a >> 2) & 1);
                const long long j = node_index(g, ax, ay, az);
                const bool dj = is_dirichlet(g, ax, ay, az);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    xe[c][a] = x[c * nn + j];
                    ve[c][a] = dj ? T(0) : v[c * nn + j];
                }
                kp[a] = (KIND == JFNK_INVCOEF) ? kap[j] : T(0);
            }
            if (!zero_fd) elem_eval<DIM, KIND, MODE, T, NC, NV>(xe, ve, kp, e, ph, h, r8);
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int a = 0; a < NV; ++a) ew[(c * ne + el) * NV + a] = zero_fd ? T(0) : r8[c][a];
        }
        __syncthreads();
        NODE_LOOP(i, nn) {
            int X, Y, Z;
            node_coords(g, i, X, Y, Z);
            const bool dir = is_dirichlet(g, X, Y, Z);
            T val[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) val[c] = T(0);
            if (!dir && !zero_fd) {
#pragma unroll
                for (int a = 0; a < NV; ++a) {   // the element whose corner a is this node
                    const int ex = X - (a & 1), ey = Y - ((a >> 1) & 1), ez = DIM == 3 ? Z - ((a >> 2) & 1) : 0;
                    if (ex < 0 || ex >= g.nx || ey < 0 || ey >= g.ny) continue;
                    if (DIM == 3 && (ez < 0 || ez >= g.nz)) continue;
                    const long long el = ((long long)ez * g.ny + ey) * g.nx + ex;
#pragma unroll
                    for (int c = 0; c < NC; ++c) val[c] += ew[(c * ne + el) * NV + a];
                }
                if constexpr (MODE == M_FD_PLAIN) {
#pragma unroll
                    for (int c = 0; c < NC; ++c) val[c] = (val[c] - Ax[c * nn + i]) * (T)(1.0 / eps);
                }
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const long long k = c * nn + i;
                q[k] = dir ? T(0) : val[c] - (T)shift * v[k];
            }
        }
        __syncthreads();
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

    // L-BFGS preconditioner (CG-QN), as in k_coarse_small below but with the
    // vectors, recorded steps and pairs in global memory (entry k of a pair
    // is touched by the thread that owns entry k of every vector)
    T *rec_s = (T *)ca.qn_rec, *rec_y = rec_s ? rec_s + (size_t)ca.qn_cap * n : nullptr;
    T *ps = (T *)ca.qn_pairs, *py = ps ? ps + (size_t)ca.qn_m * n : nullptr;
    __shared__ QnLds L;
    const bool qn_on = ca.qn_m > 0;
    bool recording = qn_on && ca.qn_state[0] == 0.0;
    int np = (qn_on && !recording) ? (int)ca.qn_state[1] : 0;
    double gam = np > 0 ? ca.qn_state[2] : 1.0;
    if (np > 0) qn_load(L, ca.qn_state, np);
    __syncthreads();
    int nrec = 0;
    // z = H r by the compact recursion (np > 0)
    auto prec = [&]() __attribute__((always_inline)) {
        qn_sums(L, 2 * np, [&](int k) -> double {
            const T *w = ((k & 1) ? py : ps) + (size_t)(k >> 1) * n;
            double d = 0.0;
            NODE_LOOP(i, n) d += (double)w[i] * (double)r[i];
            return d;
        });
        if (threadIdx.x < 64) qn_coeffs(L, np, gam);
        __syncthreads();
        NODE_LOOP(i, n) {
            T zi = (T)gam * r[i];
            for (int k = 0; k < np; ++k) zi += (T)L.cs[k] * ps[(size_t)k * n + i] + (T)L.cy[k] * py[(size_t)k * n + i];
            z[i] = zi;
        }
    };

    auto cg = [&](double shift) __attribute__((always_inline)) -> double {
        if (s_nonzero) {
            double ss = 0.0;
            NODE_LOOP(i, n) ss += (double)s[i] * (double)s[i];
            apply(s, cg_bsum(ss), shift);
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
        double pp = rr;             // ||p||^2, carried from the p update
        double rz = rr;             // r.z (z = r without pairs)
        if (np > 0) {
            prec();
            double d1 = 0.0, d2 = 0.0;
            NODE_LOOP(i, n) {
                p[i] = z[i];
                d1 += (double)r[i] * (double)z[i];
                d2 += (double)z[i] * (double)z[i];
            }
            rz = cg_bsum(d1);
            pp = cg_bsum(d2);
        }
        for (int it = 1; it <= ca.maxit; ++it) {
            apply(p, pp, shift);
            ++fd;
            ++iters;
            double pq = 0.0;
            NODE_LOOP(i, n) pq += (double)p[i] * (double)q[i];
            pq = cg_bsum(pq);
            if (pq <= 0.0) return pq / pp;
            const double alpha = rz / pq;
            const T a = (T)alpha;
            if (recording && nrec < ca.qn_cap) {
                T *rs = rec_s + (size_t)nrec * n, *ry = rec_y + (size_t)nrec * n;
                NODE_LOOP(i, n) {
                    rs[i] = a * p[i];
                    ry[i] = a * q[i];
                }
                ++nrec;
            }
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
            double pn = 0.0;
            if (np > 0) {
                prec();
                double d = 0.0;
                NODE_LOOP(i, n) d += (double)r[i] * (double)z[i];
                const double rzn = cg_bsum(d);
                const T beta = (T)(rzn / rz);
                NODE_LOOP(i, n) {
                    const T pi = z[i] + beta * p[i];
                    p[i] = pi;
                    pn += (double)pi * (double)pi;
                }
                rz = rzn;
            } else {
                const T beta = (T)(rn / rz);
                NODE_LOOP(i, n) {
                    const T pi = r[i] + beta * p[i];
                    p[i] = pi;
                    pn += (double)pi * (double)pi;
                }
                rz = rn;
            }
            pp = cg_bsum(pn);
        }
        return 0.0;
    };

    // after the recording CG: keep the uniform sample floor(k t / m) with
    // positive curvature, oldest first; rho_k and gamma to the state
    auto keep_pairs = [&]() __attribute__((always_inline)) {
        const int t = nrec, m = ca.qn_m;
        const int nsel = t <= m ? t : m;
        int kept = 0;
        double g_s = 0.0;
        for (int k = 0; k < nsel; ++k) {
            const int src = t <= m ? k : (int)(((long long)k * t) / m);
            const T *rs = rec_s + (size_t)src * n, *ry = rec_y + (size_t)src * n;
            double d = 0.0;
            NODE_LOOP(i, n) d += (double)rs[i] * (double)ry[i];
            const double sy = cg_bsum(d);
            if (sy > 0.0) {
                double d2 = 0.0;
                T *qs = ps + (size_t)kept * n, *qy = py + (size_t)kept * n;
                NODE_LOOP(i, n) {
                    qs[i] = rs[i];
                    qy[i] = ry[i];
                    d2 += (double)ry[i] * (double)ry[i];
                }
                const double yy = cg_bsum(d2);
                if (threadIdx.x == 0) {
                    ca.qn_state[3 + kept] = 1.0 / sy;
                    L.rho[kept] = 1.0 / sy;
                }
                g_s = sy / yy;
                ++kept;
            }
        }
        if (threadIdx.x == 0) {
            ca.qn_state[0] = 1.0;
            ca.qn_state[1] = (double)kept;
            ca.qn_state[2] = kept > 0 ? g_s : 1.0;
        }
        __threadfence_block();
        __syncthreads();
        qn_gram(L, ca.qn_state, kept, [&](int sy, int a, int b) -> double {
            const T *u = (sy ? ps : py) + (size_t)a * n, *w = py + (size_t)b * n;
            double d = 0.0;
            NODE_LOOP(i, n) d += (double)u[i] * (double)w[i];
            return d;
        });
        np = kept;
        gam = kept > 0 ? g_s : 1.0;
        recording = false;
    };

    double shift = 0.0;
    double lam_c = cg(shift);
    if (recording) {
        __syncthreads();
        keep_pairs();
    }
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

// The same solver for a scalar coarse level with at most CBLOCK nodes: thread
// i owns node i and keeps its entries of r, p, q, s, b in registers; the
// state x, e^m, the direction being applied and the element contributions
// live in LDS, so an iteration touches no global memory.
template <int DIM, int KIND, int MODE, typename T>
__global__ __launch_bounds__(CBLOCK) void k_coarse_small(Grid g, Phys ph, const T *kap, const T *x, const T *Ax,
                                                         const double *num, const T *b, T *s_out, CoarseArgs ca) {
    constexpr int NV = Cell<DIM>::NV;
    constexpr bool INV = KIND == JFNK_INVCOEF;
    extern __shared__ __align__(16) unsigned char smem[];
    const int nn = (int)g.nn;
    const int ne = g.nx * g.ny * (DIM == 3 ? g.nz : 1);
    T *sx = (T *)smem, *sv = sx + nn, *sk = sv + nn, *ew = sk + (INV ? nn : 0);
    const int i = threadIdx.x;
    const bool act = i < nn;
    CgSum cg_bsum;
    const double epsn = *num;
    const T h = (T)g.h;
    int X = 0, Y = 0, Z = 0;
    bool dir = true;
    T bi = T(0), axi = T(0);
    if (act) {
        node_coords(g, i, X, Y, Z);
        dir = is_dirichlet(g, X, Y, Z);
        sx[i] = x[i];
        if (INV) sk[i] = kap[i];
        bi = b[i];
        if (MODE == M_FD_PLAIN) axi = Ax[i];
    }
    // this thread's element (if any): element i of the level
    int ex = 0, ey = 0, ez = 0;
    const bool has_el = i < ne;
    if (has_el) {
        ex = i % g.nx;
        const int rest = i / g.nx;
        ey = DIM == 3 ? rest % g.ny : rest;
        ez = DIM == 3 ? rest / g.ny : 0;
    }
    __syncthreads();

    // q_i = ((J - shift I) v)_i for the direction whose entry here is vi, vv = v.v
    auto apply = [&](T vi, double vv, double shift) __attribute__((always_inline)) -> T {
        const double eps = vv > 0.0 ? epsn / sqrt(vv) : 0.0;
        const T e = (T)eps;
        if (act) sv[i] = dir ? T(0) : vi;
        __syncthreads();
        if (has_el && eps != 0.0) {
            T xe[1][NV], ve[1][NV], kp[NV], r8[1][NV];
#pragma unroll
            for (int a = 0; a < NV; ++a) {
                const int j = (int)node_index(g, ex + (a & 1), ey + ((a >> 1) & 1), ez + ((a >> 2) & 1));
                xe[0][a] = sx[j];
                ve[0][a] = sv[j];
                kp[a] = INV ? sk[j] : T(0);
            }
            elem_eval<DIM, KIND, MODE, T, 1, NV>(xe, ve, kp, e, ph, h, r8);
#pragma unroll
            for (int a = 0; a < NV; ++a) ew[a * ne + i] = r8[0][a];
        }
        __syncthreads();
        T val = T(0);
        if (act && !dir && eps != 0.0) {
#pragma unroll
            for (int a = 0; a < NV; ++a) {   // the element whose corner a is this node
                const int cx = X - (a & 1), cy = Y - ((a >> 1) & 1), cz = DIM == 3 ? Z - ((a >> 2) & 1) : 0;
                if (cx < 0 || cx >= g.nx || cy < 0 || cy >= g.ny) continue;
                if (DIM == 3 && (cz < 0 || cz >= g.nz)) continue;
                val += ew[a * ne + (cz * g.ny + cy) * g.nx + cx];
            }
            if constexpr (MODE == M_FD_PLAIN) val = (val - axi) * (T)(1.0 / eps);
        }
        return dir ? T(0) : val - (T)shift * vi;
    };

    const double bb = cg_bsum((double)bi * (double)bi);
    const double tol = fmax(ca.atol, ca.rtol * sqrt(bb));
    long long fd = 0, iters = 0;
    bool s_nonzero = false;
    T si = T(0), ri = T(0), pi = T(0), qi = T(0);

    // L-BFGS preconditioner (CG-QN): the first solve with no pairs records
    // every step of its first CG; pairs kept afterwards precondition all CG
    // runs (the compact two-loop recursion, H_0 = gamma I of the newest
    // pair).  Each lane touches only its own node's pair entries; the
    // coefficients and Gram entries live in LDS.
    T *rec_s = (T *)ca.qn_rec, *rec_y = rec_s ? rec_s + (size_t)ca.qn_cap * nn : nullptr;
    T *ps = (T *)ca.qn_pairs, *py = ps ? ps + (size_t)ca.qn_m * nn : nullptr;
    __shared__ QnLds L;
    const bool qn_on = ca.qn_m > 0;
    bool recording = qn_on && ca.qn_state[0] == 0.0;
    int np = (qn_on && !recording) ? (int)ca.qn_state[1] : 0;
    double gam = np > 0 ? ca.qn_state[2] : 1.0;
    if (np > 0) qn_load(L, ca.qn_state, np);
    __syncthreads();
    int nrec = 0;
    auto prec = [&](T r) __attribute__((always_inline)) -> T {
        if (np == 0) return r;
        qn_sums(L, 2 * np, [&](int k) -> double {
            const T w = act ? ((k & 1) ? py : ps)[(size_t)(k >> 1) * nn + i] : T(0);
            return (double)w * (double)r;
        });
        if (threadIdx.x < 64) qn_coeffs(L, np, gam);
        __syncthreads();
        T z = (T)gam * r;
        for (int k = 0; k < np; ++k) {
            const T sk = act ? ps[(size_t)k * nn + i] : T(0), yk = act ? py[(size_t)k * nn + i] : T(0);
            z += (T)L.cs[k] * sk + (T)L.cy[k] * yk;
        }
        return z;
    };

    auto cg = [&](double shift) __attribute__((always_inline)) -> double {
        if (s_nonzero) {
            const double ss = cg_bsum((double)si * (double)si);
            qi = apply(si, ss, shift);
            ++fd;
            ri = bi - qi;
        } else {
            ri = bi;
        }
        double rr = cg_bsum((double)ri * (double)ri);
        if (sqrt(rr) <= tol) return 0.0;
        T zi = prec(ri);
        pi = zi;
        double rz = np > 0 ? cg_bsum((double)ri * (double)zi) : rr;
        double pp = np > 0 ? cg_bsum((double)pi * (double)pi) : rr;
        for (int it = 1; it <= ca.maxit; ++it) {
            qi = apply(pi, pp, shift);
            ++fd;
            ++iters;
            const double pq = cg_bsum((double)pi * (double)qi);
            if (pq <= 0.0) return pq / pp;
            const double alpha = rz / pq;
            const T a = (T)alpha;
            if (recording && nrec < ca.qn_cap) {
                if (act) {
                    rec_s[(size_t)nrec * nn + i] = a * pi;
                    rec_y[(size_t)nrec * nn + i] = a * qi;
                }
                ++nrec;
            }
            si += a * pi;
            ri -= a * qi;
            s_nonzero = true;
            const double rn = cg_bsum((double)ri * (double)ri);
            if (sqrt(rn) <= tol) return 0.0;
            zi = prec(ri);
            const double rzn = np > 0 ? cg_bsum((double)ri * (double)zi) : rn;
            const T beta = (T)(rzn / rz);
            pi = zi + beta * pi;
            pp = cg_bsum((double)pi * (double)pi);
            rz = rzn;
        }
        return 0.0;
    };

    // after the recording CG: keep the uniform sample floor(k t / m) with
    // positive curvature, oldest first; rho_k and gamma to the state
    auto keep_pairs = [&]() __attribute__((always_inline)) {
        const int t = nrec, m = ca.qn_m;
        const int nsel = t <= m ? t : m;
        int kept = 0;
        double g_s = 0.0;
        for (int k = 0; k < nsel; ++k) {
            const int src = t <= m ? k : (int)(((long long)k * t) / m);
            const T sk = act ? rec_s[(size_t)src * nn + i] : T(0), yk = act ? rec_y[(size_t)src * nn + i] : T(0);
            const double sy = cg_bsum((double)sk * (double)yk);
            if (sy > 0.0) {
                const double yy = cg_bsum((double)yk * (double)yk);
                if (act) {
                    ps[(size_t)kept * nn + i] = sk;
                    py[(size_t)kept * nn + i] = yk;
                }
                if (threadIdx.x == 0) {
                    ca.qn_state[3 + kept] = 1.0 / sy;
                    L.rho[kept] = 1.0 / sy;
                }
                g_s = sy / yy;
                ++kept;
            }
        }
        if (threadIdx.x == 0) {
            ca.qn_state[0] = 1.0;
            ca.qn_state[1] = (double)kept;
            ca.qn_state[2] = kept > 0 ? g_s : 1.0;
        }
        __threadfence_block();
        __syncthreads();
        qn_gram(L, ca.qn_state, kept, [&](int sy, int a, int b) -> double {
            if (!act) return 0.0;
            return (double)(sy ? ps : py)[(size_t)a * nn + i] * (double)py[(size_t)b * nn + i];
        });
        np = kept;
        gam = kept > 0 ? g_s : 1.0;
        recording = false;
    };

    double shift = 0.0;
    double lam_c = cg(shift);
    if (recording) {
        __syncthreads();
        keep_pairs();
    }
    int rounds = 0;
    int negc = lam_c < 0.0 ? 1 : 0;
    while (lam_c < 0.0 && rounds < ca.shift_max) {
        shift = ca.gamma * fmin(lam_c, shift);
        lam_c = cg(shift);
        if (lam_c < 0.0) ++negc;
        ++rounds;
    }
    if (act) s_out[i] = si;
    if (threadIdx.x == 0) {
        ca.stats[0] = shift;
        ca.stats[1] += (double)iters;
        ca.stats[2] = rounds;
        ca.stats[3] += (double)fd;
        ca.stats[4] += (double)negc;
        ca.stats[5] += 1.0;
    }
}

static size_t coarse_small_lds(const Grid &g, int kind, size_t eb) {
    const long long ne = (long long)g.nx * g.ny * (g.dim == 3 ? g.nz : 1);
    return (size_t)((kind == JFNK_INVCOEF ? 3 : 2) * g.nn + (g.dim == 3 ? 8 : 4) * ne) * eb;
}
bool coarse_small(const Grid &g, int kind, size_t eb) {
    return kind != JFNK_NEOHOOKE && g.nn <= CBLOCK && coarse_small_lds(g, kind, eb) <= 64 * 1024;
}
// elements of the generic solver's work array: r, p, q, z and 2^d
// contributions per element and component
size_t coarse_work_elems(const Grid &g, int nc) {
    const long long ne = (long long)g.nx * g.ny * (g.dim == 3 ? g.nz : 1);
    return (size_t)(4 * g.nn * nc + (g.dim == 3 ? 8 : 4) * ne * nc);
}

// The small kernel's static LDS (the CG-QN arrays) plus up to 64 KB of
// dynamic LDS can pass the default 64 KB per workgroup: raise its dynamic
// limit once per device; if the runtime refuses, the generic kernel runs.
static bool coarse_lds_ok(const void *fn, size_t dyn) {
    static std::mutex mu;
    static std::map<std::pair<int, const void *>, bool> ok;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_pair(dev, fn);
    auto it = ok.find(key);
    if (it == ok.end()) {
        const bool r = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024) == hipSuccess;
        if (!r) (void)hipGetLastError();
        it = ok.emplace(key, r).first;
    }
    return it->second && dyn <= 64 * 1024;
}

template <int DIM, int KIND, typename T>
static void launch_coarse(const Exec &ex, int mode, const Grid &g, const Phys &ph, const T *kap, const T *x,
                          const T *Ax, const double *num, const T *b, T *s, T *work, const CoarseArgs &ca) {
    if constexpr (KIND != JFNK_NEOHOOKE) {
        const size_t lds = coarse_small_lds(g, KIND, sizeof(T));
        if (coarse_small(g, KIND, sizeof(T))) {
            if (mode == M_FD_DIFF) {
                const void *fn = (const void *)k_coarse_small<DIM, KIND, M_FD_DIFF, T>;
                if (coarse_lds_ok(fn, lds)) {
                    k_coarse_small<DIM, KIND, M_FD_DIFF, T><<<1, CBLOCK, lds, ex.st>>>(g, ph, kap, x, Ax, num, b, s,
                                                                                      ca);
                    return;
                }
            } else {
                const void *fn = (const void *)k_coarse_small<DIM, KIND, M_FD_PLAIN, T>;
                if (coarse_lds_ok(fn, lds)) {
                    k_coarse_small<DIM, KIND, M_FD_PLAIN, T><<<1, CBLOCK, lds, ex.st>>>(g, ph, kap, x, Ax, num, b,
                                                                                       s, ca);
                    return;
                }
            }
        }
    }
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
    case JFNK_PLAP_GAUSS:
        if (g.dim == 2) launch_coarse<2, JFNK_PLAP_GAUSS, T>(ex, mode, g, ph, kap, x, Ax, num, b, s, work, ca);
        else launch_coarse<3, JFNK_PLAP_GAUSS, T>(ex, mode, g, ph, kap, x, Ax, num, b, s, work, ca);
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
