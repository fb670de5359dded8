// FP64 instantiation of the stencil launchers, the mixed-precision outer
// Jacobian action (FP64 state, FP32 preconditioned direction), the energy
// and the exact vector-Jacobian products.
#define JFNK_T double
#include "ops_stencil.inc"

namespace jfnk {

template <>
void op_jv<double, float>(const Exec &ex, int mode, const Grid &g, const Phys &ph, const double *kap,
                          const double *x, const double *Ax, const float *v, const double *num, const double *vn2,
                          double eps_fixed, double *Jv) {
    dispatch_fd<double, float, EpiJv>(ex, mode, g, ph, kap, x, v, Ax, make_fd(ex, num, vn2, eps_fixed), Jv, g.nn);
}

// ---- energy: sum over elements of Psi_e(u) ----------------------------------
template <int DIM, int KIND>
__global__ __launch_bounds__(BLOCK) void k_energy(Grid g, Phys ph, const double *u, Red red, double *out) {
    constexpr int NV = Cell<DIM>::NV;
    constexpr int NC = (KIND == JFNK_NEOHOOKE) ? 3 : 1;
    const long long ne = (long long)g.nx * g.ny * (DIM == 3 ? g.nz : 1);
    double sum[1] = {0.0};
    const long long stride = (long long)gridDim.x * blockDim.x;
    const double rnx = 1.0 / g.nx, rny = 1.0 / g.ny;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += stride) {
        unsigned q, r, q2, r2;
        udivmod((unsigned)e, (unsigned)g.nx, rnx, q, r);
        udivmod(q, (unsigned)g.ny, rny, q2, r2);
        const int ex = (int)r, ey = (int)r2, ez = (int)q2;
        double w[NC][NV];
#pragma unroll
        for (int a = 0; a < NV; ++a) {
            const long long j = node_index(g, ex + (a & 1), ey + ((a >> 1) & 1), ez + ((a >> 2) & 1));
#pragma unroll
            for (int c = 0; c < NC; ++c) w[c][a] = u[c * g.nn + j];
        }
        if constexpr (KIND == JFNK_NEOHOOKE) sum[0] += elem_neohooke_energy<double>(w, ph, g.h);
        else sum[0] += elem_scalar_energy<DIM, KIND, double>(w[0], ph, g.h);
    }
    block_partials<1>(sum, red);
}

void op_energy(const Exec &ex, const Grid &g, const Phys &ph, const double *u, double *out) {
    const long long ne = (long long)g.nx * g.ny * (g.dim == 3 ? g.nz : 1);
    const int nb = node_blocks(ne);
    if (ph.kind == JFNK_BRATU && g.dim == 2) k_energy<2, JFNK_BRATU><<<nb, BLOCK, 0, ex.st>>>(g, ph, u, ex.red, out);
    else if (ph.kind == JFNK_BRATU) k_energy<3, JFNK_BRATU><<<nb, BLOCK, 0, ex.st>>>(g, ph, u, ex.red, out);
    else if (ph.kind == JFNK_PLAP && g.dim == 2) k_energy<2, JFNK_PLAP><<<nb, BLOCK, 0, ex.st>>>(g, ph, u, ex.red, out);
    else if (ph.kind == JFNK_PLAP) k_energy<3, JFNK_PLAP><<<nb, BLOCK, 0, ex.st>>>(g, ph, u, ex.red, out);
    else if (ph.kind == JFNK_NEOHOOKE) k_energy<3, JFNK_NEOHOOKE><<<nb, BLOCK, 0, ex.st>>>(g, ph, u, ex.red, out);
    else if (ph.kind == JFNK_PLAP_GAUSS && g.dim == 2)
        k_energy<2, JFNK_PLAP_GAUSS><<<nb, BLOCK, 0, ex.st>>>(g, ph, u, ex.red, out);
    else if (ph.kind == JFNK_PLAP_GAUSS) k_energy<3, JFNK_PLAP_GAUSS><<<nb, BLOCK, 0, ex.st>>>(g, ph, u, ex.red, out);
    finish<1>(ex.st, ex.red, nb, FinStore<1>{out});
}

// ---- exact VJP ---------------------------------------------------------------------
// wrt 0: out_i = sum_e (J_e^T lam_e)_{a(i)} on DoFs (lam taken as 0 on Dirichlet nodes)
// wrt 1: out_i = e^{m_i} sum_e (1 + ubar_e^2)(lam_e^T K_e u_e) / 2^d at every node
// (both times scale: -1 gives the coefficient gradient -(dF/dm)^T lam exactly)
template <int DIM, int KIND>
__global__ __launch_bounds__(BLOCK) void k_vjp(Grid g, Phys ph, const double *kap, const double *u,
                                               const double *lam, int wrt, double scale, double *out) {
    constexpr int NV = Cell<DIM>::NV;
    constexpr int NC = (KIND == JFNK_NEOHOOKE) ? 3 : 1;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.nn; i += stride) {
        int x, y, z;
        node_coords(g, i, x, y, z);
        const bool dir = is_dirichlet(g, x, y, z);
        double acc[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = 0.0;
        if (wrt == 0 && dir) {
#pragma unroll
            for (int c = 0; c < NC; ++c) out[c * g.nn + i] = 0.0;
            continue;
        }
        for (int e = 0; e < NV; ++e) {
            const int ex = x - (e & 1), ey = y - ((e >> 1) & 1), ez = (DIM == 3) ? z - ((e >> 2) & 1) : 0;
            if (ex < 0 || ex >= g.nx || ey < 0 || ey >= g.ny) continue;
            if (DIM == 3 && (ez < 0 || ez >= g.nz)) continue;
            double w[NC][NV], l[NC][NV], kp[NV];
#pragma unroll
            for (int a = 0; a < NV; ++a) {
                const int ax = ex + (a & 1), ay = ey + ((a >> 1) & 1), az = ez + ((a >> 2) & 1);
                const long long j = node_index(g, ax, ay, az);
                const bool dj = is_dirichlet(g, ax, ay, az);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    w[c][a] = u[c * g.nn + j];
                    l[c][a] = dj ? 0.0 : lam[c * g.nn + j];
                }
                kp[a] = (KIND == JFNK_INVCOEF) ? kap[j] : 0.0;
            }
            if constexpr (KIND == JFNK_NEOHOOKE) {
                double r[3][8];
                elem_neohooke_jvp<double>(w, l, ph, g.h, r);
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[c] += r[c][e];
            } else if (KIND == JFNK_INVCOEF) {
                if (wrt == 1) {
                    acc[0] += elem_coef_factor<DIM, double>(w[0], l[0], g.h);
                } else {
                    double r[NV];
                    elem_scalar_vjp<DIM, KIND, double>(w[0], kp, l[0], ph, g.h, r);
                    acc[0] += r[e];
                }
            } else {
                double r[NV];
                elem_scalar_vjp<DIM, KIND, double>(w[0], kp, l[0], ph, g.h, r);
                acc[0] += r[e];
            }
        }
        if (wrt == 1) acc[0] *= kap[i];
#pragma unroll
        for (int c = 0; c < NC; ++c) out[c * g.nn + i] = scale * acc[c];
    }
}

void op_vjp(const Exec &ex, const Grid &g, const Phys &ph, const double *kap, const double *u, const double *lam,
            int wrt, double *out, double scale) {
    const int nb = node_blocks(g.nn);
    switch (ph.kind) {
    case JFNK_BRATU:
        if (g.dim == 2) k_vjp<2, JFNK_BRATU><<<nb, BLOCK, 0, ex.st>>>(g, ph, kap, u, lam, wrt, scale, out);
        else k_vjp<3, JFNK_BRATU><<<nb, BLOCK, 0, ex.st>>>(g, ph, kap, u, lam, wrt, scale, out);
        break;
    case JFNK_PLAP:
        if (g.dim == 2) k_vjp<2, JFNK_PLAP><<<nb, BLOCK, 0, ex.st>>>(g, ph, kap, u, lam, wrt, scale, out);
        else k_vjp<3, JFNK_PLAP><<<nb, BLOCK, 0, ex.st>>>(g, ph, kap, u, lam, wrt, scale, out);
        break;
    case JFNK_INVCOEF:
        if (g.dim == 2) k_vjp<2, JFNK_INVCOEF><<<nb, BLOCK, 0, ex.st>>>(g, ph, kap, u, lam, wrt, scale, out);
        else k_vjp<3, JFNK_INVCOEF><<<nb, BLOCK, 0, ex.st>>>(g, ph, kap, u, lam, wrt, scale, out);
        break;
    case JFNK_NEOHOOKE:
        k_vjp<3, JFNK_NEOHOOKE><<<nb, BLOCK, 0, ex.st>>>(g, ph, kap, u, lam, wrt, scale, out);
        break;
    case JFNK_PLAP_GAUSS:
        if (g.dim == 2) k_vjp<2, JFNK_PLAP_GAUSS><<<nb, BLOCK, 0, ex.st>>>(g, ph, kap, u, lam, wrt, scale, out);
        else k_vjp<3, JFNK_PLAP_GAUSS><<<nb, BLOCK, 0, ex.st>>>(g, ph, kap, u, lam, wrt, scale, out);
        break;
    }
}

}  // namespace jfnk
