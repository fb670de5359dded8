// Row-marching LDS-tiled evaluation for 3D levels of the scalar kinds.
//
// A block spans the whole x extent of the level: thread t owns the element
// column ex = t (ceil(nx / 64) wavefronts, so every global access is a
// coalesced row) and a tile of a few node rows in y and a chunk of
// node planes in z.  The block marches up in z with the two node planes
// that bound the current element layer in LDS (state x, direction v,
// coefficient e^m), one halo row on each side in y.  For every element
// layer each thread walks its column through the tile's element rows,
// keeping the shared corner row in registers, so every element of the tile
// is evaluated exactly once and the y and z neighbours of a node are summed
// in registers.  The contributions that belong to the node column t + 1 are
// handed over once per node through a small LDS row buffer.  Because a
// block covers all of x, a level with 2^k + 1 nodes per row costs no
// partial tile in x; in y and z the tiles are sized evenly.
//
// The next plane is fetched into registers before the element layer is
// evaluated and written to LDS afterwards, so its global latency overlaps
// the arithmetic.  Tiles are numbered y-fastest inside each z chunk and
// workgroup ids are remapped so the blocks dispatched to one XCD (ids are
// dealt round-robin over the 8 XCDs) own a contiguous range of tiles,
// keeping the shared halo rows in that XCD's L2.
#pragma once
#include "stencil.hpp"

namespace jfnk {

// node rows per tile (register arrays), chosen by measurement at 256^3:
// FP32 4 (under 128 VGPRs, 4 waves per SIMD; faster than 3, 5, 6 or 8
// despite the larger y halo); FP64: 4 for the plain FD quotient without
// epilogue inputs (the outer J v: 166 VGPRs, 3 waves per SIMD, faster than
// 6 rows at 2 waves), 3 for the residual (124 VGPRs, 4 waves per SIMD),
// 4 otherwise.  The FP64 Gauss-point p-Laplacian takes 3 in every mode
// (p = 3 instantiation: the residual at 136 VGPRs, 3 waves per SIMD, beats
// 2 rows at 116 VGPRs and 4 waves, 346 against 379 us at 256^3; in the FD
// modes 2 rows gain no occupancy and 4 spill).
constexpr int GAUSS_ROWS64 = 3;
template <typename T, int MODE, class Epi, int KIND> struct TileRows {
    static constexpr bool jv64 = sizeof(T) == 8 && MODE == M_FD_PLAIN && Epi::NIN == 0;
    static constexpr bool res64 = sizeof(T) == 8 && MODE == M_RESID;
    static constexpr bool gauss64 = sizeof(T) == 8 && KIND == JFNK_PLAP_GAUSS;
    static constexpr int value = gauss64 ? GAUSS_ROWS64 : (jv64 ? 4 : (res64 ? 3 : 4));
};
constexpr int TMAX_THREADS = 512;   // nx <= 512 elements per row

struct TileArgs {
    int nty, ntz;      // tiles along y and z
    int pitch;         // LDS row pitch in entries (>= NX)
    int srows;         // rows per LDS plane slot (node rows + 2)
};

__device__ __forceinline__ int xcd_tile(int id, int nb) {
    const int q = nb / 8, r = nb % 8;
    const int xcd = id % 8, loc = id / 8;
    return xcd < r ? xcd * (q + 1) + loc : r * (q + 1) + (xcd - r) * q + loc;
}

// Dynamic LDS of one block: two plane slots of x (T), e^m (T, INVCOEF) and
// v (TV, FD modes), plus the (tile rows) x pitch hand-over buffer (T).
template <typename T, typename TV, int MODE, class Epi, int KIND>
inline size_t tiled_lds_bytes(int pitch, int srows) {
    constexpr bool FD = MODE != M_RESID;
    constexpr bool INV = KIND == JFNK_INVCOEF;
    const size_t plane = (size_t)srows * pitch;
    return 2 * plane * sizeof(T) * (INV ? 2 : 1) + (size_t)TileRows<T, MODE, Epi, KIND>::value * pitch * sizeof(T) +
           (FD ? 2 * plane * sizeof(TV) : 0);
}

// PF = 3: p-Laplacian with p = 3 fixed at compile time (no exponent branches)
template <int KIND, int MODE, typename T, typename TV, class Epi, int PF = 0>
__global__ __launch_bounds__(TMAX_THREADS) void k_tiled(Grid g, Phys ph, const T *kap, const T *x, const TV *v,
                                                        const T *Ax, FdStep fd, Epi epi, Red red, TileArgs ta) {
    constexpr bool FD = MODE != M_RESID;
    constexpr bool INV = KIND == JFNK_INVCOEF;
    constexpr int R = TileRows<T, MODE, Epi, KIND>::value;
    extern __shared__ __align__(16) unsigned char smem[];
    const int P = ta.pitch;
    const int plane = ta.srows * P;
    T *sx = (T *)smem;                            // [2][plane]
    T *sk = sx + 2 * plane;                       // [2][plane] (INVCOEF)
    T *xb = sk + (INV ? 2 * plane : 0);           // [R][P] hand-over rows
    TV *sv = (TV *)(xb + R * P);                  // [2][plane] (FD)

    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tiy = tile % ta.nty, tiz = tile / ta.nty;
    const int y0 = (int)((long long)tiy * g.NY / ta.nty), y1 = (int)((long long)(tiy + 1) * g.NY / ta.nty);
    const int z0 = (int)((long long)tiz * g.NZ / ta.ntz), z1 = (int)((long long)(tiz + 1) * g.NZ / ta.ntz);
    const int rows = y1 - y0;
    const int t = threadIdx.x, nthr = blockDim.x;
    const double eps = fd_eps_prepare(fd, epi);
    const bool zero_fd = FD && eps == 0.0;
    const T e = (T)eps;
    const T ie = eps > 0.0 ? (T)(1.0 / eps) : T(0);
    const T h = (T)g.h;
    double sums[Epi::NS > 0 ? Epi::NS : 1];
#pragma unroll
    for (int k = 0; k < (Epi::NS > 0 ? Epi::NS : 1); ++k) sums[k] = 0.0;

    const bool own_col = t < g.NX;                 // loads and outputs node column t
    const bool own_elem = t < g.nx;                // evaluates element column t
    const bool extra = g.NX > nthr;                // column nx (= nthr) needs an extra loader
    const bool xdir_t = ((g.dir & JFNK_FACE_XLO) && t == 0) || ((g.dir & JFNK_FACE_XHI) && t == g.nx);
    const bool xdir_e = (g.dir & JFNK_FACE_XHI) != 0;   // column nx
    auto ydir = [&](int gy) { return ((g.dir & JFNK_FACE_YLO) && gy == 0) || ((g.dir & JFNK_FACE_YHI) && gy == g.ny); };
    auto zdir = [&](int gz) { return ((g.dir & JFNK_FACE_ZLO) && gz == 0) || ((g.dir & JFNK_FACE_ZHI) && gz == g.nz); };

    // Block-uniform row flags, bit r for the LDS row r (grid row y0 - 1 + r):
    // rfree: inside the grid and not a Dirichlet row (direction entries are
    // free there); eok: element row y0 - 1 + r inside the grid; odir: output
    // row y0 + r on a Dirichlet face.  Lane factors: vlane switches off the
    // direction entries of a column outside the grid or on a Dirichlet face
    // in x, elane the element of a column outside the grid.
    unsigned rfree = 0, eok = 0, odir = 0;
#pragma unroll
    for (int r = 0; r < R + 2; ++r) {
        const int gy = y0 - 1 + r;
        if (gy >= 0 && gy < g.NY && !ydir(gy)) rfree |= 1u << r;
        if (r <= R && gy >= 0 && gy < g.ny) eok |= 1u << r;
        if (r < R && ydir(y0 + r)) odir |= 1u << r;
    }
    const TV vlane = (own_col && !xdir_t) ? TV(1) : TV(0);
    const T elane = own_elem ? T(1) : T(0);

    // Block-uniform scalars used inside the plane loop.  They pass an empty
    // register barrier at the top of every iteration, so what the compiler
    // derives from them (row offsets, row and face tests) is recomputed there
    // by scalar instructions instead of being kept live, as dozens of scalar
    // registers, across the loop.
    auto sc = [](int v) { return __builtin_amdgcn_readfirstlane(v); };
    int uNX = sc(g.NX), uNY = sc(g.NY), uNZ = sc(g.NZ), unx = sc(g.nx), unz = sc(g.nz), udir = sc(g.dir);
    int uy0 = sc(y0), urows = sc(rows), usrows = sc(ta.srows);
    unsigned ufree = sc(rfree), ueok = sc(eok), uodir = sc(odir);
    // (the barrier's outputs count as divergent to the compiler, hence the
    // lane reads that mark them uniform again; on scalar registers they are
    // plain copies).  The Gauss-point kinds go without the barrier: with
    // their element routine the compiler fails to keep its operands in
    // scalar registers.
    auto refresh = [&]() {
        if constexpr (KIND != JFNK_PLAP_GAUSS)
            asm volatile("" : "+s"(uNX), "+s"(uNY), "+s"(uNZ), "+s"(unx), "+s"(unz), "+s"(udir), "+s"(uy0),
                         "+s"(urows), "+s"(usrows), "+s"(ufree), "+s"(ueok), "+s"(uodir));
        uNX = sc(uNX); uNY = sc(uNY); uNZ = sc(uNZ); unx = sc(unx); unz = sc(unz); udir = sc(udir);
        uy0 = sc(uy0); urows = sc(urows); usrows = sc(usrows); ufree = sc(ufree); ueok = sc(ueok);
        uodir = sc(uodir);
    };
    auto zdir_u = [&](int gz) { return ((udir & JFNK_FACE_ZLO) && gz == 0) || ((udir & JFNK_FACE_ZHI) && gz == unz); };
    auto ydir_u = [&](int gy) { return ((udir & JFNK_FACE_YLO) && gy == 0) || ((udir & JFNK_FACE_YHI) && gy == uNY - 1); };

    // ---- plane fetch (global -> registers) and store (registers -> LDS) ----
    // Loads use clamped urows and columns and are always issued.  Off the grid
    // the state is a copy of the edge row or plane, read only by elements that
    // are switched off; the direction is zeroed there and on Dirichlet nodes.
    //
    // LATE (the residual, whose fetch is the state alone): the fetched
    // registers keep the raw loaded values, every mask is applied by store(),
    // and settle() marks them used on every path before that, so nothing
    // between the fetch and the store waits for the loads.  An early use, or
    // a register write that could overtake a load left pending on some path,
    // makes the compiler drain every outstanding access at that point, and
    // the fetch then no longer overlaps the element work (FP64 F(u) at 256^3:
    // 144 us that way, 136 us late).  The FD modes keep masking the direction
    // as it arrives, which waits for the fetch before the element work: their
    // VALU is about two thirds busy, and with the fetch and the epilogue
    // inputs in flight across the element work the FP32 Chebyshev step at
    // 256^3 took 148 us instead of 136 us (150 us with the fetch spread over
    // the element rows).
    constexpr bool LATE = !FD;
    const int tc = t < uNX ? t : uNX - 1;
    T px[R + 2], pk[R + 2], qx = T(0), qk = T(0);
    TV pv[R + 2], qv = TV(0);
    auto fetch = [&](int pz) {
        const int pzc = pz < 0 ? 0 : (pz >= uNZ ? uNZ - 1 : pz);
        const bool zin = pz == pzc;
        const bool zd = zdir_u(pz);
        const bool zfree = zin && !zd;
#pragma unroll
        for (int r = 0; r < R + 2; ++r) {
            const int gy = uy0 - 1 + r;
            const int gyc = gy < 0 ? 0 : (gy >= uNY ? uNY - 1 : gy);
            const BufAt at{(unsigned)((pzc * uNY + gyc) * uNX), (unsigned)tc};
            px[r] = at.ld(x, 0);
            if constexpr (FD) {
                const TV vv = at.ld(v, 0);
                pv[r] = (zfree && ((ufree >> r) & 1u)) ? vv * vlane : TV(0);
            }
            if constexpr (INV) pk[r] = at.ld(kap, 0);
        }
        if (extra) {       // column nx, row t
            const int gy = uy0 - 1 + t;
            const int gyc = gy < 0 ? 0 : (gy >= uNY ? uNY - 1 : gy);
            const bool in = zin && gy == gyc && t < urows + 2;
            const int idx = (pzc * uNY + gyc) * uNX + unx;
            const T xv = x[idx];
            if constexpr (LATE) {
                qx = xv;
            } else {
                qx = in ? xv : T(0);
            }
            if constexpr (FD) {
                const TV vv = v[idx];
                qv = (in && !(xdir_e || zd || ydir_u(gy))) ? vv : TV(0);
            }
            if constexpr (INV) {
                const T kv = kap[idx];
                if constexpr (LATE) {
                    qk = kv;
                } else {
                    qk = in ? kv : T(0);
                }
            }
        }
    };
    auto settle = [&]() {
#pragma unroll
        for (int r = 0; r < R + 2; ++r) {
            asm volatile("" ::"v"(px[r]));
            if constexpr (INV) asm volatile("" ::"v"(pk[r]));
        }
        if (extra) {
            asm volatile("" ::"v"(qx));
            if constexpr (INV) asm volatile("" ::"v"(qk));
        }
    };
    auto store = [&](int pz) {
        const int sl = pz & 1;
        if constexpr (LATE) settle();
        if (own_col) {
#pragma unroll
            for (int r = 0; r < R + 2; ++r) {
                if (r < usrows) {
                    sx[sl * plane + r * P + t] = px[r];
                    if constexpr (FD) sv[sl * plane + r * P + t] = pv[r];
                    if constexpr (INV) sk[sl * plane + r * P + t] = pk[r];
                }
            }
        }
        if (extra && t < usrows) {
            bool in = true;
            if constexpr (LATE) {
                const int gy = uy0 - 1 + t;
                in = pz >= 0 && pz < uNZ && gy >= 0 && gy < uNY && t < urows + 2;
            }
            sx[sl * plane + t * P + unx] = in ? qx : T(0);
            if constexpr (FD) sv[sl * plane + t * P + unx] = qv;
            if constexpr (INV) sk[sl * plane + t * P + unx] = in ? qk : T(0);
        }
    };

    // ---- element layer ez, walked row by row --------------------------------
    // C0/C1[k]: contributions of the layer below to node row y0 + k, columns
    // t and t + 1 (the carry); O[k]: the finished value of column t.  The walk
    // over the element urows is unrolled, so all indices are compile-time; a
    // row k is finished when element row k + 1 is done, and its carry slot
    // then takes this layer's contribution to the plane above.  The part for
    // column t + 1 goes to the hand-over buffer.
    T C0[R], C1[R], O[R];
#pragma unroll
    for (int k = 0; k < R; ++k) { C0[k] = T(0); C1[k] = T(0); O[k] = T(0); }
    auto layer = [&](int ez) {
        const bool lz = !zero_fd && ez >= 0 && ez < unz;
        const int lo = (ez & 1) * plane + t, hi = ((ez + 1) & 1) * plane + t;
        // corners on the current row: [plane lo/hi][column t / t+1]
        T cx[4], ck[4];
        TV cv[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) { cx[c] = T(0); ck[c] = T(0); cv[c] = TV(0); }
        auto row = [&](int r, T(&ox)[4], TV(&ov)[4], T(&ok)[4]) {
            const int o = (r < usrows ? r : usrows - 1) * P;
            ox[0] = sx[lo + o]; ox[1] = sx[lo + o + 1]; ox[2] = sx[hi + o]; ox[3] = sx[hi + o + 1];
            if constexpr (FD) { ov[0] = sv[lo + o]; ov[1] = sv[lo + o + 1]; ov[2] = sv[hi + o]; ov[3] = sv[hi + o + 1]; }
            if constexpr (INV) { ok[0] = sk[lo + o]; ok[1] = sk[lo + o + 1]; ok[2] = sk[hi + o]; ok[3] = sk[hi + o + 1]; }
        };
        if (lz) row(0, cx, cv, ck);
        T pS0 = T(0), pS1 = T(0), pN0 = T(0), pN1 = T(0);
        // every element row of the walk is evaluated (rows past the tile
        // produce values no epilogue stores; past the grid they are
        // switched off): straight-line code without early exits
#pragma unroll
        for (int re = 0; re <= R; ++re) {
            T r8[1][8];
#pragma unroll
            for (int a = 0; a < 8; ++a) r8[0][a] = T(0);
            if (lz) {
                T ux[4], uk[4];
                TV uv[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) { uk[c] = T(0); uv[c] = TV(0); }
                row(re + 1, ux, uv, uk);
                // element rows and columns outside the grid are switched off by
                // the factor m (no branch); their corners hold finite copies
                const T m = ((ueok >> re) & 1u) ? elane : T(0);
                // corner a = ax + 2 ay + 4 az
                const T xe[1][8] = {{cx[0], cx[1], ux[0], ux[1], cx[2], cx[3], ux[2], ux[3]}};
                T ve[1][8], kp[8];
                const TV vv[8] = {cv[0], cv[1], uv[0], uv[1], cv[2], cv[3], uv[2], uv[3]};
                const T kk[8] = {ck[0], ck[1], uk[0], uk[1], ck[2], ck[3], uk[2], uk[3]};
#pragma unroll
                for (int a = 0; a < 8; ++a) { ve[0][a] = (T)vv[a]; kp[a] = kk[a]; }
                elem_eval<3, KIND, MODE, T, 1, 8, PF>(xe, ve, kp, e, ph, h, r8, m);
#pragma unroll
                for (int c = 0; c < 4; ++c) { cx[c] = ux[c]; cv[c] = uv[c]; ck[c] = uk[c]; }
            }
            if (re >= 1) {     // node row re - 1 is complete for this layer
                const int k = re - 1;
                O[k] = C0[k] + (pS0 + r8[0][0]);
                const T t1 = C1[k] + (pS1 + r8[0][1]);
                C0[k] = pN0 + r8[0][4];
                C1[k] = pN1 + r8[0][5];
                if (own_elem && k < urows) xb[k * P + t + 1] = t1;
            }
            pS0 = r8[0][2]; pS1 = r8[0][3]; pN0 = r8[0][6]; pN1 = r8[0][7];
        }
    };

    if (t < R) xb[t * P] = T(0);        // node column 0 has no left element
    // columns NX..P-1 of every plane row: read as corners by the lanes past
    // the last element column, so they must hold finite values
    if (P > g.NX) {
        const int pad = P - g.NX;
        for (int q = t; q < 2 * ta.srows * pad; q += nthr) {
            const int o = (q / pad) * P + g.NX + q % pad;
            sx[o] = T(0);
            if constexpr (FD) sv[o] = TV(0);
            if constexpr (INV) sk[o] = T(0);
        }
    }

    // prologue: planes z0-1 and z0 in LDS; element layer z0-1 builds the
    // carry while plane z0+1 is fetched
    fetch(z0 - 1);
    store(z0 - 1);
    fetch(z0);
    store(z0);
    __syncthreads();
    refresh();
    fetch(z0 + 1);
    layer(z0 - 1);
    __syncthreads();
    store(z0 + 1);
    __syncthreads();

    // iteration z evaluates element layer z (planes z, z+1 in LDS) and
    // finishes node plane z.  The epilogue inputs of plane z (and A(x) for
    // the plain FD quotient) are read before the element work.  Node
    // (nx, y0 + k) of the last column is finished by thread k.
    constexpr int NIN = Epi::NIN > 0 ? Epi::NIN : 1;
    constexpr bool PLAIN = MODE == M_FD_PLAIN;
    constexpr bool VLDS = FD && Epi::VIN >= 0 && Epi::NCOMP == 1;
    for (int z = z0; z < z1; ++z) {
        refresh();
        T pin[R][NIN], pax[R], qin[NIN], qax = T(0);
        {
            if (z + 2 <= z1) fetch(z + 2);
            // clamped row and column: always a valid node, unused where out of the tile.
            // An input that is the direction itself is read from its LDS plane
            // (slot z & 1 holds plane z until store(z + 2)), masked like the
            // element corners: equal to the array on every free node, and the
            // epilogues use it on free nodes only.
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int kc = k < urows ? k : urows - 1;
                const BufAt at{(unsigned)((z * uNY + uy0 + kc) * uNX), (unsigned)tc};
                epi.template load<VLDS>(at, pin[k]);
                pax[k] = PLAIN ? at.ld(Ax, 0) : T(0);
                if constexpr (VLDS) pin[k][Epi::VIN] = (T)sv[(z & 1) * plane + (kc + 1) * P + t];
            }
            if (extra) {
                const int kc = t < urows ? t : urows - 1;
                const PtrAt at{(long long)((z * uNY + uy0 + kc) * uNX + unx)};
                epi.template load<VLDS>(at, qin);
                if constexpr (PLAIN) qax = at.ld(Ax, 0);
                if constexpr (VLDS) qin[Epi::VIN] = (T)sv[(z & 1) * plane + (kc + 1) * P + unx];
            }
        }
        layer(z);
        __syncthreads();
        if (z + 2 <= z1) store(z + 2);
        {
            const bool zd = zdir_u(z);
            // LATE: the epilogue inputs are marked used on every path (see settle)
#pragma unroll
            for (int k = 0; k < (LATE ? R : 0); ++k) {
#pragma unroll
                for (int c = 0; c < Epi::NIN; ++c) asm volatile("" ::"v"(pin[k][c]));
                if constexpr (PLAIN) asm volatile("" ::"v"(pax[k]));
            }
            if (LATE && extra) {
#pragma unroll
                for (int c = 0; c < Epi::NIN; ++c) asm volatile("" ::"v"(qin[c]));
                if constexpr (PLAIN) asm volatile("" ::"v"(qax));
            }
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int gy = uy0 + k;
                if (own_col && k < urows) {
                    const BufAt at{(unsigned)((z * uNY + gy) * uNX), (unsigned)t};
                    const bool dir = zd || ((uodir >> k) & 1u) || xdir_t;
                    T val[1] = {T(0)};
                    if (!dir && !zero_fd) {
                        T acc = O[k] + xb[k * P + t];
                        if constexpr (PLAIN) acc = (acc - pax[k]) * ie;
                        val[0] = acc;
                    }
                    epi.node(at, val, dir, sums, pin[k]);
                }
            }
            if (extra && t < urows) {
                const int gy = uy0 + t;
                const PtrAt at{(long long)((z * uNY + gy) * uNX + unx)};
                const bool dir = zd || ydir_u(gy) || xdir_e;
                T val[1] = {T(0)};
                if (!dir && !zero_fd) {
                    T acc = xb[t * P + unx];
                    if constexpr (PLAIN) acc = (acc - qax) * ie;
                    val[0] = acc;
                }
                epi.node(at, val, dir, sums, qin);
            }
        }
        __syncthreads();
    }
    if constexpr (Epi::NS > 0) block_partials<Epi::NS>(sums, red);
}

}  // namespace jfnk
