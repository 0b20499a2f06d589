// Stage kernels: everything in one RK4 stage evaluation except the pressure
// solve.  One thread per cell; each kernel reads its operands straight from
// HBM with x-contiguous (coalesced) rows, neighbours reused through L1/L2.
#include "tpf_internal.hpp"

namespace tpf {

// ------------------------------------------------------------------ kernels
// One thread per cell; the bodies are the op_* functions of tpf_stage_ops.hpp.
template <typename T, int DIM, bool W = false>
__global__ __launch_bounds__(BLOCK) void k_cell(Dims d, int kz, Phys P, const T* __restrict__ phi,
                                                T* __restrict__ n0, T* __restrict__ n1,
                                                T* __restrict__ n2, T* __restrict__ mu) {
    for_cells_zchunk<W>(d, kz, [&](const Cell& C) { op_cell<T, DIM>(P, C, phi, n0, n1, n2, mu); });
}

template <typename T, int DIM, bool W = false>
__global__ __launch_bounds__(BLOCK) void k_kappa(Dims d, int kz, Phys P, const T* __restrict__ n0,
                                                 const T* __restrict__ n1,
                                                 const T* __restrict__ n2, T* __restrict__ kappa) {
    for_cells_zchunk<W>(d, kz, [&](const Cell& C) { op_kappa<T, DIM>(P, C, n0, n1, n2, kappa); });
}

template <typename T, int DIM, bool W = false>
__global__ __launch_bounds__(BLOCK) void k_face(Dims d, int kz, Phys P, const T* __restrict__ phi,
                                                const T* __restrict__ n0, const T* __restrict__ n1,
                                                const T* __restrict__ n2, const T* __restrict__ u0,
                                                const T* __restrict__ u1, const T* __restrict__ u2,
                                                T* __restrict__ r0, T* __restrict__ r1,
                                                T* __restrict__ r2, T* __restrict__ m0,
                                                T* __restrict__ m1, T* __restrict__ m2) {
    for_cells_zchunk<W>(d, kz, [&](const Cell& C) {
        op_face<T, DIM>(P, C, phi, n0, n1, n2, u0, u1, u2, r0, r1, r2, m0, m1, m2);
    });
}

template <typename T, int DIM, bool W = false>
__global__ __launch_bounds__(BLOCK) void k_momentum(
    Dims d, int kz, Phys P, const T* __restrict__ phi, const T* __restrict__ u0,
    const T* __restrict__ u1, const T* __restrict__ u2, const T* __restrict__ m0,
    const T* __restrict__ m1, const T* __restrict__ m2, const T* __restrict__ mu,
    const T* __restrict__ kappa, T* __restrict__ f0, T* __restrict__ f1, T* __restrict__ f2,
    T* __restrict__ F0, T* __restrict__ F1, T* __restrict__ F2) {
    for_cells_zchunk<W>(d, kz, [&](const Cell& C) {
        op_momentum<T, DIM>(P, C, phi, u0, u1, u2, m0, m1, m2, mu, kappa, f0, f1, f2, F0, F1, F2);
    });
}

// the phase-field update and the momentum right-hand side of one cell in one
// pass: both read phi and u at the same cells
template <typename T, int DIM, bool W = false>
__global__ __launch_bounds__(BLOCK) void k_phase_momentum(
    Dims d, int kz, Phys P, RKArgs rk, const T* __restrict__ phi, const T* __restrict__ u0,
    const T* __restrict__ u1, const T* __restrict__ u2, const T* __restrict__ r0,
    const T* __restrict__ r1, const T* __restrict__ r2, const T* __restrict__ kappa,
    const T* __restrict__ yn, T* __restrict__ acc, T* __restrict__ ynext, int* __restrict__ flags,
    const T* __restrict__ m0, const T* __restrict__ m1, const T* __restrict__ m2,
    const T* __restrict__ mu, T* __restrict__ f0, T* __restrict__ f1, T* __restrict__ f2,
    T* __restrict__ F0, T* __restrict__ F1, T* __restrict__ F2) {
    for_cells_zchunk<W>(d, kz, [&](const Cell& C) {
        op_phase<T, DIM>(P, rk, C, phi, u0, u1, u2, r0, r1, r2, kappa, yn, acc, ynext, flags);
        op_momentum<T, DIM>(P, C, phi, u0, u1, u2, m0, m1, m2, mu, kappa, f0, f1, f2, F0, F1, F2);
    });
}

// k_cell and k_face in one pass (3D), from a ring of three phi planes in LDS.
// Per z plane k the block first forms the normals of its BX x BY tile and of
// the cells one below it in x and y (the c - e_a a face needs) into a
// two-plane LDS ring of n, then the face fluxes r (CDI) and m of its cells,
// with n_a(c - e_z) from the ring's previous plane.  phi is read once per
// cell (plus halo), n and mu are written once, and n is not read back.  The
// arithmetic is that of op_cell and op_face.
template <typename T, bool CDI, bool MU>
__global__ __launch_bounds__(BLOCK) void k_cell_face_lds(
    Dims d, int kz, Phys P, const T* __restrict__ phi, const T* __restrict__ u0, const T* __restrict__ u1,
    const T* __restrict__ u2, T* __restrict__ n0, T* __restrict__ n1, T* __restrict__ n2, T* __restrict__ mu,
    T* __restrict__ r0, T* __restrict__ r1, T* __restrict__ r2, T* __restrict__ m0, T* __restrict__ m1,
    T* __restrict__ m2) {
    constexpr int PX = BX + 3, PY = BY + 3;   // phi tile: tile x/y index X in [-2, BX] at column X + 2
    constexpr int NX = BX + 1, NY = BY + 1;   // n tile: X in [-1, BX - 1] at column X + 1
    __shared__ T fr[3][PY][PX];
    __shared__ T nr[2][3][NY][NX];
    int bx, by, bz;
    if (!block_tile(d.xcd, (d.nx + BX - 1) / BX, (d.ny + BY - 1) / BY, (d.nz + kz - 1) / kz, bx, by, bz)) return;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * BX + tx;
    const int i = bx * BX + tx, j = by * BY + ty;
    const bool valid = i < d.nx && j < d.ny;
    const int k0 = bz * kz, k1 = min(d.nz, k0 + kz);
    const unsigned plane = (unsigned)(d.nx * d.ny);
    const T* u[3] = {u0, u1, u2};
    T* nout[3] = {n0, n1, n2};
    T* rout[3] = {r0, r1, r2};
    T* mout[3] = {m0, m1, m2};
    // phi plane q (periodic) into ring slot (q - k0 + 3) % 3; tile positions
    // past the grid land on periodic neighbours of the last valid cells
    auto stage = [&](int q) {
        const unsigned base = (unsigned)((q + d.nz) % d.nz) * plane;
        T(*dst)[PX] = fr[(q - k0 + 3) % 3];
        for (int e = tid; e < PX * PY; e += BLOCK) {
            const int py = e / PX, px = e - py * PX;
            const int gi = (bx * BX + px - 2 + 2 * d.nx) % d.nx;
            const int gj = (by * BY + py - 2 + 2 * d.ny) % d.ny;
            dst[py][px] = ld(phi, base + (unsigned)(gj * d.nx + gi));
        }
    };
    const T ih = T(P.inv_h), ih2 = T(0.5 * P.inv_h);
    // normals of plane q (tile and the low halo) from ring planes q - 1, q, q + 1
    auto normals = [&](int q) {
        const T(*fm)[PX] = fr[(q - 1 - k0 + 3) % 3];
        const T(*fc)[PX] = fr[(q - k0 + 3) % 3];
        const T(*fp)[PX] = fr[(q + 1 - k0 + 3) % 3];
        const int sl = (q - k0 + 2) % 2;
        for (int e = tid; e < NX * NY; e += BLOCK) {
            const int ny_ = e / NX, nx_ = e - ny_ * NX;
            const int cx = nx_ + 1, cy = ny_ + 1;        // phi tile column / row of this cell
            T g[3];
            g[0] = (fc[cy][cx + 1] - fc[cy][cx - 1]) * ih2;
            g[1] = (fc[cy + 1][cx] - fc[cy - 1][cx]) * ih2;
            g[2] = (fp[cy][cx] - fm[cy][cx]) * ih2;
            T gg = T(0);
#pragma unroll
            for (int a = 0; a < 3; ++a) gg += g[a] * g[a];
            const T inv = rsqrt_of(gg + T(P.delta2));
#pragma unroll
            for (int a = 0; a < 3; ++a) nr[sl][a][ny_][nx_] = g[a] * inv;
        }
    };
    stage(k0 - 2);
    stage(k0 - 1);
    stage(k0);
    __syncthreads();
    normals(k0 - 1);
    __syncthreads();
    stage(k0 + 1);                      // into the slot of plane k0 - 2
    for (int k = k0; k < k1; ++k) {
        __syncthreads();                // phi planes k - 1, k, k + 1 are in the ring
        normals(k);
        __syncthreads();
        if (valid) {
            const T(*fm)[PX] = fr[(k - 1 - k0 + 3) % 3];
            const T(*fc)[PX] = fr[(k - k0 + 3) % 3];
            const T(*fp)[PX] = fr[(k + 1 - k0 + 3) % 3];
            const int sc = (k - k0 + 2) % 2, sm = (k - 1 - k0 + 2) % 2;
            const int cx = tx + 2, cy = ty + 2;         // phi tile
            const int qx = tx + 1, qy = ty + 1;         // n tile
            const unsigned c = (unsigned)k * plane + (unsigned)(j * d.nx + i);
            const T f = fc[cy][cx];
            if (nout[0]) {
#pragma unroll
                for (int a = 0; a < 3; ++a) st(nout[a], c, nr[sc][a][qy][qx]);
            }
            if (MU) {
                const T fxp = fc[cy][cx + 1], fxm = fc[cy][cx - 1], fyp = fc[cy + 1][cx], fym = fc[cy - 1][cx];
                const T fzp = fp[cy][cx], fzm = fm[cy][cx];
                T lap = T(0);
                lap += ((fxp - f) * ih - (f - fxm) * ih) * ih;
                lap += ((fyp - f) * ih - (f - fym) * ih) * ih;
                lap += ((fzp - f) * ih - (f - fzm) * ih) * ih;
                st(mu, c, T(P.sigma_hat / P.eps) * dpsi(f) - T(P.sigma_hat * P.eps) * lap);
            }
            const T drho = T(P.rho1 - P.rho2);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const T fm_ = a == 0 ? fc[cy][cx - 1] : (a == 1 ? fc[cy - 1][cx] : fm[cy][cx]);
                const T rho_f = T(0.5) * (rho_of(P, fm_) + rho_of(P, f));
                T ra = T(0);
                if (CDI) {
                    const T nam = a == 0 ? nr[sc][0][qy][qx - 1] : (a == 1 ? nr[sc][1][qy - 1][qx] : nr[sm][2][qy][qx]);
                    const T wm = fm_ * (T(1) - fm_) * nam;
                    const T wc = f * (T(1) - f) * nr[sc][a][qy][qx];
                    ra = T(P.gamma) * (T(P.eps) * ((f - fm_) * T(P.inv_h)) - T(0.5) * (wm + wc));
                    st(rout[a], c, ra);
                }
                st(mout[a], c, rho_f * ld(u[a], c) - drho * ra);
            }
        }
        __syncthreads();                // plane k - 1's phi and n slots are free
        if (k + 2 <= k1) stage(k + 2);  // into the slot of plane k - 1
    }
}

// The same pass with the neighbourhoods staged in LDS (3D).  A block owns a
// BX x BY column piece of kz planes.  It keeps a ring of three z planes
// (k - 1, k, k + 1) of the fields it reads z neighbours and z diagonals of
// (phi, u, m), each plane its BX x BY tile plus a one-cell halo, and a
// single-plane tile of the fields it reads only in-plane (mu or kappa, and r_x,
// r_y for CDI).  What else a cell reads is its own column: mu or kappa one
// plane below, r_z (CDI) or kappa (the other models with the energy-based
// force) at the cell, r_z one plane above, and the RK state and accumulator.
// Every global load is issued one plane ahead, while the block computes the
// plane before it: the ring and the single tile through coalesced loads of one
// new plane per step, the column values into registers.  The compute phase
// reads only LDS and registers.
template <typename T>
using Tile = T[BY + 2][BX + 2];

// ZF: single-plane field whose value one plane below the cell comes from a
// register (zm); CF: field read at the cell from a register (zc), and one
// plane above it (zp) when CP; -1: none
template <typename T, unsigned RMASK, unsigned OMASK, int ZF, int CF, bool CP>
struct LAcc {
    const Cell& C;
    const T* p[F_NF];
    const Tile<T>* t[3];   // ring fields (RMASK), planes k - 1, k, k + 1: t[z][slot(f)]
    const Tile<T>* t1;     // single-plane fields (OMASK), plane k: t1[slot1(f)]
    int lx, ly;            // this cell in the tile (halo offset 1)
    T zm, zc, zp;          // column values, see above
    T yv[2];               // the cell's RK state y_n and accumulator
    static constexpr bool ring(int f) { return (RMASK >> f) & 1u; }
    static constexpr bool one(int f) { return (OMASK >> f) & 1u; }
    static constexpr int slot(int f) { return __builtin_popcount(RMASK & ((1u << f) - 1u)); }
    static constexpr int slot1(int f) { return __builtin_popcount(OMASK & ((1u << f) - 1u)); }
    __device__ __forceinline__ T c(int f) const {
        if (ring(f)) return t[1][slot(f)][ly][lx];
        if (one(f)) return t1[slot1(f)][ly][lx];
        if (f == CF) return zc;
        return ld(p[f], C.id);
    }
    __device__ __forceinline__ T nb(int f, int a, int s) const {
        if (ring(f)) return t[1 + (a == 2 ? s : 0)][slot(f)][ly + (a == 1 ? s : 0)][lx + (a == 0 ? s : 0)];
        if (one(f) && a != 2) return t1[slot1(f)][ly + (a == 1 ? s : 0)][lx + (a == 0 ? s : 0)];
        if (f == ZF && a == 2 && s < 0) return zm;
        if (CP && f == CF && a == 2 && s > 0) return zp;
        return ld(p[f], C.off(a, s));
    }
    __device__ __forceinline__ T nb2(int f, int a, int s, int b, int u) const {
        if (ring(f))
            return t[1 + (a == 2 ? s : 0) + (b == 2 ? u : 0)][slot(f)][ly + (a == 1 ? s : 0) + (b == 1 ? u : 0)]
                    [lx + (a == 0 ? s : 0) + (b == 0 ? u : 0)];
        if (one(f) && a != 2 && b != 2)
            return t1[slot1(f)][ly + (a == 1 ? s : 0) + (b == 1 ? u : 0)][lx + (a == 0 ? s : 0) + (b == 0 ? u : 0)];
        return ld(p[f], C.off2(a, s, b, u));
    }
    __device__ __forceinline__ T own(const T* __restrict__, int w) const { return yv[w]; }
};

template <typename T, bool CDI, bool EB>
__global__ __launch_bounds__(BLOCK) void k_phase_momentum_lds(
    Dims d, int kz, Phys P, RKArgs rk, const T* __restrict__ phi, const T* __restrict__ u0,
    const T* __restrict__ u1, const T* __restrict__ u2, const T* __restrict__ r0,
    const T* __restrict__ r1, const T* __restrict__ r2, const T* __restrict__ kappa,
    const T* __restrict__ yn, T* __restrict__ acc, T* __restrict__ ynext, int* __restrict__ flags,
    const T* __restrict__ m0, const T* __restrict__ m1, const T* __restrict__ m2,
    const T* __restrict__ mu, T* __restrict__ f0, T* __restrict__ f1, T* __restrict__ f2,
    T* __restrict__ F0, T* __restrict__ F1, T* __restrict__ F2) {
    constexpr unsigned RMASK = (1u << F_PHI) | (7u << F_U0) | (7u << F_M0);
    constexpr unsigned OMASK = (EB ? (1u << F_MU) : (1u << F_KAP)) | (CDI ? ((1u << F_R0) | (1u << F_R1)) : 0u);
    constexpr int ZF = EB ? F_MU : F_KAP;
    constexpr int CF = CDI ? F_R2 : (EB ? F_KAP : -1);
    constexpr bool CP = CDI;
    constexpr int NS = __builtin_popcount(RMASK), NS1 = __builtin_popcount(OMASK);
    using A_t = LAcc<T, RMASK, OMASK, ZF, CF, CP>;
    __shared__ Tile<T> ring[3][NS];
    __shared__ Tile<T> tile1[NS1];
    int bx, by, bz;
    if (!block_tile(d.xcd, (d.nx + BX - 1) / BX, (d.ny + BY - 1) / BY, (d.nz + kz - 1) / kz, bx, by, bz)) return;
    const int tid = threadIdx.y * BX + threadIdx.x;
    const int i = bx * BX + threadIdx.x, j = by * BY + threadIdx.y;
    const bool valid = i < d.nx && j < d.ny;
    const int k0 = bz * kz, k1 = min(d.nz, k0 + kz);
    const T* p[F_NF] = {phi, u0, u1, u2, m0, m1, m2, mu, kappa, r0, r1, r2};
    // Each thread copies tile positions tid and tid + BLOCK (when inside the
    // (BX + 2) x (BY + 2) tile).  Positions are periodic; for a ragged tile
    // the positions past the grid land on the periodic neighbours of its last
    // valid cells.
    constexpr int TP = (BX + 2) * (BY + 2);
    unsigned pos[2];
    int py[2], px[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int e = min(tid + h * BLOCK, TP - 1);
        py[h] = e / (BX + 2);
        px[h] = e - py[h] * (BX + 2);
        const int gi = (bx * BX + px[h] - 1 + d.nx) % d.nx;
        const int gj = (by * BY + py[h] - 1 + d.ny) % d.ny;
        pos[h] = (unsigned)(gj * d.nx + gi);
    }
    const bool second = tid + BLOCK < TP;
    const unsigned plane = (unsigned)(d.nx * d.ny);
    // the thread's own column (cell 0 of the plane for threads outside the
    // grid, whose values are never used)
    const unsigned col = valid ? (unsigned)(j * d.nx + i) : 0u;
    auto at = [&](int q) { return (unsigned)((q + d.nz) % d.nz) * plane + col; };
    const bool rd_y = !rk.eval_only, rd_acc = !rk.eval_only && rk.stage != 0;
    T pre[2][NS], pre1[2][NS1 > 0 ? NS1 : 1];
    T ny[2] = {T(0), T(0)}, nc = T(0);
    // ring fields of plane q and single-plane fields of plane q1 (periodic in
    // z) into registers; stored to ring slot r and the single tile
    auto load = [&](int q, int q1) {
        const unsigned base = (unsigned)((q + d.nz) % d.nz) * plane;
        const unsigned base1 = (unsigned)((q1 + d.nz) % d.nz) * plane;
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int f = 0; f < F_NF; ++f) {
                if ((RMASK >> f) & 1u) pre[h][A_t::slot(f)] = ld(p[f], base + pos[h]);
                if ((OMASK >> f) & 1u) pre1[h][A_t::slot1(f)] = ld(p[f], base1 + pos[h]);
            }
    };
    // column values of plane q1: y_n, the accumulator, and CF at q1 (at
    // q1 + 1 when CP: its value at q1 was loaded one plane earlier)
    auto load_col = [&](int q1) {
        if (rd_y) ny[0] = ld(yn, at(q1));
        if (rd_acc) ny[1] = ld(acc, at(q1));
        if (CF >= 0) nc = ld(p[CF >= 0 ? CF : 0], at(CP ? q1 + 1 : q1));
    };
    auto store = [&](int r, bool with1) {
#pragma unroll
        for (int f = 0; f < F_NF; ++f) {
            if ((RMASK >> f) & 1u) {
                ring[r][A_t::slot(f)][py[0]][px[0]] = pre[0][A_t::slot(f)];
                if (second) ring[r][A_t::slot(f)][py[1]][px[1]] = pre[1][A_t::slot(f)];
            }
            if (with1 && ((OMASK >> f) & 1u)) {
                tile1[A_t::slot1(f)][py[0]][px[0]] = pre1[0][A_t::slot1(f)];
                if (second) tile1[A_t::slot1(f)][py[1]][px[1]] = pre1[1][A_t::slot1(f)];
            }
        }
    };
    T zm = ld(p[ZF], at(k0 - 1)), zc = T(0), zp = T(0);
    if (CP) zp = ld(p[CF >= 0 ? CF : 0], at(k0));
    load(k0 - 1, k0);
    store(0, false);
    load(k0, k0);
    store(1, true);
    load(k0 + 1, k0 + 1);
    load_col(k0);
    for (int k = k0; k < k1; ++k) {
        const int rm = (k - k0) % 3, rc = (k - k0 + 1) % 3, rp = (k - k0 + 2) % 3;
        // the column values of plane k, loaded one step earlier
        const T yv0 = ny[0], yv1 = ny[1];
        if (CP) {
            zc = zp;
            zp = nc;
        } else {
            zc = nc;
        }
        // ring plane k + 1 into the slot plane k - 2 used, and (after the
        // first plane, whose single tile the prologue stored) the
        // single-plane fields of plane k, both loaded one step earlier
        store(rp, k > k0);
        __syncthreads();
        if (k + 1 < k1) {                       // in flight while plane k is computed
            load(k + 2, k + 1);
            load_col(k + 1);
        }
        if (valid) {
            const Cell C = make_cell(d, i, j, k);
            const A_t A{C, {phi, u0, u1, u2, m0, m1, m2, mu, kappa, r0, r1, r2}, {ring[rm], ring[rc], ring[rp]},
                        tile1, (int)threadIdx.x + 1, (int)threadIdx.y + 1, zm, zc, zp, {yv0, yv1}};
            op_phase_g<T, 3, A_t, CDI ? MODEL_CDI : -1>(P, rk, C, A, yn, acc, ynext, flags);
            op_momentum_g<T, 3, A_t, EB ? FORCE_EB : -1>(P, C, A, f0, f1, f2, F0, F1, F2);
        }
        zm = tile1[A_t::slot1(ZF)][threadIdx.y + 1][threadIdx.x + 1];   // ZF of plane k, for plane k + 1
        __syncthreads();           // plane k - 1's ring slot and the single tile are free
    }
}

// b = D f* in FP64, plus the block sums of b (for the mean)
template <typename T, int DIM, bool W = false>
__global__ __launch_bounds__(BLOCK) void k_div(Dims d, int kz, Phys P, const T* __restrict__ f0,
                                               const T* __restrict__ f1,
                                               const T* __restrict__ f2, double* __restrict__ b,
                                               double* __restrict__ partials) {
    double v[1] = {0.0};
    for_cells_zchunk<W>(d, kz, [&](const Cell& C) { v[0] += op_div<T, DIM>(P, C, f0, f1, f2, b); });
    block_partials<1>(v, partials);
}

template <typename T, int DIM, bool W = false>
__global__ __launch_bounds__(BLOCK) void k_project(Dims d, int kz, Phys P, RKArgs rk,
                                                   const T* __restrict__ phi,
                                                   const double* __restrict__ p,
                                                   const T* __restrict__ f0, const T* __restrict__ f1,
                                                   const T* __restrict__ f2, const T* yn0,
                                                   const T* yn1, const T* yn2, T* acc0, T* acc1,
                                                   T* acc2, T* nx0, T* nx1, T* nx2,
                                                   int* __restrict__ flags, double* __restrict__ hist,
                                                   const double* __restrict__ hsub, double* __restrict__ guess,
                                                   const double* __restrict__ gsrc, double ga, double gb) {
    for_cells_zchunk<W>(d, kz, [&](const Cell& C) {
        op_project<T, DIM>(P, rk, C, phi, p, f0, f1, f2, yn0, yn1, yn2, acc0, acc1, acc2, nx0, nx1, nx2, flags);
        // the pressure history of the warm starts (hist = p, or p - hsub),
        // and the next stage's starting guess (ga p + gb gsrc; both weights
        // are 1 or 2 in magnitude, so the products are exact)
        if (hist || guess) {
            const double pc = ld(p, C.id);
            if (hist) stn(hist, C.id, hsub ? pc - ld(hsub, C.id) : pc);
            if (guess) stn(guess, C.id, ga * pc + gb * ld(gsrc, C.id));
        }
    });
}

template <typename T, int DIM>
__global__ __launch_bounds__(BLOCK) void k_init_droplet(Dims d, double h, double eps, double c0,
                                                        double c1, double c2, double a0, double a1,
                                                        double a2, T* __restrict__ phi) {
    Cell C;
    if (!cell_of_thread(d, C)) return;
    op_init_droplet<T, DIM>(d, C, h, eps, c0, c1, c2, a0, a1, a2, phi);
}

template <typename T>
__global__ void k_convert_in(long N, const double* __restrict__ src, T* __restrict__ dst) {
    long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < N) dst[q] = T(src[q]);
}
template <typename T>
__global__ void k_convert_out(long N, const T* __restrict__ src, double* __restrict__ dst) {
    long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < N) dst[q] = (double)src[q];
}
template <typename T>
__global__ void k_fill(long N, T* __restrict__ dst, T v) {
    long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < N) dst[q] = v;
}

// ------------------------------------------------------------------ diagnostics
template <typename T, int DIM, bool W = false>
__global__ __launch_bounds__(BLOCK) void k_diag(Dims d, Phys P, const T* __restrict__ phi,
                                                const T* __restrict__ u0, const T* __restrict__ u1,
                                                const T* __restrict__ u2,
                                                const double* __restrict__ p,
                                                double* __restrict__ part) {
    Cell C;
    double s[ND_SUM] = {0, 0, 0, 0, 0, 0, 0};
    double mx[ND_MAX] = {0.0, 0.0, -1e300, -1e300};
    if (cell_of_thread<W>(d, C)) op_diag<T, DIM>(P, C, phi, u0, u1, u2, p, s, mx);
    block_sum<ND_SUM>(s);
    block_max<ND_MAX>(mx);
    if (thread_linear() == 0) {
        const int b = block_linear(), nb = nblocks_linear();
        for (int q = 0; q < ND_SUM; ++q) part[(long)q * nb + b] = s[q];
        for (int q = 0; q < ND_MAX; ++q) part[(long)(ND_SUM + q) * nb + b] = mx[q];
    }
}

__global__ __launch_bounds__(BLOCK) void k_diag_final(int nb, const double* __restrict__ part,
                                                      double* __restrict__ out) {
    double s[ND_SUM] = {0, 0, 0, 0, 0, 0, 0};
    double mx[ND_MAX] = {0.0, 0.0, -1e300, -1e300};
    for (int b = thread_linear(); b < nb; b += BLOCK) {
        for (int q = 0; q < ND_SUM; ++q) s[q] += part[(long)q * nb + b];
        for (int q = 0; q < ND_MAX; ++q) mx[q] = fmax(mx[q], part[(long)(ND_SUM + q) * nb + b]);
    }
    block_sum<ND_SUM>(s);
    block_max<ND_MAX>(mx);
    if (thread_linear() == 0) {
        for (int q = 0; q < ND_SUM; ++q) out[q] = s[q];
        for (int q = 0; q < ND_MAX; ++q) out[ND_SUM + q] = mx[q];
    }
}

// ================================================================== launchers

template <typename T>
static inline T* tp(void* p) { return static_cast<T*>(p); }
template <typename T>
static inline const T* ctp(const void* p) { return static_cast<const T*>(p); }

template <typename T, int DIM, bool W>
static hipError_t stage_fields_impl(tpf_ctx* c, const void* phi_s) {
    const Phys P = phys_of(c);
    const Dims d = dims_of(c->n, c->walls);
    const int kz = c->stage_kz;
    const dim3 g = zchunk_grid(c->n, kz), b(BX, BY);
    const bool need_mu = c->P.force == FORCE_EB;
    const bool need_kappa = c->P.model != MODEL_CDI || c->P.force != FORCE_EB;
    prof_begin(c, PC_CELL, (double)c->N * c->tsz * (1 + DIM + (need_mu ? 1 : 0)));
    k_cell<T, DIM, W><<<g, b, 0, c->stream>>>(d, kz, P, ctp<T>(phi_s), tp<T>(c->nrm[0]), tp<T>(c->nrm[1]),
                                           tp<T>(c->nrm[2]), need_mu ? tp<T>(c->mu) : nullptr);
    prof_end(c);
    if (need_kappa) {
        prof_begin(c, PC_KAPPA, (double)c->N * c->tsz * (DIM + 1));
        k_kappa<T, DIM, W><<<g, b, 0, c->stream>>>(d, kz, P, ctp<T>(c->nrm[0]), ctp<T>(c->nrm[1]),
                                                ctp<T>(c->nrm[2]), tp<T>(c->kappa));
        prof_end(c);
    }
    return hipGetLastError();
}

// the instantiation with or without wall bits
template <typename T, int DIM, typename... A>
static hipError_t stage_fields_impl_w(tpf_ctx* c, A... a) {
    return c->walls ? stage_fields_impl<T, DIM, true>(c, a...) : stage_fields_impl<T, DIM, false>(c, a...);
}

template <typename T, int DIM, bool W>
static hipError_t face_impl(tpf_ctx* c, const void* phi_s, const void* const u_s[3]) {
    const Phys P = phys_of(c);
    const Dims d = dims_of(c->n, c->walls);
    const int kz = c->stage_kz;
    const dim3 g = zchunk_grid(c->n, kz), b(BX, BY);
    const int cdi = c->P.model == MODEL_CDI;
    prof_begin(c, PC_FACE, (double)c->N * c->tsz * (1 + DIM * (cdi ? 4 : 2)));
    k_face<T, DIM, W><<<g, b, 0, c->stream>>>(
        d, kz, P, ctp<T>(phi_s), ctp<T>(c->nrm[0]), ctp<T>(c->nrm[1]), ctp<T>(c->nrm[2]),
        ctp<T>(u_s[0]), ctp<T>(u_s[1]), ctp<T>(u_s[2]), tp<T>(c->rflux[0]), tp<T>(c->rflux[1]),
        tp<T>(c->rflux[2]), tp<T>(c->mflux[0]), tp<T>(c->mflux[1]), tp<T>(c->mflux[2]));
    prof_end(c);
    return hipGetLastError();
}

// the instantiation with or without wall bits
template <typename T, int DIM, typename... A>
static hipError_t face_impl_w(tpf_ctx* c, A... a) {
    return c->walls ? face_impl<T, DIM, true>(c, a...) : face_impl<T, DIM, false>(c, a...);
}

// the LDS form of k_cell + k_face, then k_kappa where kappa is needed (3D)
template <typename T>
static hipError_t cell_face_lds_impl(tpf_ctx* c, const void* phi_s, const void* const u_s[3], bool normals) {
    const Phys P = phys_of(c);
    const Dims d = dims_of(c->n, c->walls);
    const int lkz = c->stage_lds_kz;
    const dim3 lg = zchunk_grid(c->n, lkz), b(BX, BY);
    const bool cdi = c->P.model == MODEL_CDI, need_mu = c->P.force == FORCE_EB;
    const bool need_kappa = !cdi || !need_mu;
    // n is read only by the kappa pass (and by the callers that ask for it)
    const bool store_n = normals || need_kappa;
    prof_begin(c, PC_FACE, (double)c->N * c->tsz * (1 + 3 + (store_n ? 3 : 0) + (need_mu ? 1 : 0) + 3 * (cdi ? 2 : 1)));
    auto kern = cdi ? (need_mu ? k_cell_face_lds<T, true, true> : k_cell_face_lds<T, true, false>)
                    : (need_mu ? k_cell_face_lds<T, false, true> : k_cell_face_lds<T, false, false>);
    kern<<<lg, b, 0, c->stream>>>(d, lkz, P, ctp<T>(phi_s), ctp<T>(u_s[0]), ctp<T>(u_s[1]), ctp<T>(u_s[2]),
                                  store_n ? tp<T>(c->nrm[0]) : nullptr, tp<T>(c->nrm[1]), tp<T>(c->nrm[2]), tp<T>(c->mu),
                                  tp<T>(c->rflux[0]), tp<T>(c->rflux[1]), tp<T>(c->rflux[2]), tp<T>(c->mflux[0]),
                                  tp<T>(c->mflux[1]), tp<T>(c->mflux[2]));
    prof_end(c);
    if (need_kappa) {
        const int kz = c->stage_kz;
        const dim3 g = zchunk_grid(c->n, kz);
        prof_begin(c, PC_KAPPA, (double)c->N * c->tsz * 4);
        k_kappa<T, 3><<<g, b, 0, c->stream>>>(d, kz, P, ctp<T>(c->nrm[0]), ctp<T>(c->nrm[1]), ctp<T>(c->nrm[2]),
                                              tp<T>(c->kappa));
        prof_end(c);
    }
    return hipGetLastError();
}

hipError_t launch_stage_fields(tpf_ctx* c, const void* phi_s, const void* const u_s[3], bool normals) {
    hipError_t e;
    if (c->dim == 3 && c->stage_lds)
        return c->mixed ? cell_face_lds_impl<float>(c, phi_s, u_s, normals)
                        : cell_face_lds_impl<double>(c, phi_s, u_s, normals);
    if (c->mixed) {
        e = c->dim == 2 ? stage_fields_impl_w<float, 2>(c, phi_s) : stage_fields_impl_w<float, 3>(c, phi_s);
        if (e != hipSuccess) return e;
        return c->dim == 2 ? face_impl_w<float, 2>(c, phi_s, u_s) : face_impl_w<float, 3>(c, phi_s, u_s);
    }
    e = c->dim == 2 ? stage_fields_impl_w<double, 2>(c, phi_s) : stage_fields_impl_w<double, 3>(c, phi_s);
    if (e != hipSuccess) return e;
    return c->dim == 2 ? face_impl_w<double, 2>(c, phi_s, u_s) : face_impl_w<double, 3>(c, phi_s, u_s);
}

template <typename T, int DIM, bool W>
static hipError_t mom_impl(tpf_ctx* c, const void* phi_s, const void* const u_s[3], int want_force) {
    const Phys P = phys_of(c);
    const int kz = c->stage_kz;
    const dim3 g = zchunk_grid(c->n, kz), b(BX, BY);
    prof_begin(c, PC_MOM, (double)c->N * c->tsz * (1 + 3 * DIM + 1));
    k_momentum<T, DIM, W><<<g, b, 0, c->stream>>>(
        dims_of(c->n, c->walls), kz, P, ctp<T>(phi_s), ctp<T>(u_s[0]), ctp<T>(u_s[1]), ctp<T>(u_s[2]),
        ctp<T>(c->mflux[0]), ctp<T>(c->mflux[1]), ctp<T>(c->mflux[2]), ctp<T>(c->mu),
        ctp<T>(c->kappa), tp<T>(c->fs[0]), tp<T>(c->fs[1]), tp<T>(c->fs[2]),
        want_force ? tp<T>(c->force[0]) : nullptr, tp<T>(c->force[1]), tp<T>(c->force[2]));
    prof_end(c);
    return hipGetLastError();
}

// the instantiation with or without wall bits
template <typename T, int DIM, typename... A>
static hipError_t mom_impl_w(tpf_ctx* c, A... a) {
    return c->walls ? mom_impl<T, DIM, true>(c, a...) : mom_impl<T, DIM, false>(c, a...);
}

hipError_t launch_momentum(tpf_ctx* c, const void* phi_s, const void* const u_s[3], int want_force) {
    if (c->mixed)
        return c->dim == 2 ? mom_impl_w<float, 2>(c, phi_s, u_s, want_force)
                           : mom_impl_w<float, 3>(c, phi_s, u_s, want_force);
    return c->dim == 2 ? mom_impl_w<double, 2>(c, phi_s, u_s, want_force)
                       : mom_impl_w<double, 3>(c, phi_s, u_s, want_force);
}

template <typename T, int DIM, bool W>
static hipError_t phase_mom_impl(tpf_ctx* c, const void* phi_s, const void* const u_s[3], const RKArgs& rk,
                                 void* out, int want_force) {
    const Phys P = phys_of(c);
    const int kz = c->stage_kz;
    const dim3 g = zchunk_grid(c->n, kz), b(BX, BY);
    const int cdi = c->P.model == MODEL_CDI;
    T* yn = tp<T>(c->phi[c->s_yn]);
    T* acc = tp<T>(c->phi[c->s_acc]);
    // phi and u once; r (CDI) or kappa, phase history; m, mu or kappa; f* out
    const double phase = 1 + (cdi ? DIM : 1) + (rk.eval_only ? 1 : 3 + (rk.stage < 3));
    prof_begin(c, PC_MOM, (double)c->N * c->tsz * (1 + DIM + phase - 1 + DIM + 1 + DIM));
    if (DIM == 3 && c->stage_lds) {
        const int lkz = c->stage_lds_kz;
        const dim3 lg = zchunk_grid(c->n, lkz);
        const bool eb = c->P.force == TPF_EB;
        auto kern = cdi ? (eb ? k_phase_momentum_lds<T, true, true> : k_phase_momentum_lds<T, true, false>)
                        : (eb ? k_phase_momentum_lds<T, false, true> : k_phase_momentum_lds<T, false, false>);
        kern<<<lg, b, 0, c->stream>>>(
            dims_of(c->n, c->walls), lkz, P, rk, ctp<T>(phi_s), ctp<T>(u_s[0]), ctp<T>(u_s[1]), ctp<T>(u_s[2]),
            ctp<T>(c->rflux[0]), ctp<T>(c->rflux[1]), ctp<T>(c->rflux[2]), ctp<T>(c->kappa), yn, acc, tp<T>(out),
            c->flags, ctp<T>(c->mflux[0]), ctp<T>(c->mflux[1]), ctp<T>(c->mflux[2]), ctp<T>(c->mu),
            tp<T>(c->fs[0]), tp<T>(c->fs[1]), tp<T>(c->fs[2]), want_force ? tp<T>(c->force[0]) : nullptr,
            tp<T>(c->force[1]), tp<T>(c->force[2]));
        prof_end(c);
        return hipGetLastError();
    }
    k_phase_momentum<T, DIM, W><<<g, b, 0, c->stream>>>(
        dims_of(c->n, c->walls), kz, P, rk, ctp<T>(phi_s), ctp<T>(u_s[0]), ctp<T>(u_s[1]), ctp<T>(u_s[2]),
        ctp<T>(c->rflux[0]), ctp<T>(c->rflux[1]), ctp<T>(c->rflux[2]), ctp<T>(c->kappa), yn, acc, tp<T>(out),
        c->flags, ctp<T>(c->mflux[0]), ctp<T>(c->mflux[1]), ctp<T>(c->mflux[2]), ctp<T>(c->mu),
        tp<T>(c->fs[0]), tp<T>(c->fs[1]), tp<T>(c->fs[2]), want_force ? tp<T>(c->force[0]) : nullptr,
        tp<T>(c->force[1]), tp<T>(c->force[2]));
    prof_end(c);
    return hipGetLastError();
}

// the instantiation with or without wall bits
template <typename T, int DIM, typename... A>
static hipError_t phase_mom_impl_w(tpf_ctx* c, A... a) {
    return c->walls ? phase_mom_impl<T, DIM, true>(c, a...) : phase_mom_impl<T, DIM, false>(c, a...);
}

hipError_t launch_phase_momentum(tpf_ctx* c, const void* phi_s, const void* const u_s[3], const RKArgs& rk,
                                 void* out, int want_force) {
    if (c->mixed)
        return c->dim == 2 ? phase_mom_impl_w<float, 2>(c, phi_s, u_s, rk, out, want_force)
                           : phase_mom_impl_w<float, 3>(c, phi_s, u_s, rk, out, want_force);
    return c->dim == 2 ? phase_mom_impl_w<double, 2>(c, phi_s, u_s, rk, out, want_force)
                       : phase_mom_impl_w<double, 3>(c, phi_s, u_s, rk, out, want_force);
}

template <typename T, int DIM, bool W>
static hipError_t div_impl(tpf_ctx* c) {
    const Phys P = phys_of(c);
    const int kz = c->stage_kz;
    const dim3 g = zchunk_grid(c->n, kz), b(BX, BY);
    prof_begin(c, PC_DIV, (double)c->N * (c->tsz * DIM + 8));
    k_div<T, DIM, W><<<g, b, 0, c->stream>>>(dims_of(c->n, c->walls), kz, P, ctp<T>(c->fs[0]), ctp<T>(c->fs[1]),
                                          ctp<T>(c->fs[2]), c->b, c->partials);
    prof_end(c);
    return hipGetLastError();
}

// the instantiation with or without wall bits
template <typename T, int DIM, typename... A>
static hipError_t div_impl_w(tpf_ctx* c, A... a) {
    return c->walls ? div_impl<T, DIM, true>(c, a...) : div_impl<T, DIM, false>(c, a...);
}

hipError_t launch_divergence(tpf_ctx* c) {
    hipError_t e;
    if (c->mixed) e = c->dim == 2 ? div_impl_w<float, 2>(c) : div_impl_w<float, 3>(c);
    else e = c->dim == 2 ? div_impl_w<double, 2>(c) : div_impl_w<double, 3>(c);
    if (e != hipSuccess) return e;
    return launch_finalize(c, (int)zchunk_grid(c->n, c->stage_kz).x, 1, FIN_MEAN);
}

template <typename T, int DIM, bool W>
static hipError_t proj_impl(tpf_ctx* c, const void* phi_s, const RKArgs& rk, void* const out[3]) {
    const Phys P = phys_of(c);
    const int kz = c->stage_kz;
    const dim3 g = zchunk_grid(c->n, kz), b(BX, BY);
    const int yn = c->s_yn, ac = c->s_acc;
    prof_begin(c, PC_PROJ, (double)c->N * (c->tsz * (1 + DIM + (rk.eval_only ? DIM : DIM * (3 + (rk.stage < 3)))) + 8 +
                                           (c->proj_hist ? 8 : 0) + (c->proj_hsub ? 8 : 0) +
                                           (c->proj_guess ? 16 : 0)));
    k_project<T, DIM, W><<<g, b, 0, c->stream>>>(
        dims_of(c->n, c->walls), kz, P, rk, ctp<T>(phi_s), c->p, ctp<T>(c->fs[0]), ctp<T>(c->fs[1]),
        ctp<T>(c->fs[2]), ctp<T>(c->u[0][yn]), ctp<T>(c->u[1][yn]), ctp<T>(c->u[2][yn]),
        tp<T>(c->u[0][ac]), tp<T>(c->u[1][ac]), tp<T>(c->u[2][ac]), tp<T>(out[0]), tp<T>(out[1]),
        tp<T>(out[2]), c->flags, c->proj_hist, c->proj_hist ? c->proj_hsub : nullptr,
        c->proj_guess ? c->p_alt : nullptr, c->proj_guess ? c->proj_gsrc : nullptr, c->proj_ga, c->proj_gb);
    prof_end(c);
    return hipGetLastError();
}

// the instantiation with or without wall bits
template <typename T, int DIM, typename... A>
static hipError_t proj_impl_w(tpf_ctx* c, A... a) {
    return c->walls ? proj_impl<T, DIM, true>(c, a...) : proj_impl<T, DIM, false>(c, a...);
}

hipError_t launch_project_update(tpf_ctx* c, const void* phi_s, const RKArgs& rk, void* const out[3]) {
    if (c->mixed)
        return c->dim == 2 ? proj_impl_w<float, 2>(c, phi_s, rk, out) : proj_impl_w<float, 3>(c, phi_s, rk, out);
    return c->dim == 2 ? proj_impl_w<double, 2>(c, phi_s, rk, out) : proj_impl_w<double, 3>(c, phi_s, rk, out);
}

hipError_t launch_init_droplet(tpf_ctx* c, const double center[3], const double axes[3]) {
    const dim3 g = grid_of(c->n), b(BX, BY);
    const Dims d = dims_of(c->n, c->walls);
    void* dst = c->phi[c->s_yn];
    const double eps = c->P.eps;
#define TPF_INIT(T, D)                                                                        \
    k_init_droplet<T, D><<<g, b, 0, c->stream>>>(d, c->h, eps, center[0], center[1], center[2], \
                                                 axes[0], axes[1], axes[2], tp<T>(dst))
    if (c->mixed) { if (c->dim == 2) TPF_INIT(float, 2); else TPF_INIT(float, 3); }
    else { if (c->dim == 2) TPF_INIT(double, 2); else TPF_INIT(double, 3); }
#undef TPF_INIT
    return hipGetLastError();
}

hipError_t launch_convert_in(tpf_ctx* c, const double* src, void* dst) {
    const int bs = 256;
    const unsigned nb = (unsigned)((c->N + bs - 1) / bs);
    if (c->mixed) k_convert_in<float><<<nb, bs, 0, c->stream>>>(c->N, src, tp<float>(dst));
    else k_convert_in<double><<<nb, bs, 0, c->stream>>>(c->N, src, tp<double>(dst));
    return hipGetLastError();
}

hipError_t launch_convert_out(tpf_ctx* c, const void* src, double* dst) {
    const int bs = 256;
    const unsigned nb = (unsigned)((c->N + bs - 1) / bs);
    if (c->mixed) k_convert_out<float><<<nb, bs, 0, c->stream>>>(c->N, ctp<float>(src), dst);
    else k_convert_out<double><<<nb, bs, 0, c->stream>>>(c->N, ctp<double>(src), dst);
    return hipGetLastError();
}

hipError_t launch_zero_state(tpf_ctx* c, void* dst) {
    const int bs = 256;
    const unsigned nb = (unsigned)((c->N + bs - 1) / bs);
    if (c->mixed) k_fill<float><<<nb, bs, 0, c->stream>>>(c->N, tp<float>(dst), 0.0f);
    else k_fill<double><<<nb, bs, 0, c->stream>>>(c->N, tp<double>(dst), 0.0);
    return hipGetLastError();
}

template <typename T, int DIM, bool W>
static hipError_t diag_impl(hipStream_t st, const int n[3], int walls, const Phys& P, const void* phi,
                            const void* const u[3], const double* p, double* part, double* out) {
    const dim3 g = grid_of(n), b(BX, BY);
    k_diag<T, DIM, W><<<g, b, 0, st>>>(dims_of(n, walls), P, ctp<T>(phi), ctp<T>(u[0]), ctp<T>(u[1]),
                                    ctp<T>(u[2] ? u[2] : u[1]), p, part);
    k_diag_final<<<1, BLOCK, 0, st>>>((int)nblocks_of(n), part, out);
    return hipGetLastError();
}

// the instantiation with or without wall bits
template <typename T, int DIM, typename... A>
static hipError_t diag_impl_w(hipStream_t st, const int n[3], int walls, A... a) {
    return walls ? diag_impl<T, DIM, true>(st, n, walls, a...) : diag_impl<T, DIM, false>(st, n, walls, a...);
}

hipError_t launch_diagnostics_arrays(hipStream_t st, int dim, const int n[3], int walls, int fp32, const Phys& P,
                                     const void* phi, const void* const u[3], const double* p, double* part,
                                     double* out) {
    if (fp32)
        return dim == 2 ? diag_impl_w<float, 2>(st, n, walls, P, phi, u, p, part, out)
                        : diag_impl_w<float, 3>(st, n, walls, P, phi, u, p, part, out);
    return dim == 2 ? diag_impl_w<double, 2>(st, n, walls, P, phi, u, p, part, out)
                    : diag_impl_w<double, 3>(st, n, walls, P, phi, u, p, part, out);
}

hipError_t launch_diagnostics(tpf_ctx* c, const void* phi, const void* const u[3], const double* p) {
    return launch_diagnostics_arrays(c->stream, c->dim, c->n, c->walls, c->mixed, phys_of(c), phi, u, p, c->diag_part,
                                     c->diag_out);
}

}  // namespace tpf
