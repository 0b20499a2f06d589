// Index arithmetic of the [z][y][x] cell grid: block shape, the XCD-aware
// block -> tile map, a cell's six neighbour offsets (periodic, or mirrored at
// free-slip walls) and the column offsets of the z-marching kernels.
// Everything here is plain integer code callable from the host too, so the
// CPU test-suite runs these exact functions over whole grids and checks every
// offset against the wrapped or mirrored coordinates (tests/index_check.cpp).
#pragma once

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define TPF_HD __host__ __device__ __forceinline__
#else
#define TPF_HD inline
#endif

namespace tpf {

// 256-thread blocks laid out as 64 consecutive x cells (one wave64 = one
// coalesced row segment) by 4 rows in y; grid z walks the z planes.
constexpr int BX = 64;
constexpr int BY = 4;
constexpr int BLOCK = BX * BY;

struct Dims {
    int nx, ny, nz;
    int xcd;        // 1: XCD slab tiling of the 1D block grid, 0: tile = block id
    int walls;      // bit a: free-slip walls at both ends of axis a (make_cell_w)
};

// wrap an index that is at most one period out of range
TPF_HD int wrapc(int v, int n) {
    v = v < 0 ? v + n : v;
    return v >= n ? v - n : v;
}

// A cell and the offsets of its six neighbours; a, b are physical axes
// (0 = x).  Indices are 32-bit (grids up to 2^31 cells): neighbour
// addressing is one integer add, and the loads use a scalar base plus a
// 32-bit vector offset.  The offsets land inside the grid for every cell
// (checked cell by cell on the CPU); a build with TPF_BOUNDS_CLAMP defined
// also clamps every neighbour index to [0, N-1], for debugging an index
// change without risking an access outside the array.
//
// Free-slip walls.  wl has bit 4a set when the cell is the first cell of a
// walled axis a, bit 4a+1 when it is the last and bit 4a+2 when it is the
// second (its lower neighbour's lower face is the wall).  off() and off2() then
// read a cell field's mirror image: the neighbour across the wall is the
// cell itself (an even reflection).  nb() stays periodic: the pressure
// solver closes the box by zero face coefficients on the wall faces instead,
// and the wrapped neighbour it reads there is multiplied by that zero.  What
// other field kinds read across a wall (odd normals, face fields that are 0
// on the wall) is decided by the operator bodies through wall().  Cells made
// by make_cell() have wl = 0, which folds every wall test away.
struct Cell {
    int i, j, k;
    unsigned id;
    unsigned last;  // N - 1
    unsigned wl;    // wall bits, see above
    int o[3][2];    // o[a][0]: offset to c - e_a, o[a][1]: offset to c + e_a (periodic)
    TPF_HD unsigned bound(unsigned q) const {
#ifdef TPF_BOUNDS_CLAMP
        return q < last ? q : last;
#else
        return q;
#endif
    }
    // the cell is next to a wall on side s of axis a
    TPF_HD bool wall(int a, int s) const { return (wl >> (4 * a + (s > 0))) & 1u; }
    // the cell is the second along a walled axis a
    TPF_HD bool second(int a) const { return (wl >> (4 * a + 2)) & 1u; }
    TPF_HD unsigned mo(int a, int s) const { return wall(a, s) ? 0u : (unsigned)o[a][s > 0]; }
    TPF_HD unsigned off(int a, int s) const { return bound(id + mo(a, s)); }
    // the periodic neighbour, never clamped (pressure-solver kernels)
    TPF_HD unsigned nb(int a, int s) const { return id + (unsigned)o[a][s > 0]; }
    // c + s e_a + t e_b for a != b only: each offset is the one of cell c, so
    // two shifts compose only when they move along different axes
    TPF_HD unsigned off2(int a, int s, int b, int t) const { return bound(id + mo(a, s) + mo(b, t)); }
};

TPF_HD Cell make_cell(const Dims& d, int i, int j, int k) {
    Cell C;
    C.i = i;
    C.j = j;
    C.k = k;
    const int nx = d.nx, plane = d.nx * d.ny;
    C.id = (unsigned)((k * d.ny + j) * nx + i);
    C.last = (unsigned)(plane * d.nz - 1);
    C.wl = 0u;
    C.o[0][0] = i == 0 ? nx - 1 : -1;
    C.o[0][1] = i == nx - 1 ? 1 - nx : 1;
    C.o[1][0] = j == 0 ? (d.ny - 1) * nx : -nx;
    C.o[1][1] = j == d.ny - 1 ? (1 - d.ny) * nx : nx;
    C.o[2][0] = k == 0 ? (d.nz - 1) * plane : -plane;
    C.o[2][1] = k == d.nz - 1 ? (1 - d.nz) * plane : plane;
    return C;
}

// make_cell with the wall bits of d.walls
TPF_HD Cell make_cell_w(const Dims& d, int i, int j, int k) {
    Cell C = make_cell(d, i, j, k);
    const int v[3] = {i, j, k}, n[3] = {d.nx, d.ny, d.nz};
    for (int a = 0; a < 3; ++a) {
        if (!((d.walls >> a) & 1)) continue;
        if (v[a] == 0) C.wl |= 1u << (4 * a);
        if (v[a] == n[a] - 1) C.wl |= 2u << (4 * a);
        if (v[a] == 1) C.wl |= 4u << (4 * a);
    }
    return C;
}

// XCD-aware tiling.  Workgroups are dealt to the 8 XCDs round robin by their
// linear id, and each XCD has its own L2.  Grids are therefore 1D (padded to a
// multiple of 8) and block b of nb works on tile (b % 8) * (nb / 8) + b / 8:
// every XCD owns one contiguous run of tiles (a slab of z planes), so the y
// and z neighbours a stencil reads sit in the same L2.  Tiles are x-fastest.
constexpr int NXCD = 8;

TPF_HD int tile_of_block(int xcd, int nb, int b) {
    return xcd ? (b % NXCD) * (nb / NXCD) + b / NXCD : b;
}

// tile -> (bx, by, bz) of a gx x gy x gz tiling; false for padding tiles
TPF_HD bool tile_coords(int tile, int gx, int gy, int gz, int& bx, int& by, int& bz) {
    if (tile >= gx * gy * gz) return false;
    bx = tile % gx;
    by = (tile / gx) % gy;
    bz = tile / (gx * gy);
    return true;
}

// Periodic in-plane offsets of one (i, j) column of the z-marching kernels;
// a plane k of the column is cell k * plane + row.
struct ColIndex {
    int nx, ny, nz;
    int i, j;
    unsigned plane, row;
    int oxm, oxp, oym, oyp;   // periodic in-plane neighbour offsets
    int im, ip, jm, jp;       // neighbour coordinates
    TPF_HD void set(int nx_, int ny_, int nz_, int i_, int j_) {
        nx = nx_;
        ny = ny_;
        nz = nz_;
        i = i_;
        j = j_;
        plane = (unsigned)(nx * ny);
        row = (unsigned)(j * nx + i);
        oxm = i == 0 ? nx - 1 : -1;
        oxp = i == nx - 1 ? 1 - nx : 1;
        oym = j == 0 ? (ny - 1) * nx : -nx;
        oyp = j == ny - 1 ? (1 - ny) * nx : nx;
        im = i == 0 ? nx - 1 : i - 1;
        ip = i == nx - 1 ? 0 : i + 1;
        jm = j == 0 ? ny - 1 : j - 1;
        jp = j == ny - 1 ? 0 : j + 1;
    }
    TPF_HD unsigned at(int k) const { return (unsigned)k * plane + row; }
    TPF_HD int kwrap(int k) const { return k < 0 ? k + nz : (k >= nz ? k - nz : k); }
};

}  // namespace tpf
