// CPU check of the library's index arithmetic (tpf_index.hpp, the
// same header the kernels include, compiled here for the host).  For every
// cell of each grid given on the command line (nx ny nz ...) it checks:
//   - Cell::off / nb / off2 (a != b) against the wrapped coordinates, and
//     that every neighbour index lies in [0, N);
//   - with free-slip walls on any set of axes (make_cell_w): off / off2
//     against the mirrored coordinates, nb still wrapped, the wall bits;
//   - ColIndex (z-marching columns): in-plane offsets and neighbour
//     coordinates against the wrapped coordinates, kwrap at both ends;
//   - the XCD block -> tile map: with the grid padded to a multiple of 8
//     blocks, every real tile is taken by exactly one block.
// Prints "ok <cells checked>" and exits 0, or prints the first mismatch and
// exits 1.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "tpf_index.hpp"

using namespace tpf;

static long wrapped(const Dims& d, int i, int j, int k) {
    i = (i % d.nx + d.nx) % d.nx;
    j = (j % d.ny + d.ny) % d.ny;
    k = (k % d.nz + d.nz) % d.nz;
    return ((long)k * d.ny + j) * d.nx + i;
}

static int fail(const char* what, int nx, int ny, int nz, int i, int j, int k, long got, long want) {
    std::printf("MISMATCH %s grid %dx%dx%d cell (%d,%d,%d): got %ld want %ld\n", what, nx, ny, nz, i, j, k, got,
                want);
    return 1;
}

static int check_cells(const Dims& d) {
    const long N = (long)d.nx * d.ny * d.nz;
    for (int k = 0; k < d.nz; ++k)
        for (int j = 0; j < d.ny; ++j)
            for (int i = 0; i < d.nx; ++i) {
                const Cell C = make_cell(d, i, j, k);
                if ((long)C.id != wrapped(d, i, j, k)) return fail("id", d.nx, d.ny, d.nz, i, j, k, C.id, wrapped(d, i, j, k));
                if ((long)C.last != N - 1) return fail("last", d.nx, d.ny, d.nz, i, j, k, C.last, N - 1);
                for (int a = 0; a < 3; ++a)
                    for (int s = -1; s <= 1; s += 2) {
                        int v[3] = {i, j, k};
                        v[a] += s;
                        const long want = wrapped(d, v[0], v[1], v[2]);
                        const long got = C.off(a, s), gnb = C.nb(a, s);
                        if (got != want || gnb != want || want < 0 || want >= N)
                            return fail("off", d.nx, d.ny, d.nz, i, j, k, got, want);
                        for (int b = 0; b < 3; ++b) {
                            if (b == a) continue;
                            for (int t = -1; t <= 1; t += 2) {
                                int w[3] = {v[0], v[1], v[2]};
                                w[b] += t;
                                const long want2 = wrapped(d, w[0], w[1], w[2]);
                                const long got2 = C.off2(a, s, b, t);
                                if (got2 != want2) return fail("off2", d.nx, d.ny, d.nz, i, j, k, got2, want2);
                            }
                        }
                    }
            }
    return 0;
}

// the mirror image of coordinate v on an axis of n cells walled at both ends
static int mirrored(int v, int n) { return v < 0 ? -1 - v : (v >= n ? 2 * n - 1 - v : v); }

// make_cell_w for every wall mask of the grid's axes: off / off2 read the
// mirror image across a walled axis and wrap across the others; nb() wraps
// everywhere; wall(a, s) is set exactly on the first and last cell of a
// walled axis
static int check_walls(const Dims& d0) {
    const int n[3] = {d0.nx, d0.ny, d0.nz};
    for (int walls = 1; walls < 8; ++walls) {
        Dims d = d0;
        d.walls = walls;
        auto want_at = [&](int v0, int v1, int v2) {
            int v[3] = {v0, v1, v2};
            for (int a = 0; a < 3; ++a)
                if ((walls >> a) & 1) v[a] = mirrored(v[a], n[a]);
            return wrapped(d, v[0], v[1], v[2]);
        };
        for (int k = 0; k < d.nz; ++k)
            for (int j = 0; j < d.ny; ++j)
                for (int i = 0; i < d.nx; ++i) {
                    const Cell C = make_cell_w(d, i, j, k);
                    const int c[3] = {i, j, k};
                    for (int a = 0; a < 3; ++a)
                        for (int s = -1; s <= 1; s += 2) {
                            const bool wl = ((walls >> a) & 1) && (s < 0 ? c[a] == 0 : c[a] == n[a] - 1);
                            if (C.wall(a, s) != wl) return fail("wall bit", d.nx, d.ny, d.nz, i, j, k, C.wall(a, s), wl);
                            const bool w2 = ((walls >> a) & 1) && c[a] == 1;
                            if (C.second(a) != w2) return fail("wall second", d.nx, d.ny, d.nz, i, j, k, C.second(a), w2);
                            int v[3] = {i, j, k};
                            v[a] += s;
                            if ((long)C.off(a, s) != want_at(v[0], v[1], v[2]))
                                return fail("wall off", d.nx, d.ny, d.nz, i, j, k, C.off(a, s), want_at(v[0], v[1], v[2]));
                            if ((long)C.nb(a, s) != wrapped(d, v[0], v[1], v[2]))
                                return fail("wall nb", d.nx, d.ny, d.nz, i, j, k, C.nb(a, s), wrapped(d, v[0], v[1], v[2]));
                            for (int b = 0; b < 3; ++b) {
                                if (b == a) continue;
                                for (int t = -1; t <= 1; t += 2) {
                                    int w[3] = {v[0], v[1], v[2]};
                                    w[b] += t;
                                    if ((long)C.off2(a, s, b, t) != want_at(w[0], w[1], w[2]))
                                        return fail("wall off2", d.nx, d.ny, d.nz, i, j, k, C.off2(a, s, b, t),
                                                    want_at(w[0], w[1], w[2]));
                                }
                            }
                        }
                }
    }
    return 0;
}

static int check_columns(const Dims& d) {
    for (int j = 0; j < d.ny; ++j)
        for (int i = 0; i < d.nx; ++i) {
            ColIndex q;
            q.set(d.nx, d.ny, d.nz, i, j);
            for (int k = 0; k < d.nz; ++k) {
                const long c = q.at(k);
                if (c != wrapped(d, i, j, k)) return fail("col at", d.nx, d.ny, d.nz, i, j, k, c, wrapped(d, i, j, k));
                const long xm = (long)(unsigned)(c + q.oxm), xp = (long)(unsigned)(c + q.oxp);
                const long ym = (long)(unsigned)(c + q.oym), yp = (long)(unsigned)(c + q.oyp);
                if (xm != wrapped(d, i - 1, j, k)) return fail("col oxm", d.nx, d.ny, d.nz, i, j, k, xm, wrapped(d, i - 1, j, k));
                if (xp != wrapped(d, i + 1, j, k)) return fail("col oxp", d.nx, d.ny, d.nz, i, j, k, xp, wrapped(d, i + 1, j, k));
                if (ym != wrapped(d, i, j - 1, k)) return fail("col oym", d.nx, d.ny, d.nz, i, j, k, ym, wrapped(d, i, j - 1, k));
                if (yp != wrapped(d, i, j + 1, k)) return fail("col oyp", d.nx, d.ny, d.nz, i, j, k, yp, wrapped(d, i, j + 1, k));
            }
            if (q.im != (i + d.nx - 1) % d.nx || q.ip != (i + 1) % d.nx || q.jm != (j + d.ny - 1) % d.ny ||
                q.jp != (j + 1) % d.ny)
                return fail("col coords", d.nx, d.ny, d.nz, i, j, 0, q.im, (i + d.nx - 1) % d.nx);
            if (q.kwrap(-1) != d.nz - 1 || q.kwrap(d.nz) != 0 || q.kwrap(0) != 0)
                return fail("col kwrap", d.nx, d.ny, d.nz, i, j, 0, q.kwrap(-1), d.nz - 1);
        }
    return 0;
}

// every real tile of a gx x gy x gz tiling is owned by exactly one block of
// the padded 1D grid, with and without the XCD map
static int check_tiles(int gx, int gy, int gz) {
    const long nt = (long)gx * gy * gz;
    const int nb = (int)((nt + NXCD - 1) / NXCD * NXCD);
    for (int xcd = 0; xcd <= 1; ++xcd) {
        std::vector<int> hits((size_t)nt, 0);
        for (int b = 0; b < nb; ++b) {
            int bx, by, bz;
            const int tile = tile_of_block(xcd, nb, b);
            if (tile < 0 || tile >= nb) return fail("tile range", gx, gy, gz, b, xcd, 0, tile, nb);
            if (!tile_coords(tile, gx, gy, gz, bx, by, bz)) continue;
            if (bx < 0 || bx >= gx || by < 0 || by >= gy || bz < 0 || bz >= gz)
                return fail("tile coords", gx, gy, gz, b, xcd, 0, tile, nt);
            hits[(size_t)tile] += 1;
        }
        for (long t = 0; t < nt; ++t)
            if (hits[(size_t)t] != 1) return fail("tile cover", gx, gy, gz, (int)t, xcd, 0, hits[(size_t)t], 1);
    }
    return 0;
}

int main(int argc, char** argv) {
    long cells = 0;
    for (int q = 1; q + 2 < argc; q += 3) {
        const Dims d{std::atoi(argv[q]), std::atoi(argv[q + 1]), std::atoi(argv[q + 2]), 1, 0};
        if (check_cells(d) || check_columns(d)) return 1;
        if ((long)d.nx * d.ny * d.nz <= 100000 && check_walls(d)) return 1;
        // the tilings the kernels launch: 64 x 4 tiles per plane, z-chunks of 1, 8 and 32 planes
        for (int kz : {1, 8, 32})
            if (check_tiles((d.nx + BX - 1) / BX, (d.ny + BY - 1) / BY, (d.nz + kz - 1) / kz)) return 1;
        cells += (long)d.nx * d.ny * d.nz;
    }
    std::printf("ok %ld\n", cells);
    return 0;
}
