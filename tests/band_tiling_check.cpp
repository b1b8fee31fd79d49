// Host-only brute force over random grids: the band kernel's tiles (band_box
// boxes, band_xtiles x tiles, rows of BAND_TY, z chunks of 32 except z boxes,
// which are walked whole) cover every band point of the compute box exactly
// once, and along x the points up to the whole-tile bounds of the non-band x
// range (band_range_x), and nothing else; and, on geometries the library fuses (each x band at most BAND_TX wide,
// the x bands and the z bands each far enough apart), every x-layer point lies
// in the same tile row as each band point that reads it, and every z-layer
// point in the same z-box walk as its readers, with the walk's first planes
// outside the layers and at least 5 planes deep.  And the LDS staging of every
// tile (tiles of BAND_TY rows in even cases, BAND_TY_TALL in odd ones): each x and y stencil tap of each of its points is found in the slot that
// the tile's lanes fill with that position (their own u^n, or a halo value from
// band_halo), loaded from a position the field buffer holds (rows within the
// frame of fy = max(4, ext + 4), columns within 4 of the grid).  Prints
// "ok <cases> <fused>".
#include "fdtd_dev.hpp"

#include <array>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

namespace {
bool fused(const int *n, const int *lo, const int *hi) {
    if (lo[0] + hi[0] > 0 && (lo[0] + FDTD_R > BAND_TX || hi[0] + FDTD_R > BAND_TX || n[0] < lo[0] + hi[0] + 2 * FDTD_R))
        return false;
    return lo[2] + hi[2] == 0 || n[2] >= lo[2] + hi[2] + 2 * FDTD_R;
}
struct Owner {
    int box = -1, tx, ty, zc, za, zb;
};
// dense owner table over the compute box (x in [0, nx), y, z in [-ext, n + ext))
struct Table {
    int nx, ny, nz, ext;
    std::vector<Owner> v;
    Table(int nx_, int ny_, int nz_, int ext_) : nx(nx_), ny(ny_ + 2 * ext_), nz(nz_ + 2 * ext_), ext(ext_) {
        v.resize((size_t)nx * ny * nz);
    }
    bool inside(int x, int y, int z) const {
        return x >= 0 && x < nx && y + ext >= 0 && y + ext < ny && z + ext >= 0 && z + ext < nz;
    }
    Owner &at(int x, int y, int z) { return v[((size_t)(z + ext) * ny + (y + ext)) * nx + x]; }
};
// Replay of one tile's LDS staging (the band kernel's slots and band_halo):
// every tap of every point of the tile is the position its slot is filled
// with, from a position inside the field buffer's rows [-fy, ny + fy) and
// columns [-4, nx + 4).
bool staging_ok(const int *n, int fy, int x0, int x1, int yt, int yend, int ty) {
    struct Fill {
        int x, y;
        bool held;
    };
    const int LB = band_lds(ty);
    std::vector<Fill> slot(LB, Fill{0, 0, false});
    std::vector<bool> set(LB, false);
    auto held = [&](int xp, int yp) { return xp >= -4 && xp < n[0] + 4 && yp >= -fy && yp < n[1] + fy; };
    auto put = [&](int c, int r) {
        const int i = r * kBandLW + c, xp = x0 - FDTD_R + c, yp = yt - FDTD_R + r;
        if (i < 0 || i >= LB - 1) return false;
        slot[i] = Fill{xp, yp, held(xp, yp)};
        set[i] = true;
        return true;
    };
    for (int t = 0; t < BAND_TX * ty; ++t) {
        if (!put(FDTD_R + t % BAND_TX, FDTD_R + t / BAND_TX)) return false;
        for (int k = 0; k < 2; ++k) {
            int c, r;
            band_halo(t, k, ty, c, r);
            if (c >= 0 && !put(c, r)) return false;
        }
    }
    for (int t = 0; t < BAND_TX * ty; ++t) {
        const int lx = t % BAND_TX, ly = t / BAND_TX, x = x0 + lx, y = yt + ly;
        if (x >= x1 || y >= yend) continue;
        const int own = (ly + FDTD_R) * kBandLW + lx + FDTD_R;
        for (int l = 1; l <= FDTD_R; ++l) {
            const int idx[4] = {own - l, own + l, own - l * kBandLW, own + l * kBandLW};
            const int px[4] = {x - l, x + l, x, x}, py[4] = {y, y, y - l, y + l};
            for (int j = 0; j < 4; ++j) {
                const Fill &f = slot[idx[j]];
                if (!set[idx[j]] || f.x != px[j] || f.y != py[j] || !f.held) return false;
            }
        }
    }
    return true;
}
}  // namespace

int main(int argc, char **argv) {
    if (argc > 1 && std::string(argv[1]) == "ranges") {
        // "n lo hi" per line on stdin -> the z-march's x range "a b" (band_range_x)
        int n, lo, hi;
        while (scanf("%d %d %d", &n, &lo, &hi) == 3) {
            int a, b, e0, e1;
            band_range_x(n, lo, hi, a, b, e0, e1);
            printf("%d %d\n", a, b);
        }
        return 0;
    }
    const int cases = argc > 1 ? atoi(argv[1]) : 2000;
    srand(7);
    long nf = 0;
    for (int it = 0; it < cases; ++it) {
        const int th = it % 2 ? BAND_TY_TALL : BAND_TY;   // tile rows: both heights the library uses
        int n[3], lo[3], hi[3], gh[3] = {0, 0, 0};
        for (int d = 0; d < 3; ++d) {
            n[d] = 9 + rand() % 60;
            const int m = (n[d] - 1) / 2;
            lo[d] = rand() % 3 ? rand() % (m + 1) : 0;
            hi[d] = rand() % 3 ? rand() % (m + 1) : 0;
        }
        int ext = 0;
        if (rand() % 4 == 0) {   // ghost (loopback) y, maybe z: no layers there
            gh[1] = 1;
            lo[1] = hi[1] = 0;
            if (rand() % 2) {
                gh[2] = 1;
                lo[2] = hi[2] = 0;
            }
            ext = rand() % 13;
        }
        Table own(n[0], n[1], n[2], ext);
        for (int b = 0; b < 6; ++b) {
            int blo[3], bhi[3];
            band_box(n, lo, hi, gh, ext, b, blo, bhi);
            if (bhi[0] <= blo[0] || bhi[1] <= blo[1] || bhi[2] <= blo[2]) continue;
            int x0, x1;
            const int ntx = band_xtiles(n[0], lo[0], hi[0], b, blo[0], bhi[0], 0, &x0, &x1);
            const int nty = (bhi[1] - blo[1] + th - 1) / th;
            const int nzc = b < 2 ? 1 : (bhi[2] - blo[2] + 31) / 32;
            for (int zc = 0; zc < nzc; ++zc)
                for (int ty = 0; ty < nty; ++ty)
                    for (int tx = 0; tx < ntx; ++tx) {
                        band_xtiles(n[0], lo[0], hi[0], b, blo[0], bhi[0], tx, &x0, &x1);
                        if (x1 <= x0 || x1 - x0 > BAND_TX) {
                            printf("FAIL tile width %d\n", x1 - x0);
                            return 1;
                        }
                        if (!staging_ok(n, gh[1] ? ext + 4 : 4, x0, x1, blo[1] + ty * th, bhi[1], th)) {
                            printf("FAIL LDS staging of tile box %d tx %d ty %d\n", b, tx, ty);
                            return 1;
                        }
                        const int za = b < 2 ? blo[2] : blo[2] + 32 * zc, zb = b < 2 ? bhi[2] : std::min(za + 32, bhi[2]);
                        for (int z = za; z < zb; ++z)
                            for (int r = 0; r < th; ++r) {
                                const int y = blo[1] + ty * th + r;
                                if (y >= bhi[1]) continue;
                                for (int x = x0; x < x1; ++x) {
                                    Owner &w = own.at(x, y, z);
                                    if (w.box >= 0) {
                                        printf("FAIL point (%d,%d,%d) in two tiles\n", x, y, z);
                                        return 1;
                                    }
                                    w = Owner{b, tx, ty, zc, za, zb};
                                }
                            }
                    }
            band_xtiles(n[0], lo[0], hi[0], b, blo[0], bhi[0], 1 << 20, &x0, &x1);   // idle work item
            if (x1 > x0) {
                printf("FAIL idle item has points\n");
                return 1;
            }
        }
        auto in_band_d = [&](int d, int c) {
            return (lo[d] > 0 && c < lo[d] + FDTD_R) || (hi[d] > 0 && c >= n[d] - hi[d] - FDTD_R);
        };
        auto in_slab_d = [&](int d, int c) { return c >= 0 && c < n[d] && (c < lo[d] || c >= n[d] - hi[d]); };
        int e0[3], e1[3];
        for (int d = 0; d < 3; ++d) {
            int a, b;
            band_range(n[d], lo[d], hi[d], gh[d], ext, a, b, e0[d], e1[d]);
        }
        // the x band boxes also hold the points between an x band and the whole-tile
        // bound of the non-band x range (band_range_x), which lie in no band
        int xa, xb, xe0, xe1;
        band_range_x(n[0], lo[0], hi[0], xa, xb, xe0, xe1);
        {
            // the range only narrows, to [BAND_TX, ...) at the low end, and stays non-empty
            int a0, b0, f0, f1;
            band_range(n[0], lo[0], hi[0], 0, 0, a0, b0, f0, f1);
            if (xa < a0 || xb > b0 || xa > xb || (xa != a0 && xa != BAND_TX)) {
                printf("FAIL x range [%d, %d) for n %d, layers %d %d\n", xa, xb, n[0], lo[0], hi[0]);
                return 1;
            }
        }
        for (int z = e0[2]; z < e1[2]; ++z)
            for (int y = e0[1]; y < e1[1]; ++y)
                for (int x = 0; x < n[0]; ++x) {
                    const bool band = in_band_d(0, x) || in_band_d(1, y) || in_band_d(2, z) || x < xa || x >= xb;
                    if (band != (own.at(x, y, z).box >= 0)) {
                        printf("FAIL coverage at (%d,%d,%d): band %d\n", x, y, z, band);
                        return 1;
                    }
                }
        if (!fused(n, lo, hi)) continue;
        ++nf;
        for (int z = e0[2]; z < e1[2]; ++z)
        for (int y = e0[1]; y < e1[1]; ++y)
        for (int x = 0; x < n[0]; ++x) {
            const Owner &o = own.at(x, y, z);
            if (o.box < 0) continue;
            if (in_band_d(0, x))
                for (int l = -FDTD_R; l <= FDTD_R; ++l) {
                    if (!l || !in_slab_d(0, x + l)) continue;
                    const Owner &p = own.at(x + l, y, z);
                    if (p.box != o.box || p.tx != o.tx || p.ty != o.ty || p.zc != o.zc) {
                        printf("FAIL x-layer point (%d,%d,%d) outside its reader's tile row\n", x + l, y, z);
                        return 1;
                    }
                }
            if (in_slab_d(2, z) && o.box >= 2) {
                printf("FAIL z-layer point outside the z boxes\n");
                return 1;
            }
            if (in_band_d(2, z)) {
                for (int l = -FDTD_R; l <= FDTD_R; ++l) {
                    if (!l || !in_slab_d(2, z + l)) continue;
                    const Owner &p = own.at(x, y, z + l);
                    if (p.box != o.box || p.tx != o.tx || p.ty != o.ty) {
                        printf("FAIL z-layer point outside its reader's walk\n");
                        return 1;
                    }
                }
                for (int p = o.za - FDTD_R; p < o.za; ++p)
                    if (in_slab_d(2, p)) {
                        printf("FAIL z walk starts next to a layer plane\n");
                        return 1;
                    }
                if (o.zb - o.za < FDTD_R + 1) {
                    printf("FAIL z walk shorter than 5 planes\n");
                    return 1;
                }
            }
        }
    }
    printf("ok %d %ld\n", cases, nf);
    return 0;
}
