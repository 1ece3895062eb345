// Tile geometry shared by the neighbor build and the kernels that read a
// tiled list (force gather/scatter, adjoint, export).
//
// The cell grid is cut into strips of up to kTileMaxStrip consecutive cells
// along x; one workgroup owns one strip (its "home" cells).  The strip's
// 27-cell stencil is the 3 x 3 block of rows (dy, dz in -1..1) times the
// strip's cells plus one on each side.  Staged cell c = rr * (bs + 2) + t,
// with rr = 3 (dz + 1) + (dy + 1) and t = 0 .. bs + 1 for raw x index
// cx0 - 1 + t.  Concatenating the staged cells' atoms (cell-sorted order) in
// that order numbers them 0 .. total - 1: these "slots" are what a tiled
// neighbor entry stores, in 16 bits.  A staged cell whose raw index wrapped
// around the box carries one periodic image; the kernels add that shift to
// the staged positions, so x_i - staged_j is the minimum-image displacement.
// Tiling therefore needs at least 3 cells in every dimension.
#pragma once

#include "common.hpp"

namespace ljmd {

constexpr int kTileMaxStrip = 30;
constexpr int kTileRows = 9;
constexpr int kTileMaxCells = kTileRows * (kTileMaxStrip + 2);  // 288
constexpr int kTileSlots = 65536;                              // 16-bit slots

struct TileArgs {
    const int32_t *cell_start;  // [ncell + 1], cell-sorted starts
    const int32_t *perm;        // cell-sorted position -> atom index
    Grid g;
    Box box;
    int strip;    // home cells per strip
    int nstrips;  // strips per x row
};

struct TileLds {
    int32_t cs[kTileMaxCells];       // first cell-sorted index of staged cell c
    int32_t off[kTileMaxCells + 1];  // first slot of staged cell c
    int32_t home[kTileMaxStrip + 1]; // cell-sorted starts of the home cells
};

struct TileGeom {
    int cx0, bs, cy, cz, ncells;
};

// Packed tiled entries: 4 slots per 64-bit word; word w of tile row s sits at
// ((s / 64) * capw + w) * 64 + s % 64 (rows interleaved per 64-lane wave).
__device__ __forceinline__ int64_t tile_word(int64_t s, int w, int capw) {
    return ((s >> 6) * (int64_t)capw + w) * kWave + (s & 63);
}

// Fill the LDS tables of the strip handled by logical block lb.  Ends with a
// barrier; every thread of the block must call it.
__device__ __forceinline__ TileGeom tile_setup(const TileArgs &a, int64_t lb, TileLds &L) {
    const int nx = a.g.nc[0], ny = a.g.nc[1], nz = a.g.nc[2];
    TileGeom t;
    const int sx = (int)(lb % a.nstrips);
    const int64_t row = lb / a.nstrips;
    t.cy = (int)(row % ny);
    t.cz = (int)(row / ny);
    t.cx0 = sx * a.strip;
    t.bs = min(a.strip, nx - t.cx0);
    const int w = t.bs + 2;
    t.ncells = kTileRows * w;
    for (int c = threadIdx.x; c < t.ncells; c += blockDim.x) {
        const int rr = c / w, tt = c - rr * w;
        const int zz = (t.cz + rr / 3 - 1 + nz) % nz;
        const int yy = (t.cy + rr % 3 - 1 + ny) % ny;
        const int xx = (t.cx0 - 1 + tt + nx) % nx;
        const int64_t cell = ((int64_t)zz * ny + yy) * nx + xx;
        const int32_t c0 = a.cell_start[cell];
        L.cs[c] = c0;
        L.off[c + 1] = a.cell_start[cell + 1] - c0;
    }
    if ((int)threadIdx.x <= t.bs)
        L.home[threadIdx.x] = a.cell_start[((int64_t)t.cz * ny + t.cy) * nx + t.cx0 + threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) {
        L.off[0] = 0;
        for (int c = 1; c <= t.ncells; ++c) L.off[c] += L.off[c - 1];
    }
    __syncthreads();
    return t;
}

// Periodic shift of staged cell c (added to the staged positions).
__device__ __forceinline__ void tile_shift(const TileArgs &a, const TileGeom &t, int c,
                                           double &sx, double &sy, double &sz) {
    const int w = t.bs + 2;
    const int rr = c / w, tt = c - rr * w;
    const int xr = t.cx0 - 1 + tt, yr = t.cy + rr % 3 - 1, zr = t.cz + rr / 3 - 1;
    sx = xr < 0 ? -a.box.L[0] : (xr >= a.g.nc[0] ? a.box.L[0] : 0.0);
    sy = yr < 0 ? -a.box.L[1] : (yr >= a.g.nc[1] ? a.box.L[1] : 0.0);
    sz = zr < 0 ? -a.box.L[2] : (zr >= a.g.nc[2] ? a.box.L[2] : 0.0);
}

// Image code of staged cell c (bits 2d..2d+1: 1 = subtract L, 2 = add L to
// x_i - x_j), as stored by the global list format.
__device__ __forceinline__ uint32_t tile_code(const TileArgs &a, const TileGeom &t, int c) {
    const int w = t.bs + 2;
    const int rr = c / w, tt = c - rr * w;
    const int xr = t.cx0 - 1 + tt, yr = t.cy + rr % 3 - 1, zr = t.cz + rr / 3 - 1;
    uint32_t code = xr < 0 ? 2u : (xr >= a.g.nc[0] ? 1u : 0u);
    code |= yr < 0 ? 8u : (yr >= a.g.nc[1] ? 4u : 0u);
    code |= zr < 0 ? 32u : (zr >= a.g.nc[2] ? 16u : 0u);
    return code;
}

// Staged cell holding slot q (largest c with off[c] <= q).
__device__ __forceinline__ int tile_cell_of(const TileLds &L, int ncells, int32_t q) {
    int lo = 0, hi = ncells - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.off[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Per-row staging table.  Within stencil row rr the staged cells are the
// strip's cells plus one on each side; the middle cells (t = 1 .. bs) are
// consecutive cells of one grid row, hence one contiguous cell-sorted range,
// and only the end cells (t = 0, t = bs + 1) can wrap around the box.  So a
// slot q of row rr lies in one of three segments and its cell-sorted index is
// q + g[seg]; the x shift is nonzero only for the end segments.
struct RowTab {
    int32_t b1[kTileRows];  // first slot after segment 0 (cell t = 0)
    int32_t b2[kTileRows];  // first slot after segment 1 (cells t = 1 .. bs)
    int32_t r1[kTileRows];  // first slot after the row
    int32_t g0[kTileRows], g1[kTileRows], g2[kTileRows];
    double sx0[kTileRows], sx2[kTileRows], sy[kTileRows], sz[kTileRows];
};

// Fill R from the tile tables; threads 0..8 each fill one row.  The caller
// synchronizes before reading R.
__device__ __forceinline__ void tile_rows(const TileArgs &a, const TileGeom &t, const TileLds &L,
                                          RowTab &R) {
    const int rr = threadIdx.x;
    if (rr >= kTileRows) return;
    const int w = t.bs + 2;
    const int c0 = rr * w, c2 = rr * w + t.bs + 1;
    R.b1[rr] = L.off[c0 + 1];
    R.b2[rr] = L.off[c2];
    R.r1[rr] = L.off[c2 + 1];
    R.g0[rr] = L.cs[c0] - L.off[c0];
    R.g1[rr] = L.cs[c0 + 1] - L.off[c0 + 1];
    R.g2[rr] = L.cs[c2] - L.off[c2];
    double sx, sy, sz;
    tile_shift(a, t, c0, sx, sy, sz);
    R.sx0[rr] = sx;
    R.sy[rr] = sy;
    R.sz[rr] = sz;
    tile_shift(a, t, c2, sx, sy, sz);
    R.sx2[rr] = sx;
}

// Stage slots [lo, hi) of the strip into LDS (index q - lo): positions plus
// their periodic shift, and optionally types, atom indices and a second
// per-atom vector (the adjoint's upstream gradient).  Loads are issued in
// batches of four slots per thread before any of them is used, so their
// latencies overlap.  `sorted`: the cell order is the atom order (perm is the
// identity) and the perm lookup is skipped.
template <int T, bool IDX, bool VEC>
__device__ __forceinline__ void tile_stage(const TileArgs &a, const RowTab &R, int32_t lo,
                                           int32_t hi, bool sorted, const double *x,
                                           const int32_t *type, const double *vec, double *sx,
                                           double *sy, double *sz, uint8_t *st, int32_t *su,
                                           double *vx, double *vy, double *vz) {
    const int32_t step = (int32_t)blockDim.x;
    for (int32_t base = lo + (int32_t)threadIdx.x; base < hi; base += 4 * step) {
        int64_t u[4];
        int rr[4], seg[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int32_t q = base + i * step;
            int r = 0;
#pragma unroll
            for (int k = 0; k < kTileRows - 1; ++k) r += q >= R.r1[k] ? 1 : 0;
            const int sg = q < R.b1[r] ? 0 : (q < R.b2[r] ? 1 : 2);
            const int32_t g = q + (sg == 0 ? R.g0[r] : (sg == 1 ? R.g1[r] : R.g2[r]));
            rr[i] = r;
            seg[i] = sg;
            u[i] = q < hi ? (int64_t)g : 0;
        }
        if (!sorted) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (base + i * step < hi) u[i] = a.perm[u[i]];
        }
        double px[4], py[4], pz[4], gx[4], gy[4], gz[4];
        int tt[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (base + i * step < hi) {
                px[i] = x[3 * u[i]];
                py[i] = x[3 * u[i] + 1];
                pz[i] = x[3 * u[i] + 2];
                if (T > 1) tt[i] = type[u[i]];
                if (VEC) {
                    gx[i] = vec[3 * u[i]];
                    gy[i] = vec[3 * u[i] + 1];
                    gz[i] = vec[3 * u[i] + 2];
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int32_t q = base + i * step;
            if (q < hi) {
                const int r = rr[i];
                const double shx = seg[i] == 0 ? R.sx0[r] : (seg[i] == 2 ? R.sx2[r] : 0.0);
                const int32_t m = q - lo;
                sx[m] = px[i] + shx;
                sy[m] = py[i] + R.sy[r];
                sz[m] = pz[i] + R.sz[r];
                if (T > 1) st[m] = (uint8_t)tt[i];
                if (IDX) su[m] = (int32_t)u[i];
                if (VEC) {
                    vx[m] = gx[i];
                    vy[m] = gy[i];
                    vz[m] = gz[i];
                }
            }
        }
    }
}

// Home cell (0 .. bs-1) of cell-sorted index s inside the strip.
__device__ __forceinline__ int tile_home_cell(const TileLds &L, const TileGeom &t, int32_t s) {
    int hx = 0;
    while (hx + 1 < t.bs && s >= L.home[hx + 1]) ++hx;
    return hx;
}

}  // namespace ljmd
