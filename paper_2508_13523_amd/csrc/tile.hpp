// Tile geometry shared by the neighbor build and the kernels that read a
// tiled list (force gather/scatter, adjoint, export).
//
// The cell grid is cut into tiles of up to ext[0] x ext[1] x ext[2] cells
// (fewer at the upper edge of the grid); one workgroup owns one tile (its
// "home" cells).  The tile's 27-cell stencil is the block of cells one wider
// on every side: (b[1] + 2) (b[2] + 2) "staged rows" along x, each of
// b[0] + 2 cells.  Staged cell c = r * w + t, w = b[0] + 2, with stencil row
// r = (dz + 1) (b[1] + 2) + (dy + 1) for dy = -1 .. b[1], dz = -1 .. b[2], and
// raw x index c0[0] - 1 + t.  Concatenating the staged cells' atoms
// (cell-sorted order) in that order numbers them 0 .. total - 1: these
// "slots" are what a tiled neighbor entry stores, in 16 bits.  A staged cell
// whose raw index wrapped around the box carries one periodic image; the
// force kernels add that shift to the staged positions, so that
// x_i - staged_j is the minimum-image displacement.  Tiling needs at least 3
// cells in every dimension for a single system; in a batch a dimension may
// have 2 cells (then a staged row holds the same cell twice, under two
// periodic images, and the neighbor cutoff, at most half the box, admits at
// most one of the images of any atom).
//
// The home cells of one staged row (t = 1 .. b[0]) are consecutive cells of
// one grid row, so a tile's home atoms are b[1] b[2] contiguous runs of the
// cell order ("home rows"), enumerated one after the other.
#pragma once

#include "common.hpp"

namespace ljmd {

constexpr int kTileThreads = 512;  // workgroup size of every tiled kernel
constexpr int kTileMaxRows = 32;    // staged rows (b[1] + 2) (b[2] + 2)
constexpr int kTileMaxHome = 16;    // home rows b[1] b[2]
constexpr int kTileMaxCells = 288;  // staged cells (b[0] + 2) * rows
constexpr int kTileSlots = 65536;   // 16-bit slots

// Home atoms a tile of a tiled batch list is cut for when the batch does not
// set it (ljmd_batch.tile_atoms); the autotuner searches other values.
constexpr int kBatchTileAtomsDefault = 300;
constexpr int kBatchTileAtomsMin = 32, kBatchTileAtomsMax = 4096;

// Strip length along x of a batch system's tiles and build strips: about
// `target` home atoms, at most 30 cells and at most the grid row, then
// evened out over the strips of the row so that none is a short remainder (a
// one-cell strip stages 27 cells for one cell's atoms).
__host__ __device__ inline int batch_strip(double mean, int nc0, int target) {
    // clamped before the conversion: a nearly empty system has a tiny mean
    const double want = mean > 0.0 ? (double)target / mean : 30.0;
    int b = want >= 30.0 ? 30 : (want < 1.0 ? 1 : (int)want);
    if (b > nc0) b = nc0;
    const int ns = (nc0 + b - 1) / b;
    return (nc0 + ns - 1) / ns;
}

// Cells along y of the tiles of a tiled batch list (one strip along x, one
// cell along z): about `target` home atoms within the tile tables' limits
// (staged rows, home rows, staged cells), evened out over the row.  Small
// systems have short grid rows, so their strips alone are small tiles.
__host__ __device__ inline int batch_tile_rows(double mean, int strip, int nc1, int target) {
    const double per_row = mean * strip;
    const double want = per_row > 0.0 ? (double)target / per_row : 1.0;
    int e = want >= (double)kTileMaxHome ? kTileMaxHome : (int)want;
    const int lim_rows = kTileMaxRows / 3 - 2;
    const int lim_cells = kTileMaxCells / (3 * (strip + 2)) - 2;
    if (e > lim_rows) e = lim_rows;
    if (e > kTileMaxHome) e = kTileMaxHome;
    if (e > lim_cells) e = lim_cells;
    if (e > nc1) e = nc1;
    if (e < 1) e = 1;
    const int nt = (nc1 + e - 1) / e;
    return (nc1 + nt - 1) / nt;
}

struct TileArgs {
    const int32_t *cell_start;  // [ncell + 1], cell-sorted starts
    const int32_t *perm;        // cell-sorted position -> atom index
    Grid g;
    Box box;
    int ext[3];    // home cells per tile along x, y, z
    int ntile[3];  // tiles along x, y, z
    // Batch of independent systems (reps non-null): workgroup b takes tile
    // b - reps[r].tile_base of system r = tile_rep[b]; system r's tiles are
    // reps[r].strip cells along x, reps[r].ey along y and one along z, its
    // cells start at reps[r].cell_base of cell_start, and nbatch is the
    // number of tiles of all systems.
    const RepInfo *reps;
    const int32_t *tile_rep;
    int64_t nbatch;
};

// The tile arguments of workgroup lb and its tile within its own system.
__device__ __forceinline__ TileArgs tile_args_of(const TileArgs &a, int64_t lb, int64_t &lbl) {
    if (!a.reps) {
        lbl = lb;
        return a;
    }
    const RepInfo &r = a.reps[a.tile_rep[lb]];
    TileArgs t = a;
    t.cell_start = a.cell_start + r.cell_base;
    t.g = r.g;
    t.box = r.box;
    t.ext[0] = r.strip;
    t.ext[1] = r.ey;
    t.ext[2] = 1;
    t.ntile[0] = r.nstripx;
    t.ntile[1] = (r.g.nc[1] + r.ey - 1) / r.ey;
    t.ntile[2] = r.g.nc[2];
    lbl = lb - r.tile_base;
    return t;
}

struct TileLds {
    int32_t cs[kTileMaxCells];       // first cell-sorted index of staged cell c
    int32_t off[kTileMaxCells + 1];  // first slot of staged cell c
    int32_t hs[kTileMaxHome];        // first cell-sorted index of home row h
    int32_t hoff[kTileMaxHome + 1];  // home atoms in the home rows before h
};

struct TileGeom {
    int c0[3];   // first home cell
    int b[3];    // home cells per dimension
    int w;       // cells per staged row, b[0] + 2
    int nrows;   // staged rows
    int ncells;  // staged cells
    int nhome;   // home rows, b[1] b[2]
};

// Packed tiled entries: 4 slots per 64-bit word; word w of tile row s sits at
// ((s / 64) * capw + w) * 64 + s % 64 (rows interleaved per 64-lane wave).
// A row of nn entries is padded to a multiple of kRowPad entries (two words)
// with the "null slot" `total` (the tile's slot count): readers that stage a
// null position there, far from every atom, may then process whole pairs of
// words without masking.  capw, the words per row, is a multiple of 2.
constexpr int kRowPad = 8;
__host__ __device__ __forceinline__ int tile_row_words(int nn) {
    return (nn + kRowPad - 1) / kRowPad * (kRowPad / 4);
}
__host__ __device__ __forceinline__ int tile_capw(int cap) { return tile_row_words(cap); }

__device__ __forceinline__ int64_t tile_word(int64_t s, int w, int capw) {
    return ((s >> 6) * (int64_t)capw + w) * kWave + (s & 63);
}

// Zero an FP64 reciprocal square distance outside the cutoff by clearing
// its upper 32 bits: what remains is below 2^-1022, so r^-6 underflows to
// zero and with it the pair force and energy (one select instead of two).
__device__ __forceinline__ double cut_r2i(double r2i, bool in) {
    const uint64_t b = __double_as_longlong(r2i);
    const uint32_t hi = in ? (uint32_t)(b >> 32) : 0u;
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | (uint32_t)b));
}

// 1/a and 1/b from one reciprocal: y = 1/(a b) (hardware estimate and one
// Newton step), 1/a = b y, 1/b = a y.  Relative error a few 1e-15 for the
// square distances met here (products far from over- and underflow).
__device__ __forceinline__ void recip2(double a, double b, double &ia, double &ib) {
    const double p = a * b;
    const double y0 = __builtin_amdgcn_rcp(p);
    const double y = fma(y0, fma(-p, y0, 1.0), y0);
    ia = b * y;
    ib = a * y;
}

// The tiles of this workgroup when gridDim.x workgroups (at most ntiles, at
// least 8 when fewer than ntiles) walk ntiles tiles: the hardware hands
// workgroup b to XCD b % 8, and each XCD takes one contiguous range of tiles
// (its own L2 then holds the stencil atoms its tiles share), its workgroups
// striding through the range.  With one workgroup per tile this is the
// xcd_remap order.
struct TileWalk {
    int64_t first, end, step;
};
__device__ __forceinline__ TileWalk tile_walk(int64_t ntiles) {
    const int64_t nb = gridDim.x;
    const int x = (int)(blockIdx.x % kXcds);
    const int64_t l = blockIdx.x / kXcds;
    const int64_t step = nb / kXcds + (x < nb % kXcds ? 1 : 0);
    const int64_t q = ntiles / kXcds, r = ntiles % kXcds;
    const int64_t start = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    const int64_t len = q + (x < r ? 1 : 0);
    return TileWalk{start + l, start + len, step};
}

// Lanes per home atom chosen per tile from its home count nh: the most lanes
// (8, 4, 2 or 1) that still cover all home atoms in one pass of the workgroup.
__device__ __forceinline__ int tile_pass_lanes(int32_t nh) {
    return nh <= kTileThreads / 8   ? 8
           : nh <= kTileThreads / 4 ? 4
           : nh <= kTileThreads / 2 ? 2
                                    : 1;
}

// Coordinate staged at the null slot: the null partner is then more than
// 1e9 away from any atom of a box shorter than 1e9 (checked by the API), far
// outside every cutoff, while r^2 (about 3e20) stays far from overflow when
// two of them are multiplied.
constexpr double kNullCoord = 1.0e10;

__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = (int)(threadIdx.x & 63);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}

struct RowTab;
__device__ __forceinline__ void tile_row_fill(const TileArgs &a, const TileGeom &t,
                                              const TileLds &L, RowTab &R, int r);

// Fill the LDS tables of tile lb, and with R its per-row staging table (by
// the lanes after the first wave, while the first wave fills the home-row
// table).  Ends with a barrier; every thread of the block must call it
// (blockDim.x >= 64, and >= 64 + kTileMaxRows with R).
__device__ __forceinline__ TileGeom tile_setup(const TileArgs &a, int64_t lb, TileLds &L,
                                               RowTab *R = nullptr) {
    const int nx = a.g.nc[0], ny = a.g.nc[1], nz = a.g.nc[2];
    TileGeom t;
    const int ix = (int)(lb % a.ntile[0]);
    const int64_t rest = lb / a.ntile[0];
    const int iy = (int)(rest % a.ntile[1]);
    const int iz = (int)(rest / a.ntile[1]);
    t.c0[0] = ix * a.ext[0];
    t.c0[1] = iy * a.ext[1];
    t.c0[2] = iz * a.ext[2];
    t.b[0] = min(a.ext[0], nx - t.c0[0]);
    t.b[1] = min(a.ext[1], ny - t.c0[1]);
    t.b[2] = min(a.ext[2], nz - t.c0[2]);
    t.w = t.b[0] + 2;
    const int ry = t.b[1] + 2;
    t.nrows = ry * (t.b[2] + 2);
    t.ncells = t.w * t.nrows;
    t.nhome = t.b[1] * t.b[2];
    for (int c = threadIdx.x; c < t.ncells; c += blockDim.x) {
        const int r = c / t.w, tt = c - r * t.w;
        const int zz = (t.c0[2] + r / ry - 1 + nz) % nz;
        const int yy = (t.c0[1] + r % ry - 1 + ny) % ny;
        const int xx = (t.c0[0] - 1 + tt + nx) % nx;
        const int64_t cell = ((int64_t)zz * ny + yy) * nx + xx;
        const int32_t s0 = a.cell_start[cell];
        L.cs[c] = s0;
        L.off[c + 1] = a.cell_start[cell + 1] - s0;
    }
    __syncthreads();
    if (threadIdx.x < kWave) {
        // exclusive prefix of the cell counts: each lane sums a run of cells
        const int lane = (int)threadIdx.x;
        const int per = (t.ncells + kWave - 1) / kWave;
        const int c_lo = min(lane * per, t.ncells), c_hi = min(c_lo + per, t.ncells);
        int sum = 0;
        for (int c = c_lo; c < c_hi; ++c) sum += L.off[c + 1];
        int run = wave_incl_scan(sum) - sum;
        for (int c = c_lo; c < c_hi; ++c) {
            run += L.off[c + 1];
            L.off[c + 1] = run;
        }
        if (lane == 0) L.off[0] = 0;
    }
    __syncthreads();
    if (threadIdx.x < kWave) {
        const int h = (int)threadIdx.x;
        int cnt = 0;
        if (h < t.nhome) {
            const int hy = h % t.b[1], hz = h / t.b[1];
            const int c = ((hz + 1) * ry + hy + 1) * t.w + 1;
            L.hs[h] = L.cs[c];
            cnt = L.off[c + t.b[0]] - L.off[c];
        }
        const int incl = wave_incl_scan(cnt);
        if (h < t.nhome) L.hoff[h + 1] = incl;
        if (h == 0) L.hoff[0] = 0;
    } else if (R && (int)threadIdx.x - kWave < t.nrows) {
        tile_row_fill(a, t, L, *R, (int)threadIdx.x - kWave);
    }
    __syncthreads();
    return t;
}

// Home atoms of the tile.
__device__ __forceinline__ int32_t tile_home_count(const TileLds &L, const TileGeom &t) {
    return L.hoff[t.nhome];
}

// Home row of home atom h (0 <= h < tile_home_count).
__device__ __forceinline__ int tile_home_row(const TileLds &L, const TileGeom &t, int32_t h) {
    int hr = 0;
    for (int k = 1; k < t.nhome; ++k) hr += h >= L.hoff[k] ? 1 : 0;
    return hr;
}

// Cell-sorted index of home atom h.
__device__ __forceinline__ int32_t tile_home_s(const TileLds &L, const TileGeom &t, int32_t h) {
    const int hr = tile_home_row(L, t, h);
    return L.hs[hr] + (h - L.hoff[hr]);
}

// Periodic shift of staged cell c (added to the staged positions).
__device__ __forceinline__ void tile_shift(const TileArgs &a, const TileGeom &t, int c,
                                           double &sx, double &sy, double &sz) {
    const int ry = t.b[1] + 2;
    const int r = c / t.w, tt = c - r * t.w;
    const int xr = t.c0[0] - 1 + tt, yr = t.c0[1] + r % ry - 1, zr = t.c0[2] + r / ry - 1;
    sx = xr < 0 ? -a.box.L[0] : (xr >= a.g.nc[0] ? a.box.L[0] : 0.0);
    sy = yr < 0 ? -a.box.L[1] : (yr >= a.g.nc[1] ? a.box.L[1] : 0.0);
    sz = zr < 0 ? -a.box.L[2] : (zr >= a.g.nc[2] ? a.box.L[2] : 0.0);
}

// Image code of staged cell c (bits 2d..2d+1: 1 = subtract L, 2 = add L to
// x_i - x_j), as stored by the global list format.
__device__ __forceinline__ uint32_t tile_code(const TileArgs &a, const TileGeom &t, int c) {
    const int ry = t.b[1] + 2;
    const int r = c / t.w, tt = c - r * t.w;
    const int xr = t.c0[0] - 1 + tt, yr = t.c0[1] + r % ry - 1, zr = t.c0[2] + r / ry - 1;
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

// Per-row staging table.  Within staged row r the middle cells
// (t = 1 .. b[0]) are one contiguous cell-sorted range, and only the end
// cells (t = 0, t = b[0] + 1) can wrap around the box.  So a slot q of row r
// lies in one of three segments and its cell-sorted index is q + g[seg]; the
// x shift is nonzero only for the end segments.
struct RowTab {
    int32_t r0[kTileMaxRows];  // first slot of the row
    int32_t b1[kTileMaxRows];  // first slot after segment 0 (cell t = 0)
    int32_t b2[kTileMaxRows];  // first slot after segment 1 (cells t = 1 .. b[0])
    int32_t r1[kTileMaxRows];  // first slot after the row
    int32_t g0[kTileMaxRows], g1[kTileMaxRows], g2[kTileMaxRows];
    double sx0[kTileMaxRows], sx2[kTileMaxRows], sy[kTileMaxRows], sz[kTileMaxRows];
};

// Fill row r of R from the tile tables (tile_setup calls it for every row,
// one thread each).
__device__ __forceinline__ void tile_row_fill(const TileArgs &a, const TileGeom &t,
                                              const TileLds &L, RowTab &R, int r) {
    const int c0 = r * t.w, c2 = c0 + t.b[0] + 1;
    R.r0[r] = L.off[c0];
    R.b1[r] = L.off[c0 + 1];
    R.b2[r] = L.off[c2];
    R.r1[r] = L.off[c2 + 1];
    R.g0[r] = L.cs[c0] - L.off[c0];
    R.g1[r] = L.cs[c0 + 1] - L.off[c0 + 1];
    R.g2[r] = L.cs[c2] - L.off[c2];
    double sx, sy, sz;
    tile_shift(a, t, c0, sx, sy, sz);
    R.sx0[r] = sx;
    R.sy[r] = sy;
    R.sz[r] = sz;
    tile_shift(a, t, c2, sx, sy, sz);
    R.sx2[r] = sx;
}

// Stage slots [lo, hi) of the tile into LDS (index q - lo): positions as
// (x, y) pairs plus a separate z array, plus their periodic shift when SHIFT,
// and optionally types, atom indices (with the type in bits 30..31 when
// IDX == 2) and a second per-atom vector in the same layout (the adjoint's
// upstream gradient).  The pair layout matters for the random reads of the
// force kernels: one 16-byte read of (x, y) and one of z spread over more LDS
// banks than three 8-byte reads from three arrays whose bases sit in the same
// bank.  Each wave takes whole staged rows, so the row's table values are
// uniform across the wave; loads are issued for four slots per lane before
// any of them is used.  `sorted`: the cell order is the atom order (perm is
// the identity) and the perm lookup is skipped.
template <int T, int IDX, bool VEC, bool SHIFT>
__device__ __forceinline__ void tile_stage(const TileArgs &a, const TileGeom &tg,
                                           const RowTab &R, int32_t lo, int32_t hi, bool sorted,
                                           const double *x, const int32_t *type,
                                           const double *vec, double2 *sxy, double *sz,
                                           uint8_t *st, uint32_t *su, double2 *vxy,
                                           double *vz) {
    const int wv = (int)(threadIdx.x >> 6), nwv = (int)(blockDim.x >> 6);
    const int lane = (int)(threadIdx.x & 63);
    for (int r = wv; r < tg.nrows; r += nwv) {
        const int32_t a0 = max(R.r0[r], lo), a1 = min(R.r1[r], hi);
        const int32_t b1 = R.b1[r], b2 = R.b2[r];
        const int32_t g0 = R.g0[r], g1 = R.g1[r], g2 = R.g2[r];
        const double sx0 = R.sx0[r], sx2 = R.sx2[r], shy = R.sy[r], shz = R.sz[r];
        for (int32_t base = a0 + lane; base < a1; base += 4 * kWave) {
            int64_t u[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int32_t q = base + i * kWave;
                const int32_t g = q + (q < b1 ? g0 : (q < b2 ? g1 : g2));
                u[i] = q < a1 ? (int64_t)g : 0;
            }
            if (!sorted) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (base + i * kWave < a1) u[i] = a.perm[u[i]];
            }
            double px[4], py[4], pz[4], gx[4], gy[4], gz[4];
            int tt[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (base + i * kWave < a1) {
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
                const int32_t q = base + i * kWave;
                if (q < a1) {
                    const int32_t m = q - lo;
                    if (SHIFT) {
                        const double shx = q < b1 ? sx0 : (q < b2 ? 0.0 : sx2);
                        sxy[m] = make_double2(px[i] + shx, py[i] + shy);
                        sz[m] = pz[i] + shz;
                    } else {
                        sxy[m] = make_double2(px[i], py[i]);
                        sz[m] = pz[i];
                    }
                    if (T > 1 && IDX != 2) st[m] = (uint8_t)tt[i];
                    if (IDX == 1) su[m] = (uint32_t)u[i];
                    if (IDX == 2) su[m] = (uint32_t)u[i] | (T > 1 ? (uint32_t)tt[i] << 30 : 0u);
                    if (VEC) {
                        vxy[m] = make_double2(gx[i], gy[i]);
                        vz[m] = gz[i];
                    }
                }
            }
        }
    }
}

}  // namespace ljmd
