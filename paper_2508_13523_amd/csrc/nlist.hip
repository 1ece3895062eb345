// Verlet neighbor-list build over the cell-sorted atoms, and the export of a
// list to atom indices.
//
// Sec. 4 of the paper: pair sums run over a neighbor list that is built and
// periodically updated.  Sec. 4.1: a full list holds every partner j of i in
// row i (each pair twice); a half list holds each pair once, here in the row
// of the lower atom index.  Rows are interleaved across consecutive atoms (the
// GPU layout of Sec. 4.1) in blocks of one 64-lane wave.  A row that would
// exceed the capacity is cut and the count needed is reported, in the spirit
// of the count / resize / fill pattern of Sec. 4.2.
//
// One workgroup owns a strip of home cells along x and walks the 27-cell
// stencil one stencil row (3 x-cells wider than the strip) at a time, each
// row staged through LDS.  The distance test is FP64 with a fixed operation
// order, so that the list is exactly reproducible: d = x_i - x_j, minimum
// image, r^2 = fma(dz,dz, fma(dy,dy, dx*dx)), accepted when
// r^2 < (rc_ij + skin)^2.
//
// Two storage formats:
//  - tiled (every dimension has >= 3 cells): rows in cell-sorted order,
//    entries are 16-bit tile slots (tile.hpp), 4 per 64-bit word;
//  - global: rows by atom index, entries are 32-bit atom index | image code.
#include "tile.hpp"

namespace ljmd {

namespace {

constexpr int kNbThreads = 256;
constexpr int kChunk = 1024;  // stencil-row atoms staged in LDS at a time

struct NlArgs {
    TileArgs t;
    const double4 *pos;  // cell-sorted wrapped positions, w = type
    int cap;
    void *neigh;
    int32_t *numneigh;
    int32_t *status;
    double rnb2[kTab];
};

// Per-candidate minimum image in branch form (used by the global format on
// boxes with fewer than 3 cells in some dimension, where one staged cell can
// hold partners under two images).
__device__ __forceinline__ double branch_image(double d, double L, double h, uint32_t &code,
                                               uint32_t sub, uint32_t add) {
    if (d > h) {
        code |= sub;
        return d - L;
    }
    if (d < -h) {
        code |= add;
        return d + L;
    }
    return d;
}

// Tiled build.  Every staged cell has a single image, fixed by whether its
// raw index wrapped around the box, and (x_i - x_j) - shift equals the
// branch-form minimum image bit for bit on every pair inside the neighbor
// cutoff: the two choices differ only when both displacements exceed a cell
// width, which is at least the cutoff.
template <int T, bool HALF>
__global__ __launch_bounds__(kNbThreads) void k_nl_build_tiled(NlArgs a) {
    __shared__ TileLds L;
    __shared__ double s_x[kChunk], s_y[kChunk], s_z[kChunk];
    __shared__ uint32_t s_id[kChunk];
    __shared__ double s_rnb2[kTab];
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    if (T > 1 && threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kTab; ++k) s_rnb2[k] = a.rnb2[k];
    }
    const TileGeom tg = tile_setup(a.t, lb, L);
    const int w = tg.bs + 2;
    const int32_t total = L.off[tg.ncells];
    const int32_t hs = L.home[0], he = L.home[tg.bs];
    if (total >= kTileSlots) {  // slots would not fit 16 bits: report, store nothing
        for (int32_t s = hs + (int32_t)threadIdx.x; s < he; s += kNbThreads) a.numneigh[s] = 0;
        if (threadIdx.x == 0) atomicOr(&a.status[0], 2);
        return;
    }
    const int capw = (a.cap + 3) >> 2;
    uint64_t *words = static_cast<uint64_t *>(a.neigh);

    for (int32_t h0 = hs; h0 < he; h0 += kNbThreads) {
        const int32_t s = h0 + (int32_t)threadIdx.x;
        const bool active = s < he;
        double xi = 0.0, yi = 0.0, zi = 0.0;
        int ti = 0, hx = 0, cnt = 0;
        int32_t ui = -1;
        uint64_t word = 0;
        if (active) {
            const double4 p = a.pos[s];
            xi = p.x;
            yi = p.y;
            zi = p.z;
            ti = (int)p.w;
            ui = a.t.perm[s];
            hx = tile_home_cell(L, tg, s);
        }
        for (int rr = 0; rr < kTileRows; ++rr) {
            const int32_t r0 = L.off[rr * w], r1 = L.off[rr * w + w];
            for (int32_t lo = r0; lo < r1; lo += kChunk) {
                const int32_t hi = min(r1, lo + kChunk);
                __syncthreads();
                for (int32_t q = lo + (int32_t)threadIdx.x; q < hi; q += kNbThreads) {
                    int c = rr * w;
                    while (q >= L.off[c + 1]) ++c;
                    const int32_t gi = L.cs[c] + (q - L.off[c]);
                    const double4 pq = a.pos[gi];
                    s_x[q - lo] = pq.x;
                    s_y[q - lo] = pq.y;
                    s_z[q - lo] = pq.z;
                    s_id[q - lo] = (uint32_t)a.t.perm[gi] | ((uint32_t)(int)pq.w << 30);
                }
                __syncthreads();
                if (!active) continue;
                for (int ox = 0; ox < 3; ++ox) {
                    const int c = rr * w + hx + ox;
                    const int32_t b0 = max(L.off[c], lo), b1 = min(L.off[c + 1], hi);
                    if (b0 >= b1) continue;
                    double shx, shy, shz;
                    tile_shift(a.t, tg, c, shx, shy, shz);
                    for (int32_t q = b0; q < b1; ++q) {
                        const int32_t k = q - lo;
                        const double dx = (xi - s_x[k]) - shx;
                        const double dy = (yi - s_y[k]) - shy;
                        const double dz = (zi - s_z[k]) - shz;
                        const double rsq = fma(dz, dz, fma(dy, dy, dx * dx));
                        const uint32_t id = s_id[k];
                        const int32_t j = (int32_t)(id & 0x3FFFFFFFu);
                        const double cut2 = T > 1 ? s_rnb2[ti * T + (int)(id >> 30)] : a.rnb2[0];
                        bool ok = rsq < cut2 && j != ui;
                        if (HALF) ok = ok && j > ui;
                        if (ok) {
                            if (cnt < a.cap) {
                                word |= (uint64_t)(uint32_t)q << (16 * (cnt & 3));
                                if ((cnt & 3) == 3) {
                                    words[tile_word(s, cnt >> 2, capw)] = word;
                                    word = 0;
                                }
                            }
                            ++cnt;
                        }
                    }
                }
            }
        }
        if (active) {
            const int kept = cnt < a.cap ? cnt : a.cap;
            if (kept & 3) words[tile_word(s, kept >> 2, capw)] = word;
            a.numneigh[s] = kept;
        }
        const int m = wave_max(active ? cnt : 0);
        if ((threadIdx.x & 63) == 0 && m > 0) {
            atomicMax(&a.status[1], m);
            if (m > a.cap) atomicOr(&a.status[0], 1);
        }
    }
}

// Global-format build (rows by atom index, 32-bit index | image code).  With
// SMALL (some dimension has fewer than 3 cells) the stencil is de-duplicated
// and the image is chosen per candidate by the branch form; otherwise it is
// the staged cell's image as in the tiled build.
template <int T, bool HALF, bool SMALL>
__global__ __launch_bounds__(kNbThreads) void k_nl_build_global(NlArgs a) {
    __shared__ double s_x[kChunk], s_y[kChunk], s_z[kChunk];
    __shared__ uint32_t s_id[kChunk];
    __shared__ int32_t s_cs[kTileMaxStrip + 2];
    __shared__ int32_t s_off[kTileMaxStrip + 3];
    __shared__ int32_t s_home[kTileMaxStrip + 1];
    __shared__ double s_rnb2[kTab];

    const int nx = a.t.g.nc[0], ny = a.t.g.nc[1], nz = a.t.g.nc[2];
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int sx = (int)(lb % a.t.nstrips);
    const int64_t rowid = lb / a.t.nstrips;
    const int cy = (int)(rowid % ny), cz = (int)(rowid / ny);
    const int cx0 = sx * a.t.strip;
    const int bs = min(a.t.strip, nx - cx0);
    const int64_t homebase = ((int64_t)cz * ny + cy) * nx;
    if (T > 1 && threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kTab; ++k) s_rnb2[k] = a.rnb2[k];
    }
    if ((int)threadIdx.x <= bs) s_home[threadIdx.x] = a.t.cell_start[homebase + cx0 + threadIdx.x];
    __syncthreads();
    const int32_t hs = s_home[0], he = s_home[bs];
    const int ox_lo = nx >= 2 ? -1 : 0, ox_hi = nx >= 3 ? 1 : 0;
    const int oy_lo = ny >= 2 ? -1 : 0, oy_hi = ny >= 3 ? 1 : 0;
    const int oz_lo = nz >= 2 ? -1 : 0, oz_hi = nz >= 3 ? 1 : 0;
    const double Lx = a.t.box.L[0], Ly = a.t.box.L[1], Lz = a.t.box.L[2];
    const double hx_ = a.t.box.hL[0], hy_ = a.t.box.hL[1], hz_ = a.t.box.hL[2];
    uint32_t *neigh = static_cast<uint32_t *>(a.neigh);

    for (int32_t h0 = hs; h0 < he; h0 += kNbThreads) {
        const int32_t s = h0 + (int32_t)threadIdx.x;
        const bool active = s < he;
        double xi = 0.0, yi = 0.0, zi = 0.0;
        int ti = 0, hx = 0, cnt = 0;
        int32_t ui = -1;
        if (active) {
            const double4 p = a.pos[s];
            xi = p.x;
            yi = p.y;
            zi = p.z;
            ti = (int)p.w;
            ui = a.t.perm[s];
            while (hx + 1 < bs && s >= s_home[hx + 1]) ++hx;
        }
        for (int dz = oz_lo; dz <= oz_hi; ++dz) {
            const int zr = cz + dz;
            const int zz = (zr + nz) % nz;
            const double shz = zr < 0 ? -Lz : (zr >= nz ? Lz : 0.0);
            const uint32_t cdz = zr < 0 ? 32u : (zr >= nz ? 16u : 0u);
            for (int dy = oy_lo; dy <= oy_hi; ++dy) {
                const int yr = cy + dy;
                const int yy = (yr + ny) % ny;
                const double shy = yr < 0 ? -Ly : (yr >= ny ? Ly : 0.0);
                const uint32_t cdy = yr < 0 ? 8u : (yr >= ny ? 4u : 0u);
                const int64_t rb = ((int64_t)zz * ny + yy) * nx;
                __syncthreads();
                if ((int)threadIdx.x < bs + 2) {
                    int xx = cx0 - 1 + (int)threadIdx.x;
                    xx = (xx % nx + nx) % nx;
                    const int32_t c0 = a.t.cell_start[rb + xx], c1 = a.t.cell_start[rb + xx + 1];
                    s_cs[threadIdx.x] = c0;
                    s_off[threadIdx.x + 1] = c1 - c0;
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    s_off[0] = 0;
                    for (int t = 1; t <= bs + 2; ++t) s_off[t] += s_off[t - 1];
                }
                __syncthreads();
                const int32_t total = s_off[bs + 2];
                for (int32_t lo = 0; lo < total; lo += kChunk) {
                    const int32_t hi = min(total, lo + kChunk);
                    if (lo > 0) __syncthreads();
                    for (int32_t q = lo + (int32_t)threadIdx.x; q < hi; q += kNbThreads) {
                        int t = 0;
                        while (q >= s_off[t + 1]) ++t;
                        const int32_t gi = s_cs[t] + (q - s_off[t]);
                        const double4 pq = a.pos[gi];
                        s_x[q - lo] = pq.x;
                        s_y[q - lo] = pq.y;
                        s_z[q - lo] = pq.z;
                        s_id[q - lo] = (uint32_t)a.t.perm[gi] | ((uint32_t)(int)pq.w << 30);
                    }
                    __syncthreads();
                    if (!active) continue;
                    for (int ox = ox_lo; ox <= ox_hi; ++ox) {
                        const int t = hx + 1 + ox;
                        const int32_t b0 = max(s_off[t], lo) - lo;
                        const int32_t b1 = min(s_off[t + 1], hi) - lo;
                        const int xr = cx0 + hx + ox;
                        const double shx = xr < 0 ? -Lx : (xr >= nx ? Lx : 0.0);
                        const uint32_t cell_code =
                            (xr < 0 ? 2u : (xr >= nx ? 1u : 0u)) | cdy | cdz;
                        for (int32_t q = b0; q < b1; ++q) {
                            uint32_t code;
                            double dx, dy2, dz2;
                            if (SMALL) {
                                code = 0;
                                dx = branch_image(xi - s_x[q], Lx, hx_, code, 1u, 2u);
                                dy2 = branch_image(yi - s_y[q], Ly, hy_, code, 4u, 8u);
                                dz2 = branch_image(zi - s_z[q], Lz, hz_, code, 16u, 32u);
                            } else {
                                code = cell_code;
                                dx = (xi - s_x[q]) - shx;
                                dy2 = (yi - s_y[q]) - shy;
                                dz2 = (zi - s_z[q]) - shz;
                            }
                            const double rsq = fma(dz2, dz2, fma(dy2, dy2, dx * dx));
                            const uint32_t id = s_id[q];
                            const int32_t j = (int32_t)(id & 0x3FFFFFFFu);
                            const double cut2 =
                                T > 1 ? s_rnb2[ti * T + (int)(id >> 30)] : a.rnb2[0];
                            bool ok = rsq < cut2 && j != ui;
                            if (HALF) ok = ok && j > ui;
                            if (ok) {
                                if (cnt < a.cap)
                                    neigh[nl_slot(ui, cnt, a.cap)] =
                                        (uint32_t)j | (code << kCodeShift);
                                ++cnt;
                            }
                        }
                    }
                }
            }
        }
        if (active) a.numneigh[ui] = cnt < a.cap ? cnt : a.cap;
        const int m = wave_max(active ? cnt : 0);
        if ((threadIdx.x & 63) == 0 && m > 0) {
            atomicMax(&a.status[1], m);
            if (m > a.cap) atomicOr(&a.status[0], 1);
        }
    }
}

// Tiled list -> global format (rows by atom index, atom index | image code).
__global__ __launch_bounds__(kNbThreads) void k_export_tiled(TileArgs t, const uint64_t *words,
                                                             const int32_t *numneigh, int cap,
                                                             uint32_t *out, int32_t *counts) {
    __shared__ TileLds L;
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const TileGeom tg = tile_setup(t, lb, L);
    const int capw = (cap + 3) >> 2;
    for (int32_t s = L.home[0] + (int32_t)threadIdx.x; s < L.home[tg.bs]; s += kNbThreads) {
        const int32_t u = t.perm[s];
        const int nn = numneigh[s];
        for (int k = 0; k < nn; ++k) {
            const uint64_t wd = words[tile_word(s, k >> 2, capw)];
            const int32_t q = (int32_t)((wd >> (16 * (k & 3))) & 0xFFFFu);
            const int c = tile_cell_of(L, tg.ncells, q);
            const int32_t g = L.cs[c] + (q - L.off[c]);
            out[nl_slot(u, k, cap)] = (uint32_t)t.perm[g] | (tile_code(t, tg, c) << kCodeShift);
        }
        counts[u] = nn;
    }
}

__global__ __launch_bounds__(kNbThreads) void k_export_global(int64_t n, const uint32_t *neigh,
                                                              const int32_t *numneigh, int cap,
                                                              uint32_t *out, int32_t *counts) {
    const int64_t i = (int64_t)blockIdx.x * kNbThreads + threadIdx.x;
    if (i >= n) return;
    const int nn = numneigh[i];
    for (int k = 0; k < nn; ++k) out[nl_slot(i, k, cap)] = neigh[nl_slot(i, k, cap)];
    counts[i] = nn;
}

template <int T>
hipError_t launch_t(const NlArgs &a, int half, int tiled, unsigned blocks, hipStream_t s) {
    const bool small = a.t.g.nc[0] < 3 || a.t.g.nc[1] < 3 || a.t.g.nc[2] < 3;
    if (tiled) {
        if (half) k_nl_build_tiled<T, true><<<blocks, kNbThreads, 0, s>>>(a);
        else k_nl_build_tiled<T, false><<<blocks, kNbThreads, 0, s>>>(a);
    } else if (small) {
        if (half) k_nl_build_global<T, true, true><<<blocks, kNbThreads, 0, s>>>(a);
        else k_nl_build_global<T, false, true><<<blocks, kNbThreads, 0, s>>>(a);
    } else {
        if (half) k_nl_build_global<T, true, false><<<blocks, kNbThreads, 0, s>>>(a);
        else k_nl_build_global<T, false, false><<<blocks, kNbThreads, 0, s>>>(a);
    }
    return hipGetLastError();
}

}  // namespace

int64_t tile_blocks(const TileArgs &t) { return (int64_t)t.nstrips * t.g.nc[1] * t.g.nc[2]; }

hipError_t launch_nl_build(int64_t n, const TileArgs &t, const PairTab &tab, int half, int tiled,
                           const char *ws, const Workspace &w, void *neigh, int32_t *numneigh,
                           int cap, int32_t *status, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    NlArgs a;
    a.t = t;
    a.pos = reinterpret_cast<const double4 *>(ws + w.pos);
    a.cap = cap;
    a.neigh = neigh;
    a.numneigh = numneigh;
    a.status = status;
    for (int k = 0; k < kTab; ++k) a.rnb2[k] = tab.rnb2[k];
    const unsigned blocks = (unsigned)tile_blocks(t);
    switch (tab.ntypes) {
        case 1: return launch_t<1>(a, half, tiled, blocks, s);
        case 2: return launch_t<2>(a, half, tiled, blocks, s);
        case 3: return launch_t<3>(a, half, tiled, blocks, s);
        default: return launch_t<4>(a, half, tiled, blocks, s);
    }
}

hipError_t launch_nl_export(int64_t n, const TileArgs &t, int tiled, const void *neigh,
                            const int32_t *numneigh, int cap, uint32_t *out, int32_t *counts,
                            hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (tiled)
        k_export_tiled<<<(unsigned)tile_blocks(t), kNbThreads, 0, s>>>(
            t, static_cast<const uint64_t *>(neigh), numneigh, cap, out, counts);
    else
        k_export_global<<<(unsigned)((n + kNbThreads - 1) / kNbThreads), kNbThreads, 0, s>>>(
            n, static_cast<const uint32_t *>(neigh), numneigh, cap, out, counts);
    return hipGetLastError();
}

}  // namespace ljmd
