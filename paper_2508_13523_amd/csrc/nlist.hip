// Verlet neighbor-list build over the cell-sorted atoms, and the export of a
// list to atom indices.
//
// Sec. 4 of the paper: pair sums run over a neighbor list that is built and
// periodically updated.  Sec. 4.1: a full list holds every partner j of i in
// row i (each pair twice); a half list holds each pair once: in the tiled
// format in the row of the atom that comes first in the stencil order (the
// forward half of the stencil, below), in the global format in the row of
// the lower atom index.  Rows are interleaved across consecutive atoms (the
// GPU layout of Sec. 4.1) in blocks of one 64-lane wave.  A row that would
// exceed the capacity is cut and the count needed is reported, in the spirit
// of the count / resize / fill pattern of Sec. 4.2.
//
// One workgroup owns a tile of home cells (tile.hpp) and stages the atoms of
// its stencil through LDS.  The distance test is FP64 with a fixed operation
// order, so that the list is exactly reproducible: d = x_i - x_j, minimum
// image, r^2 = fma(dz,dz, fma(dy,dy, dx*dx)), accepted when
// r^2 < (rc_ij + skin)^2.
//
// Two storage formats:
//  - tiled (every dimension has >= 3 cells): rows in cell-sorted order,
//    entries are 16-bit tile slots (tile.hpp), 4 per 64-bit word;
//  - global: rows by atom index, entries are 32-bit atom index | image code.
#include "tile.hpp"

#include <type_traits>

#include <cstring>

namespace ljmd {

namespace {

constexpr int kNbThreads = 256;
constexpr int kChunk = 1024;  // stencil-row atoms staged in LDS at a time (global build)
constexpr int kGlobalMaxStrip = 30;  // cells per strip of the global build
constexpr int kSubBins = 8;          // x sub-bins per staged cell (tiled build windows)

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

// Append a 16-bit slot to a list word held as two halves: the word moves
// down by 16 bits and the slot enters at the top, so after four appends the
// k-th one sits at bits 16 k (the layout of the tiled list) -- two funnel
// shifts instead of a variable 64-bit shift and two ors.
__device__ __forceinline__ void push_slot(uint32_t &lo, uint32_t &hi, uint32_t slot) {
    lo = __builtin_amdgcn_alignbit(hi, lo, 16);
    hi = __builtin_amdgcn_alignbit(slot, hi, 16);
}

// Tiled build.  Every staged cell has a single image, fixed by whether its
// raw index wrapped around the box, and (x_i - x_j) - shift equals the
// branch-form minimum image bit for bit on every pair inside the neighbor
// cutoff: the two choices differ only when both displacements exceed a cell
// width, which is at least the cutoff.
//
// The tile's stencil atoms are staged into LDS (positions without their
// shift, as an (x, y) pair and z, and the type when there are several), all
// at once when they fit and in chunks of K slots otherwise.  Each home atom
// then scans its own 27 cells: 9 staged rows, in each of them the 3
// consecutive cells around its own, one contiguous slot range cut to the x
// window its cutoff sphere reaches in that row.  Rows are visited in
// increasing order and the slots of a row in increasing order, so every list
// row comes out sorted by slot (the chunked readers rely on that).
//
// Half list: staged rows are ordered by z, then y, and cells within a row by
// x, so for any two atoms of neighboring cells the one in the cell that
// comes later in (z, y, x) -- unwrapped around the tile -- has the larger
// slot in every tile that stages both, and within one cell the cell order
// decides.  A home atom keeps the partners whose slot is larger than its
// own (its forward half stencil: 13 cells and the rest of its own cell), so
// each pair is listed exactly once, and all its partners lie at or after the
// tile's first home cell in the stage.  A stencil that fits is staged
// once for all passes.  NT threads, one per home atom and pass: 512 with
// K = 2560, or 256 with K = 1280 for batches whose tiles average fewer than
// 256 atoms, so that four workgroups share a compute unit and the few home
// atoms of such a tile still keep it busy.
template <int T, bool HALF, int NT, int K>
__global__ __launch_bounds__(NT, 4) void k_nl_build_tiled(NlArgs a) {
    constexpr bool kTypes = T > 1;  // partner types for the per-pair cutoffs
    constexpr int S = NT >= 512 ? kSubBins : kSubBins / 2;  // small workgroups: keep 4 per CU
    __shared__ TileLds L;
    __shared__ RowTab R;
    __shared__ double2 s_xy[K];
    __shared__ double s_z[K];
    __shared__ uint8_t s_ty[kTypes ? K : 1];
    __shared__ double s_rnb2[kTab];
    __shared__ uint16_t s_sb[kTileMaxCells * S + 1];
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    int64_t lbl = 0;
    const TileArgs ta = tile_args_of(a.t, lb, lbl);
    if (T > 1 && threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kTab; ++k) s_rnb2[k] = a.rnb2[k];
    }
    const TileGeom tg = tile_setup(ta, lbl, L, &R);
    const int32_t total = L.off[tg.ncells];
    const int32_t nh = tile_home_count(L, tg);
    if (total >= kTileSlots) {  // slots would not fit 16 bits: report, store nothing
        for (int32_t h = (int32_t)threadIdx.x; h < nh; h += NT)
            a.numneigh[tile_home_s(L, tg, h)] = 0;
        if (threadIdx.x == 0) atomicOr(&a.status[0], 2);
        return;
    }
    const int capw = tile_capw(a.cap);
    const int ry = tg.b[1] + 2;
    uint64_t *words = static_cast<uint64_t *>(a.neigh);
    // stage the stencil slots [lo, hi): each wave takes whole staged rows
    auto stage = [&](int32_t lo, int32_t hi) {
        for (int r = (int)(threadIdx.x >> 6); r < tg.nrows; r += NT / kWave) {
            const int32_t a0 = max(R.r0[r], lo), a1 = min(R.r1[r], hi);
            const int32_t b1 = R.b1[r], b2 = R.b2[r];
            const int32_t g0 = R.g0[r], g1 = R.g1[r], g2 = R.g2[r];
            for (int32_t q = a0 + (int32_t)(threadIdx.x & 63); q < a1; q += kWave) {
                const int32_t gi = q + (q < b1 ? g0 : (q < b2 ? g1 : g2));
                const double4 pq = a.pos[gi];
                s_xy[q - lo] = make_double2(pq.x, pq.y);
                s_z[q - lo] = pq.z;
                if (kTypes) s_ty[q - lo] = (uint8_t)(int)pq.w;
            }
        }
    };
    const bool once = total <= K;  // the whole stencil fits: staged once for all passes
    if (once) {
        stage(0, total);
        __syncthreads();
    }
    // Sub-bin table: staged cell c is cut along x into S sub-bins at
    // x = (xw S + k) / (S cinv_x) (xw: the cell's grid index); s_sb[c S + k]
    // is the first slot of c at or beyond boundary k.  The atoms of a cell
    // are sorted by x (binning), so this is a binary search; it splits
    // every staged row into S (b[0] + 2) runs of increasing x.
    const double cinv_s = ta.g.cinv[0] * S;
    for (int idx = (int)threadIdx.x; idx < tg.ncells * (S - 1); idx += NT) {
        const int c = idx / (S - 1), k = idx - c * (S - 1) + 1;
        const int xw = (tg.c0[0] - 1 + c % tg.w + ta.g.nc[0]) % ta.g.nc[0];
        const double bound = ((double)xw * S + k) / cinv_s;
        const int32_t o = L.off[c];
        int32_t lo = 0, hi = L.off[c + 1] - o;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            const double xm = once ? s_xy[o + mid].x : a.pos[L.cs[c] + mid].x;
            if (xm < bound) lo = mid + 1;
            else hi = mid;
        }
        s_sb[c * S + k] = (uint16_t)(o + lo);
    }
    for (int c = (int)threadIdx.x; c <= tg.ncells; c += NT) s_sb[c * S] = (uint16_t)L.off[c];
    bool any_shift = false, any_xshift = false;
    for (int r = (int)threadIdx.x; r < tg.nrows; r += NT) {
        any_shift = any_shift || R.sy[r] != 0.0 || R.sz[r] != 0.0;
        any_xshift = any_xshift || R.sx0[r] != 0.0 || R.sx2[r] != 0.0;
    }
    const bool wraps = __syncthreads_or(any_shift) != 0;
    const bool wraps_x = __syncthreads_or(any_xshift) != 0;

    for (int32_t h0 = 0; h0 < nh; h0 += NT) {
        const int32_t h = h0 + (int32_t)threadIdx.x;
        const bool active = h < nh;
        double xi = 0.0, yi = 0.0, zi = 0.0;
        int ti = 0, hx = 0, hy = 0, hz = 0, cnt = 0;
        int32_t s = 0, qself = -1;
        uint32_t wlo = 0, whi = 0;  // the row's current list word, low and high half
        double r2max = 0.0, dy_lo = 0.0, dy_hi = 0.0, dz_lo = 0.0, dz_hi = 0.0;
        if (active) {
            const int hr = tile_home_row(L, tg, h);
            hy = hr % tg.b[1];
            hz = hr / tg.b[1];
            s = L.hs[hr] + (h - L.hoff[hr]);
            const double4 p = a.pos[s];
            xi = p.x;
            yi = p.y;
            zi = p.z;
            ti = (int)p.w;
            const int c1 = ((hz + 1) * ry + hy + 1) * tg.w;  // own staged row, cell t = 0
            for (int t = 2; t <= tg.b[0]; ++t) hx += s >= L.cs[c1 + t] ? 1 : 0;
            qself = L.off[c1 + hx + 1] + (s - L.cs[c1 + hx + 1]);
            if (T > 1) {
#pragma unroll
                for (int tj = 0; tj < T; ++tj) r2max = fmax(r2max, s_rnb2[ti * T + tj]);
            } else {
                r2max = a.rnb2[0];
            }
            // distances to the y and z faces of the own cell
            const double wy = ta.box.L[1] / ta.g.nc[1], wz = ta.box.L[2] / ta.g.nc[2];
            dy_lo = yi - (double)(tg.c0[1] + hy) * wy;
            dy_hi = (double)(tg.c0[1] + hy + 1) * wy - yi;
            dz_lo = zi - (double)(tg.c0[2] + hz) * wz;
            dz_hi = (double)(tg.c0[2] + hz + 1) * wz - zi;
        }
        uint64_t *rowp = words + tile_word(s, 0, capw);  // word w of the row at rowp[64 w]
        const double mg = 1e-10 * (ta.box.L[0] + ta.box.L[1] + ta.box.L[2]);
        for (int32_t lo = 0; lo < total; lo += K) {
            const int32_t hi = min(total, lo + K);
            if (!once) {
                __syncthreads();
                stage(lo, hi);
            }
            __syncthreads();
            if (!active) continue;
            // SH: the tile's stencil wraps around the box (some staged cell
            // has a periodic shift); without it the shifts are all zero and
            // are not subtracted (x - 0.0 == x, so the distances are the same)
            auto scan = [&](auto sh_tag, auto shx_tag) {
                constexpr bool SH = decltype(sh_tag)::value;
                constexpr bool SHX = decltype(shx_tag)::value;
                for (int oz = 0; oz < 3; ++oz) {
                    for (int oy = 0; oy < 3; ++oy) {
                        // half list: the rows behind the own one hold no partner
                        if (HALF && (oz == 0 || (oz == 1 && oy == 0))) continue;
                        const int r = (hz + oz) * ry + hy + oy;
                        // The x window of this row: a partner lies at least dy
                        // and dz from the home atom across the cell faces, so
                        // |dx| < sqrt(rnb^2 - dy^2 - dz^2).  Every bound is
                        // widened by mg (far above the rounding of these
                        // expressions), so no pair the FP64 test accepts is cut.
                        const double dyf = oy == 0 ? dy_lo : (oy == 2 ? dy_hi : 0.0);
                        const double dzf = oz == 0 ? dz_lo : (oz == 2 ? dz_hi : 0.0);
                        const double ey = fmax(dyf - mg, 0.0), ez = fmax(dzf - mg, 0.0);
                        const double h2 = r2max - ey * ey - ez * ez;
                        if (!(h2 > 0.0)) continue;
                        const double hw = sqrt(h2) + mg;
                        const double row0 = (double)(tg.c0[0] - 1) * S;
                        const double blo = (double)hx * S, bhi = (double)(hx + 3) * S;
                        const double gs = fmin(fmax(floor((xi - hw - mg) * cinv_s) - row0, blo), bhi);
                        const double ge = fmin(fmax(floor((xi + hw + mg) * cinv_s) - row0 + 1.0, blo), bhi);
                        const int32_t wq0 = s_sb[r * tg.w * S + (int)gs];
                        const int32_t wq1 = s_sb[r * tg.w * S + (int)ge];
                        const double shy = SH ? R.sy[r] : 0.0, shz = SH ? R.sz[r] : 0.0;
                        // the window spans up to three consecutive cells of the
                        // staged row, one contiguous slot range: one loop over it
                        // (so a wave runs as long as its longest window, not its
                        // longest cell three times over); only the row's end
                        // cells (t = 0, t = b[0] + 1) can carry an x shift
                        const int32_t b1 = R.b1[r], b2 = R.b2[r];
                        const double sx0 = SHX ? R.sx0[r] : 0.0, sx2 = SHX ? R.sx2[r] : 0.0;
                        const int32_t q0 = max(wq0, lo), q1 = min(wq1, hi);
                        auto test = [&](int32_t q, bool valid) {
                            const int32_t k = q - lo;
                            const double2 pxy = s_xy[k];
                            double dx = xi - pxy.x, dy = yi - pxy.y, dz = zi - s_z[k];
                            if (SHX) dx -= q < b1 ? sx0 : (q >= b2 ? sx2 : 0.0);
                            if (SH) {
                                dy -= shy;
                                dz -= shz;
                            }
                            const double rsq = fma(dz, dz, fma(dy, dy, dx * dx));
                            const double cut2 = T > 1 ? s_rnb2[ti * T + (int)s_ty[k]] : a.rnb2[0];
                            return valid && rsq < cut2;
                        };
                        auto accept = [&](int32_t q) {
                            push_slot(wlo, whi, (uint32_t)q);
                            if ((cnt & 3) == 3 && cnt < a.cap)
                                rowp[((uint32_t)cnt >> 2) * (uint32_t)kWave] =
                                    ((uint64_t)whi << 32) | wlo;
                            ++cnt;
                        };
                        // two candidates per iteration: both tests issue their
                        // LDS reads together, and the loop control is shared
                        auto run = [&](int32_t a0, int32_t a1) {
                            for (int32_t q = a0; q < a1; q += 2) {
                                const bool two = q + 1 < a1;
                                const bool ok0 = test(q, true);
                                const bool ok1 = test(two ? q + 1 : q, two);
                                if (ok0) accept(q);
                                if (ok1) accept(q + 1);
                            }
                        };
                        // Full list: the home atom's own slot (in the middle row,
                        // which holds its cell) is skipped by splitting the
                        // window around it; every other image of the home atom
                        // lies at least a box length (at least twice the
                        // neighbor cutoff) away, so it is the only self pair
                        // inside the cutoff.  Half list: only slots after the
                        // own one (the forward half of the stencil, see above).
                        if (HALF) {
                            run(max(q0, qself + 1), q1);
                        } else {
                            const int32_t hole = (oy == 1 && oz == 1) ? qself : q1;
                            run(q0, min(q1, hole));
                            run(max(q0, hole + 1), q1);
                        }
                    }
                }
            };
            if (wraps_x) {
                if (wraps) scan(std::true_type{}, std::true_type{});
                else scan(std::false_type{}, std::true_type{});
            } else {
                if (wraps) scan(std::true_type{}, std::false_type{});
                else scan(std::false_type{}, std::false_type{});
            }
        }
        if (active) {
            // pad the row to a multiple of kRowPad entries with the null slot
            const int kept = cnt < a.cap ? cnt : a.cap;
            const int padded = tile_row_words(kept) * 4;
            for (int k = kept; k < padded; ++k) {
                push_slot(wlo, whi, (uint32_t)total);
                if ((k & 3) == 3)
                    rowp[((uint32_t)k >> 2) * (uint32_t)kWave] = ((uint64_t)whi << 32) | wlo;
            }
            a.numneigh[s] = kept;
        }
        const int m = wave_max(active ? cnt : 0);
        if ((threadIdx.x & 63) == 0 && m > 0) {
            atomicMax(&a.status[1], m);
            if (m > a.cap) atomicOr(&a.status[0], 1);
        }
    }
}

// Global-format build (rows by atom index, 32-bit index | image code) of one
// strip of `bs` cells along x starting at cell (cx0, cy, cz) of the grid g.
// `cs` is the cell-start table of this grid (cell-sorted positions are global,
// so in a batch it points at the system's first cell).  With SMALL (some
// dimension has fewer than 3 cells) the stencil is de-duplicated and the image
// is chosen per candidate by the branch form; otherwise it is the staged
// cell's image as in the tiled build.  Shared memory comes from the caller.
struct GlobalLds {
    double x[kChunk], y[kChunk], z[kChunk];
    uint32_t id[kChunk];
    int32_t cs[kGlobalMaxStrip + 2];
    int32_t off[kGlobalMaxStrip + 3];
    int32_t home[kGlobalMaxStrip + 1];
    double rnb2[kTab];
};

template <int T, bool HALF, bool SMALL>
__device__ void build_strip_global(const NlArgs &a, GlobalLds &S, const Box &box, const Grid &g,
                                   const int32_t *cs, int cx0, int cy, int cz, int bs) {
    const int nx = g.nc[0], ny = g.nc[1], nz = g.nc[2];
    const int64_t homebase = ((int64_t)cz * ny + cy) * nx;
    if ((int)threadIdx.x <= bs) S.home[threadIdx.x] = cs[homebase + cx0 + threadIdx.x];
    __syncthreads();
    const int32_t hs = S.home[0], he = S.home[bs];
    const int ox_lo = nx >= 2 ? -1 : 0, ox_hi = nx >= 3 ? 1 : 0;
    const int oy_lo = ny >= 2 ? -1 : 0, oy_hi = ny >= 3 ? 1 : 0;
    const int oz_lo = nz >= 2 ? -1 : 0, oz_hi = nz >= 3 ? 1 : 0;
    const double Lx = box.L[0], Ly = box.L[1], Lz = box.L[2];
    const double hx_ = box.hL[0], hy_ = box.hL[1], hz_ = box.hL[2];
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
            while (hx + 1 < bs && s >= S.home[hx + 1]) ++hx;
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
                    const int32_t c0 = cs[rb + xx], c1 = cs[rb + xx + 1];
                    S.cs[threadIdx.x] = c0;
                    S.off[threadIdx.x + 1] = c1 - c0;
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    S.off[0] = 0;
                    for (int t = 1; t <= bs + 2; ++t) S.off[t] += S.off[t - 1];
                }
                __syncthreads();
                const int32_t total = S.off[bs + 2];
                for (int32_t lo = 0; lo < total; lo += kChunk) {
                    const int32_t hi = min(total, lo + kChunk);
                    if (lo > 0) __syncthreads();
                    for (int32_t q = lo + (int32_t)threadIdx.x; q < hi; q += kNbThreads) {
                        int t = 0;
                        while (q >= S.off[t + 1]) ++t;
                        const int32_t gi = S.cs[t] + (q - S.off[t]);
                        const double4 pq = a.pos[gi];
                        S.x[q - lo] = pq.x;
                        S.y[q - lo] = pq.y;
                        S.z[q - lo] = pq.z;
                        S.id[q - lo] = (uint32_t)a.t.perm[gi] | ((uint32_t)(int)pq.w << 30);
                    }
                    __syncthreads();
                    if (!active) continue;
                    for (int ox = ox_lo; ox <= ox_hi; ++ox) {
                        const int t = hx + 1 + ox;
                        const int32_t b0 = max(S.off[t], lo) - lo;
                        const int32_t b1 = min(S.off[t + 1], hi) - lo;
                        const int xr = cx0 + hx + ox;
                        const double shx = xr < 0 ? -Lx : (xr >= nx ? Lx : 0.0);
                        const uint32_t cell_code =
                            (xr < 0 ? 2u : (xr >= nx ? 1u : 0u)) | cdy | cdz;
                        for (int32_t q = b0; q < b1; ++q) {
                            uint32_t code;
                            double dx, dy2, dz2;
                            if (SMALL) {
                                code = 0;
                                dx = branch_image(xi - S.x[q], Lx, hx_, code, 1u, 2u);
                                dy2 = branch_image(yi - S.y[q], Ly, hy_, code, 4u, 8u);
                                dz2 = branch_image(zi - S.z[q], Lz, hz_, code, 16u, 32u);
                            } else {
                                code = cell_code;
                                dx = (xi - S.x[q]) - shx;
                                dy2 = (yi - S.y[q]) - shy;
                                dz2 = (zi - S.z[q]) - shz;
                            }
                            const double rsq = fma(dz2, dz2, fma(dy2, dy2, dx * dx));
                            const uint32_t id = S.id[q];
                            const int32_t j = (int32_t)(id & 0x3FFFFFFFu);
                            const double cut2 =
                                T > 1 ? S.rnb2[ti * T + (int)(id >> 30)] : a.rnb2[0];
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

// One workgroup per strip of ext[0] cells along x (ext[1] = ext[2] = 1).
template <int T, bool HALF, bool SMALL>
__global__ __launch_bounds__(kNbThreads) void k_nl_build_global(NlArgs a) {
    __shared__ GlobalLds S;
    if (T > 1 && threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kTab; ++k) S.rnb2[k] = a.rnb2[k];
    }
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int nx = a.t.g.nc[0], ny = a.t.g.nc[1];
    const int sx = (int)(lb % a.t.ntile[0]);
    const int64_t rowid = lb / a.t.ntile[0];
    const int cx0 = sx * a.t.ext[0];
    build_strip_global<T, HALF, SMALL>(a, S, a.t.box, a.t.g, a.t.cell_start, cx0,
                                       (int)(rowid % ny), (int)(rowid / ny),
                                       min(a.t.ext[0], nx - cx0));
}

// Batch of independent systems: work item -> (system, strip), each system
// with its own box and grid.
template <int T, bool HALF>
__global__ __launch_bounds__(kNbThreads) void k_nl_build_batch(NlArgs a, BatchView b,
                                                               int64_t nitems) {
    __shared__ GlobalLds S;
    __shared__ int32_t s_rep;
    if (T > 1 && threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kTab; ++k) S.rnb2[k] = a.rnb2[k];
    }
    const int64_t item = xcd_remap(blockIdx.x, gridDim.x);
    if (item >= nitems) return;
    if (threadIdx.x == 0) {
        int lo = 0, hi = b.nrep - 1;  // last system whose first item is <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (b.reps[mid].item_base <= item) lo = mid;
            else hi = mid - 1;
        }
        s_rep = lo;
    }
    __syncthreads();
    const RepInfo &r = b.reps[s_rep];
    const int64_t li = item - r.item_base;
    const int nx = r.g.nc[0], ny = r.g.nc[1];
    const int sx = (int)(li % r.nstripx);
    const int64_t rowid = li / r.nstripx;
    const int cx0 = sx * r.strip;
    const int bs = min(r.strip, nx - cx0);
    const int32_t *cs = a.t.cell_start + r.cell_base;
    if (r.small)
        build_strip_global<T, HALF, true>(a, S, r.box, r.g, cs, cx0, (int)(rowid % ny),
                                          (int)(rowid / ny), bs);
    else
        build_strip_global<T, HALF, false>(a, S, r.box, r.g, cs, cx0, (int)(rowid % ny),
                                           (int)(rowid / ny), bs);
}

// Tiled list -> global format (rows by atom index, atom index | image code).
// Export writes entry k of atom u's row as index | image code at the
// interleaved position nl_slot(u, k, cap), or with KMAJOR the plain atom
// index at k * n + u (the layout of an index list with one row per atom).
template <bool KMAJOR>
__global__ __launch_bounds__(kTileThreads) void k_export_tiled(TileArgs t, const uint64_t *words,
                                                               const int32_t *numneigh, int cap,
                                                               int64_t n, uint32_t *out,
                                                               int32_t *counts) {
    __shared__ TileLds L;
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    int64_t lbl = 0;
    const TileArgs ta = tile_args_of(t, lb, lbl);
    const TileGeom tg = tile_setup(ta, lbl, L);
    const int capw = tile_capw(cap);
    const int32_t nh = tile_home_count(L, tg);
    for (int32_t h = (int32_t)threadIdx.x; h < nh; h += kTileThreads) {
        const int32_t s = tile_home_s(L, tg, h);
        const int32_t u = ta.perm[s];
        const int nn = numneigh[s];
        for (int k = 0; k < nn; ++k) {
            const uint64_t wd = words[tile_word(s, k >> 2, capw)];
            const int32_t q = (int32_t)((wd >> (16 * (k & 3))) & 0xFFFFu);
            const int c = tile_cell_of(L, tg.ncells, q);
            const int32_t g = L.cs[c] + (q - L.off[c]);
            if (KMAJOR)
                out[(int64_t)k * n + u] = (uint32_t)ta.perm[g];
            else
                out[nl_slot(u, k, cap)] =
                    (uint32_t)ta.perm[g] | (tile_code(ta, tg, c) << kCodeShift);
        }
        counts[u] = nn;
    }
}

template <bool KMAJOR>
__global__ __launch_bounds__(kNbThreads) void k_export_global(int64_t n, const uint32_t *neigh,
                                                              const int32_t *numneigh, int cap,
                                                              uint32_t *out, int32_t *counts) {
    const int64_t i = (int64_t)blockIdx.x * kNbThreads + threadIdx.x;
    if (i >= n) return;
    const int nn = numneigh[i];
    for (int k = 0; k < nn; ++k) {
        const uint32_t e = neigh[nl_slot(i, k, cap)];
        if (KMAJOR)
            out[(int64_t)k * n + i] = e & kIndexMask;
        else
            out[nl_slot(i, k, cap)] = e;
    }
    counts[i] = nn;
}

template <int T>
hipError_t launch_t(int64_t n, const NlArgs &a, int half, int tiled, unsigned blocks,
                    hipStream_t s) {
    const bool small = a.t.g.nc[0] < 3 || a.t.g.nc[1] < 3 || a.t.g.nc[2] < 3;
    if (tiled && a.t.reps && (double)n < 256.0 * (double)blocks) {  // small batch tiles
        if (half) k_nl_build_tiled<T, true, 256, 1280><<<blocks, 256, 0, s>>>(a);
        else k_nl_build_tiled<T, false, 256, 1280><<<blocks, 256, 0, s>>>(a);
    } else if (tiled) {
        if (half) k_nl_build_tiled<T, true, kTileThreads, 2560><<<blocks, kTileThreads, 0, s>>>(a);
        else k_nl_build_tiled<T, false, kTileThreads, 2560><<<blocks, kTileThreads, 0, s>>>(a);
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

int64_t tile_blocks(const TileArgs &t) {
    return t.reps ? t.nbatch : (int64_t)t.ntile[0] * t.ntile[1] * t.ntile[2];
}

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
        case 1: return launch_t<1>(n, a, half, tiled, blocks, s);
        case 2: return launch_t<2>(n, a, half, tiled, blocks, s);
        case 3: return launch_t<3>(n, a, half, tiled, blocks, s);
        default: return launch_t<4>(n, a, half, tiled, blocks, s);
    }
}

hipError_t launch_nl_build_batch(int64_t n, const BatchView &b, int64_t nitems,
                                 const int32_t *cell_start, const int32_t *perm,
                                 const PairTab &tab, int half, const char *ws,
                                 const Workspace &w, uint32_t *neigh, int32_t *numneigh, int cap,
                                 int32_t *status, hipStream_t s) {
    if (n <= 0 || nitems <= 0) return hipSuccess;
    NlArgs a;
    std::memset(&a, 0, sizeof(a));
    a.t.cell_start = cell_start;
    a.t.perm = perm;
    a.pos = reinterpret_cast<const double4 *>(ws + w.pos);
    a.cap = cap;
    a.neigh = neigh;
    a.numneigh = numneigh;
    a.status = status;
    for (int k = 0; k < kTab; ++k) a.rnb2[k] = tab.rnb2[k];
    const unsigned blocks = (unsigned)nitems;
    switch (tab.ntypes) {
#define LJMD_BATCH_BUILD(TT)                                                        \
    case TT:                                                                        \
        if (half) k_nl_build_batch<TT, true><<<blocks, kNbThreads, 0, s>>>(a, b, nitems);  \
        else k_nl_build_batch<TT, false><<<blocks, kNbThreads, 0, s>>>(a, b, nitems);      \
        break;
        LJMD_BATCH_BUILD(1)
        LJMD_BATCH_BUILD(2)
        LJMD_BATCH_BUILD(3)
        LJMD_BATCH_BUILD(4)
#undef LJMD_BATCH_BUILD
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_nl_export(int64_t n, const TileArgs &t, int tiled, const void *neigh,
                            const int32_t *numneigh, int cap, uint32_t *out, int32_t *counts,
                            hipStream_t s, int kmajor) {
    if (n <= 0) return hipSuccess;
    const uint64_t *words = static_cast<const uint64_t *>(neigh);
    const uint32_t *idx = static_cast<const uint32_t *>(neigh);
    const unsigned gb = (unsigned)((n + kNbThreads - 1) / kNbThreads);
    if (tiled && kmajor)
        k_export_tiled<true><<<(unsigned)tile_blocks(t), kTileThreads, 0, s>>>(
            t, words, numneigh, cap, n, out, counts);
    else if (tiled)
        k_export_tiled<false><<<(unsigned)tile_blocks(t), kTileThreads, 0, s>>>(
            t, words, numneigh, cap, n, out, counts);
    else if (kmajor)
        k_export_global<true><<<gb, kNbThreads, 0, s>>>(n, idx, numneigh, cap, out, counts);
    else
        k_export_global<false><<<gb, kNbThreads, 0, s>>>(n, idx, numneigh, cap, out, counts);
    return hipGetLastError();
}

}  // namespace ljmd
