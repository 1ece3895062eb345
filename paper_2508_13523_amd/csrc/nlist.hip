// Verlet neighbor-list build over the cell-sorted atoms: one workgroup per
// strip of consecutive cells along x, the 27-cell stencil walked row by row
// with each stencil row staged through LDS.
//
// Sec. 4 of the paper: pair sums run over a neighbor list that is built and
// periodically updated.  Sec. 4.1: a full list holds every partner j of i in
// row i (each pair twice); a half list holds each pair once, here in row
// min(i, j).  The rows are interleaved across consecutive atoms (the GPU
// layout of Sec. 4.1) in blocks of one 64-lane wave.  Rows that would exceed
// the capacity are cut and the count needed is reported, in the spirit of
// the count / resize / fill pattern of Sec. 4.2.
//
// The distance test is FP64 with a fixed operation order so that the list
// is exactly reproducible: d = x_i - x_j, minimum image in branch form
// (d > L/2 -> d - L, d < -L/2 -> d + L), r^2 = fma(dz,dz, fma(dy,dy, dx*dx)),
// accepted when r^2 < (rc_ij + skin)^2.  The branch taken per dimension is
// stored with the entry (the image code) so the force kernels reproduce the
// same displacement without the comparisons.
#include "common.hpp"

namespace ljmd {

namespace {

constexpr int kNbThreads = 256;
constexpr int kChunk = 1024;     // stencil-row atoms staged in LDS at a time
constexpr int kMaxStrip = 30;    // home cells per workgroup

struct NlArgs {
    const double4 *pos;        // cell-sorted wrapped positions, w = type
    const int32_t *perm;       // cell-sorted position -> atom index
    const int32_t *cell_start; // [ncell + 1]
    Box box;
    Grid g;
    int strip;                 // home cells per strip
    int nstrips;               // strips per x row
    int cap;
    uint32_t *neigh;
    int32_t *numneigh;
    int32_t *status;
    double rnb2[kTab];
};

// SMALL: some dimension has fewer than 3 cells.  Its stencil is
// de-duplicated, so one staged cell can hold partners under either image and
// the image is chosen per candidate by the branch form.  Otherwise every
// staged cell has one image, fixed by whether its cell index wrapped around
// the box, and (x_i - x_j) - shift reproduces the branch form bit for bit on
// every pair inside the cutoff (both choices differ only when both displace-
// ments exceed a cell width, i.e. the cutoff).
template <int T, bool HALF, bool SMALL>
__global__ __launch_bounds__(kNbThreads) void k_nl_build(NlArgs a) {
    __shared__ double s_x[kChunk], s_y[kChunk], s_z[kChunk];
    __shared__ uint32_t s_id[kChunk];
    __shared__ int32_t s_cs[kMaxStrip + 2];
    __shared__ int32_t s_off[kMaxStrip + 3];
    __shared__ int32_t s_home[kMaxStrip + 1];
    __shared__ double s_rnb2[kTab];

    const int nx = a.g.nc[0], ny = a.g.nc[1], nz = a.g.nc[2];
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int sx = (int)(lb % a.nstrips);
    const int64_t rowid = lb / a.nstrips;
    const int cy = (int)(rowid % ny), cz = (int)(rowid / ny);
    const int cx0 = sx * a.strip;
    const int bs = min(a.strip, nx - cx0);
    const int64_t homebase = ((int64_t)cz * ny + cy) * nx;

    if (T > 1 && threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kTab; ++k) s_rnb2[k] = a.rnb2[k];
    }
    if ((int)threadIdx.x <= bs) s_home[threadIdx.x] = a.cell_start[homebase + cx0 + threadIdx.x];
    __syncthreads();
    const int32_t hs = s_home[0], he = s_home[bs];

    // stencil offsets, de-duplicated when a dimension has 1 or 2 cells
    const int ox_lo = nx >= 2 ? -1 : 0, ox_hi = nx >= 3 ? 1 : 0;
    const int oy_lo = ny >= 2 ? -1 : 0, oy_hi = ny >= 3 ? 1 : 0;
    const int oz_lo = nz >= 2 ? -1 : 0, oz_hi = nz >= 3 ? 1 : 0;
    const double Lx = a.box.L[0], Ly = a.box.L[1], Lz = a.box.L[2];
    const double hx_ = a.box.hL[0], hy_ = a.box.hL[1], hz_ = a.box.hL[2];

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
            ui = a.perm[s];
            while (hx + 1 < bs && s >= s_home[hx + 1]) ++hx;
        }
        for (int dz = oz_lo; dz <= oz_hi; ++dz) {
            const int zr = cz + dz;
            const int zz = (zr + nz) % nz;
            // image of this stencil row in z and y (used when !SMALL)
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
                    const int32_t c0 = a.cell_start[rb + xx], c1 = a.cell_start[rb + xx + 1];
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
                        s_id[q - lo] = (uint32_t)a.perm[gi] | ((uint32_t)(int)pq.w << 30);
                    }
                    __syncthreads();
                    if (!active) continue;
                    for (int ox = ox_lo; ox <= ox_hi; ++ox) {
                        const int t = hx + 1 + ox;
                        const int32_t b0 = max(s_off[t], lo) - lo;
                        const int32_t b1 = min(s_off[t + 1], hi) - lo;
                        const int xr = cx0 + hx + ox;
                        const double shx = xr < 0 ? -Lx : (xr >= nx ? Lx : 0.0);
                        const uint32_t cell_code = (xr < 0 ? 2u : (xr >= nx ? 1u : 0u)) | cdy | cdz;
                        for (int32_t q = b0; q < b1; ++q) {
                            uint32_t code;
                            double dx, dy2, dz2;
                            if (SMALL) {
                                code = 0;
                                dx = xi - s_x[q];
                                if (dx > hx_) {
                                    dx -= Lx;
                                    code = 1u;
                                } else if (dx < -hx_) {
                                    dx += Lx;
                                    code = 2u;
                                }
                                dy2 = yi - s_y[q];
                                if (dy2 > hy_) {
                                    dy2 -= Ly;
                                    code |= 4u;
                                } else if (dy2 < -hy_) {
                                    dy2 += Ly;
                                    code |= 8u;
                                }
                                dz2 = zi - s_z[q];
                                if (dz2 > hz_) {
                                    dz2 -= Lz;
                                    code |= 16u;
                                } else if (dz2 < -hz_) {
                                    dz2 += Lz;
                                    code |= 32u;
                                }
                            } else {
                                code = cell_code;
                                dx = (xi - s_x[q]) - shx;
                                dy2 = (yi - s_y[q]) - shy;
                                dz2 = (zi - s_z[q]) - shz;
                            }
                            const double rsq = fma(dz2, dz2, fma(dy2, dy2, dx * dx));
                            const uint32_t id = s_id[q];
                            const int32_t j = (int32_t)(id & 0x3FFFFFFFu);
                            const double cut2 = T > 1 ? s_rnb2[ti * T + (int)(id >> 30)] : a.rnb2[0];
                            bool ok = rsq < cut2 && j != ui;
                            if (HALF) ok = ok && j > ui;
                            if (ok) {
                                if (cnt < a.cap)
                                    a.neigh[nl_slot(ui, cnt, a.cap)] =
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

template <int T>
hipError_t launch_t(const NlArgs &a, int half, unsigned blocks, hipStream_t s) {
    const bool small = a.g.nc[0] < 3 || a.g.nc[1] < 3 || a.g.nc[2] < 3;
    if (small) {
        if (half)
            k_nl_build<T, true, true><<<blocks, kNbThreads, 0, s>>>(a);
        else
            k_nl_build<T, false, true><<<blocks, kNbThreads, 0, s>>>(a);
    } else {
        if (half)
            k_nl_build<T, true, false><<<blocks, kNbThreads, 0, s>>>(a);
        else
            k_nl_build<T, false, false><<<blocks, kNbThreads, 0, s>>>(a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_nl_build(int64_t n, const Box &box, const Grid &g, const PairTab &tab,
                           int half, int strip, char *ws, const Workspace &w, uint32_t *neigh,
                           int32_t *numneigh, int cap, int32_t *status, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    NlArgs a;
    a.pos = reinterpret_cast<const double4 *>(ws + w.pos);
    a.perm = reinterpret_cast<const int32_t *>(ws + w.perm);
    a.cell_start = reinterpret_cast<const int32_t *>(ws + w.cell_count);
    a.box = box;
    a.g = g;
    a.strip = strip < 1 ? 1 : (strip > kMaxStrip ? kMaxStrip : strip);
    if (a.strip > g.nc[0]) a.strip = g.nc[0];
    a.nstrips = (g.nc[0] + a.strip - 1) / a.strip;
    a.cap = cap;
    a.neigh = neigh;
    a.numneigh = numneigh;
    a.status = status;
    for (int k = 0; k < kTab; ++k) a.rnb2[k] = tab.rnb2[k];
    const int64_t blocks64 = (int64_t)a.nstrips * g.nc[1] * g.nc[2];
    const unsigned blocks = (unsigned)blocks64;
    switch (tab.ntypes) {
        case 1: return launch_t<1>(a, half, blocks, s);
        case 2: return launch_t<2>(a, half, blocks, s);
        case 3: return launch_t<3>(a, half, blocks, s);
        default: return launch_t<4>(a, half, blocks, s);
    }
}

}  // namespace ljmd
