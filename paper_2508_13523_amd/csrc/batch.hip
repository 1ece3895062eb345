// Batches of independent periodic systems: the device plan (per-system box,
// cell grid, offsets into the batch-wide cell order and build work items),
// the system of every atom, and per-system thermo sums.
//
// The systems of a batch share the force field; each has its own box.  The
// plan mirrors the host's arithmetic exactly (same IEEE operations), so the
// host can size buffers and grids from its own copy of the offsets and boxes
// while the kernels read the device table.
#include "tile.hpp"

namespace ljmd {

namespace {

constexpr int kPlanThreads = 1024;
constexpr int kThreads = 256;

// Block-wide exclusive scan of one int64 per thread (blockDim.x threads, a
// multiple of 64); also returns the block total.
__device__ int64_t block_scan_i64(int64_t v, int64_t *s_wave, int64_t *total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t incl = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int64_t o = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += o;
    }
    if (lane == 63) s_wave[wv] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
            const int64_t t = s_wave[k];
            s_wave[k] = run;
            run += t;
        }
        *total = run;
    }
    __syncthreads();
    const int64_t r = incl - v + s_wave[wv];
    __syncthreads();
    return r;
}

// One workgroup: systems in chunks of 1024 with running cell and item bases.
__global__ __launch_bounds__(kPlanThreads) void k_batch_plan(int32_t nrep,
                                                             const int64_t *__restrict__ off,
                                                             const double *__restrict__ boxes,
                                                             double max_rnb, int tile_atoms,
                                                             RepInfo *__restrict__ reps) {
    __shared__ int64_t s_wave[kPlanThreads / kWave];
    __shared__ int64_t s_total;
    int64_t cell_carry = 0, item_carry = 0, tile_carry = 0;
    for (int32_t c0 = 0; c0 < nrep; c0 += kPlanThreads) {
        const int32_t r = c0 + (int32_t)threadIdx.x;
        RepInfo ri;
        int64_t ncell = 0, items = 0, tiles = 0;
        if (r < nrep) {
            ri.g.ncell = 1;
            ri.small = 0;
            for (int d = 0; d < 3; ++d) {
                const double L = boxes[3 * r + d];
                ri.box.L[d] = L;
                ri.box.hL[d] = 0.5 * L;
                int nc = (int)floor(L / (max_rnb * (1.0 + 1e-12)));
                if (nc < 1) nc = 1;
                ri.g.nc[d] = nc;
                ri.g.cinv[d] = nc / L;
                ri.g.ncell *= nc;
                if (nc < 3) ri.small = 1;
            }
            ri.atom_base = off[r];
            ri.natoms = off[r + 1] - off[r];
            const double mean = (double)ri.natoms / (double)ri.g.ncell;
            const int b = batch_strip(mean, ri.g.nc[0], tile_atoms);
            ri.strip = b;
            ri.nstripx = (ri.g.nc[0] + b - 1) / b;
            ri.ey = batch_tile_rows(mean, b, ri.g.nc[1], tile_atoms);
            ncell = ri.g.ncell;
            items = (int64_t)ri.nstripx * ri.g.nc[1] * ri.g.nc[2];
            tiles = (int64_t)ri.nstripx * ((ri.g.nc[1] + ri.ey - 1) / ri.ey) * ri.g.nc[2];
        }
        const int64_t cb = block_scan_i64(ncell, s_wave, &s_total);
        const int64_t ctot = s_total;
        const int64_t ib = block_scan_i64(items, s_wave, &s_total);
        const int64_t itot = s_total;
        const int64_t tb = block_scan_i64(tiles, s_wave, &s_total);
        const int64_t ttot = s_total;
        if (r < nrep) {
            ri.cell_base = cell_carry + cb;
            ri.item_base = item_carry + ib;
            ri.tile_base = tile_carry + tb;
            reps[r] = ri;
        }
        cell_carry += ctot;
        item_carry += itot;
        tile_carry += ttot;
    }
}

// System of every atom: one workgroup per system writes its atoms' entries.
__global__ __launch_bounds__(kThreads) void k_batch_rid(const int64_t *__restrict__ off,
                                                        int32_t *__restrict__ rid) {
    const int32_t r = (int32_t)blockIdx.x;
    const int64_t a1 = off[r + 1];
    for (int64_t i = off[r] + threadIdx.x; i < a1; i += kThreads) rid[i] = r;
}

// System of every tile of the tiled batch list: the last r with
// reps[r].tile_base <= b.
__global__ __launch_bounds__(kThreads) void k_batch_tile_rep(int64_t ntiles,
                                                             const RepInfo *__restrict__ reps,
                                                             int32_t nrep,
                                                             int32_t *__restrict__ tile_rep) {
    const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (b >= ntiles) return;
    int lo = 0, hi = nrep - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (reps[mid].tile_base <= b) lo = mid;
        else hi = mid - 1;
    }
    tile_rep[b] = lo;
}

// One workgroup per system: E and W from the per-atom arrays (each already
// holding half of every pair term), KE = sum m v^2 / 2, in a fixed order: each
// thread sums its strided share of the system's atoms for all eight values in
// one pass, then the block adds the threads' partial sums (wave butterflies,
// then the waves in order).
// rows[r] = [step, E, KE, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz] when rows != nullptr;
// ev_out[r] = [E, W...] when ev_out != nullptr.
__global__ __launch_bounds__(kThreads) void k_batch_thermo(const RepInfo *__restrict__ reps,
                                                           const double *__restrict__ v,
                                                           const int32_t *__restrict__ type,
                                                           double m0, double m1, double m2,
                                                           double m3,
                                                           const double *__restrict__ ev_atom,
                                                           int64_t n, int64_t step,
                                                           double *__restrict__ rows,
                                                           double *__restrict__ ev_out) {
    __shared__ double s[kThreads / kWave][8];
    const RepInfo &r = reps[blockIdx.x];
    const int64_t a0 = r.atom_base, a1 = r.atom_base + r.natoms;
    double t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = a0 + threadIdx.x; i < a1; i += kThreads) {
        if (ev_atom) {
#pragma unroll
            for (int k = 0; k < 7; ++k) t[k] += ev_atom[k * n + i];
        }
        if (v) {
            const int ty = type ? type[i] : 0;
            const double m = ty == 0 ? m0 : (ty == 1 ? m1 : (ty == 2 ? m2 : m3));
            const double vx = v[3 * i], vy = v[3 * i + 1], vz = v[3 * i + 2];
            t[7] += 0.5 * m * (vx * vx + vy * vy + vz * vz);
        }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) t[k] = wave_sum(t[k]);
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) s[threadIdx.x >> 6][k] = t[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double out[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            double u = 0.0;
            for (int w = 0; w < kThreads / kWave; ++w) u += s[w][k];
            out[k] = u;
        }
        if (rows) {
            double *row = rows + 9 * (int64_t)blockIdx.x;
            row[0] = (double)step;
            row[1] = out[0];
            row[2] = out[7];
            for (int k = 1; k < 7; ++k) row[2 + k] = out[k];
        }
        if (ev_out)
            for (int k = 0; k < 7; ++k) ev_out[7 * (int64_t)blockIdx.x + k] = out[k];
    }
}

// flag[0] becomes 1 if some cell-order position does not hold its own atom
// (the caller zeroes it first).
__global__ __launch_bounds__(kThreads) void k_perm_identity(const int32_t *__restrict__ perm,
                                                            int64_t n, int32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const bool bad = i < n && perm[i] != (int32_t)i;
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

}  // namespace

hipError_t launch_perm_identity(const int32_t *perm, int64_t n, int32_t *flag, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_perm_identity<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(perm, n, flag);
    return hipGetLastError();
}

hipError_t launch_batch_plan(int32_t nrep, const int64_t *offsets, const double *boxes,
                             double max_rnb, int tile_atoms, RepInfo *reps, int32_t *rid, int64_t n,
                             int32_t *tile_rep, int64_t ntiles, hipStream_t s) {
    k_batch_plan<<<1, kPlanThreads, 0, s>>>(nrep, offsets, boxes, max_rnb, tile_atoms, reps);
    if (n > 0) k_batch_rid<<<(unsigned)nrep, kThreads, 0, s>>>(offsets, rid);
    if (ntiles > 0 && tile_rep)
        k_batch_tile_rep<<<(unsigned)((ntiles + kThreads - 1) / kThreads), kThreads, 0, s>>>(
            ntiles, reps, nrep, tile_rep);
    return hipGetLastError();
}

hipError_t launch_batch_thermo(const BatchView &b, const double *v, const int32_t *type,
                               const double *mass, int ntypes, const double *ev_atom, int64_t n,
                               int64_t step, double *rows, double *ev_out, hipStream_t s) {
    if (b.nrep <= 0) return hipSuccess;
    double m[4] = {0, 0, 0, 0};
    for (int t = 0; t < ntypes && t < 4; ++t) m[t] = mass ? mass[t] : 0.0;
    k_batch_thermo<<<(unsigned)b.nrep, kThreads, 0, s>>>(b.reps, v, ntypes > 1 ? type : nullptr,
                                                         m[0], m[1], m[2], m[3], ev_atom, n, step,
                                                         rows, ev_out);
    return hipGetLastError();
}

}  // namespace ljmd
