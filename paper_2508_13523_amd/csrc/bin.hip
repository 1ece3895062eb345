// Cell binning by a stable counting sort (wrap -> cell id -> histogram ->
// exclusive scan -> scatter -> in-cell ranking), producing cell-sorted SoA
// copies of the wrapped positions for the neighbor build.
//
// The paper delegates list construction to LAMMPS (Sec. 4: the list is built
// and periodically updated); binning atoms into cells at least one neighbor
// cutoff wide, so that only the 27 surrounding cells can hold partners, is
// the textbook way to make that build O(n).
#include "common.hpp"

namespace ljmd {

namespace {

constexpr int kThreads = 256;

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t len, int32_t value) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < len) p[i] = value;
}

__global__ void k_fill_f64(double *__restrict__ p, int64_t len) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < len) p[i] = 0.0;
}

// Wrap one coordinate into [0, L): x < 0 -> x + L, x >= L -> x - L, and a
// result equal to L (rounding of a tiny negative x) becomes 0.
__device__ __forceinline__ double wrap1(double x, double L) {
    if (x < 0.0)
        x += L;
    else if (x >= L)
        x -= L;
    if (x == L) x = 0.0;
    return x;
}

__device__ __forceinline__ int cell_coord(double w, double cinv, int nc) {
    int c = (int)(w * cinv);
    c = c < 0 ? 0 : c;
    return c >= nc ? nc - 1 : c;
}

// Compute the cell of each atom (from its position wrapped into the box) and
// count the cell occupancy; the atomic's return value is a provisional slot.
// Atoms that are already in cell order (after a sort at the previous rebuild)
// come in runs of equal cells, so each run of equal cells inside a wave takes
// one atomic for the whole run and hands its members consecutive slots.
// With write_wrapped the wrapped positions are stored in x (and xref);
// otherwise the sort that follows writes them.  The block's positions are
// read and written through LDS so that every global access is contiguous.
// In a batch (reps != nullptr) each atom uses the box and cell grid of its
// own system, and the cell ids are offset into the batch-wide cell order.
// With disp_status, the list being replaced is checked first: status[2]
// becomes 1 if some atom has moved more than sqrt(disp_lim2) (half the skin)
// since that list's build, as recorded in xref (positions are not wrapped
// between builds, so x - xref is the displacement); two atoms may then have
// closed in from beyond the neighbor cutoff unseen.
__global__ __launch_bounds__(kThreads) void k_bin_count(double *__restrict__ x, int64_t n,
                                                        Box box, Grid g,
                                                        double *__restrict__ xref,
                                                        int32_t *__restrict__ cell_count,
                                                        int32_t *__restrict__ atom_cell,
                                                        int32_t *__restrict__ atom_slot,
                                                        const RepInfo *__restrict__ reps,
                                                        const int32_t *__restrict__ rid,
                                                        double disp_lim2,
                                                        int32_t *__restrict__ disp_status,
                                                        int write_wrapped) {
    __shared__ double s_x[3 * kThreads];
    __shared__ double s_r[3 * kThreads];
    const int64_t i0 = (int64_t)blockIdx.x * kThreads;
    const int64_t i = i0 + threadIdx.x;
    const int t = (int)threadIdx.x;
    const int m3 = 3 * (int)(n - i0 < kThreads ? n - i0 : kThreads);  // this block's doubles
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int e = k * kThreads + t;
        if (e < m3) {
            s_x[e] = x[3 * i0 + e];
            if (disp_status) s_r[e] = xref[3 * i0 + e];
        }
    }
    __syncthreads();
    const bool active = i < n;
    const int lane = (int)(threadIdx.x & 63);
    int32_t c = -1 - lane;  // distinct from every neighbor when inactive
    bool far = false;
    if (active) {
        int64_t base = 0;
        if (reps) {
            const RepInfo &r = reps[rid[i]];
            box = r.box;
            g = r.g;
            base = r.cell_base;
        }
        double w[3];
        double dsq = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double xd = s_x[3 * t + d];
            if (disp_status) {
                const double dd = xd - s_r[3 * t + d];
                dsq = fma(dd, dd, dsq);
            }
            w[d] = wrap1(xd, box.L[d]);
            s_x[3 * t + d] = w[d];  // only this thread reads these three
        }
        far = dsq > disp_lim2;
        const int cx = cell_coord(w[0], g.cinv[0], g.nc[0]);
        const int cy = cell_coord(w[1], g.cinv[1], g.nc[1]);
        const int cz = cell_coord(w[2], g.cinv[2], g.nc[2]);
        c = (int32_t)(base + ((int64_t)cz * g.nc[1] + cy) * g.nc[0] + cx);
        atom_cell[i] = c;
    }
    if (write_wrapped) {  // uniform
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int e = k * kThreads + t;
            if (e < m3) {
                x[3 * i0 + e] = s_x[e];
                if (xref) xref[3 * i0 + e] = s_x[e];
            }
        }
    }
    const int32_t prev = __shfl_up(c, 1, kWave);
    const bool head = lane == 0 || prev != c;
    const uint64_t heads = __ballot(head);
    // lanes 0..lane, and lanes above lane
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    const int first = 63 - __clzll(heads & upto);
    const uint64_t later = heads & ~upto;
    const int end = later ? __ffsll((unsigned long long)later) - 1 : kWave;
    int32_t base = 0;
    if (active && head) base = atomicAdd(&cell_count[c], end - first);
    base = __shfl(base, first, kWave);
    if (active) atom_slot[i] = base + (lane - first);
    // one flag update per block, and none once the flag is already raised
    // (disp_status is uniform, so every thread reaches the block-wide or)
    if (disp_status && __syncthreads_or(far) && threadIdx.x == 0 &&
        __hip_atomic_load(&disp_status[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
        atomicOr(&disp_status[2], 1);
}

// The box of atom i (its own system's in a batch).
__device__ __forceinline__ const double *box_of(const Box &box, const RepInfo *reps,
                                               const int32_t *rid, int64_t i) {
    return reps ? reps[rid[i]].box.L : box.L;
}

// ---- exclusive scan of int32 counts: block sums, top-level scan, down-sweep ----

__global__ __launch_bounds__(kThreads) void k_scan_reduce(const int32_t *__restrict__ a,
                                                          int64_t len,
                                                          int32_t *__restrict__ bsum) {
    __shared__ int32_t s[kThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanItems + threadIdx.x * 4;
    int32_t v = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + k < len) v += a[base + k];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int k = 0; k < kThreads / kWave; ++k) t += s[k];
        bsum[blockIdx.x] = t;
    }
}

// Block-wide exclusive scan of one value per thread (1024 threads).
__device__ int32_t block_exclusive_scan_1024(int32_t v, int32_t *s_wave, int32_t *total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int32_t incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t o = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += o;
    }
    if (lane == 63) s_wave[wv] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
            const int32_t t = s_wave[k];
            s_wave[k] = run;
            run += t;
        }
        *total = run;
    }
    __syncthreads();
    return incl - v + s_wave[wv];
}

__global__ __launch_bounds__(1024) void k_scan_top(int32_t *__restrict__ bsum, int64_t nb) {
    __shared__ int32_t s_wave[16];
    __shared__ int32_t s_total;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t lo = threadIdx.x * per;
    int32_t local = 0;
    for (int64_t k = lo; k < lo + per && k < nb; ++k) local += bsum[k];
    int32_t run = block_exclusive_scan_1024(local, s_wave, &s_total);
    for (int64_t k = lo; k < lo + per && k < nb; ++k) {
        const int32_t t = bsum[k];
        bsum[k] = run;
        run += t;
    }
}

__global__ __launch_bounds__(kThreads) void k_scan_down(int32_t *__restrict__ a, int64_t len,
                                                        const int32_t *__restrict__ bsum) {
    __shared__ int32_t s_wave[kThreads / kWave];
    __shared__ int32_t s_total;
    const int64_t base = (int64_t)blockIdx.x * kScanItems + threadIdx.x * 4;
    int32_t v[4];
    int32_t t = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = (base + k < len) ? a[base + k] : 0;
        t += v[k];
    }
    // block scan over 256 threads
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int32_t incl = t;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t o = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += o;
    }
    if (lane == 63) s_wave[wv] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int k = 0; k < kThreads / kWave; ++k) {
            const int32_t u = s_wave[k];
            s_wave[k] = run;
            run += u;
        }
        s_total = run;
    }
    __syncthreads();
    int32_t run = incl - t + s_wave[wv] + bsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (base + k < len) a[base + k] = run;
        run += v[k];
    }
}

// Provisional cell-sorted order (the atomics' slots), with each atom's
// wrapped x beside it for the in-cell ranking (wrapping is the identity on
// positions already wrapped).
__global__ __launch_bounds__(kThreads) void k_bin_scatter(int64_t n, const double *__restrict__ x,
                                                          Box box, const RepInfo *__restrict__ reps,
                                                          const int32_t *__restrict__ rid,
                                                          const int32_t *__restrict__ atom_cell,
                                                          const int32_t *__restrict__ atom_slot,
                                                          const int32_t *__restrict__ cell_start,
                                                          int32_t *__restrict__ tmp,
                                                          double *__restrict__ tmpx) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const int32_t q = cell_start[atom_cell[i]] + atom_slot[i];
    tmp[q] = (int32_t)i;
    tmpx[q] = wrap1(x[3 * i], box_of(box, reps, rid, i)[0]);
}

// Order inside each cell: ascending (wrapped) x, ties by atom index, so the
// cells of one grid row, taken in order, are sorted along x (the neighbor
// build cuts each stencil row to the x window a home atom can reach).  An
// atom's final slot is the cell start plus the number of cell-mates that
// precede it.  Also writes the cell-sorted copy of the positions with the
// type in w.  A block stages the (atom, x) pairs of the cells its positions
// fall in (at most kRankSpan of them; more only when cells hold hundreds of
// atoms, and then the cell-mates are read from global memory).
constexpr int kRankSpan = 2048;

__global__ __launch_bounds__(kThreads) void k_bin_finalize(
    int64_t n, const double *__restrict__ x, Box box, const RepInfo *__restrict__ reps,
    const int32_t *__restrict__ rid, const int32_t *__restrict__ type,
    const int32_t *__restrict__ atom_cell, const int32_t *__restrict__ cell_start,
    const int32_t *__restrict__ tmp, const double *__restrict__ tmpx,
    int32_t *__restrict__ perm, double4 *__restrict__ pos) {
    __shared__ int32_t s_a[kRankSpan];
    __shared__ double s_x[kRankSpan];
    const int64_t p0 = (int64_t)blockIdx.x * kThreads;
    const int64_t p = p0 + threadIdx.x;
    const int64_t p1 = p0 + kThreads < n ? p0 + kThreads : n;  // p0 < n: grid from n
    // positions are in provisional cell order, so the cells of [p0, p1)
    // cover the positions [lo, hi)
    const int32_t lo = cell_start[atom_cell[tmp[p0]]];
    const int32_t hi = cell_start[atom_cell[tmp[p1 - 1]] + 1];
    const bool staged = hi - lo <= kRankSpan;
    if (staged) {
        for (int32_t q = lo + (int32_t)threadIdx.x; q < hi; q += kThreads) {
            s_a[q - lo] = tmp[q];
            s_x[q - lo] = tmpx[q];
        }
    }
    __syncthreads();
    if (p >= n) return;
    const int32_t a = tmp[p];
    const int32_t c = atom_cell[a];
    const int32_t s = cell_start[c], e = cell_start[c + 1];
    const double xa = tmpx[p];
    int32_t rank = 0;
    if (staged) {
        for (int32_t q = s - lo; q < e - lo; ++q) {
            const int32_t b = s_a[q];
            const double xb = s_x[q];
            rank += (xb < xa || (xb == xa && b < a)) ? 1 : 0;
        }
    } else {
        for (int32_t q = s; q < e; ++q) {
            const int32_t b = tmp[q];
            const double xb = tmpx[q];
            rank += (xb < xa || (xb == xa && b < a)) ? 1 : 0;
        }
    }
    const int32_t d = s + rank;
    perm[d] = a;
    const double *L = box_of(box, reps, rid, a);
    pos[d] = make_double4(wrap1(x[3 * (int64_t)a], L[0]), wrap1(x[3 * (int64_t)a + 1], L[1]),
                          wrap1(x[3 * (int64_t)a + 2], L[2]), type ? (double)type[a] : 0.0);
}

// Atom sorting, step 1: gather velocity, type and id into cell order.
__global__ __launch_bounds__(kThreads) void k_sort_gather(int64_t n,
                                                          const int32_t *__restrict__ perm,
                                                          const double *__restrict__ v,
                                                          const int32_t *__restrict__ type,
                                                          const int32_t *__restrict__ id,
                                                          double *__restrict__ sv,
                                                          int32_t *__restrict__ stype,
                                                          int32_t *__restrict__ sid) {
    const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (s >= n) return;
    const int64_t a = perm[s];
#pragma unroll
    for (int d = 0; d < 3; ++d) sv[3 * s + d] = v[3 * a + d];
    if (type) stype[s] = type[a];
    if (id) sid[s] = id[a];
}

// Atom sorting, step 2: write the cell-ordered state back (positions come
// from the sorted copy of the wrapped positions), make the permutation the
// identity and record the build positions.
__global__ __launch_bounds__(kThreads) void k_sort_commit(
    int64_t n, const double4 *__restrict__ pos, const double *__restrict__ sv,
    const int32_t *__restrict__ stype, const int32_t *__restrict__ sid, double *__restrict__ x,
    double *__restrict__ v, int32_t *__restrict__ type, int32_t *__restrict__ id,
    int32_t *__restrict__ perm, double *__restrict__ xref) {
    const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (s >= n) return;
    const double4 p = pos[s];
    x[3 * s] = p.x;
    x[3 * s + 1] = p.y;
    x[3 * s + 2] = p.z;
    if (xref) {
        xref[3 * s] = p.x;
        xref[3 * s + 1] = p.y;
        xref[3 * s + 2] = p.z;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) v[3 * s + d] = sv[3 * s + d];
    if (type) type[s] = stype[s];
    if (id) id[s] = sid[s];
    perm[s] = (int32_t)s;
}

inline unsigned blocks_for(int64_t len, int per) { return (unsigned)((len + per - 1) / per); }

}  // namespace

hipError_t launch_sort(int64_t n, double *x, double *v, int32_t *type, int32_t *id, double *xref,
                       int32_t *perm, char *ws, const Workspace &w, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const double4 *pos = reinterpret_cast<const double4 *>(ws + w.pos);
    double *sv = reinterpret_cast<double *>(ws + w.sort_v);
    int32_t *stype = reinterpret_cast<int32_t *>(ws + w.sort_i);
    int32_t *sid = stype + n;
    k_sort_gather<<<blocks_for(n, kThreads), kThreads, 0, s>>>(n, perm, v, type, id, sv, stype, sid);
    k_sort_commit<<<blocks_for(n, kThreads), kThreads, 0, s>>>(n, pos, sv, stype, sid, x, v, type,
                                                               id, perm, xref);
    return hipGetLastError();
}

hipError_t launch_set_i32(int32_t *p, int64_t len, int32_t value, hipStream_t s) {
    if (len <= 0) return hipSuccess;
    k_fill_i32<<<blocks_for(len, kThreads), kThreads, 0, s>>>(p, len, value);
    return hipGetLastError();
}

hipError_t launch_zero_i32(int32_t *p, int64_t len, hipStream_t s) {
    return launch_set_i32(p, len, 0, s);
}

hipError_t launch_zero_f64(double *p, int64_t len, hipStream_t s) {
    if (len <= 0) return hipSuccess;
    k_fill_f64<<<blocks_for(len, kThreads), kThreads, 0, s>>>(p, len);
    return hipGetLastError();
}

hipError_t launch_bin(double *x, const int32_t *type, int64_t n, const Box &box, const Grid &g,
                      double *xref, char *ws, const Workspace &w, int32_t *cell_count,
                      int32_t *perm, hipStream_t s, const RepInfo *reps, const int32_t *rid,
                      int64_t ncell_total, double disp_lim2, int32_t *disp_status,
                      bool sorting) {
    if (!xref) disp_status = nullptr;
    int32_t *bsum = reinterpret_cast<int32_t *>(ws + w.scan_bsum);
    int32_t *atom_cell = reinterpret_cast<int32_t *>(ws + w.atom_cell);
    int32_t *atom_slot = reinterpret_cast<int32_t *>(ws + w.atom_slot);
    int32_t *tmp = reinterpret_cast<int32_t *>(ws + w.tmp);
    double4 *pos = reinterpret_cast<double4 *>(ws + w.pos);
    const int64_t len = (reps ? ncell_total : g.ncell) + 1;  // the extra element becomes the total
    hipError_t e = launch_zero_i32(cell_count, len, s);
    if (e != hipSuccess) return e;
    if (n > 0) {
        k_bin_count<<<blocks_for(n, kThreads), kThreads, 0, s>>>(x, n, box, g, xref, cell_count,
                                                                 atom_cell, atom_slot, reps, rid,
                                                                 disp_lim2, disp_status,
                                                                 sorting ? 0 : 1);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int64_t nb = (len + kScanItems - 1) / kScanItems;
    k_scan_reduce<<<(unsigned)nb, kThreads, 0, s>>>(cell_count, len, bsum);
    k_scan_top<<<1, 1024, 0, s>>>(bsum, nb);
    k_scan_down<<<(unsigned)nb, kThreads, 0, s>>>(cell_count, len, bsum);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (n > 0) {
        // the in-cell ranking's copy of x lives in the sorting buffer, which
        // is free until the binning is done
        double *tmpx = reinterpret_cast<double *>(ws + w.sort_v);
        k_bin_scatter<<<blocks_for(n, kThreads), kThreads, 0, s>>>(
            n, x, box, reps, rid, atom_cell, atom_slot, cell_count, tmp, tmpx);
        k_bin_finalize<<<blocks_for(n, kThreads), kThreads, 0, s>>>(
            n, x, box, reps, rid, type, atom_cell, cell_count, tmp, tmpx, perm, pos);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace ljmd
